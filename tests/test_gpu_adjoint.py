"""Adjoint of the 2D stream-function advance against the oracle's
complex-step derivatives, the transpose identity of each step, checkpointing
invariance, the autograd wrappers, and central finite differences at the
1024^2, 200-step size."""
import numpy as np
import pytest

import oracle
import paper_0905_3409_amd as pkg
from paper_0905_3409_amd import inputs

pytestmark = pytest.mark.gpu

NC = (37, 29)
LO, HI = (0.0, 0.0), (1.0, 1.0)


def _grid(dtype, mixed=pkg.MIXED_CENTRAL, ncell=NC):
    return pkg.Grid(ncell, LO, HI, dtype=dtype, mixed=mixed)


def _case(seed, nmodes=8, vmax=1.5):
    rng = np.random.default_rng(seed)
    params = inputs.stream_modes(rng, nmodes, NC, vmax)
    phi, psi = inputs.sdf_union(inputs.node_grid(NC), [[0.45, 0.5], [0.7, 0.35]], [0.2, 0.12])
    return params, phi, psi


def _lam_to_dense(g, lam):
    return np.concatenate([g._grid_view(lam[a]).cpu().numpy().ravel() for a in range(3)])


def _lam_from_dense(g, dense):
    import torch
    lam = g.empty_adjoint()
    n = g.num_nodes
    for a in range(3):
        g._grid_view(lam[a]).copy_(torch.from_numpy(
            np.ascontiguousarray(dense[a * n:(a + 1) * n].reshape(g.nodes[1], g.nodes[0]))))
    return lam


def _dense_state(g, st):
    phi, psi = g.to_numpy(st)
    return np.concatenate([phi, psi])


# FP32: each entry of M du is rounded to FP32 once as stored (u/2 of the
# entry) after a few roundings inside the Hermite sums, each relative to the
# sum of the magnitudes of its terms. For random data those terms do not
# cancel, so their magnitudes are of the size of the entry, and both errors
# stay within a few u of the scale sum |lam| |M du| used below: 8 u bounds
# the relative difference (measured about 2e-9, the roundings of different
# entries cancelling).
U32 = 2.0 ** -24


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 8 * U32)])
@pytest.mark.parametrize("mixed,ncell,dt", [(pkg.MIXED_CENTRAL, NC, 0.03),
                                            (pkg.MIXED_ZERO, NC, 0.03),
                                            (pkg.MIXED_CENTRAL, (150, 140), 0.08)])
def test_adjoint_step_is_the_transpose_of_the_step(dtype, tol, mixed, ncell, dt):
    """<lam, M du> = <M^T lam, du> for random du and lam: the step is linear
    in the state, and the adjoint step must be its exact transpose. The last
    case moves feet up to about 18 cells, so blocks whose feet spread beyond
    the scatter's LDS tile take the direct path."""
    import torch
    params, _, _ = _case(21)
    g = _grid(dtype, mixed, ncell)
    g.set_velocity(pkg.STREAM_SIN, params, 1.3)
    rng = np.random.default_rng(22)
    n = g.num_nodes
    du = rng.normal(size=3 * n)
    lam = rng.normal(size=3 * n)
    st = g.from_numpy(du[:n], du[n:])
    du32 = _dense_state(g, st)  # the state as stored (rounded for FP32)
    t = 0.2
    out = st.clone()
    g.advance(out, t, dt, 1)
    torch.cuda.synchronize()
    Mdu = _dense_state(g, out)
    lam_prev, _ = g.adjoint_step(st, t, dt, _lam_from_dense(g, lam))
    torch.cuda.synchronize()
    lhs = float(lam @ Mdu)
    rhs = float(_lam_to_dense(g, lam_prev) @ du32)
    scale = float(np.abs(lam) @ np.abs(Mdu))
    print(f"{dtype} mixed={mixed}: <lam, M du> {lhs:.12e} <M^T lam, du> {rhs:.12e} "
          f"rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= tol * scale


@pytest.mark.parametrize("mixed,period", [(pkg.MIXED_CENTRAL, 0.0), (pkg.MIXED_CENTRAL, 1.3),
                                          (pkg.MIXED_ZERO, 0.0)])
def test_step_parameter_derivative_matches_oracle(mixed, period):
    """d/dS <lam, M(u; S)> for one step, FP64, against the oracle's complex
    step."""
    import torch
    params, phi, psi = _case(23)
    g = _grid("float64", mixed)
    g.set_velocity(pkg.STREAM_SIN, params, period)
    n = g.num_nodes
    lam = np.random.default_rng(24).normal(size=3 * n)
    t, dt = 0.15, 0.025
    st = g.from_numpy(phi, psi)
    _, dS = g.adjoint_step(st, t, dt, _lam_from_dense(g, lam))
    torch.cuda.synchronize()
    gpu = dS.cpu().numpy().reshape(4, 4)
    _, ref = oracle.grad_cs(NC, LO, HI, params, period, phi, psi, t, dt, 1, lam=lam,
                            mixed_mode=mixed)
    err = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
    print(f"mixed={mixed} period={period}: max|dF/dS| {np.max(np.abs(ref)):.3e}, rel err {err:.2e}")
    assert err <= 1e-10


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_step_parameter_derivative_is_deterministic(dtype):
    """The 16 parameter partials are summed in a fixed order (lane swaps and
    row sums within a wave, the waves and then the blocks in order): the
    same step twice gives the same bits."""
    import torch
    params, phi, psi = _case(26)
    g = _grid(dtype, ncell=(150, 140))
    g.set_velocity(pkg.STREAM_SIN, params, 1.3)
    lam = _lam_from_dense(g, np.random.default_rng(27).normal(size=3 * g.num_nodes))
    st = g.from_numpy(np.resize(phi, g.num_nodes), np.resize(psi, 2 * g.num_nodes))
    _, a = g.adjoint_step(st, 0.1, 0.03, lam)
    _, b = g.adjoint_step(st, 0.1, 0.03, lam)
    torch.cuda.synchronize()
    assert torch.count_nonzero(a).item() == 16
    assert torch.equal(a, b)


def _loss_case(seed=25, steps=11):
    params, phi, psi = _case(seed)
    tgt_params = params.copy()
    tgt_params[0::3] *= 1.4
    t0, dt = 0.0, 0.02
    tphi, _ = oracle.advance(2, NC, LO, HI, oracle.STREAM_SIN, tgt_params, 0.0, phi, psi, t0, dt,
                             steps)
    return params, phi, psi, tphi, t0, dt, steps, 1.5 / NC[0]


def _gpu_loss_grad(dtype, params, phi, psi, tphi, t0, dt, steps, eps, every):
    import torch
    g = _grid(dtype)
    g.set_velocity(pkg.STREAM_SIN, params, 0.0)
    st = g.from_numpy(phi, psi)
    ref = g.from_numpy(tphi, np.zeros(2 * tphi.size))
    ckpt = g.advance_save(st, t0, dt, steps, every)
    loss, lam = g.shape_loss(st, ref, eps)
    dS = g.adjoint(ckpt, t0, dt, steps, every, lam)
    torch.cuda.synchronize()
    return g, loss, dS.cpu().numpy().reshape(4, 4), lam


def test_loss_gradient_matches_oracle():
    """11 steps in checkpoint segments of 4, 4 and 3: loss and dL/dS in FP64
    against the oracle's complex-step derivative of its own advance."""
    params, phi, psi, tphi, t0, dt, steps, eps = _loss_case()
    _, loss, gpu, _ = _gpu_loss_grad("float64", params, phi, psi, tphi, t0, dt, steps, eps, 4)
    val, ref = oracle.grad_cs(NC, LO, HI, params, 0.0, phi, psi, t0, dt, steps, phi_target=tphi,
                              eps=eps)
    err = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
    print(f"loss gpu {loss:.15e} oracle {val:.15e}; max|dL/dS| {np.max(np.abs(ref)):.3e} "
          f"rel err {err:.2e}")
    assert abs(loss - val) <= 1e-12 * abs(val)
    assert err <= 1e-9


def test_checkpoint_spacing_does_not_change_the_result():
    params, phi, psi, tphi, t0, dt, steps, eps = _loss_case(seed=26)
    runs = [_gpu_loss_grad("float64", params, phi, psi, tphi, t0, dt, steps, eps, every)
            for every in (1, 3, 11, 50)]
    g0, l0, d0, lam0 = runs[0]
    for g, loss, d, lam in runs[1:]:
        assert loss == l0
        assert np.max(np.abs(d - d0)) <= 1e-13 * np.max(np.abs(d0))
        a, b = _lam_to_dense(g0, lam0), _lam_to_dense(g, lam)
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_initial_state_adjoint_is_the_transpose_of_the_advance():
    """<lam_T, A du_0> = <lam_0, du_0>, A the (linear) 11-step advance."""
    import torch
    params, phi, psi, tphi, t0, dt, steps, eps = _loss_case(seed=27)
    g, _, _, lam0 = _gpu_loss_grad("float64", params, phi, psi, tphi, t0, dt, steps, eps, 4)
    # lam_T again (the sweep overwrote it)
    st = g.from_numpy(phi, psi)
    g.advance(st, t0, dt, steps)
    _, lamT = g.shape_loss(st, g.from_numpy(tphi, np.zeros(2 * tphi.size)), eps)
    n = g.num_nodes
    du = np.random.default_rng(28).normal(size=3 * n)
    sd = g.from_numpy(du[:n], du[n:])
    g.advance(sd, t0, dt, steps)
    torch.cuda.synchronize()
    lhs = float(_lam_to_dense(g, lamT) @ _dense_state(g, sd))
    rhs = float(_lam_to_dense(g, lam0) @ du)
    print(f"<lam_T, A du> {lhs:.12e} <lam_0, du> {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-300)


def test_fp32_gradient_is_close_to_fp64():
    params, phi, psi, tphi, t0, dt, steps, eps = _loss_case(seed=29)
    _, l64, d64, _ = _gpu_loss_grad("float64", params, phi, psi, tphi, t0, dt, steps, eps, 4)
    _, l32, d32, _ = _gpu_loss_grad("float32", params, phi, psi, tphi, t0, dt, steps, eps, 4)
    err = np.max(np.abs(d32 - d64)) / np.max(np.abs(d64))
    print(f"loss fp32 {l32:.9e} fp64 {l64:.9e}; gradient rel diff {err:.2e}")
    assert abs(l32 - l64) <= 1e-4 * abs(l64)
    assert err <= 1e-3


def test_autograd_matches_the_direct_calls_and_finite_differences():
    import torch
    from paper_0905_3409_amd.autograd import ShapeLoss, StreamAdvance
    params, phi, psi, tphi, t0, dt, steps, eps = _loss_case(seed=30)
    modes = params.reshape(-1, 3)[:, 1:].astype(np.int64)
    g = _grid("float64")
    st0 = g.from_numpy(phi, psi)
    ref = g.from_numpy(tphi, np.zeros(2 * tphi.size))

    def loss_of(amps):
        uT = StreamAdvance.apply(amps, st0, g, modes, 0.0, t0, dt, steps, 5)
        return ShapeLoss.apply(uT, ref, g, eps)

    amps = torch.tensor(params[0::3], dtype=torch.float64, requires_grad=True)
    L = loss_of(amps)
    L.backward()
    _, _, direct, _ = _gpu_loss_grad("float64", params, phi, psi, tphi, t0, dt, steps, eps, 5)
    want = direct[modes[:, 0] - 1, modes[:, 1] - 1]
    got = amps.grad.numpy()
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    with torch.no_grad():
        for k in range(len(params) // 3):
            d = 1e-6
            e = torch.zeros_like(amps)
            e[k] = d
            fd = (float(loss_of(amps + e)) - float(loss_of(amps - e))) / (2 * d)
            assert abs(fd - got[k]) <= 1e-6 * np.max(np.abs(got)), (k, fd, got[k])


def test_full_size_gradient_matches_central_differences():
    """1024^2 cells, 16 modes, 200 steps with checkpoints every 20, FP64:
    dL/da_k from the reverse sweep against central differences with
    delta_k = 1e-5 max(|a_k|, 1e-2); the FP32 forward's gradient beside it."""
    import torch
    w = inputs.adjoint_circles()
    modes, amps, steps, dt, eps = w["modes"], w["amps"], w["steps"], w["dt"], w["eps"]
    from paper_0905_3409_amd.autograd import stream_params

    def run(dtype, a, target_state=None, grad=False):
        g = _grid(dtype, ncell=w["ncell"])
        g.set_velocity(pkg.STREAM_SIN, stream_params(a, modes), 0.0)
        st = g.from_numpy(w["phi0"], w["psi0"])
        if target_state is None:
            g.advance(st, 0.0, dt, steps)
            return g, st
        if not grad:
            g.advance(st, 0.0, dt, steps)
            return g.shape_loss(st, target_state, eps, with_grad=False)[0], None
        ckpt = g.advance_save(st, 0.0, dt, steps, 20)
        loss, lam = g.shape_loss(st, target_state, eps)
        dS = g.adjoint(ckpt, 0.0, dt, steps, 20, lam)
        torch.cuda.synchronize()
        return loss, dS.cpu().numpy()[4 * (modes[:, 0] - 1) + (modes[:, 1] - 1)]

    print("full size: target run", flush=True)
    _, tgt64 = run("float64", w["target_amps"])
    loss, grad = run("float64", amps, tgt64, grad=True)
    print(f"loss {loss:.6e}, |dL/da| max {np.max(np.abs(grad)):.3e}", flush=True)
    fd = np.zeros_like(grad)
    for k in range(len(amps)):
        d = 1e-5 * max(abs(amps[k]), 1e-2)
        ap, am = amps.copy(), amps.copy()
        ap[k] += d
        am[k] -= d
        fd[k] = (run("float64", ap, tgt64)[0] - run("float64", am, tgt64)[0]) / (2 * d)
    err = np.max(np.abs(fd - grad)) / np.max(np.abs(grad))
    print(f"adjoint vs central differences: rel err {err:.2e}", flush=True)
    _, tgt32 = run("float32", w["target_amps"])
    loss32, grad32 = run("float32", amps, tgt32, grad=True)
    err32 = np.max(np.abs(grad32 - grad)) / np.max(np.abs(grad))
    print(f"FP32 forward: loss {loss32:.6e}, gradient rel diff to FP64 {err32:.2e}", flush=True)
    assert err <= 1e-4
    assert err32 <= 2e-2
