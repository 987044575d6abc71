"""The paper's variants on the GPU against the oracle: cell-based cross
derivatives (approach B, sec. 2.3) and Heun's gradient update (sec. 4), in
every kernel family (generic 2D/3D, stream-function, point evaluation,
batch, adjoint)."""
import zlib

import numpy as np
import pytest

import oracle
import paper_0905_3409_amd as pkg
from gpu_util import TOL64, U32, fp32_tolerances, gpu_advance, oracle_advance, rel, rel_psi
from paper_0905_3409_amd import inputs
from test_gpu_step import CASES_2D, CASES_3D, _random_smooth_state

pytestmark = pytest.mark.gpu

MODES = [(pkg.MIXED_CELL, pkg.PSI_SUPERCONSISTENT), (pkg.MIXED_CENTRAL, pkg.PSI_HEUN),
         (pkg.MIXED_CELL, pkg.PSI_HEUN)]


@pytest.mark.parametrize("mixed,psi", MODES)
@pytest.mark.parametrize("name,kind,params,period,dt,steps", CASES_2D)
def test_fp64_2d_variants(name, kind, params, period, dt, steps, mixed, psi):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    ncell, lo, hi = (37, 29), (-0.1, 0.05), (1.15, 0.95)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    print(f"case {name} mixed={mixed} psi={psi}", flush=True)
    args = (2, ncell, lo, hi, kind, params, period, phi0, psi0, 0.1, dt, steps)
    g = gpu_advance(*args, dtype="float64", mixed=mixed, psi=psi)
    o = oracle_advance(*args, mixed=mixed, psi=psi)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(2))
    print(f"  phi {rel(g[0], o[0]):.2e} psi/scale {rel_psi(g[1], o[1], o[0], hmin):.2e}")
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


@pytest.mark.parametrize("mixed,psi", MODES)
@pytest.mark.parametrize("name,kind,params,period,dt,steps", CASES_3D)
def test_fp64_3d_variants(name, kind, params, period, dt, steps, mixed, psi):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    ncell, lo, hi = (13, 11, 9), (0.0, -0.05, 0.1), (1.0, 1.0, 0.95)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    print(f"case 3d {name} mixed={mixed} psi={psi}", flush=True)
    args = (3, ncell, lo, hi, kind, params, period, phi0, psi0, 0.0, dt, steps)
    g = gpu_advance(*args, dtype="float64", mixed=mixed, psi=psi)
    o = oracle_advance(*args, mixed=mixed, psi=psi)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(3))
    print(f"  phi {rel(g[0], o[0]):.2e} psi/scale {rel_psi(g[1], o[1], o[0], hmin):.2e}")
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


@pytest.mark.parametrize("mixed,psi", MODES)
@pytest.mark.parametrize("n", [160, 512])
def test_fp32_stream_variants(mixed, psi, n):
    """FP32 stream-function kernel (Taylor stages, and for Heun grad v at the
    foot from the node's jet) against the FP64 oracle; n = 512 mixes the
    Taylor and exact branches."""
    w = inputs.stream_circles(seed=5, n=n, steps=n // 2)
    steps = 3
    args = (2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
            w["phi0"], w["psi0"], 0.0, w["dt"], steps)
    g = gpu_advance(*args, dtype="float32", mixed=mixed, psi=psi)
    o = oracle_advance(*args, mixed=mixed, psi=psi)
    tp, tg = fp32_tolerances(o[0], o[1], 1 / n, steps)
    ep, eg = rel(g[0], o[0]), rel(g[1], o[1])
    print(f"fp32 n={n} mixed={mixed} psi={psi}: phi {ep:.2e} (tol {tp:.1e}) "
          f"psi {eg:.2e} (tol {tg:.1e})")
    assert ep <= tp and eg <= tg


@pytest.mark.parametrize("mixed,psi", MODES)
def test_fp64_stream_kernel_variants(mixed, psi):
    """The FP64 stream-function kernel (tables, exact stages) with the
    variants, 2 steps at 160^2 against the oracle."""
    w = inputs.stream_circles(seed=6, n=160, steps=80)
    args = (2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
            w["phi0"], w["psi0"], 0.0, w["dt"], 2)
    g = gpu_advance(*args, dtype="float64", mixed=mixed, psi=psi)
    o = oracle_advance(*args, mixed=mixed, psi=psi)
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], 1 / 160) <= TOL64


@pytest.mark.parametrize("dim,ncell", [(2, (45, 38)), (3, (17, 14, 19))])
def test_eval_points_cell_based(dim, ncell):
    import torch
    rng = np.random.default_rng(40 + dim)
    coords = inputs.node_grid(ncell)
    phi, psi = inputs.sdf_union(coords, rng.uniform(0.3, 0.7, (3, dim)), rng.uniform(0.1, 0.2, 3))
    pts = rng.uniform(-0.05, 1.05, (5000, dim))
    g = pkg.Grid(ncell, dtype="float64", mixed=pkg.MIXED_CELL)
    st = g.from_numpy(phi, psi)
    val, nrm, cur = g.eval_points(st, pts)
    torch.cuda.synchronize()
    o = oracle.eval_points(dim, ncell, np.zeros(dim), np.ones(dim), phi, psi, pts,
                           mixed_mode=oracle.MIXED_CELL)
    assert rel(val.cpu().numpy(), o["val"]) <= TOL64
    ok = np.linalg.norm(o["grad"], axis=1) > 1e-3
    assert rel(cur.cpu().numpy()[ok], o["kappa"][ok]) <= 1e-10


def test_batch_cell_based_equals_single_grids():
    import torch
    sizes = [(20, 20), (33, 47), (70, 41), (130, 64), (9, 200), (300, 120)]
    w = inputs.batched_stream_circles(seed=41, steps=64, sizes=sizes)
    b = pkg.Batch([p["ncell"] for p in w["problems"]], dtype="float32", mixed=pkg.MIXED_CELL)
    for k, p in enumerate(w["problems"]):
        b.set_velocity(k, w["kind"], p["params"], w["period"])
    b.set_tiles((16, 0, 64, 32))
    st = b.from_numpy([(p["phi0"], p["psi0"]) for p in w["problems"]])
    b.advance(st, 0.0, w["dt"], 3)
    torch.cuda.synchronize()
    for k, p in enumerate(w["problems"]):
        g = pkg.Grid(p["ncell"], dtype="float32", mixed=pkg.MIXED_CELL)
        g.set_velocity(w["kind"], p["params"], w["period"])
        s1 = g.from_numpy(p["phi0"], p["psi0"])
        g.advance(s1, 0.0, w["dt"], 3)
        torch.cuda.synchronize()
        a, c = b.to_numpy(st, k), g.to_numpy(s1)
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), k


def test_adjoint_cell_based_matches_oracle():
    """Transpose identity and the 8-step loss gradient with (B)."""
    import torch
    from test_gpu_adjoint import _dense_state, _lam_from_dense, _lam_to_dense
    NC, LO, HI = (37, 29), (0.0, 0.0), (1.0, 1.0)
    rng = np.random.default_rng(42)
    params = inputs.stream_modes(rng, 8, NC, 1.5)
    g = pkg.Grid(NC, LO, HI, dtype="float64", mixed=pkg.MIXED_CELL)
    g.set_velocity(pkg.STREAM_SIN, params, 0.0)
    n = g.num_nodes
    du, lam = rng.normal(size=3 * n), rng.normal(size=3 * n)
    st = g.from_numpy(du[:n], du[n:])
    out = st.clone()
    g.advance(out, 0.1, 0.03, 1)
    lam_prev, _ = g.adjoint_step(st, 0.1, 0.03, _lam_from_dense(g, lam))
    torch.cuda.synchronize()
    lhs, rhs = float(lam @ _dense_state(g, out)), float(_lam_to_dense(g, lam_prev) @ du)
    assert abs(lhs - rhs) <= 1e-12 * float(np.abs(lam) @ np.abs(_dense_state(g, out)))
    phi, psi = inputs.sdf_union(inputs.node_grid(NC), [[0.45, 0.5], [0.7, 0.35]], [0.2, 0.12])
    tgt_params = params.copy()
    tgt_params[0::3] *= 1.4
    steps, dt, eps = 8, 0.02, 1.5 / NC[0]
    tphi, _ = oracle.advance(2, NC, LO, HI, oracle.STREAM_SIN, tgt_params, 0.0, phi, psi, 0.0,
                             dt, steps, mixed_mode=oracle.MIXED_CELL)
    st = g.from_numpy(phi, psi)
    ckpt = g.advance_save(st, 0.0, dt, steps, 3)
    loss, lamT = g.shape_loss(st, g.from_numpy(tphi, np.zeros(2 * tphi.size)), eps)
    dS = g.adjoint(ckpt, 0.0, dt, steps, 3, lamT)
    torch.cuda.synchronize()
    val, ref = oracle.grad_cs(NC, LO, HI, params, 0.0, phi, psi, 0.0, dt, steps,
                              phi_target=tphi, eps=eps, mixed_mode=oracle.MIXED_CELL)
    err = np.max(np.abs(dS.cpu().numpy().reshape(4, 4) - ref)) / np.max(np.abs(ref))
    print(f"(B) loss {loss:.12e} oracle {val:.12e}, dL/dS rel err {err:.2e}")
    assert abs(loss - val) <= 1e-12 * abs(val)
    assert err <= 1e-9


def test_heun_changes_phi_by_far_less_than_a_tenth_of_a_percent():
    """The paper's remark on Heun's method, on the GPU: vortex in a box,
    64^2, T = 2 (128 steps), FP64."""
    n = 64
    coords = inputs.node_grid((n, n))
    phi, psi = inputs.gaussian_bump(coords, (0.5, 0.75))
    args = (2, (n, n), (0.0, 0.0), (1.0, 1.0), inputs.VORTEX, np.zeros(0), 2.0, phi, psi, 0.0,
            1.0 / n, 2 * n)
    sc = gpu_advance(*args, dtype="float64")
    he = gpu_advance(*args, dtype="float64", psi=pkg.PSI_HEUN)
    d = np.abs(sc[0] - he[0]).max() / np.abs(phi).max()
    print(f"max |phi_heun - phi_sc| / max |phi| = {d:.2e}")
    assert 0 < d < 1e-3
