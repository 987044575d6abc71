"""The step at the largest grids the library accepts: square and cubic grids
whose state planes (rows padded to 64 nodes) are just under the 2 GiB a plane
may hold, so that the kernels' 32-bit byte offsets, tile counts and node-index
divisions run at the top of their range.

* the stream-function step (2D, the benchmark's kernel) and the
  vector-potential step (3D): windows at the corners of the grid (the
  highest and lowest addresses) and at its centre against the oracle, run on
  the window alone with the same node coordinates and data; nodes closer than
  a margin to a window side inside the domain are not compared, as the
  oracle's window has a boundary there that the full grid has not;
* properties of the whole output: every value finite and the row padding
  never written;
* the generic 2D step with v dt an integer number of cells: an exact shift of
  the data at every node, checked bit for bit on the device;
* the same on the longest thin 3D grid (64 x 3 nodes per plane, as many
  planes as a plane of state may hold), where the 3D kernels' estimate of a
  node's z-plane meets its largest quotients;
* a batch whose state spans more than 4 GiB (two of the largest grids around
  a small one): every problem bit for bit equal to the same grid advanced
  alone, for each wave shape of the tile list.
"""
import numpy as np
import pytest

import oracle
import paper_0905_3409_amd as pkg
from gpu_util import TOL64, fp32_tolerances, rel, rel_psi
from helpers import PLANE_LIMIT, interior_mask, largest_ncell, windows
from paper_0905_3409_amd import inputs

pytestmark = pytest.mark.gpu


def _fill(views, F, dF):
    """The separable state into dense device views (phi, psi_x, psi_y[, psi_z]),
    products in the generator's order."""
    import torch
    dim = len(F)
    dev = views[0].device
    f = [torch.from_numpy(F[a]).to(dev) for a in range(dim)]
    df = [torch.from_numpy(dF[a]).to(dev) for a in range(dim)]
    for a in range(1 + dim):
        fs = f if a == 0 else [df[b] if b == a - 1 else f[b] for b in range(dim)]
        v = fs[1][:, None] * fs[0][None, :]
        if dim == 3:
            v = fs[2][:, None, None] * v[None, :, :]
        views[a].copy_(v)
        del v


def _fill_state(g, F, dF):
    st = g.empty_state()
    _fill([g._grid_view(st[a]) for a in range(1 + g.dim)], F, dF)
    return st


def _whole_output_checks(g, st):
    import torch
    assert bool(torch.isfinite(st).all())
    pad = st.view(1 + g.dim, -1, g.pitch)[:, :, g.nodes[0]:]
    assert pad.numel() == 0 or not bool(pad.any())  # padding still as allocated (zero)


def _window_parity(g, st, ncell, axes, F, dF, kind, params, period, dt, steps, dtype, margin):
    dim = len(ncell)
    n_nodes = ncell[0] + 1
    m = 48 if dim == 2 else 16
    for win in windows(n_nodes, m, dim):
        print(f"window {win}", flush=True)
        lo_w = [axes[a][win[a][0]] for a in range(dim)]
        hi_w = [axes[a][win[a][1] - 1] for a in range(dim)]
        phi_w, psi_w = inputs.separable_dense(F, dF, win)
        op, og = oracle.advance(dim, (m,) * dim, lo_w, hi_w, kind, params, period, phi_w, psi_w,
                                0.0, dt, steps)
        sl = tuple(slice(*w) for w in reversed(win))
        gp = g._grid_view(st[0])[sl].double().cpu().numpy().ravel()
        gg = np.concatenate([g._grid_view(st[1 + a])[sl].double().cpu().numpy().ravel()
                             for a in range(dim)])
        keep = interior_mask(win, n_nodes, margin)
        kp = np.tile(keep, dim)
        if dtype == "float64":
            ep = rel(gp[keep], op[keep])
            eg = rel_psi(gg[kp], og[kp], op[keep], 1.0 / ncell[0])
            assert ep <= TOL64 and eg <= TOL64, (win, ep, eg)
        else:
            tp, tg = fp32_tolerances(phi_w, psi_w, 1.0 / ncell[0], steps)
            ep, eg = rel(gp[keep], op[keep]), rel(gg[kp], og[kp])
            print(f"  phi {ep:.2e} (tol {tp:.1e}) psi {eg:.2e} (tol {tg:.1e})", flush=True)
            assert ep <= tp and eg <= tg, (win, ep, eg)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_stream_step_at_the_largest_2d_grid(dtype):
    """Two stream-function steps (one into the workspace, one back into the
    caller's state) on the largest square grid of the precision."""
    import torch
    es = 4 if dtype == "float32" else 8
    n = largest_ncell(2, es)
    ncell = (n, n)
    print(f"case stream 2D {dtype} ncell {n}", flush=True)
    params = inputs.stream_modes(np.random.default_rng(11), 8, (256, 256), 1.0)
    dt, steps = 0.8 / n, 2
    F, dF = inputs.separable_sines(12, ncell)
    axes = inputs.node_axes(ncell)
    g = pkg.Grid(ncell, dtype=dtype)
    assert g.plane * es < PLANE_LIMIT
    g.set_velocity(inputs.STREAM_SIN, params, 2.0)
    st = _fill_state(g, F, dF)
    g.advance(st, 0.0, dt, steps)
    torch.cuda.synchronize()
    _whole_output_checks(g, st)
    _window_parity(g, st, ncell, axes, F, dF, inputs.STREAM_SIN, params, 2.0, dt, steps, dtype,
                   margin=8)


def test_vecpot_step_at_the_largest_3d_grid():
    """One vector-potential step on the largest FP32 cube."""
    import torch
    n = largest_ncell(3, 4)
    ncell = (n, n, n)
    print(f"case vecpot 3D float32 ncell {n}", flush=True)
    params = inputs.vecpot_modes(np.random.default_rng(13), 6, (32, 32, 32), 1.0)
    dt = 0.9 / n
    F, dF = inputs.separable_sines(14, ncell)
    axes = inputs.node_axes(ncell)
    g = pkg.Grid(ncell, dtype="float32")
    assert g.plane * 4 < PLANE_LIMIT
    g.set_velocity(inputs.VECPOT_SIN, params, 3.0)
    st = _fill_state(g, F, dF)
    g.advance(st, 0.0, dt, 1)
    torch.cuda.synchronize()
    _whole_output_checks(g, st)
    _window_parity(g, st, ncell, axes, F, dF, inputs.VECPOT_SIN, params, 3.0, dt, 1, "float32",
                   margin=4)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("k,axis", [(1, 0), (2, 1)])
def test_integer_shift_at_the_largest_2d_grid(dtype, k, axis):
    """v dt = k h with h, dt powers of two (the ratios of the small-grid
    shift test): the foot of every node is a node, xi = 0, and the step
    shifts arbitrary data exactly (sec. 5.4, xi = 1 case) at all interior
    nodes of the largest grid."""
    import torch
    es = 4 if dtype == "float32" else 8
    n = largest_ncell(2, es)
    ncell = (n, n)
    print(f"case shift {dtype} ncell {n} k {k} axis {axis}", flush=True)
    h, dt = 2.0 ** -15, 2.0 ** -14
    hi = (n * h, n * h)
    F, dF = inputs.separable_sines(15, ncell, (0.0, 0.0), hi)
    g = pkg.Grid(ncell, (0.0, 0.0), hi, dtype=dtype)
    vel = np.zeros(2)
    vel[axis] = k * h / dt
    g.set_velocity(inputs.AFFINE, inputs.affine_params(vel, [0, 0], np.zeros((2, 2))), 0.0)
    st = _fill_state(g, F, dF)
    ref = st.clone()
    g.advance(st, 0.0, dt, 1)
    torch.cuda.synchronize()
    _whole_output_checks(g, st)
    for a in range(3):
        new, old = g._grid_view(st[a]), g._grid_view(ref[a])
        if axis == 0:
            assert torch.equal(new[:, k:], old[:, :-k])
        else:
            assert torch.equal(new[k:, :], old[:-k, :])


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("k,axis", [(1, 2), (2, 0)])
def test_integer_shift_on_the_longest_thin_3d_grid(dtype, k, axis):
    """The 3D step on 64 x 3 nodes per z-plane and as many planes as a 2 GiB
    state plane holds (2.8 M in FP32, 1.4 M in FP64). Each XCD's band of a
    plane is then 24 nodes, so a thread finds its plane as id / 24 with id
    up to 6.7e7 and the quotient up to 2^21.4: the largest quotients the
    kernels' FP32 estimate of that division meets, and one correction must
    still make it exact. v dt = k h with h, dt powers of two, so the step is
    an exact shift of arbitrary data at every interior node."""
    import torch
    es = 4 if dtype == "float32" else 8
    nz = (PLANE_LIMIT - 1) // (64 * 3 * es)  # nodes along z
    ncell = (63, 2, nz - 1)
    print(f"case thin 3D shift {dtype} ncell {ncell} k {k} axis {axis}", flush=True)
    h, dt = 2.0 ** -15, 2.0 ** -14
    hi = tuple(c * h for c in ncell)
    F, dF = inputs.separable_sines(18, ncell, (0.0, 0.0, 0.0), hi)
    g = pkg.Grid(ncell, (0.0, 0.0, 0.0), hi, dtype=dtype)
    assert g.pitch == 64 and g.plane * es < PLANE_LIMIT
    vel = np.zeros(3)
    vel[axis] = k * h / dt
    g.set_velocity(inputs.AFFINE, inputs.affine_params(vel, [0, 0, 0], np.zeros((3, 3))), 0.0)
    st = _fill_state(g, F, dF)
    ref = st.clone()
    g.advance(st, 0.0, dt, 1)
    torch.cuda.synchronize()
    _whole_output_checks(g, st)
    for a in range(4):
        new, old = g._grid_view(st[a]), g._grid_view(ref[a])  # (z, y, x)
        if axis == 0:
            assert torch.equal(new[:, :, k:], old[:, :, :-k]), a
        else:
            assert torch.equal(new[k:], old[:-k]), a


@pytest.mark.parametrize("dtype,widths", [("float32", (64, 64, 64, 64)),
                                          ("float32", (0, 0, 0, 0)),
                                          ("float32", (16, 16, 16, 16)),
                                          ("float64", (32, 32, 32, 32))])
def test_batch_beyond_4_gib_equals_single_grids(dtype, widths):
    """The third problem's planes start past 4 GiB into the batch state
    (64-bit problem offsets, 32-bit offsets within a plane); two steps, the
    second read back from the workspace."""
    import torch
    es = 4 if dtype == "float32" else 8
    n = largest_ncell(2, es)
    ncells = [(n, n), (700, 1000), (n, n)]
    print(f"case batch {dtype} widths {widths} ncells {ncells}", flush=True)
    b = pkg.Batch(ncells, dtype=dtype)
    b.set_tiles(widths)
    assert int(b.offset[2]) * es > 2 ** 32
    rng = np.random.default_rng(16)
    params = [inputs.stream_modes(rng, 8, (256, 256), 1.0) for _ in ncells]
    dt, steps = 0.8 / n, 2
    fields = [inputs.separable_sines(17 + p, ncells[p]) for p in range(len(ncells))]
    st = b.empty_state()
    for p in range(len(ncells)):
        b.set_velocity(p, inputs.STREAM_SIN, params[p], 2.0)
        _fill(b._views(st, p), *fields[p])
    b.advance(st, 0.0, dt, steps)
    torch.cuda.synchronize()
    for p in range(len(ncells)):
        print(f"  problem {p} against a single grid", flush=True)
        g = pkg.Grid(ncells[p], dtype=dtype)
        g.set_velocity(inputs.STREAM_SIN, params[p], 2.0)
        sg = _fill_state(g, *fields[p])
        assert not torch.equal(b._views(st, p)[0], g._grid_view(sg[0]))  # the batch moved it
        g.advance(sg, 0.0, dt, steps)
        torch.cuda.synchronize()
        for a, v in enumerate(b._views(st, p)):
            assert torch.equal(v, g._grid_view(sg[a])), (p, a)
        del g, sg
