"""GPU step parity against the FP64 oracle at sizes the oracle finishes in
seconds: several 256-thread blocks, ragged rows (node counts that are not
multiples of 64), every velocity field, both cross-derivative modes, CFL
numbers above 1 and feet outside the domain."""
import zlib

import numpy as np
import pytest

import oracle
import paper_0905_3409_amd as pkg
from gpu_util import TOL64, fp32_tolerances, gpu_advance, oracle_advance, rel, rel_psi
from paper_0905_3409_amd import inputs

pytestmark = pytest.mark.gpu


def _random_smooth_state(rng, ncell, lo, hi):
    coords = inputs.node_grid(ncell, lo, hi)
    dim = len(ncell)
    x0 = [lo[a] + (hi[a] - lo[a]) * rng.uniform(0.3, 0.7) for a in range(dim)]
    phi, psi = inputs.gaussian_bump(coords, x0)
    # plus a random perturbation: the step is linear in the data, so parity
    # must hold for arbitrary (not only consistent) phi and psi
    phi = phi + 0.01 * rng.normal(size=phi.shape)
    psi = psi + 0.01 * rng.normal(size=psi.shape)
    return phi, psi


CASES_2D = [
    # name, kind, params, period, dt, steps
    ("rotation_shear_cfl2.5", inputs.AFFINE,
     inputs.affine_params([0.1, -0.05], [0.4, 0.55], [[0.3, -6.0], [5.0, -0.3]]), 0.0, 0.02, 7),
    ("stream_modulated", inputs.STREAM_SIN,
     np.array([0.05, 1, 3, -0.03, 4, 2, 0.02, 2, 2, 0.04, 3, 1, -0.01, 1, 1]), 1.5, 0.03, 6),
    ("vortex", inputs.VORTEX, np.zeros(0), 2.0, 0.04, 5),
    ("pseudo1d", inputs.PSEUDO1D, np.zeros(0), 0.0, 0.02, 5),
]


@pytest.mark.parametrize("mixed", [pkg.MIXED_CENTRAL, pkg.MIXED_ZERO])
@pytest.mark.parametrize("name,kind,params,period,dt,steps", CASES_2D)
def test_fp64_2d_parity(name, kind, params, period, dt, steps, mixed):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    ncell, lo, hi = (37, 29), (-0.1, 0.05), (1.15, 0.95)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    print(f"case {name} mixed={mixed}", flush=True)
    g = gpu_advance(2, ncell, lo, hi, kind, params, period, phi0, psi0, 0.1, dt, steps,
                    "float64", mixed)
    o = oracle_advance(2, ncell, lo, hi, kind, params, period, phi0, psi0, 0.1, dt, steps, mixed)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(2))
    print(f"  phi {rel(g[0], o[0]):.2e} psi {rel(g[1], o[1]):.2e} "
          f"psi/scale {rel_psi(g[1], o[1], o[0], hmin):.2e}")
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


def test_fp64_stream_both_stage_branches():
    """FP64 stream-function kernel with offsets |pi d| from about 0 to 0.4:
    stage angles by angle addition where |pi d| <= 0.1, sincospi beyond;
    both against the oracle."""
    rng = np.random.default_rng(31)
    ncell, lo, hi = (41, 37), (-0.1, 0.05), (1.15, 0.95)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    params = np.array([0.5, 1, 2, -0.3, 2, 1, 0.2, 3, 3])
    v = oracle.max_speed(2, ncell, lo, hi, inputs.STREAM_SIN, params, 0.0, 0.0)
    dt = 0.4 / (np.pi * v)  # the fastest nodes move 0.4 / pi: beyond the series' range
    args = (2, ncell, lo, hi, inputs.STREAM_SIN, params, 0.0, phi0, psi0, 0.0, dt, 4)
    g = gpu_advance(*args, dtype="float64")
    o = oracle_advance(*args)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(2))
    print(f"fp64 stream, max |pi d| 0.4: phi {rel(g[0], o[0]):.2e} "
          f"psi/scale {rel_psi(g[1], o[1], o[0], hmin):.2e}")
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


def test_fp32_stream_all_stage_branches():
    """FP32 stream-function kernel with offsets |pi d| from about 0 to 0.4:
    Taylor stages where k |d| <= 0.03, the modal sum with angles by angle
    addition where |pi d| <= 0.25, sincospi beyond; against the oracle."""
    rng = np.random.default_rng(32)
    ncell, lo, hi = (41, 37), (-0.1, 0.05), (1.15, 0.95)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    params = np.array([0.5, 1, 2, -0.3, 2, 1, 0.2, 3, 3])
    v = oracle.max_speed(2, ncell, lo, hi, inputs.STREAM_SIN, params, 0.0, 0.0)
    dt = 0.4 / (np.pi * v)
    steps = 4
    args = (2, ncell, lo, hi, inputs.STREAM_SIN, params, 0.0, phi0, psi0, 0.0, dt, steps)
    g = gpu_advance(*args, dtype="float32")
    o = oracle_advance(*args)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(2))
    tp, tg = fp32_tolerances(o[0], o[1], hmin, steps)
    ep, eg = rel(g[0], o[0]), rel(g[1], o[1])
    print(f"fp32 stream, max |pi d| 0.4: phi {ep:.2e} (tol {tp:.2e}) psi {eg:.2e} (tol {tg:.2e})")
    assert ep <= tp and eg <= tg


CASES_3D = [
    ("affine", inputs.AFFINE,
     inputs.affine_params([0.05, 0.0, -0.1], [0.5, 0.5, 0.5],
                          [[0.2, -4.0, 0.5], [4.0, 0.1, -0.3], [0.2, 0.6, -0.3]]), 0.0, 0.03, 4),
    ("vecpot", inputs.VECPOT_SIN,
     np.array([0.05, -0.01, 0.02, 1, 3, 2, -0.02, 0.04, 0.01, 4, 2, 1, 0.03, 0.02, -0.02, 2, 2, 3]),
     3.0, 0.05, 3),
    ("leveque", inputs.LEVEQUE3D, np.zeros(0), 2.5, 0.04, 3),
]


@pytest.mark.parametrize("mixed", [pkg.MIXED_CENTRAL, pkg.MIXED_ZERO])
@pytest.mark.parametrize("name,kind,params,period,dt,steps", CASES_3D)
def test_fp64_3d_parity(name, kind, params, period, dt, steps, mixed):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    ncell, lo, hi = (13, 11, 9), (0.0, -0.05, 0.1), (1.0, 1.0, 0.95)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    print(f"case 3d {name} mixed={mixed}", flush=True)
    g = gpu_advance(3, ncell, lo, hi, kind, params, period, phi0, psi0, 0.0, dt, steps,
                    "float64", mixed)
    o = oracle_advance(3, ncell, lo, hi, kind, params, period, phi0, psi0, 0.0, dt, steps, mixed)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(3))
    print(f"  phi {rel(g[0], o[0]):.2e} psi {rel(g[1], o[1]):.2e} "
          f"psi/scale {rel_psi(g[1], o[1], o[0], hmin):.2e}")
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


@pytest.mark.parametrize("ncell", [(2, 2, 40), (5, 3, 7), (31, 2, 9), (3, 17, 2)])
@pytest.mark.parametrize("name,kind,params,period,dt,steps", CASES_3D[:2])
def test_fp64_3d_parity_thin_grids(name, kind, params, period, dt, steps, ncell):
    """Grids whose planes hold few nodes: each XCD's eighth of a plane is a
    node or two, part of a row, or spans rows; every node still updated once
    (the oracle at every node)."""
    rng = np.random.default_rng(zlib.crc32((name + str(ncell)).encode()))
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    print(f"case 3d {name} {ncell}", flush=True)
    g = gpu_advance(3, ncell, lo, hi, kind, params, period, phi0, psi0, 0.0, dt, steps,
                    "float64")
    o = oracle_advance(3, ncell, lo, hi, kind, params, period, phi0, psi0, 0.0, dt, steps)
    hmin = min((hi[a] - lo[a]) / ncell[a] for a in range(3))
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


def test_rotation_circle_full_run_fp64():
    """The 64^2 rotating circle: one revolution in 128 steps (CFL up to 2.2 at
    the corners), every node against the oracle."""
    w = inputs.rotation_circle(seed=11)
    args = (2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
            w["phi0"], w["psi0"], 0.0, w["dt"], w["steps"])
    g = gpu_advance(*args, dtype="float64")
    o = oracle_advance(*args)
    print(f"  phi {rel(g[0], o[0]):.2e} psi {rel(g[1], o[1]):.2e}")
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], 1 / 64) <= TOL64
    # the Neumann treatment keeps the corners bounded
    assert np.abs(g[0]).max() <= 1.01 * np.abs(w["phi0"]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_extrapolation_boundary_parity(dim):
    """The extrapolating boundary treatment, with feet up to ~1.5 cells out."""
    rng = np.random.default_rng(21 + dim)
    ncell = (23, 19) if dim == 2 else (12, 10, 11)
    lo, hi = (0.0,) * dim, (1.0,) * dim
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    A = rng.normal(size=(dim, dim)) * 2.0
    params = inputs.affine_params(rng.normal(size=dim), [0.5] * dim, A)
    args = (dim, ncell, lo, hi, inputs.AFFINE, params, 0.0, phi0, psi0, 0.0, 0.04, 3)
    g = gpu_advance(*args, dtype="float64", bc=pkg.BC_EXTRAPOLATE)
    o = oracle_advance(*args, bc=pkg.BC_EXTRAPOLATE)
    hmin = 1 / max(ncell)
    assert rel(g[0], o[0]) <= TOL64
    assert rel_psi(g[1], o[1], o[0], hmin) <= TOL64


@pytest.mark.parametrize("dim", [2, 3])
def test_minimal_grid(dim):
    """ncell = 2 per axis: every cell touches both boundaries."""
    rng = np.random.default_rng(7 + dim)
    ncell = (2,) * dim
    lo, hi = (0.0,) * dim, (1.0,) * dim
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    A = rng.normal(size=(dim, dim))
    params = inputs.affine_params(rng.normal(size=dim) * 0.3, [0.5] * dim, A)
    args = (dim, ncell, lo, hi, inputs.AFFINE, params, 0.0, phi0, psi0, 0.0, 0.1, 3)
    g = gpu_advance(*args, dtype="float64")
    o = oracle_advance(*args)
    assert rel(g[0], o[0]) <= TOL64 and rel_psi(g[1], o[1], o[0], 0.5) <= TOL64


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("k,axis", [(1, 0), (2, 1), (3, 0)])
def test_integer_shift_bit_exact(dtype, k, axis):
    """v dt = k h exactly: the foot is a node, xi = 0, and the scheme is an
    exact shift of arbitrary data (sec. 5.4, xi = 1 case) on interior nodes."""
    rng = np.random.default_rng(90 + k)
    n = 70  # 71 nodes per row: two 64-wide chunks, ragged
    ncell = (n, 40)
    h, dt = 1.0 / 64, 1.0 / 32
    lo, hi = (0.0, 0.0), (n * h, 40 * h)
    npdt = np.float32 if dtype == "float32" else np.float64
    phi = rng.normal(size=(n + 1) * 41).astype(npdt).astype(np.float64)
    psi = rng.normal(size=2 * (n + 1) * 41).astype(npdt).astype(np.float64)
    vel = np.zeros(2)
    vel[axis] = k * h / dt
    params = inputs.affine_params(vel, [0, 0], np.zeros((2, 2)))
    ph, ps = gpu_advance(2, ncell, lo, hi, inputs.AFFINE, params, 0.0, phi, psi, 0.0, dt, 1,
                         dtype)
    P = phi.reshape(41, n + 1)
    S = psi.reshape(2, 41, n + 1)
    PH = ph.reshape(41, n + 1)
    SH = ps.reshape(2, 41, n + 1)
    if axis == 0:
        np.testing.assert_array_equal(PH[:, k:], P[:, :-k])
        np.testing.assert_array_equal(SH[:, :, k:], S[:, :, :-k])
    else:
        np.testing.assert_array_equal(PH[k:, :], P[:-k, :])
        np.testing.assert_array_equal(SH[:, k:, :], S[:, :-k, :])


def test_split_advance_equals_single_advance():
    """advance(3) then advance(2) from t0 + 3 dt is bitwise advance(5): times
    are computed from t0 + n dt, odd step counts copy back from the workspace,
    and the kernels are deterministic."""
    import torch
    w = inputs.stream_circles(seed=3, n=96, steps=64)
    for dtype in ("float64", "float32"):
        g = pkg.Grid(w["ncell"], dtype=dtype)
        g.set_velocity(w["kind"], w["params"], w["period"])
        a = g.from_numpy(w["phi0"], w["psi0"])
        b = g.from_numpy(w["phi0"], w["psi0"])
        g.advance(a, 0.0, w["dt"], 5)
        g.advance(b, 0.0, w["dt"], 3)
        g.advance(b, 3 * w["dt"], w["dt"], 2)
        g.advance(b, 0.0, w["dt"], 0)  # no-op
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_side_stream_matches_default_stream():
    import torch
    w = inputs.stream_circles(seed=4, n=80, steps=64)
    g = pkg.Grid(w["ncell"], dtype="float32")
    g.set_velocity(w["kind"], w["params"], w["period"])
    a = g.from_numpy(w["phi0"], w["psi0"])
    b = a.clone()
    g.advance(a, 0.0, w["dt"], 4)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g2 = pkg.Grid(w["ncell"], dtype="float32")
        g2.set_velocity(w["kind"], w["params"], w["period"])
        g2.advance(b, 0.0, w["dt"], 4, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("dtype,steps", [("float32", 3), ("float64", 2)])
def test_caller_captured_graph_replays_equal_eager(dtype, steps):
    """A caller may capture gals_advance (the table kernel, the steps and, for
    an odd step count, the copy back from the workspace) in a HIP graph: each
    replay, with eager work and synchronisations between replays, equals the
    eager advance bit for bit."""
    import torch
    w = inputs.stream_circles(seed=5, n=96, steps=64)
    g = pkg.Grid(w["ncell"], dtype=dtype)
    g.set_velocity(w["kind"], w["params"], w["period"])
    init = g.from_numpy(w["phi0"], w["psi0"])
    eager = init.clone()
    g.advance(eager, 0.1, w["dt"], steps)  # also allocates the workspace before capture
    torch.cuda.synchronize()
    assert not torch.equal(eager, init)
    st = init.clone()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=side):
        g.advance(st, 0.1, w["dt"], steps)
    torch.cuda.synchronize()
    other = init.clone()
    for r in range(3):
        st.copy_(init)
        torch.cuda.synchronize()
        graph.replay()
        g.advance(other, 0.0, w["dt"], 1)  # eager work on the same workspace between replays
        torch.cuda.synchronize()
        assert torch.equal(st, eager), f"replay {r}"


@pytest.mark.parametrize("steps", [1, 8])
def test_fp32_against_fp64_oracle_2d(steps):
    w = inputs.stream_circles(seed=5, n=160, steps=128)
    args = (2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
            w["phi0"], w["psi0"], 0.0, w["dt"], steps)
    g = gpu_advance(*args, dtype="float32")
    o = oracle_advance(*args)
    tp, tg = fp32_tolerances(o[0], o[1], 1 / 160, steps)
    ep, eg = rel(g[0], o[0]), rel(g[1], o[1])
    print(f"fp32 2d steps={steps}: phi {ep:.2e} (tol {tp:.1e}) psi {eg:.2e} (tol {tg:.1e})")
    assert ep <= tp and eg <= tg


def test_fp32_against_fp64_oracle_3d():
    rng = np.random.default_rng(33)
    ncell = (21, 17, 19)
    lo, hi = (0.0,) * 3, (1.0,) * 3
    phi0, psi0 = _random_smooth_state(rng, ncell, lo, hi)
    params = np.array([0.05, -0.01, 0.02, 1, 3, 2, -0.02, 0.04, 0.01, 4, 2, 1])
    args = (3, ncell, lo, hi, inputs.VECPOT_SIN, params, 3.0, phi0, psi0, 0.0, 0.04, 3)
    g = gpu_advance(*args, dtype="float32")
    o = oracle_advance(*args)
    tp, tg = fp32_tolerances(o[0], o[1], 1 / 21, 3)
    ep, eg = rel(g[0], o[0]), rel(g[1], o[1])
    print(f"fp32 3d: phi {ep:.2e} (tol {tp:.1e}) psi {eg:.2e} (tol {tg:.1e})")
    assert ep <= tp and eg <= tg


def test_nan_propagates_and_is_counted():
    import torch
    w = inputs.rotation_circle(seed=2, n=40, steps=80)
    phi0 = w["phi0"].copy()
    phi0[41 * 20 + 20] = np.nan
    g = pkg.Grid(w["ncell"], dtype="float64")
    g.set_velocity(w["kind"], w["params"], w["period"])
    st = g.from_numpy(phi0, w["psi0"])
    ref = g.from_numpy(w["phi0"], w["psi0"])
    g.advance(st, 0.0, w["dt"], 2)
    torch.cuda.synchronize()
    out = g.norms(st, ref, 1.5 / 40, 3 / 40)
    assert out[6] > 0  # non-finite entries are reported
    phi, psi = g.to_numpy(st)
    assert out[6] == np.count_nonzero(~np.isfinite(phi)) + np.count_nonzero(~np.isfinite(psi))


@pytest.mark.parametrize("n", [256, 512, 1024])
def test_fp32_stream_taylor_and_exact_regimes(n):
    """FP32 stream-function steps evaluate stages 2 and 3 from the node's
    Taylor jet when the offset is small enough and exactly otherwise; n = 512
    at CFL 0.8 mixes both within waves. Two steps against the oracle."""
    w = inputs.stream_circles(seed=8, n=n, steps=n // 2)
    args = (2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
            w["phi0"], w["psi0"], 0.3, w["dt"], 2)
    g = gpu_advance(*args, dtype="float32")
    o = oracle_advance(*args)
    tp, tg = fp32_tolerances(o[0], o[1], 1 / n, 2)
    ep, eg = rel(g[0], o[0]), rel(g[1], o[1])
    print(f"fp32 stream n={n}: phi {ep:.2e} (tol {tp:.1e}) psi {eg:.2e} (tol {tg:.1e})")
    assert ep <= tp and eg <= tg
