"""GPU point evaluation, norms and max speed against the oracle."""
import numpy as np
import pytest

import oracle
import paper_0905_3409_amd as pkg
from gpu_util import TOL64, U32, rel
from paper_0905_3409_amd import inputs

pytestmark = pytest.mark.gpu


def _state(dim, ncell, seed):
    rng = np.random.default_rng(seed)
    coords = inputs.node_grid(ncell)
    centres = rng.uniform(0.3, 0.7, (3, dim))
    radii = rng.uniform(0.1, 0.2, 3)
    phi, psi = inputs.sdf_union(coords, centres, radii)
    return phi, psi


@pytest.mark.parametrize("dim,ncell", [(2, (45, 38)), (3, (17, 14, 19))])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_eval_points_parity(dim, ncell, dtype):
    import torch
    phi, psi = _state(dim, ncell, 5 + dim)
    rng = np.random.default_rng(dim)
    if dtype == "float64":
        pts = rng.uniform(-0.05, 1.05, (5000, dim))  # some outside: extrapolation
    else:
        pts = rng.uniform(0.0, 1.0, (5000, dim))     # FP32: inside (bounded weights)
    g = pkg.Grid(ncell, dtype=dtype)
    st = g.from_numpy(phi, psi)
    phi, psi = g.to_numpy(st)  # the oracle sees the same (FP32-rounded) data
    val, nrm, cur = g.eval_points(st, pts)
    torch.cuda.synchronize()
    o = oracle.eval_points(dim, ncell, np.zeros(dim), np.ones(dim), phi, psi, pts)
    val = val.double().cpu().numpy()
    nrm = nrm.double().cpu().numpy().T
    cur = cur.double().cpu().numpy()
    h = 1.0 / max(ncell)
    pmax = np.abs(phi).max()
    gn = np.linalg.norm(o["grad"], axis=1)
    if dtype == "float64":
        assert rel(val, o["val"]) <= TOL64
        # the normal is grad H / |grad H|: its rounding scale is u |phi| / (h |grad H|)
        ok = gn > 1e-3
        en = np.abs(nrm - o["normal"]).max(axis=1)[ok] * gn[ok] * h / pmax
        assert en.max() <= TOL64
        # curvature divides by |grad|^3: compare where the gradient is not tiny
        assert rel(cur[ok], o["kappa"][ok]) <= 1e-10
    else:
        # FP32 data and arithmetic: value ~u|phi|, derivatives ~u|phi|/h,
        # curvature ~u|phi|/h^2 (second differences of the data)
        h = 1.0 / min(ncell)
        assert rel(val, o["val"]) <= 64 * U32
        assert np.abs(nrm - o["normal"]).max() <= 64 * U32 / h
        ok = np.linalg.norm(o["grad"], axis=1) > 0.5
        assert np.abs(cur[ok] - o["kappa"][ok]).max() <= 64 * U32 / h**2 * np.abs(o["kappa"][ok]).max()


def test_eval_points_zero_gradient_and_empty():
    import torch
    ncell = (8, 8)
    g = pkg.Grid(ncell, dtype="float64")
    st = g.from_numpy(np.ones(81), np.zeros(162))
    val, nrm, cur = g.eval_points(st, np.array([[0.25, 0.5], [0.5, 0.5]]))  # nodes
    torch.cuda.synchronize()
    assert np.all(cur.cpu().numpy() == 0) and np.all(nrm.cpu().numpy() == 0)
    assert np.all(val.cpu().numpy() == 1.0)
    v0, n0, c0 = g.eval_points(st, np.zeros((0, 2)))
    assert v0.numel() == 0


def test_curvature_of_circle_on_device():
    """Quadratic level set |x - c|^2 - r^2: kappa = 1/|x - c| up to rounding."""
    import torch
    ncell = (33, 33)
    coords = inputs.node_grid(ncell)
    c = (0.45, 0.52)
    phi = (coords[0] - c[0]) ** 2 + (coords[1] - c[1]) ** 2 - 0.04
    psi = np.concatenate([2 * (coords[0] - c[0]), 2 * (coords[1] - c[1])])
    g = pkg.Grid(ncell, dtype="float64")
    st = g.from_numpy(phi, psi)
    pts = np.random.default_rng(1).uniform(0, 1, (2000, 2))
    r = np.hypot(pts[:, 0] - c[0], pts[:, 1] - c[1])
    pts = pts[r > 0.05]
    r = r[r > 0.05]
    _, _, cur = g.eval_points(st, pts)
    torch.cuda.synchronize()
    assert np.allclose(cur.cpu().numpy(), 1 / r, rtol=1e-10)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_norms_parity(dtype):
    import torch
    ncell = (70, 45)
    phi, psi = _state(2, ncell, 9)
    rng = np.random.default_rng(4)
    phr = phi + 0.01 * rng.normal(size=phi.shape)
    psr = psi + 0.01 * rng.normal(size=psi.shape)
    g = pkg.Grid(ncell, dtype=dtype)
    a, b = g.from_numpy(phi, psi), g.from_numpy(phr, psr)
    # the oracle sees the same (possibly FP32-rounded) values
    pa, qa = g.to_numpy(a)
    pb, qb = g.to_numpy(b)
    eps, band = 1.5 / 70, 3 / 70
    out = g.norms(a, b, eps, band)
    o = oracle.norms(2, ncell, [0, 0], [1, 1], pa, qa, pb, qb, eps, band)
    torch.cuda.synchronize()
    assert np.allclose(out, o, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim,kind,params,period", [
    (2, inputs.STREAM_SIN, np.array([0.05, 1, 3, -0.02, 4, 2]), 2.0),
    (2, inputs.AFFINE, inputs.rotation_params(), 0.0),
    (2, inputs.VORTEX, np.zeros(0), 2.0),
    (2, inputs.PSEUDO1D, np.zeros(0), 0.0),
    (3, inputs.VECPOT_SIN, np.array([0.05, -0.01, 0.02, 1, 3, 2]), 3.0),
    (3, inputs.LEVEQUE3D, np.zeros(0), 2.5),
])
def test_max_speed_parity(dim, kind, params, period):
    ncell = (40, 37) if dim == 2 else (20, 18, 23)
    for dtype, tol in (("float64", 1e-13), ("float32", 1e-6)):
        g = pkg.Grid(ncell, dtype=dtype)
        g.set_velocity(kind, params, period)
        s = g.max_speed(0.3)
        o = oracle.max_speed(dim, ncell, np.zeros(dim), np.ones(dim), kind, params, period, 0.3)
        assert s == pytest.approx(o, rel=tol)
