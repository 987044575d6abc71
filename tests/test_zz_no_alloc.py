"""The allocation-free advance (gals_advance_noalloc, through the C ABI)
against gals_advance: the same kernels, so the same state bit for bit, on two
calls in a row that share the library's static scratch, the second on a
smaller grid (and an odd step count, so the result is copied back out of the
scratch); FP32 and FP64, and the FP64 result against the oracle."""
import numpy as np
import pytest

import paper_0905_3409_amd as pkg
from gpu_util import TOL64, oracle_advance, rel, rel_psi
from paper_0905_3409_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(w, dtype, steps):
    import torch
    g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype=dtype, device=0)
    g.set_velocity(w["kind"], w["params"], w["period"])
    a = g.from_numpy(w["phi0"], w["psi0"])
    b = a.clone()
    g.advance(a, 0.0, w["dt"], steps)
    g.advance_noalloc(b, 0.0, w["dt"], steps)
    torch.cuda.synchronize()
    return g, a, b


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_noalloc_equals_advance_on_two_calls_in_a_row(dtype):
    import torch
    big = inputs.stream_circles(seed=3, n=300, steps=150)
    small = inputs.stream_circles(seed=4, n=97, steps=48)
    for w, steps in ((big, 20), (small, 7)):
        print(f"noalloc {dtype} {w['ncell']} {steps} steps", flush=True)
        g, a, b = _pair(w, dtype, steps)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1:], b[1:])
        pa, sa = g.to_numpy(a)
        assert np.isfinite(pa).all() and np.isfinite(sa).all()
    if dtype == "float64":
        o = oracle_advance(2, small["ncell"], small["lo"], small["hi"], small["kind"],
                           small["params"], small["period"], small["phi0"], small["psi0"], 0.0,
                           small["dt"], 7)
        pb, sb = g.to_numpy(b)
        assert rel(pb, o[0]) <= TOL64
        assert rel_psi(sb, o[1], o[0], 1.0 / 97) <= TOL64


def test_noalloc_affine_3d_and_rejects_grids_beyond_the_scratch():
    import torch
    w = inputs.rotation_circle(seed=1, n=48, steps=96)
    # a 3D affine case (rotation about the z axis) through the same scratch
    ncell = (21, 17, 13)
    coords = inputs.node_grid(ncell)
    phi, psi = inputs.sdf_union(coords, [np.array([0.45, 0.55, 0.5])], [0.2])
    A = np.zeros((3, 3))
    A[0, 1], A[1, 0] = -2 * np.pi, 2 * np.pi
    g = pkg.Grid(ncell, dtype="float32", device=0)
    g.set_velocity(pkg.AFFINE, inputs.affine_params(np.zeros(3), np.full(3, 0.5), A), 0.0)
    a = g.from_numpy(phi, psi)
    b = a.clone()
    g.advance(a, 0.0, 1.0 / 64, 5)
    g.advance_noalloc(b, 0.0, 1.0 / 64, 5)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # a grid whose workspace exceeds the static scratch is refused, state untouched
    big = pkg.Grid((4096, 4096), dtype="float32", device=0)
    big.set_velocity(w["kind"], w["params"], 0.0)
    st = big.empty_state().zero_()
    with pytest.raises(pkg.GalsError) as err:
        big.advance_noalloc(st, 0.0, 1e-3, 1)
    assert err.value.code == pkg.EINVAL and "static scratch" in str(err.value)
