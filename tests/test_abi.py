"""C-ABI checks that need no GPU: the library loads, exports every function
that include/gals.h declares, and validates arguments on a host-only context
(device -1) before touching HIP."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_0905_3409_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gals.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gals_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(pkg.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def _ctx(dim=2, ncell=(10, 7, 5), prec=pkg.F32, mixed=pkg.MIXED_CENTRAL, bc=pkg.BC_NEUMANN,
         device=-1):
    L = pkg.lib()
    ctx = ctypes.c_void_p()
    nc = (ctypes.c_int64 * dim)(*ncell[:dim])
    lo = (ctypes.c_double * dim)(*([0.0] * dim))
    hi = (ctypes.c_double * dim)(*([1.0] * dim))
    rc = L.gals_create(ctypes.byref(ctx), dim, nc, lo, hi, prec, mixed, bc, device)
    return rc, ctx


def test_create_validation():
    L = pkg.lib()
    assert _ctx(dim=4)[0] == pkg.EINVAL
    assert _ctx(ncell=(1, 7, 5))[0] == pkg.EINVAL
    assert _ctx(prec=3)[0] == pkg.EINVAL
    assert _ctx(mixed=7)[0] == pkg.EINVAL
    assert _ctx(mixed=pkg.MIXED_CELL)[0] == pkg.OK
    assert _ctx(bc=4)[0] == pkg.EINVAL
    assert _ctx(bc=-1)[0] == pkg.EINVAL
    assert _ctx(bc=pkg.BC_INFLOW)[0] == pkg.OK
    assert _ctx(bc=pkg.BC_INFLOW_NEUMANN)[0] == pkg.OK
    assert _ctx(bc=pkg.BC_EXTRAPOLATE)[0] == pkg.OK
    assert _ctx(device=-2)[0] in (pkg.EINVAL, pkg.EHIP)
    assert _ctx(dim=3, ncell=(2048, 2048, 1024))[0] == pkg.EINVAL  # >= 2^31 nodes
    ctx = ctypes.c_void_p()
    nc = (ctypes.c_int64 * 2)(8, 8)
    lo = (ctypes.c_double * 2)(0.0, 1.0)
    hi = (ctypes.c_double * 2)(1.0, 1.0)  # hi == lo on axis 1
    assert L.gals_create(ctypes.byref(ctx), 2, nc, lo, hi, pkg.F32, 0, 0, -1) == pkg.EINVAL
    assert b"axis 1" in L.gals_last_error()
    rc, ctx = _ctx()
    assert rc == pkg.OK
    L.gals_destroy(ctx)
    assert L.gals_destroy(None) == pkg.OK


@pytest.mark.parametrize("dim,prec,es,n,nbytes", [(2, pkg.F32, 4, 23167, 2147024896),
                                                 (2, pkg.F64, 8, 16382, 2147352576),
                                                 (3, pkg.F32, 4, 802, 2145924352),
                                                 (3, pkg.F64, 8, 639, 2097152000)])
def test_largest_grids_are_accepted_and_one_more_cell_refused(dim, prec, es, n, nbytes):
    """A plane (rows padded to 64 nodes) must stay below 2 GiB: 23168^2 FP32
    nodes take 2147024896 bytes, 16383^2 FP64 nodes (pitch 16384) 2147352576,
    803^3 FP32 nodes (pitch 832) 2145924352, 640^3 FP64 nodes 2097152000.
    One more cell per axis crosses the limit. The GPU tests step these grids."""
    L = pkg.lib()
    rc, ctx = _ctx(dim=dim, ncell=(n,) * 3, prec=prec)
    assert rc == pkg.OK
    nodes = (ctypes.c_int64 * dim)()
    pitch, plane = ctypes.c_int64(), ctypes.c_int64()
    assert L.gals_layout(ctx, nodes, ctypes.byref(pitch), ctypes.byref(plane)) == pkg.OK
    assert tuple(nodes) == (n + 1,) * dim and pitch.value % 64 == 0
    assert plane.value * es == nbytes < 2 ** 31
    L.gals_destroy(ctx)
    rc, _ = _ctx(dim=dim, ncell=(n + 1,) * 3, prec=prec)
    assert rc == pkg.EINVAL
    assert b"2 GiB" in L.gals_last_error()


@pytest.mark.parametrize("dim,ncell,prec", [(2, (2048, 2048), pkg.F32), (2, (64, 64), pkg.F64),
                                            (3, (256, 256, 256), pkg.F32), (3, (2, 3, 4), pkg.F64)])
def test_layout_and_workspace(dim, ncell, prec):
    L = pkg.lib()
    rc, ctx = _ctx(dim=dim, ncell=ncell + (1,) * (3 - dim), prec=prec)
    assert rc == pkg.OK
    nodes = (ctypes.c_int64 * dim)()
    pitch, plane = ctypes.c_int64(), ctypes.c_int64()
    assert L.gals_layout(ctx, nodes, ctypes.byref(pitch), ctypes.byref(plane)) == pkg.OK
    assert tuple(nodes) == tuple(n + 1 for n in ncell)
    assert pitch.value % 64 == 0 and ncell[0] + 1 <= pitch.value < ncell[0] + 65
    assert plane.value == pitch.value * int(np.prod([n + 1 for n in ncell[1:]]))
    ws = ctypes.c_size_t()
    assert L.gals_workspace_bytes(ctx, ctypes.byref(ws)) == pkg.OK
    es = 4 if prec == pkg.F32 else 8
    assert ws.value >= (1 + dim) * plane.value * es + 1025 * 8 * 8
    assert ws.value % 256 == 0
    L.gals_destroy(ctx)


def _setvel(ctx, kind, params, period=0.0):
    p = np.ascontiguousarray(params, dtype=np.float64)
    ptr = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if p.size else None
    return pkg.lib().gals_set_velocity(ctx, kind, ptr, p.size, period)


def test_set_velocity_validation():
    rc, c2 = _ctx(dim=2)
    rc3, c3 = _ctx(dim=3)
    assert _setvel(c2, pkg.AFFINE, np.zeros(8)) == pkg.OK
    assert _setvel(c2, pkg.AFFINE, np.zeros(7)) == pkg.EINVAL
    assert _setvel(c3, pkg.AFFINE, np.zeros(15)) == pkg.OK
    assert _setvel(c2, pkg.STREAM_SIN, [0.1, 1, 4, 0.2, 3, 2]) == pkg.OK
    assert _setvel(c2, pkg.STREAM_SIN, [0.1, 5, 1]) == pkg.ENOTSUP
    assert _setvel(c2, pkg.STREAM_SIN, [0.1, 1.5, 1]) == pkg.ENOTSUP
    assert _setvel(c2, pkg.STREAM_SIN, [0.1, 1]) == pkg.EINVAL
    assert _setvel(c2, pkg.STREAM_SIN, np.tile([0.1, 1, 1], 65)) == pkg.ENOTSUP
    assert _setvel(c3, pkg.STREAM_SIN, [0.1, 1, 1]) == pkg.EINVAL
    assert _setvel(c3, pkg.VECPOT_SIN, [0.1, 0.2, 0.3, 1, 2, 3]) == pkg.OK
    assert _setvel(c3, pkg.VECPOT_SIN, np.tile([0.1, 0.2, 0.3, 1, 2, 3], 9)) == pkg.ENOTSUP
    assert _setvel(c2, pkg.VORTEX, [], 2.0) == pkg.OK
    assert _setvel(c2, pkg.VORTEX, [1.0]) == pkg.EINVAL
    assert _setvel(c2, pkg.PSEUDO1D, []) == pkg.OK
    assert _setvel(c3, pkg.LEVEQUE3D, [], 2.5) == pkg.OK
    assert _setvel(c2, pkg.LEVEQUE3D, []) == pkg.EINVAL
    assert _setvel(c2, 99, []) == pkg.EINVAL
    assert _setvel(c2, pkg.VORTEX, [], -1.0) == pkg.EINVAL
    assert _setvel(c2, pkg.AFFINE, [np.nan] + [0.0] * 7) == pkg.EINVAL
    pkg.lib().gals_destroy(c2)
    pkg.lib().gals_destroy(c3)


def test_advance_validation_on_host_only_context():
    L = pkg.lib()
    rc, ctx = _ctx(dim=2, ncell=(10, 7))
    ws = ctypes.c_size_t()
    L.gals_workspace_bytes(ctx, ctypes.byref(ws))
    vp = ctypes.c_void_p
    # fake, never dereferenced addresses: every call below fails validation first
    phi, grad, w = vp(0x100000), vp(0x200000), vp(0x400000)
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.1, 1, w, ws.value, None) == pkg.EINVAL
    assert b"no velocity" in L.gals_last_error()
    assert _setvel(ctx, pkg.VORTEX, []) == pkg.OK
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.0, 1, w, ws.value, None) == pkg.EINVAL
    assert L.gals_advance(ctx, phi, grad, 0.0, float("nan"), 1, w, ws.value, None) == pkg.EINVAL
    assert L.gals_advance(ctx, phi, grad, float("inf"), 0.1, 1, w, ws.value, None) == pkg.EINVAL
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.1, -1, w, ws.value, None) == pkg.EINVAL
    assert L.gals_advance(ctx, None, grad, 0.0, 0.1, 1, w, ws.value, None) == pkg.EINVAL
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.1, 1, w, ws.value - 1, None) == pkg.EINVAL
    assert L.gals_advance(ctx, vp(0x100002), grad, 0.0, 0.1, 1, w, ws.value, None) == pkg.EINVAL
    # overlapping phi and grad
    assert L.gals_advance(ctx, phi, vp(0x100000 + 64), 0.0, 0.1, 1, w, ws.value, None) == pkg.EINVAL
    assert b"overlap" in L.gals_last_error()
    # overlapping state and workspace
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.1, 1, vp(0x200000), ws.value, None) == pkg.EINVAL
    # steps == 0 is a no-op that succeeds without a device
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.1, 0, w, ws.value, None) == pkg.OK
    # a valid call reaches the device check
    assert L.gals_advance(ctx, phi, grad, 0.0, 0.1, 1, w, ws.value, None) == pkg.EINVAL
    assert b"host-only" in L.gals_last_error()
    assert L.gals_eval_points(ctx, phi, grad, None, 0, None, None, None, None) == pkg.OK
    assert L.gals_eval_points(ctx, phi, grad, None, 5, None, None, None, None) == pkg.EINVAL
    assert L.gals_eval_points(ctx, phi, grad, w, -1, None, None, None, None) == pkg.EINVAL
    # point counts: 2^40 and beyond are refused before the device check; one
    # below passes validation (the kernel strides over any count, so the
    # launch's 32-bit work-item count never wraps)
    assert L.gals_eval_points(ctx, phi, grad, w, 1 << 40, None, None, None, None) == pkg.EINVAL
    assert b"too many points" in L.gals_last_error()
    assert L.gals_eval_points(ctx, phi, grad, w, (1 << 40) - 1, None, None, None, None) == pkg.EINVAL
    assert b"host-only" in L.gals_last_error()
    out = (ctypes.c_double * 8)()
    assert L.gals_norms(ctx, phi, grad, phi, grad, 0.0, 0.1, out, w, ws.value, None) == pkg.EINVAL
    assert L.gals_max_speed(ctx, 0.0, out, w, 8, None) == pkg.EINVAL
    L.gals_destroy(ctx)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        pkg.lib()


def _batch(ncells, prec=pkg.F32, mixed=pkg.MIXED_CENTRAL, bc=pkg.BC_NEUMANN, device=-1, lo=None,
           hi=None):
    L = pkg.lib()
    n = len(ncells)
    b = ctypes.c_void_p()
    nc = (ctypes.c_int64 * (2 * n))(*[v for c in ncells for v in c])
    lo = (ctypes.c_double * (2 * n))(*(lo if lo is not None else [0.0] * (2 * n)))
    hi = (ctypes.c_double * (2 * n))(*(hi if hi is not None else [1.0] * (2 * n)))
    rc = L.gals_batch_create(ctypes.byref(b), n, nc, lo, hi, prec, mixed, bc, device)
    return rc, b


def test_batch_create_validation():
    L = pkg.lib()
    b = ctypes.c_void_p()
    nc = (ctypes.c_int64 * 2)(8, 8)
    lo = (ctypes.c_double * 2)(0.0, 0.0)
    hi = (ctypes.c_double * 2)(1.0, 1.0)
    assert L.gals_batch_create(ctypes.byref(b), 0, nc, lo, hi, pkg.F32, 0, 0, -1) == pkg.EINVAL
    assert L.gals_batch_create(None, 1, nc, lo, hi, pkg.F32, 0, 0, -1) == pkg.EINVAL
    assert L.gals_batch_create(ctypes.byref(b), 65536, nc, lo, hi, pkg.F32, 0, 0, -1) == pkg.EINVAL
    assert _batch([(8, 8), (1, 8)])[0] == pkg.EINVAL
    assert b"problem 1 axis 0" in L.gals_last_error()
    assert _batch([(8, 8)], prec=5)[0] == pkg.EINVAL
    assert _batch([(8, 8)], mixed=3)[0] == pkg.EINVAL
    assert _batch([(8, 8)], mixed=pkg.MIXED_CELL)[0] == pkg.OK
    assert _batch([(8, 8)], bc=pkg.BC_INFLOW)[0] == pkg.EINVAL  # single grids only
    assert _batch([(8, 8)], bc=pkg.BC_INFLOW_NEUMANN)[0] == pkg.EINVAL
    assert _batch([(8, 8)], device=-3)[0] == pkg.EINVAL
    assert _batch([(8, 8)], lo=[0.0, 1.0], hi=[1.0, 1.0])[0] == pkg.EINVAL
    assert _batch([(40000, 20000)])[0] == pkg.EINVAL  # plane of 2 GiB or more
    rc, b = _batch([(8, 8), (30, 70)], bc=pkg.BC_EXTRAPOLATE)
    assert rc == pkg.OK
    assert L.gals_batch_destroy(b) == pkg.OK
    assert L.gals_batch_destroy(None) == pkg.OK


def test_batch_layout_and_workspace():
    L = pkg.lib()
    ncells = [(8, 8), (33, 47), (100, 3), (511, 512)]
    for prec, es in ((pkg.F32, 4), (pkg.F64, 8)):
        rc, b = _batch(ncells, prec=prec)
        assert rc == pkg.OK
        n = len(ncells)
        off, pitch, plane = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        total = ctypes.c_int64()
        assert L.gals_batch_layout(b, off, pitch, plane, ctypes.byref(total)) == pkg.OK
        o = 0
        for p, (nx, ny) in enumerate(ncells):
            assert off[p] == o
            assert pitch[p] % 64 == 0 and nx + 1 <= pitch[p] < nx + 65
            assert plane[p] == pitch[p] * (ny + 1)
            o += 3 * plane[p]
        assert total.value == o
        ws = ctypes.c_size_t()
        assert L.gals_batch_workspace_bytes(b, ctypes.byref(ws)) == pkg.OK
        tables = sum(nx + ny + 2 for nx, ny in ncells) * 24 * es  # 24 entries a column/row
        assert total.value * es + tables <= ws.value <= total.value * es + tables + 256 * (n * 64 + 2)
        L.gals_batch_destroy(b)


def test_batch_velocity_tiles_and_advance_validation():
    L = pkg.lib()
    rc, b = _batch([(8, 8), (40, 20)])
    assert rc == pkg.OK
    P = ctypes.POINTER(ctypes.c_double)
    good = np.array([0.01, 1, 2, -0.02, 4, 4], dtype=np.float64)
    assert L.gals_batch_set_velocity(b, 0, pkg.STREAM_SIN, good.ctypes.data_as(P), 6, 2.0) == pkg.OK
    assert L.gals_batch_set_velocity(b, 2, pkg.STREAM_SIN, good.ctypes.data_as(P), 6, 2.0) == pkg.EINVAL
    assert L.gals_batch_set_velocity(b, 1, pkg.AFFINE, good.ctypes.data_as(P), 6, 2.0) == pkg.ENOTSUP
    assert L.gals_batch_set_velocity(b, 1, pkg.STREAM_SIN, good.ctypes.data_as(P), 5, 2.0) == pkg.EINVAL
    bad = np.array([0.01, 5, 1], dtype=np.float64)
    assert L.gals_batch_set_velocity(b, 1, pkg.STREAM_SIN, bad.ctypes.data_as(P), 3, 2.0) == pkg.ENOTSUP
    bad = np.array([np.nan, 1, 1], dtype=np.float64)
    assert L.gals_batch_set_velocity(b, 1, pkg.STREAM_SIN, bad.ctypes.data_as(P), 3, 2.0) == pkg.EINVAL
    # one period for the whole batch
    assert L.gals_batch_set_velocity(b, 1, pkg.STREAM_SIN, good.ctypes.data_as(P), 6, 3.0) == pkg.EINVAL
    assert b"one period" in L.gals_last_error()
    tiles = (ctypes.c_int * 4)(64, 32, 16, 16)
    assert L.gals_batch_set_tiles(b, tiles) == pkg.OK
    got = (ctypes.c_int * 4)()
    assert L.gals_batch_get_tiles(b, got) == pkg.OK and list(got) == [64, 32, 16, 16]
    assert L.gals_batch_set_tiles(b, (ctypes.c_int * 4)(64, 8, 16, 16)) == pkg.EINVAL
    assert L.gals_batch_get_tiles(b, got) == pkg.OK and list(got) == [64, 32, 16, 16]
    assert L.gals_batch_set_tiles(b, (ctypes.c_int * 4)(0, 0, 16, 0)) == pkg.OK  # row-major
    assert L.gals_batch_get_tiles(b, got) == pkg.OK and list(got) == [0, 0, 16, 0]
    ws_bytes = ctypes.c_size_t()
    L.gals_batch_workspace_bytes(b, ctypes.byref(ws_bytes))
    state, ws = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 40)
    # problem 1 has no velocity yet
    assert L.gals_batch_advance(b, state, 0.0, 0.01, 1, 0, ws, ws_bytes.value, None) == pkg.EINVAL
    assert b"problem 1" in L.gals_last_error()
    assert L.gals_batch_set_velocity(b, 1, pkg.STREAM_SIN, good.ctypes.data_as(P), 6, 2.0) == pkg.OK
    args = dict(t0=0.0, dt=0.01, steps=1, ws=ws, wsb=ws_bytes.value)

    def adv(**kw):
        a = dict(args, **kw)
        return L.gals_batch_advance(b, state, a["t0"], a["dt"], a["steps"], 0, a["ws"], a["wsb"],
                                    None)

    assert adv(dt=0.0) == pkg.EINVAL
    assert adv(dt=float("inf")) == pkg.EINVAL
    assert adv(t0=float("nan")) == pkg.EINVAL
    assert adv(steps=-1) == pkg.EINVAL
    assert adv(wsb=ws_bytes.value - 1) == pkg.EINVAL
    assert adv(ws=ctypes.c_void_p((1 << 40) + 4)) == pkg.EINVAL  # workspace not 256-aligned
    assert adv(ws=ctypes.c_void_p((1 << 20) + 256)) == pkg.EINVAL  # overlaps the state
    assert adv(steps=0) == pkg.OK  # nothing to do, nothing touched
    assert adv() == pkg.EINVAL  # host-only batch cannot launch
    assert b"host-only" in L.gals_last_error()
    best = ctypes.c_double()
    assert L.gals_batch_autotune(b, state, 0.01, 0, ws, ws_bytes.value, None,
                                 ctypes.byref(best)) == pkg.EINVAL
    L.gals_batch_destroy(b)


def test_batch_binding_layout_roundtrip():
    """The Python views of each problem's planes address the documented layout."""
    bt = pkg.Batch([(8, 8), (33, 5), (70, 70)], device=-1)
    assert bt.nprob == 3 and bt.num_nodes() == 81 + 34 * 6 + 71 * 71
    assert list(bt.offset) == [0, 3 * bt.plane[0], 3 * (bt.plane[0] + bt.plane[1])]
    assert bt.total_elems == 3 * int(bt.plane.sum())


def test_adjoint_entry_points_validate_on_a_host_only_context():
    L = pkg.lib()
    P = ctypes.POINTER(ctypes.c_double)
    rc, ctx = _ctx(dim=2, ncell=(10, 7, 1), prec=pkg.F64)
    assert rc == pkg.OK
    b = ctypes.c_size_t()
    nodes = (ctypes.c_int64 * 2)()
    pitch, plane = ctypes.c_int64(), ctypes.c_int64()
    L.gals_layout(ctx, nodes, ctypes.byref(pitch), ctypes.byref(plane))
    state_b = -(-3 * plane.value * 8 // 256) * 256
    assert L.gals_checkpoint_bytes(ctx, 200, 20, ctypes.byref(b)) == pkg.OK
    assert b.value == 10 * state_b
    assert L.gals_checkpoint_bytes(ctx, 201, 20, ctypes.byref(b)) == pkg.OK
    assert b.value == 11 * state_b
    assert L.gals_checkpoint_bytes(ctx, 5, 0, ctypes.byref(b)) == pkg.EINVAL
    assert L.gals_adjoint_workspace_bytes(ctx, 0, ctypes.byref(b)) == pkg.EINVAL
    ws1, ws20 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.gals_adjoint_workspace_bytes(ctx, 1, ctypes.byref(ws1)) == pkg.OK
    assert L.gals_adjoint_workspace_bytes(ctx, 20, ctypes.byref(ws20)) == pkg.OK
    assert ws20.value - ws1.value == 19 * state_b
    lam, dS, ws = ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 31), ctypes.c_void_p(1 << 32)
    ck = ctypes.c_void_p(1 << 33)
    args = (ck, 10 * state_b, 0.0, 0.01, 200, 20, lam, dS, ws, ws20.value, None)
    # no velocity yet
    assert L.gals_adjoint(ctx, *args) == pkg.EINVAL
    good = np.array([0.01, 1, 2], dtype=np.float64)
    assert L.gals_set_velocity(ctx, pkg.AFFINE, np.zeros(8).ctypes.data_as(P), 8, 0.0) == pkg.OK
    assert L.gals_adjoint(ctx, *args) == pkg.ENOTSUP  # only sine stream functions
    assert L.gals_set_velocity(ctx, pkg.STREAM_SIN, good.ctypes.data_as(P), 3, 0.0) == pkg.OK
    bad = list(args)
    bad[1] = 10 * state_b - 1  # checkpoint store too small
    assert L.gals_adjoint(ctx, *bad) == pkg.EINVAL
    bad = list(args)
    bad[9] = ws20.value - 1  # workspace too small
    assert L.gals_adjoint(ctx, *bad) == pkg.EINVAL
    bad = list(args)
    bad[6] = ctypes.c_void_p((1 << 32) + 512)  # lam inside the workspace
    assert L.gals_adjoint(ctx, *bad) == pkg.EINVAL
    bad = list(args)
    bad[3] = 0.0  # dt
    assert L.gals_adjoint(ctx, *bad) == pkg.EINVAL
    assert L.gals_adjoint(ctx, *args) == pkg.EINVAL  # host-only context
    assert b"host-only" in L.gals_last_error()
    st = ctypes.c_void_p(1 << 34)
    lam2 = ctypes.c_void_p((1 << 30) + 8)  # overlaps lam
    assert L.gals_adjoint_step(ctx, st, st, 0.0, 0.01, lam, lam2, dS, ws, ws1.value,
                               None) == pkg.EINVAL
    out = ctypes.c_double()
    assert L.gals_shape_loss(ctx, st, st, 0.0, ctypes.byref(out), None, ws, 1 << 30,
                             None) == pkg.EINVAL  # eps
    L.gals_destroy(ctx)
    rc, ctx3 = _ctx(dim=3, ncell=(4, 4, 4), prec=pkg.F64)
    assert L.gals_shape_loss(ctx3, st, st, 0.1, ctypes.byref(out), None, ws, 1 << 30,
                             None) == pkg.ENOTSUP
    assert L.gals_set_velocity(ctx3, pkg.LEVEQUE3D, None, 0, 0.0) == pkg.OK
    assert L.gals_adjoint_step(ctx3, st, st, 0.0, 0.01, lam, ctypes.c_void_p(1 << 35), dS, ws,
                               1 << 30, None) == pkg.ENOTSUP
    L.gals_destroy(ctx3)


def test_psi_update_option():
    L = pkg.lib()
    rc, ctx = _ctx()
    assert L.gals_set_psi_update(ctx, pkg.PSI_HEUN) == pkg.OK
    assert L.gals_set_psi_update(ctx, 2) == pkg.EINVAL
    assert L.gals_set_psi_update(None, 0) == pkg.EINVAL
    # the adjoint differentiates the superconsistent update only
    P = ctypes.POINTER(ctypes.c_double)
    rc2, c2 = _ctx(dim=2, ncell=(8, 8, 1), prec=pkg.F64)
    good = np.array([0.01, 1, 2], dtype=np.float64)
    assert L.gals_set_velocity(c2, pkg.STREAM_SIN, good.ctypes.data_as(P), 3, 0.0) == pkg.OK
    assert L.gals_set_psi_update(c2, pkg.PSI_HEUN) == pkg.OK
    v = ctypes.c_void_p
    assert L.gals_adjoint_step(c2, v(1 << 30), v(1 << 31), 0.0, 0.01, v(1 << 32), v(1 << 33),
                               v(1 << 34), v(1 << 35), 1 << 30, None) == pkg.ENOTSUP
    L.gals_destroy(ctx)
    L.gals_destroy(c2)


def test_inflow_data_validation():
    L = pkg.lib()
    P = ctypes.POINTER(ctypes.c_double)
    v = ctypes.c_void_p
    rc, ctx = _ctx(dim=2, ncell=(8, 8, 1), prec=pkg.F64, bc=pkg.BC_INFLOW)
    assert rc == pkg.OK
    assert L.gals_set_velocity(ctx, pkg.AFFINE, np.zeros(8).ctypes.data_as(P), 8, 0.0) == pkg.OK
    ws = ctypes.c_size_t()
    L.gals_workspace_bytes(ctx, ctypes.byref(ws))
    # no data yet
    assert L.gals_advance(ctx, v(1 << 30), v(1 << 31), 0.0, 0.1, 1, v(1 << 32), ws.value,
                          None) == pkg.EINVAL
    assert b"gals_set_inflow_data" in L.gals_last_error()
    assert L.gals_set_inflow_data(ctx, None, v(1 << 33), v(1 << 34)) == pkg.EINVAL
    assert L.gals_set_inflow_data(ctx, v((1 << 33) + 4), v(1 << 33), v(1 << 34)) == pkg.EINVAL
    assert L.gals_set_inflow_data(ctx, v(1 << 35), v(1 << 33), v(1 << 34)) == pkg.OK
    rc, c2 = _ctx(dim=2, ncell=(8, 8, 1), prec=pkg.F64)
    assert L.gals_set_inflow_data(c2, v(1 << 35), v(1 << 33), v(1 << 34)) == pkg.EINVAL
    # no adjoint through inflow data
    good = np.array([0.01, 1, 2], dtype=np.float64)
    assert L.gals_set_velocity(ctx, pkg.STREAM_SIN, good.ctypes.data_as(P), 3, 0.0) == pkg.OK
    assert L.gals_adjoint_step(ctx, v(1 << 30), v(1 << 31), 0.0, 0.01, v(1 << 32), v(1 << 36),
                               v(1 << 37), v(1 << 38), 1 << 30, None) == pkg.ENOTSUP
    rc, c3 = _ctx(dim=2, ncell=(8, 8, 1), prec=pkg.F64, bc=pkg.BC_INFLOW_NEUMANN)
    assert L.gals_set_velocity(c3, pkg.STREAM_SIN, good.ctypes.data_as(P), 3, 0.0) == pkg.OK
    assert L.gals_adjoint_step(c3, v(1 << 30), v(1 << 31), 0.0, 0.01, v(1 << 32), v(1 << 36),
                               v(1 << 37), v(1 << 38), 1 << 30, None) == pkg.ENOTSUP
    assert L.gals_set_inflow_data(c3, v(1 << 35), v(1 << 33), v(1 << 34)) == pkg.EINVAL
    L.gals_destroy(c3)
    L.gals_destroy(ctx)
    L.gals_destroy(c2)


def test_noalloc_advance_validation_on_host_only_context():
    """gals_advance_noalloc validates like gals_advance, refuses grids whose
    workspace exceeds the library's static scratch before any HIP call, and
    refuses host-only contexts."""
    L = pkg.lib()
    vp = ctypes.c_void_p
    phi, grad = vp(0x100000), vp(0x8000000)
    rc, ctx = _ctx(dim=2, ncell=(300, 200))
    assert rc == pkg.OK
    assert L.gals_advance_noalloc(ctx, phi, grad, 0.0, 0.1, 1, None) == pkg.EINVAL
    assert b"no velocity" in L.gals_last_error()
    assert _setvel(ctx, pkg.VORTEX, []) == pkg.OK
    assert L.gals_advance_noalloc(ctx, None, grad, 0.0, 0.1, 1, None) == pkg.EINVAL
    assert L.gals_advance_noalloc(ctx, phi, grad, 0.0, -0.1, 1, None) == pkg.EINVAL
    assert L.gals_advance_noalloc(ctx, phi, grad, 0.0, 0.1, -1, None) == pkg.EINVAL
    assert L.gals_advance_noalloc(ctx, vp(0x100002), grad, 0.0, 0.1, 1, None) == pkg.EINVAL
    assert L.gals_advance_noalloc(ctx, phi, vp(0x100000 + 64), 0.0, 0.1, 1, None) == pkg.EINVAL
    assert b"overlap" in L.gals_last_error()
    assert L.gals_advance_noalloc(ctx, phi, grad, 0.0, 0.1, 0, None) == pkg.OK
    assert L.gals_advance_noalloc(ctx, phi, grad, 0.0, 0.1, 1, None) == pkg.EINVAL
    assert b"host-only" in L.gals_last_error()
    L.gals_destroy(ctx)
    # the largest square FP32 grid whose workspace fits, and one that does not
    ws = ctypes.c_size_t()
    for n, fits in ((2048, True), (4096, False)):
        rc, ctx = _ctx(dim=2, ncell=(n, n))
        assert rc == pkg.OK
        L.gals_workspace_bytes(ctx, ctypes.byref(ws))
        assert (ws.value <= 64 << 20) == fits
        assert _setvel(ctx, pkg.VORTEX, []) == pkg.OK
        assert L.gals_advance_noalloc(ctx, phi, vp(0x100000000), 0.0, 0.1, 1, None) == pkg.EINVAL
        assert (b"static scratch" in L.gals_last_error()) == (not fits)
        L.gals_destroy(ctx)


def _shape_key(prec, mixed, ncells):
    """FNV-1a over 64-bit little-endian words, as the library keys a batch
    shape for its tuning record."""
    h = 14695981039346656037
    for v in [prec, mixed, len(ncells)] + [c for nc in ncells for c in nc]:
        for k in range(8):
            h ^= (v >> (8 * k)) & 0xFF
            h = (h * 1099511628211) % (1 << 64)
    return h


def test_batch_tuning_record_is_read_at_create(tmp_path, monkeypatch):
    """A batch of a shape recorded in GALS_TUNE_FILE starts with the recorded
    wave shapes (the last valid line for the key wins); other shapes, and
    invalid lines, keep the default."""
    ncells = [(40, 40), (100, 90), (300, 300)]
    key = _shape_key(pkg.F32, pkg.MIXED_CENTRAL, ncells)
    f = tmp_path / "tune.txt"
    f.write_text(f"{key:016x} 32 32 32 32\n"
                 f"{key ^ 1:016x} 16 16 16 16\n"
                 f"{key:016x} 0 16 32 64\n"
                 f"{key:016x} 7 7 7 7\n")
    monkeypatch.setenv("GALS_TUNE_FILE", str(f))
    b = pkg.Batch(ncells, dtype="float32", device=-1)
    assert b.get_tiles() == [0, 16, 32, 64]
    other = pkg.Batch(ncells[:2], dtype="float32", device=-1)
    assert other.get_tiles() == [64, 64, 64, 64]
    monkeypatch.delenv("GALS_TUNE_FILE")
    assert pkg.Batch(ncells, dtype="float32", device=-1).get_tiles() == [64, 64, 64, 64]
