"""MI355X (gfx950) gradient-augmented level set advection.

A thin ctypes binding over ``libgals.so`` (C ABI in ``include/gals.h``).
PyTorch only supplies device memory and the stream; every step of the method
runs in the library's HIP kernels. There is no CPU fallback: if the library is
not built, every call raises.

Typical use::

    g = Grid((2048, 2048), dtype="float32")
    g.set_velocity(STREAM_SIN, params, period=2.0)
    state = g.from_numpy(phi0, psi0)        # (1+dim, plane) device tensor
    g.advance(state, t0=0.0, dt=2/1024, steps=1024)
    phi, psi = g.to_numpy(state)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgals.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSUP = 0, -1, -2, -3, -4
F32, F64 = 1, 2
MIXED_CENTRAL, MIXED_CELL, MIXED_ZERO = 0, 1, 2
PSI_SUPERCONSISTENT, PSI_HEUN = 0, 1
BC_NEUMANN, BC_EXTRAPOLATE, BC_INFLOW, BC_INFLOW_NEUMANN = 0, 1, 2, 3
AFFINE, STREAM_SIN, VECPOT_SIN, VORTEX, PSEUDO1D, LEVEQUE3D = 1, 2, 3, 4, 5, 6

EXPORTS = ("gals_create", "gals_destroy", "gals_layout", "gals_workspace_bytes",
           "gals_set_velocity", "gals_advance", "gals_eval_points", "gals_max_speed",
           "gals_norms", "gals_last_error", "gals_batch_create", "gals_batch_destroy",
           "gals_batch_layout", "gals_batch_workspace_bytes", "gals_batch_set_velocity",
           "gals_batch_set_tiles", "gals_batch_get_tiles", "gals_batch_advance",
           "gals_batch_autotune", "gals_checkpoint_bytes", "gals_advance_save",
           "gals_adjoint_workspace_bytes", "gals_adjoint", "gals_adjoint_step",
           "gals_shape_loss", "gals_set_psi_update", "gals_set_inflow_data",
           "gals_advance_noalloc")

_lib = None


class GalsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def lib():
    """Load libgals.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_0905_3409_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, i64, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P64 = ctypes.POINTER(ctypes.c_int64)
    PD = ctypes.POINTER(ctypes.c_double)
    L.gals_create.argtypes = [ctypes.POINTER(vp), i, P64, PD, PD, i, i, i, i]
    L.gals_destroy.argtypes = [vp]
    L.gals_layout.argtypes = [vp, P64, P64, P64]
    L.gals_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.gals_set_velocity.argtypes = [vp, i, PD, i64, d]
    L.gals_advance.argtypes = [vp, vp, vp, d, d, i64, vp, sz, vp]
    L.gals_advance_noalloc.argtypes = [vp, vp, vp, d, d, i64, vp]
    L.gals_eval_points.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp]
    L.gals_max_speed.argtypes = [vp, d, PD, vp, sz, vp]
    L.gals_norms.argtypes = [vp, vp, vp, vp, vp, d, d, PD, vp, sz, vp]
    PI = ctypes.POINTER(ctypes.c_int)
    L.gals_batch_create.argtypes = [ctypes.POINTER(vp), i64, P64, PD, PD, i, i, i, i]
    L.gals_batch_destroy.argtypes = [vp]
    L.gals_batch_layout.argtypes = [vp, P64, P64, P64, P64]
    L.gals_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.gals_batch_set_velocity.argtypes = [vp, i64, i, PD, i64, d]
    L.gals_batch_set_tiles.argtypes = [vp, PI]
    L.gals_batch_get_tiles.argtypes = [vp, PI]
    L.gals_batch_advance.argtypes = [vp, vp, d, d, i64, i, vp, sz, vp]
    L.gals_batch_autotune.argtypes = [vp, vp, d, i64, vp, sz, vp, PD]
    L.gals_checkpoint_bytes.argtypes = [vp, i64, i64, ctypes.POINTER(sz)]
    L.gals_advance_save.argtypes = [vp, vp, vp, d, d, i64, i64, vp, sz, vp, sz, vp]
    L.gals_adjoint_workspace_bytes.argtypes = [vp, i64, ctypes.POINTER(sz)]
    L.gals_adjoint.argtypes = [vp, vp, sz, d, d, i64, i64, vp, vp, vp, sz, vp]
    L.gals_adjoint_step.argtypes = [vp, vp, vp, d, d, vp, vp, vp, vp, sz, vp]
    L.gals_shape_loss.argtypes = [vp, vp, vp, d, PD, vp, vp, sz, vp]
    L.gals_set_psi_update.argtypes = [vp, i]
    L.gals_set_inflow_data.argtypes = [vp, vp, vp, vp]
    L.gals_last_error.argtypes = []
    L.gals_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "gals_last_error":
            getattr(L, name).restype = i
    _lib = L
    return L


def check(rc):
    if rc != OK:
        raise GalsError(rc, lib().gals_last_error().decode())
    return rc


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class Grid:
    """A uniform 2D/3D grid with its device layout and velocity field."""

    def __init__(self, ncell, lo=None, hi=None, dtype="float32", mixed=MIXED_CENTRAL,
                 bc=BC_NEUMANN, device=0):
        self.dim = len(ncell)
        self.ncell = tuple(int(n) for n in ncell)
        self.lo = tuple(float(x) for x in (lo if lo is not None else (0.0,) * self.dim))
        self.hi = tuple(float(x) for x in (hi if hi is not None else (1.0,) * self.dim))
        if dtype in ("float32", "f32", np.float32):
            self.prec, self.np_dtype = F32, np.float32
        elif dtype in ("float64", "f64", np.float64):
            self.prec, self.np_dtype = F64, np.float64
        else:
            raise ValueError(f"unsupported dtype {dtype!r}")
        self.device = int(device)
        self._ctx = ctypes.c_void_p()
        nc = (ctypes.c_int64 * self.dim)(*self.ncell)
        lo_ = (ctypes.c_double * self.dim)(*self.lo)
        hi_ = (ctypes.c_double * self.dim)(*self.hi)
        check(lib().gals_create(ctypes.byref(self._ctx), self.dim, nc, lo_, hi_, self.prec,
                                int(mixed), int(bc), self.device))
        nodes = (ctypes.c_int64 * self.dim)()
        pitch, plane = ctypes.c_int64(), ctypes.c_int64()
        check(lib().gals_layout(self._ctx, nodes, ctypes.byref(pitch), ctypes.byref(plane)))
        self.nodes = tuple(nodes)
        self.pitch = pitch.value
        self.plane = plane.value
        wsb = ctypes.c_size_t()
        check(lib().gals_workspace_bytes(self._ctx, ctypes.byref(wsb)))
        self.workspace_bytes = wsb.value
        self._ws = None

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value and _lib is not None:
            _lib.gals_destroy(ctx)
            self._ctx = None

    # ---------------------------------------------------------------- layout
    @property
    def torch_dtype(self):
        import torch
        return torch.float32 if self.prec == F32 else torch.float64

    @property
    def num_nodes(self):
        return int(np.prod(self.nodes))

    def _dev(self):
        import torch
        return torch.device("cuda", self.device)

    def empty_state(self):
        """Zero-filled (1+dim, plane) device tensor: row 0 is phi, rows 1..dim psi."""
        import torch
        return torch.zeros((1 + self.dim, self.plane), dtype=self.torch_dtype, device=self._dev())

    def _grid_view(self, plane_tensor):
        """Dense view (z, y, x) or (y, x) of one padded plane."""
        shape = tuple(reversed(self.nodes[1:])) + (self.pitch,)
        v = plane_tensor.view(*shape)
        return v[..., : self.nodes[0]]

    def from_numpy(self, phi, psi):
        """Device state from dense float64 arrays (x fastest; psi = dim planes)."""
        import torch
        st = self.empty_state()
        shape = tuple(reversed(self.nodes))
        phi = np.asarray(phi).reshape(shape)
        psi = np.asarray(psi).reshape((self.dim,) + shape)
        self._grid_view(st[0]).copy_(torch.from_numpy(np.ascontiguousarray(phi)).to(st.dtype))
        for a in range(self.dim):
            self._grid_view(st[1 + a]).copy_(
                torch.from_numpy(np.ascontiguousarray(psi[a])).to(st.dtype))
        return st

    def plane_from_numpy(self, arr):
        """One device plane (the state layout) from a dense float64 array."""
        import torch
        pl = torch.zeros(self.plane, dtype=self.torch_dtype, device=self._dev())
        shape = tuple(reversed(self.nodes))
        self._grid_view(pl).copy_(
            torch.from_numpy(np.ascontiguousarray(np.asarray(arr).reshape(shape))).to(pl.dtype))
        return pl

    def to_numpy(self, state):
        """Dense float64 (phi, psi) arrays from a device state."""
        phi = self._grid_view(state[0]).double().cpu().numpy().ravel()
        psi = np.concatenate([self._grid_view(state[1 + a]).double().cpu().numpy().ravel()
                              for a in range(self.dim)])
        return phi, psi

    def workspace(self):
        import torch
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self._dev())
        return self._ws

    def _check_state(self, state):
        if (state.dtype != self.torch_dtype or tuple(state.shape) != (1 + self.dim, self.plane)
                or not state.is_contiguous() or state.device != self._dev()):
            raise ValueError("state must be a contiguous (1+dim, plane) tensor of the grid's "
                             "dtype on the grid's device")

    # ------------------------------------------------------------------- calls
    def set_velocity(self, kind, params=(), period=0.0):
        p = np.ascontiguousarray(params, dtype=np.float64)
        ptr = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if p.size else None
        check(lib().gals_set_velocity(self._ctx, int(kind), ptr, p.size, float(period)))

    def set_inflow_data(self, state_b, phit_b):
        """Dirichlet inflow data for a BC_INFLOW grid: a state (phi, grad
        planes) and a plane of phi_t, read at boundary nodes for the end
        time of each step. The grid keeps references to both."""
        self._check_state(state_b)
        if (phit_b.dtype != self.torch_dtype or phit_b.numel() < self.plane
                or phit_b.device != self._dev() or not phit_b.is_contiguous()):
            raise ValueError("phit_b must be a contiguous plane of the grid's dtype")
        check(lib().gals_set_inflow_data(self._ctx, ctypes.c_void_p(state_b[0].data_ptr()),
                                         ctypes.c_void_p(state_b[1].data_ptr()),
                                         ctypes.c_void_p(phit_b.data_ptr())))
        self._inflow = (state_b, phit_b)

    def set_psi_update(self, mode):
        """PSI_SUPERCONSISTENT (default) or PSI_HEUN for later advances."""
        check(lib().gals_set_psi_update(self._ctx, int(mode)))

    def advance(self, state, t0, dt, steps, stream=None):
        """Advance the state in place (asynchronous on the stream)."""
        self._check_state(state)
        ws = self.workspace()
        check(lib().gals_advance(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                                 ctypes.c_void_p(state[1].data_ptr()), float(t0), float(dt),
                                 int(steps), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream_handle(stream, self._dev())))
        return state

    def advance_noalloc(self, state, t0, dt, steps, stream=None):
        """As advance, through the entry point that allocates nothing: its
        scratch is the library's static device array (calls on one GPU share
        it, so order them on one stream)."""
        self._check_state(state)
        check(lib().gals_advance_noalloc(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                                         ctypes.c_void_p(state[1].data_ptr()), float(t0),
                                         float(dt), int(steps),
                                         _stream_handle(stream, self._dev())))
        return state

    def eval_points(self, state, pts, stream=None):
        """Value, unit normal (dim, npts) and curvature at points (npts, dim)."""
        import torch
        self._check_state(state)
        pts = torch.as_tensor(pts, dtype=torch.float64, device=self._dev())
        n = pts.shape[0]
        soa = pts.t().contiguous()
        val = torch.empty(n, dtype=self.torch_dtype, device=self._dev())
        nrm = torch.empty((self.dim, n), dtype=self.torch_dtype, device=self._dev())
        cur = torch.empty(n, dtype=self.torch_dtype, device=self._dev())
        check(lib().gals_eval_points(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                                     ctypes.c_void_p(state[1].data_ptr()),
                                     ctypes.c_void_p(soa.data_ptr()), n,
                                     ctypes.c_void_p(val.data_ptr()),
                                     ctypes.c_void_p(nrm.data_ptr()),
                                     ctypes.c_void_p(cur.data_ptr()),
                                     _stream_handle(stream, self._dev())))
        # keep the SoA copy alive until the kernel has consumed it
        (stream or torch.cuda.current_stream(self._dev())).synchronize()
        return val, nrm, cur

    def max_speed(self, t, stream=None):
        out = ctypes.c_double()
        ws = self.workspace()
        check(lib().gals_max_speed(self._ctx, float(t), ctypes.byref(out),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_handle(stream, self._dev())))
        return out.value

    def norms(self, state, ref, eps, band, stream=None):
        """8 diagnostics of state against ref (see gals_norms)."""
        self._check_state(state)
        self._check_state(ref)
        out = (ctypes.c_double * 8)()
        ws = self.workspace()
        check(lib().gals_norms(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                               ctypes.c_void_p(state[1].data_ptr()),
                               ctypes.c_void_p(ref[0].data_ptr()),
                               ctypes.c_void_p(ref[1].data_ptr()), float(eps), float(band), out,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                               _stream_handle(stream, self._dev())))
        return np.array(out[:])

    # ------------------------------------------------------------ derivatives
    def empty_adjoint(self):
        """Zero FP64 adjoint state (3, plane): lam_phi, lam_x, lam_y."""
        import torch
        return torch.zeros((3, self.plane), dtype=torch.float64, device=self._dev())

    def checkpoint_bytes(self, steps, every):
        b = ctypes.c_size_t()
        check(lib().gals_checkpoint_bytes(self._ctx, int(steps), int(every), ctypes.byref(b)))
        return b.value

    def _adjoint_workspace(self, every):
        import torch
        b = ctypes.c_size_t()
        check(lib().gals_adjoint_workspace_bytes(self._ctx, int(every), ctypes.byref(b)))
        cache = getattr(self, "_adj_ws", None)
        if cache is None or cache.numel() < b.value:
            self._adj_ws = torch.empty(b.value, dtype=torch.uint8, device=self._dev())
        return self._adj_ws

    def advance_save(self, state, t0, dt, steps, every, ckpt=None, stream=None):
        """Advance in place and return the checkpoint store (uint8 device
        tensor) holding the state before steps 0, every, 2 every, ..."""
        import torch
        self._check_state(state)
        need = self.checkpoint_bytes(steps, every)
        if ckpt is None:
            ckpt = torch.empty(max(need, 256), dtype=torch.uint8, device=self._dev())
        ws = self.workspace()
        check(lib().gals_advance_save(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                                      ctypes.c_void_p(state[1].data_ptr()), float(t0), float(dt),
                                      int(steps), int(every), ctypes.c_void_p(ckpt.data_ptr()),
                                      ckpt.numel(), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream_handle(stream, self._dev())))
        return ckpt

    def _check_adjoint(self, lam):
        import torch
        if (lam.dtype != torch.float64 or tuple(lam.shape) != (3, self.plane)
                or not lam.is_contiguous() or lam.device != self._dev()):
            raise ValueError("adjoint state must be a contiguous (3, plane) float64 tensor on "
                             "the grid's device")

    def adjoint(self, ckpt, t0, dt, steps, every, lam, dS=None, stream=None):
        """Reverse sweep: lam (dF/du at the final state) becomes dF/du at the
        initial state, in place; returns dF/dS as a 16-value FP64 device
        tensor (index 4 (m-1) + (n-1))."""
        import torch
        self._check_adjoint(lam)
        if dS is None:
            dS = torch.zeros(16, dtype=torch.float64, device=self._dev())
        ws = self._adjoint_workspace(every)
        check(lib().gals_adjoint(self._ctx, ctypes.c_void_p(ckpt.data_ptr()), ckpt.numel(),
                                 float(t0), float(dt), int(steps), int(every),
                                 ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(dS.data_ptr()),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream_handle(stream, self._dev())))
        return dS

    def adjoint_step(self, state, t, dt, lam_in, lam_out=None, dS=None, stream=None):
        """One reverse step from time t; returns (lam_out, dS) with dS += the
        step's dF/dS."""
        import torch
        self._check_state(state)
        self._check_adjoint(lam_in)
        if lam_out is None:
            lam_out = self.empty_adjoint()
        self._check_adjoint(lam_out)
        if dS is None:
            dS = torch.zeros(16, dtype=torch.float64, device=self._dev())
        ws = self._adjoint_workspace(1)
        check(lib().gals_adjoint_step(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                                      ctypes.c_void_p(state[1].data_ptr()), float(t), float(dt),
                                      ctypes.c_void_p(lam_in.data_ptr()),
                                      ctypes.c_void_p(lam_out.data_ptr()),
                                      ctypes.c_void_p(dS.data_ptr()),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream_handle(stream, self._dev())))
        return lam_out, dS

    def shape_loss(self, state, ref, eps, with_grad=True, stream=None):
        """(loss, lam): the smoothed-Heaviside shape loss against ref and, if
        with_grad, its derivative as an FP64 adjoint state (else None)."""
        self._check_state(state)
        self._check_state(ref)
        lam = self.empty_adjoint() if with_grad else None
        out = ctypes.c_double()
        ws = self.workspace()
        check(lib().gals_shape_loss(self._ctx, ctypes.c_void_p(state[0].data_ptr()),
                                    ctypes.c_void_p(ref[0].data_ptr()), float(eps),
                                    ctypes.byref(out),
                                    ctypes.c_void_p(lam.data_ptr()) if lam is not None else None,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream_handle(stream, self._dev())))
        return out.value, lam


class Batch:
    """Many independent 2D grids with sine stream-function fields, advanced
    together (one launch per step, one block per tile). ``ncells`` is a list of
    (nx, ny) cell counts; every grid is the unit square unless lo/hi are
    given per problem."""

    def __init__(self, ncells, lo=None, hi=None, dtype="float32", mixed=MIXED_CENTRAL,
                 bc=BC_NEUMANN, device=0):
        self.nprob = len(ncells)
        self.ncells = [tuple(int(v) for v in n) for n in ncells]
        lo = np.zeros((self.nprob, 2)) if lo is None else np.asarray(lo, dtype=np.float64)
        hi = np.ones((self.nprob, 2)) if hi is None else np.asarray(hi, dtype=np.float64)
        if dtype in ("float32", "f32", np.float32):
            self.prec = F32
        elif dtype in ("float64", "f64", np.float64):
            self.prec = F64
        else:
            raise ValueError(f"unsupported dtype {dtype!r}")
        self.device = int(device)
        nc = np.ascontiguousarray(self.ncells, dtype=np.int64).ravel()
        lo = np.ascontiguousarray(lo, dtype=np.float64).ravel()
        hi = np.ascontiguousarray(hi, dtype=np.float64).ravel()
        self._b = ctypes.c_void_p()
        P64 = ctypes.POINTER(ctypes.c_int64)
        PD = ctypes.POINTER(ctypes.c_double)
        check(lib().gals_batch_create(ctypes.byref(self._b), self.nprob,
                                      nc.ctypes.data_as(P64), lo.ctypes.data_as(PD),
                                      hi.ctypes.data_as(PD), self.prec, int(mixed), int(bc),
                                      self.device))
        self.offset = np.zeros(self.nprob, dtype=np.int64)
        self.pitch = np.zeros(self.nprob, dtype=np.int64)
        self.plane = np.zeros(self.nprob, dtype=np.int64)
        total = ctypes.c_int64()
        check(lib().gals_batch_layout(self._b, self.offset.ctypes.data_as(P64),
                                      self.pitch.ctypes.data_as(P64),
                                      self.plane.ctypes.data_as(P64), ctypes.byref(total)))
        self.total_elems = total.value
        wsb = ctypes.c_size_t()
        check(lib().gals_batch_workspace_bytes(self._b, ctypes.byref(wsb)))
        self.workspace_bytes = wsb.value
        self._ws = None

    def __del__(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value and _lib is not None:
            _lib.gals_batch_destroy(b)
            self._b = None

    @property
    def torch_dtype(self):
        import torch
        return torch.float32 if self.prec == F32 else torch.float64

    def _dev(self):
        import torch
        return torch.device("cuda", self.device)

    def num_nodes(self):
        return sum((nx + 1) * (ny + 1) for nx, ny in self.ncells)

    def set_velocity(self, p, kind, params, period=0.0):
        arr = np.ascontiguousarray(params, dtype=np.float64)
        check(lib().gals_batch_set_velocity(self._b, int(p), int(kind),
                                            arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            arr.size, float(period)))

    def set_tiles(self, widths):
        arr = (ctypes.c_int * 4)(*[int(w) for w in widths])
        check(lib().gals_batch_set_tiles(self._b, arr))

    def get_tiles(self):
        arr = (ctypes.c_int * 4)()
        check(lib().gals_batch_get_tiles(self._b, arr))
        return list(arr)

    def empty_state(self):
        import torch
        return torch.zeros(self.total_elems, dtype=self.torch_dtype, device=self._dev())

    def _views(self, state, p):
        nx, ny = self.ncells[p]
        o, pl, pt = int(self.offset[p]), int(self.plane[p]), int(self.pitch[p])
        return [state[o + a * pl: o + (a + 1) * pl].view(ny + 1, pt)[:, : nx + 1] for a in range(3)]

    def from_numpy(self, states):
        """Device state from a list of dense (phi, psi) float64 pairs."""
        import torch
        st = self.empty_state()
        for p, (phi, psi) in enumerate(states):
            nx, ny = self.ncells[p]
            planes = [np.asarray(phi).reshape(ny + 1, nx + 1)] + list(
                np.asarray(psi).reshape(2, ny + 1, nx + 1))
            for v, arr in zip(self._views(st, p), planes):
                v.copy_(torch.from_numpy(np.ascontiguousarray(arr)).to(st.dtype))
        return st

    def to_numpy(self, state, p):
        v = self._views(state, p)
        phi = v[0].double().cpu().numpy().ravel()
        psi = np.concatenate([v[1].double().cpu().numpy().ravel(),
                              v[2].double().cpu().numpy().ravel()])
        return phi, psi

    def workspace(self):
        import torch
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self._dev())
        return self._ws

    def _check_state(self, state):
        if (state.dtype != self.torch_dtype or not state.is_cuda or not state.is_contiguous()
                or state.numel() < self.total_elems or state.device.index != self.device):
            raise ValueError("batch state must be a contiguous device tensor of "
                             f"{self.total_elems} {self.torch_dtype} elements on cuda:{self.device}")

    def advance(self, state, t0, dt, steps, graph=False, stream=None):
        self._check_state(state)
        ws = self.workspace()
        check(lib().gals_batch_advance(self._b, ctypes.c_void_p(state.data_ptr()), float(t0),
                                       float(dt), int(steps), int(bool(graph)),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream_handle(stream, self._dev())))
        return state

    def autotune(self, scratch_state, dt, steps=4, stream=None):
        """Pick the wave shape per size class by timing; advances scratch_state."""
        self._check_state(scratch_state)
        ws = self.workspace()
        best = ctypes.c_double()
        check(lib().gals_batch_autotune(self._b, ctypes.c_void_p(scratch_state.data_ptr()),
                                        float(dt), int(steps), ctypes.c_void_p(ws.data_ptr()),
                                        ws.numel(), _stream_handle(stream, self._dev()),
                                        ctypes.byref(best)))
        return best.value
