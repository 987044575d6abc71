"""ctypes binding of the plain FP64 CPU oracle (``gals_oracle.c``).

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does. Arrays are float64 numpy
arrays, dense and x fastest (index ``i + nx*(j + ny*k)``), with ``psi`` stored
as ``dim`` planes back to back.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "gals_oracle.c"), os.path.join(_HERE, "gals_oracle_cs.c")]
_LIB_PATH = os.path.join(_HERE, "libgals_oracle.so")

# Velocity kinds (same numbering as the GPU library's public header; each side
# defines its own copy).
AFFINE, STREAM_SIN, VECPOT_SIN, VORTEX, PSEUDO1D, LEVEQUE3D = 1, 2, 3, 4, 5, 6
MIXED_CENTRAL, MIXED_CELL, MIXED_ZERO = 0, 1, 2
PSI_SUPERCONSISTENT, PSI_HEUN = 0, 1
BC_NEUMANN, BC_EXTRAPOLATE, BC_INFLOW_NEUMANN = 0, 1, 3

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction). -O3 for a
    fair CPU baseline; the instruction set is x86-64-v3 (AVX2) rather than
    -march=native because the library is built on one host and run on
    another (the GPU machine's). Without FMA contraction or reassociation the
    results do not depend on these flags."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", _LIB_PATH, *_SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(_LIB_PATH)
            for s in _SRCS + [os.path.join(_HERE, "gals_oracle.h")]):
        build()  # missing or older than its sources
    lib = ctypes.CDLL(_LIB_PATH)
    D = ctypes.POINTER(ctypes.c_double)
    L = ctypes.POINTER(ctypes.c_long)
    i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
    lib.orc_basis.argtypes = [i, i, i, d, D]
    lib.orc_hermite.argtypes = [i, D, D, D, D, D, D]
    lib.orc_mixed.argtypes = [i, L, D, D, i, D, D]
    lib.orc_velocity.argtypes = [i, i, D, l, d, D, d, D, D]
    lib.orc_trace.argtypes = [i, i, D, l, d, D, d, d, D, D]
    lib.orc_advance.argtypes = [i, L, D, D, i, D, l, d, i, i, i, D, D, d, d, l]
    lib.orc_step_nodes.argtypes = [i, L, D, D, i, D, l, d, i, i, i, D, D, d, d, L, l, D, D]
    lib.orc_eval_points.argtypes = [i, L, D, D, i, D, D, D, l, D, D, D, D, D]
    lib.orc_norms.argtypes = [i, L, D, D, D, D, D, D, d, d, D]
    lib.orc_max_speed.argtypes = [i, L, D, D, i, D, l, d, d]
    lib.orc_max_speed.restype = d
    lib.orc_apply_inflow.argtypes = [i, L, D, D, i, D, l, d, d, d, D, D, D, D, D]
    lib.orc_grad_cs.argtypes = [L, D, D, D, l, d, i, i, D, D, d, d, l, D, D, d, D, D]
    lib.orc_num_threads.argtypes = []
    lib.orc_set_threads.argtypes = [i]
    lib.orc_set_sum_order.argtypes = [i]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _geom(ncell, lo, hi):
    nc = np.ascontiguousarray(ncell, dtype=np.int64).astype(np.int_)
    return (nc, _f64(lo), _f64(hi),
            nc.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))


def _params(params):
    p = _f64(params if params is not None else np.zeros(0))
    return p, (len(p))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments")


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    _check(_load().orc_set_threads(int(n)), "set_threads")


def set_sum_order(order: int) -> None:
    """Order of the Hermite sums from now on: 0 (default) the literal sum over
    every (vertex, derivative) pair, 1 axis by axis. Both evaluate the same
    definition in FP64; they differ only in rounding."""
    _check(_load().orc_set_sum_order(int(order)), "set_sum_order")


def basis(v: int, alpha: int, deriv: int, x: float) -> float:
    out = ctypes.c_double()
    _check(_load().orc_basis(v, alpha, deriv, x, ctypes.byref(out)), "basis")
    return out.value


def hermite(dim, data, h, xi):
    """Value, gradient and Hessian of the p-cubic on one cell."""
    data, h, xi = _f64(data), _f64(h), _f64(xi)
    val = np.zeros(1)
    grad = np.zeros(dim)
    hess = np.zeros(dim * dim)
    _check(_load().orc_hermite(dim, _dp(data), _dp(h), _dp(xi), _dp(val), _dp(grad),
                               _dp(hess)), "hermite")
    return val[0], grad, hess.reshape(dim, dim)


def mixed(dim, ncell, lo, hi, psi, mode=MIXED_CENTRAL):
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    psi = _f64(psi)
    nodes = int(np.prod(nc + 1))
    out = np.zeros((1 if dim == 2 else 4) * nodes)
    _check(_load().orc_mixed(dim, ncp, _dp(lo), _dp(hi), mode, _dp(psi), _dp(out)), "mixed")
    return out


def velocity(dim, kind, params, period, x, t):
    p, npar = _params(params)
    x = _f64(x)
    v = np.zeros(dim)
    G = np.zeros(dim * dim)
    _check(_load().orc_velocity(dim, kind, _dp(p), npar, period, _dp(x), t, _dp(v), _dp(G)),
           "velocity")
    return v, G.reshape(dim, dim)


def trace(dim, kind, params, period, x, t, dt):
    p, npar = _params(params)
    x = _f64(x)
    X = np.zeros(dim)
    D = np.zeros(dim * dim)
    _check(_load().orc_trace(dim, kind, _dp(p), npar, period, _dp(x), t, dt, _dp(X), _dp(D)),
           "trace")
    return X, D.reshape(dim, dim)


def advance(dim, ncell, lo, hi, kind, params, period, phi, psi, t0, dt, steps,
            mixed_mode=MIXED_CENTRAL, bc=BC_NEUMANN, psi_update=PSI_SUPERCONSISTENT):
    """Return (phi, psi) after ``steps`` steps; the inputs are not modified."""
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    p, npar = _params(params)
    phi = _f64(phi).copy()
    psi = _f64(psi).copy()
    _check(_load().orc_advance(dim, ncp, _dp(lo), _dp(hi), kind, _dp(p), npar, period,
                               mixed_mode, bc, psi_update, _dp(phi), _dp(psi), t0, dt,
                               int(steps)), "advance")
    return phi, psi


def step_nodes(dim, ncell, lo, hi, kind, params, period, phi, psi, t, dt, nodes,
               mixed_mode=MIXED_CENTRAL, bc=BC_NEUMANN, psi_update=PSI_SUPERCONSISTENT):
    """One step from t to t+dt at the given flat node indices."""
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    p, npar = _params(params)
    phi, psi = _f64(phi), _f64(psi)
    nodes = np.ascontiguousarray(nodes, dtype=np.int_)
    cnt = len(nodes)
    po = np.zeros(cnt)
    go = np.zeros(cnt * dim)
    _check(_load().orc_step_nodes(dim, ncp, _dp(lo), _dp(hi), kind, _dp(p), npar, period,
                                  mixed_mode, bc, psi_update, _dp(phi), _dp(psi), t, dt,
                                  nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), cnt,
                                  _dp(po), _dp(go)), "step_nodes")
    return po, go.reshape(cnt, dim)


def eval_points(dim, ncell, lo, hi, phi, psi, pts, mixed_mode=MIXED_CENTRAL):
    """pts: (npts, dim). Returns dict of val, grad, hess, normal, kappa."""
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    phi, psi = _f64(phi), _f64(psi)
    pts = _f64(pts).reshape(-1, dim)
    n = pts.shape[0]
    val = np.zeros(n)
    grad = np.zeros(n * dim)
    hess = np.zeros(n * dim * dim)
    normal = np.zeros(n * dim)
    kappa = np.zeros(n)
    _check(_load().orc_eval_points(dim, ncp, _dp(lo), _dp(hi), mixed_mode, _dp(phi),
                                   _dp(psi), _dp(pts), n, _dp(val), _dp(grad), _dp(hess),
                                   _dp(normal), _dp(kappa)), "eval_points")
    return {"val": val, "grad": grad.reshape(n, dim), "hess": hess.reshape(n, dim, dim),
            "normal": normal.reshape(n, dim), "kappa": kappa}


def norms(dim, ncell, lo, hi, phi, psi, phi_ref, psi_ref, eps, band):
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    out = np.zeros(8)
    args = [_f64(a) for a in (phi, psi, phi_ref, psi_ref)]
    _check(_load().orc_norms(dim, ncp, _dp(lo), _dp(hi), *[_dp(a) for a in args], eps, band,
                             _dp(out)), "norms")
    return out


def max_speed(dim, ncell, lo, hi, kind, params, period, t):
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    p, npar = _params(params)
    r = _load().orc_max_speed(dim, ncp, _dp(lo), _dp(hi), kind, _dp(p), npar, period, t)
    if r < 0:
        raise ValueError("oracle max_speed rejected its arguments")
    return r


def grad_cs(ncell, lo, hi, params, period, phi0, psi0, t0, dt, steps, lam=None,
            phi_target=None, eps=0.0, mixed_mode=MIXED_CENTRAL, bc=BC_NEUMANN):
    """Complex-step derivatives of a functional of the final 2D state with
    respect to the folded sine stream-function table S[m][n] (returned as a
    4 x 4 array, [m-1][n-1]). lam (3 N values: weights of phi, psi_x, psi_y)
    selects the linear functional sum(lam . u_T); otherwise the loss
    prod(h) sum (H_eps(phi_T) - H_eps(phi_target))^2. Returns (value, grad)."""
    nc, lo, hi, ncp = _geom(ncell, lo, hi)
    p, npar = _params(params)
    phi0, psi0 = _f64(phi0), _f64(psi0)
    lam = None if lam is None else _f64(lam)
    tgt = None if phi_target is None else _f64(phi_target)
    grad = np.zeros(16)
    val = ctypes.c_double()
    _check(_load().orc_grad_cs(ncp, _dp(lo), _dp(hi), _dp(p), npar, period, mixed_mode, bc,
                               _dp(phi0), _dp(psi0), t0, dt, steps, _dp(lam), _dp(tgt), eps,
                               ctypes.byref(val), _dp(grad)), "grad_cs")
    return val.value, grad.reshape(4, 4)


def advance_inflow(dim, ncell, lo, hi, kind, params, period, phi, psi, t0, dt, steps, inflow,
                   mixed_mode=MIXED_CENTRAL, psi_update=PSI_SUPERCONSISTENT):
    """Advance with Dirichlet inflow data: inflow(t) returns (phi_b, grad_b,
    phit_b) at every node for time t; each step is followed by
    orc_apply_inflow at its end time. Feet outside the domain are projected
    (homogeneous Neumann) as with bc 0."""
    nc, lo_, hi_, ncp = _geom(ncell, lo, hi)
    p, npar = _params(params)
    for n in range(steps):
        t = t0 + n * dt
        phi, psi = advance(dim, ncell, lo, hi, kind, params, period, phi, psi, t, dt, 1,
                           mixed_mode=mixed_mode, bc=BC_NEUMANN, psi_update=psi_update)
        pb, gb, tb = (_f64(a) for a in inflow(t + dt))
        _check(_load().orc_apply_inflow(dim, ncp, _dp(lo_), _dp(hi_), kind, _dp(p), npar, period,
                                        t + dt, dt, _dp(phi), _dp(psi), _dp(pb), _dp(gb),
                                        _dp(tb)),
               "apply_inflow")
    return phi, psi
