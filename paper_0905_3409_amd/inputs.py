"""Seeded synthetic workloads for the GA-CIR step.

This module only draws inputs: grid geometry, analytic initial level sets with
their exact gradients, and velocity-field parameters. It holds none of the
scheme's arithmetic (no tracing, interpolation or cross-derivative
reconstruction), so both the GPU library and the CPU oracle can consume what it
produces. All arrays are float64, dense, x fastest (``i + nx*(j + ny*k)``);
``psi`` is ``dim`` planes back to back.

Workloads (domain [0,1]^d, h = 1/N, nodes = N+1 per axis):

* ``rotation_circle`` - 64^2 cells, circle of radius 0.15 with a seeded centre
  in [0.35,0.65]^2, rigid rotation about (1/2,1/2) at 2 pi per unit time, one
  revolution in 128 steps.
* ``stream_circles`` - 2048^2 cells, signed distance to the union of 4 seeded
  circles (radii in [0.05,0.15]), an 8-mode sine stream function modulated by
  cos(pi t / 2); 1024 steps to t = 2 at CFL 0.8, after which the flow has
  returned every point to its start.
* ``vecpot_spheres`` - 256^3 cells, union of 8 seeded spheres (radii in
  [0.05,0.12]), velocity = curl of a 6-mode sine vector potential modulated by
  cos(pi t / 3); 512 steps to t = 3 at CFL 0.9.

The mode amplitudes are drawn N(0, 0.05^2) and then scaled by one common factor
so that the largest node speed at t = 0 equals CFL * h / dt.
"""
from __future__ import annotations

import math

import numpy as np

AFFINE, STREAM_SIN, VECPOT_SIN, VORTEX, PSEUDO1D, LEVEQUE3D = 1, 2, 3, 4, 5, 6


def node_axes(ncell, lo=None, hi=None):
    """1D node coordinate arrays, x_i = lo + i * (hi - lo) / N."""
    dim = len(ncell)
    lo = np.zeros(dim) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.ones(dim) if hi is None else np.asarray(hi, dtype=np.float64)
    axes = []
    for a in range(dim):
        h = (hi[a] - lo[a]) / ncell[a]
        axes.append(lo[a] + np.arange(ncell[a] + 1, dtype=np.float64) * h)
    return axes


def node_grid(ncell, lo=None, hi=None):
    """Coordinate arrays of every node, each flattened x fastest."""
    axes = node_axes(ncell, lo, hi)
    mesh = np.meshgrid(*axes, indexing="ij")
    # meshgrid(indexing="ij") puts x on axis 0; flatten with x fastest
    return [np.ascontiguousarray(m.transpose()).ravel() for m in mesh]


# ---------------------------------------------------------------------------
# Initial level sets (analytic values and exact gradients)
# ---------------------------------------------------------------------------
def sdf_union(coords, centres, radii):
    """Signed distance to a union of balls: min_k(|x - c_k| - r_k), negative
    inside; the gradient is that of the minimising ball (lowest k on ties),
    and zero at a ball's exact centre."""
    dim = len(coords)
    best = None
    grad = None
    for c, r in zip(centres, radii):
        diff = [coords[a] - c[a] for a in range(dim)]
        dist = np.sqrt(sum(d * d for d in diff))
        val = dist - r
        safe = np.where(dist > 0, dist, 1.0)
        g = [np.where(dist > 0, d / safe, 0.0) for d in diff]
        if best is None:
            best, grad = val, g
        else:
            take = val < best
            best = np.where(take, val, best)
            grad = [np.where(take, gn, go) for gn, go in zip(g, grad)]
    return best, np.concatenate(grad)


def sdf_box(coords, centre, half):
    """Signed distance to an axis-aligned box (centre, half side lengths),
    negative inside, with its gradient: outside, the direction from the
    nearest point of the box; inside, the outward normal of the nearest face
    (lowest axis on ties; +x side at the exact centre)."""
    dim = len(coords)
    s = [np.where(coords[a] - centre[a] >= 0, 1.0, -1.0) for a in range(dim)]
    q = [np.abs(coords[a] - centre[a]) - half[a] for a in range(dim)]
    qp = [np.maximum(qa, 0.0) for qa in q]
    outside = np.sqrt(sum(v * v for v in qp))
    qmax = np.max(np.stack(q), axis=0)
    phi = outside + np.minimum(qmax, 0.0)
    kmax = np.argmax(np.stack(q), axis=0)
    safe = np.where(outside > 0, outside, 1.0)
    grad = []
    for a in range(dim):
        g_out = qp[a] / safe * s[a]
        g_in = np.where(kmax == a, s[a], 0.0)
        grad.append(np.where(outside > 0, g_out, g_in))
    return phi, np.concatenate(grad)


def separable_sines(seed, ncell, lo=None, hi=None):
    """Factors of phi = prod_a sin(k_a x_a + p_a) on the node axes, with seeded
    wavenumbers k_a in [2 pi, 6 pi] and phases p_a in [0, 2 pi): returns the
    per-axis values F_a and derivatives dF_a. A dense state is formed from them
    by products in a fixed order (``separable_dense``), so any window of it can
    be rebuilt bit for bit without forming the whole grid, which is what a
    grid of several hundred million nodes needs."""
    dim = len(ncell)
    rng = np.random.default_rng(seed)
    k = rng.uniform(2.0 * math.pi, 6.0 * math.pi, dim)
    p = rng.uniform(0.0, 2.0 * math.pi, dim)
    axes = node_axes(ncell, lo, hi)
    F = [np.sin(k[a] * axes[a] + p[a]) for a in range(dim)]
    dF = [k[a] * np.cos(k[a] * axes[a] + p[a]) for a in range(dim)]
    return F, dF


def separable_dense(F, dF, window=None):
    """Dense phi and psi (x fastest) of the product of the factors over the
    node ranges window = [(start, stop) per axis] (default: all nodes). The
    products are taken as (F_x F_y) F_z, with dF_a in place of F_a for
    psi_a, each a single rounding, so a GPU-side broadcast product in the same
    order gives the same values."""
    dim = len(F)
    if window is None:
        window = [(0, len(F[a])) for a in range(dim)]
    sl = [slice(*w) for w in window]

    def prod(fs):
        v = fs[1][sl[1]][:, None] * fs[0][sl[0]][None, :]
        if dim == 3:
            v = fs[2][sl[2]][:, None, None] * v[None, :, :]
        return v.ravel()

    phi = prod(F)
    psi = np.concatenate([prod([dF[b] if b == a else F[b] for b in range(dim)])
                          for a in range(dim)])
    return phi, psi


def gaussian_bump(coords, x0, r0=0.15):
    """exp(-|x - x0|^2) - exp(-r0^2) and its gradient (the smooth initial data
    of the paper's accuracy tests)."""
    dim = len(coords)
    diff = [coords[a] - x0[a] for a in range(dim)]
    e = np.exp(-sum(d * d for d in diff))
    phi = e - math.exp(-r0 * r0)
    psi = np.concatenate([-2.0 * d * e for d in diff])
    return phi, psi


# ---------------------------------------------------------------------------
# Velocity parameters
# ---------------------------------------------------------------------------
def rotation_params(omega=2.0 * math.pi, centre=(0.5, 0.5)):
    """Rigid rotation v = omega (-(y - cy), x - cx) as an AFFINE field."""
    return np.array([0.0, 0.0, centre[0], centre[1], 0.0, -omega, omega, 0.0])


def affine_params(b, c, A):
    b = np.asarray(b, dtype=np.float64).ravel()
    c = np.asarray(c, dtype=np.float64).ravel()
    A = np.asarray(A, dtype=np.float64).ravel()
    return np.concatenate([b, c, A])


def _stream_speed_max(params, ncell):
    """Largest node speed of the sine stream-function field at t = 0."""
    ax = node_axes(ncell)
    x, y = ax[0][:, None], ax[1][None, :]
    u = np.zeros((len(ax[0]), len(ax[1])))
    v = np.zeros_like(u)
    for a, m, n in params.reshape(-1, 3):
        u -= a * n * math.pi * np.sin(m * math.pi * x) * np.cos(n * math.pi * y)
        v += a * m * math.pi * np.cos(m * math.pi * x) * np.sin(n * math.pi * y)
    return float(np.sqrt(u * u + v * v).max())


def _vecpot_speed_max(params, ncell):
    """Largest node speed of curl A for the sine vector potential, t = 0."""
    ax = node_axes(ncell)
    x = ax[0][:, None, None]
    best = 0.0
    modes = params.reshape(-1, 6)
    pi = math.pi
    for z0 in range(0, len(ax[2]), 16):
        z = ax[2][None, None, z0:z0 + 16]
        y = ax[1][None, :, None]
        v = [0.0, 0.0, 0.0]
        for axm, aym, azm, l, m, n in modes:
            L, M, N = l * pi, m * pi, n * pi
            sx, cx = np.sin(L * x), np.cos(L * x)
            sy, cy = np.sin(M * y), np.cos(M * y)
            sz, cz = np.sin(N * z), np.cos(N * z)
            fx = L * cx * sy * sz
            fy = M * sx * cy * sz
            fz = N * sx * sy * cz
            v[0] = v[0] + azm * fy - aym * fz
            v[1] = v[1] + axm * fz - azm * fx
            v[2] = v[2] + aym * fx - axm * fy
        s = np.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
        best = max(best, float(s.max()))
    return best


def stream_modes(rng, nmodes, ncell, vmax, maxidx=4, sigma=0.05):
    """(a, m, n) per mode, a ~ N(0, sigma^2) scaled so the max node speed at
    t = 0 is vmax; m, n uniform in 1..maxidx."""
    a = rng.normal(0.0, sigma, nmodes)
    m = rng.integers(1, maxidx + 1, nmodes)
    n = rng.integers(1, maxidx + 1, nmodes)
    params = np.stack([a, m, n], axis=1).astype(np.float64).ravel()
    s = _stream_speed_max(params, ncell)
    params.reshape(-1, 3)[:, 0] *= vmax / s
    return params


def vecpot_modes(rng, nmodes, ncell, vmax, maxidx=4, sigma=0.05):
    """(ax, ay, az, l, m, n) per mode, amplitudes N(0, sigma^2) scaled so the
    max node speed at t = 0 is vmax; l, m, n uniform in 1..maxidx."""
    amp = rng.normal(0.0, sigma, (nmodes, 3))
    idx = rng.integers(1, maxidx + 1, (nmodes, 3))
    params = np.concatenate([amp, idx], axis=1).astype(np.float64).ravel()
    s = _vecpot_speed_max(params, ncell)
    params.reshape(-1, 6)[:, :3] *= vmax / s
    return params


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def _workload(name, ncell, kind, params, period, dt, steps, phi, psi, **meta):
    dim = len(ncell)
    return dict(name=name, dim=dim, ncell=tuple(int(n) for n in ncell),
                lo=(0.0,) * dim, hi=(1.0,) * dim, kind=kind,
                params=np.asarray(params, dtype=np.float64), period=float(period),
                t0=0.0, dt=float(dt), steps=int(steps), phi0=phi, psi0=psi, **meta)


def rotation_circle(seed=0, n=64, steps=128):
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0.35, 0.65, 2)
    ncell = (n, n)
    phi, psi = sdf_union(node_grid(ncell), [centre], [0.15])
    return _workload("rotation_circle", ncell, AFFINE, rotation_params(), 0.0,
                     1.0 / steps, steps, phi, psi, seed=seed, centre=centre)


def stream_circles(seed=1, n=2048, steps=1024, cfl=0.8, period=2.0, ncircles=4,
                   nmodes=8):
    rng = np.random.default_rng(seed)
    ncell = (n, n)
    centres = rng.uniform(0.2, 0.8, (ncircles, 2))
    radii = rng.uniform(0.05, 0.15, ncircles)
    dt = period / steps
    vmax = cfl * (1.0 / n) / dt
    params = stream_modes(rng, nmodes, ncell, vmax)
    phi, psi = sdf_union(node_grid(ncell), centres, radii)
    return _workload("stream_circles", ncell, STREAM_SIN, params, period, dt, steps,
                     phi, psi, seed=seed, cfl=cfl, centres=centres, radii=radii)


def vecpot_spheres(seed=2, n=256, steps=512, cfl=0.9, period=3.0, nspheres=8,
                   nmodes=6):
    rng = np.random.default_rng(seed)
    ncell = (n, n, n)
    centres = rng.uniform(0.2, 0.8, (nspheres, 3))
    radii = rng.uniform(0.05, 0.12, nspheres)
    dt = period / steps
    vmax = cfl * (1.0 / n) / dt
    params = vecpot_modes(rng, nmodes, ncell, vmax)
    phi, psi = sdf_union(node_grid(ncell), centres, radii)
    return _workload("vecpot_spheres", ncell, VECPOT_SIN, params, period, dt, steps,
                     phi, psi, seed=seed, cfl=cfl, centres=centres, radii=radii)


def batched_stream_circles(seed=4, nprob=512, steps=256, cfl=0.8, period=2.0,
                           log2_min=5.0, log2_max=9.0, sizes=None):
    """Many independent unit-square problems: cells per side
    round(2^U(log2_min, log2_max)) (32^2 .. 512^2 by default; ``sizes``, a
    list of (nx, ny), overrides the draw), each with its own 4-circle union and
    its own 8-mode sine stream function scaled so that the largest node speed
    at t = 0 is cfl * h / dt, h the smaller cell side, dt = period / steps."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sides = np.rint(2.0 ** rng.uniform(log2_min, log2_max, nprob)).astype(int)
        sizes = [(int(n), int(n)) for n in sides]
    dt = period / steps
    probs = []
    for nx, ny in sizes:
        ncell = (int(nx), int(ny))
        centres = rng.uniform(0.2, 0.8, (4, 2))
        radii = rng.uniform(0.05, 0.15, 4)
        params = stream_modes(rng, 8, ncell, cfl * (1.0 / max(ncell)) / dt)
        phi, psi = sdf_union(node_grid(ncell), centres, radii)
        probs.append(dict(ncell=ncell, params=params, phi0=phi, psi0=psi))
    return dict(name="batched_stream_circles", kind=STREAM_SIN, period=float(period),
                dt=float(dt), steps=int(steps), t0=0.0, problems=probs, seed=seed, cfl=cfl)


def adjoint_circles(seed=5, n=1024, steps=200, nmodes=16, cfl=0.8, target_seed=6):
    """Parameter-gradient workload: 4 seeded circles (as stream_circles) on
    n^2 cells, a steady sine stream function of nmodes modes with
    (m, n) ~ U{1..4}^2 and amplitudes a ~ N(0, 0.05^2) (unscaled), target
    amplitudes for the same modes drawn from target_seed, and
    dt = cfl h / max |v_a| at the base amplitudes, steps steps."""
    rng = np.random.default_rng(seed)
    ncell = (n, n)
    centres = rng.uniform(0.2, 0.8, (4, 2))
    radii = rng.uniform(0.05, 0.15, 4)
    modes = rng.integers(1, 5, (nmodes, 2))
    amps = rng.normal(0.0, 0.05, nmodes)
    target = np.random.default_rng(target_seed).normal(0.0, 0.05, nmodes)
    params = np.stack([amps, modes[:, 0], modes[:, 1]], axis=1).astype(np.float64).ravel()
    vmax = _stream_speed_max(params, ncell)
    dt = cfl * (1.0 / n) / vmax
    phi, psi = sdf_union(node_grid(ncell), centres, radii)
    return dict(name="adjoint_circles", ncell=ncell, modes=modes, amps=amps, target_amps=target,
                dt=float(dt), steps=int(steps), period=0.0, t0=0.0, eps=1.5 / n, phi0=phi,
                psi0=psi, seed=seed, target_seed=target_seed, cfl=cfl)


def leveque_shape(shape="sphere", n=50, period=2.5):
    """The 3D deformation test with volume loss (sec. 6.2): LeVeque's field
    x cos(pi t / T), T = 2.5, on n^3 cells of [0,1]^3, dt = h, run to t = T
    (2.5 n steps); a sphere of radius 0.15 or a cube of side 0.3, centred at
    (0.35, 0.35, 0.35)."""
    ncell = (n, n, n)
    coords = node_grid(ncell)
    c = (0.35, 0.35, 0.35)
    if shape == "sphere":
        phi, psi = sdf_union(coords, [c], [0.15])
    elif shape == "cube":
        phi, psi = sdf_box(coords, c, (0.15, 0.15, 0.15))
    else:
        raise ValueError(shape)
    steps = int(round(period * n))
    return _workload(f"leveque_{shape}", ncell, LEVEQUE3D, np.zeros(0), period, 1.0 / n, steps,
                     phi, psi, shape=shape)


def random_points(seed, npts, dim, lo=0.0, hi=1.0):
    """npts uniform points, shape (npts, dim)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (npts, dim))
