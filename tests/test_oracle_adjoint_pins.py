"""Pins of the oracle's complex-step parameter derivatives (gals_oracle_cs.c)
against the real oracle: its real part must be the real advance's functional,
and its derivatives must match central finite differences of the real
advance (a brute-force derivative on small grids)."""
import math

import numpy as np
import pytest

import oracle
from paper_0905_3409_amd import inputs

NC, LO, HI = (22, 18), (0.0, 0.0), (1.0, 1.0)


def _heaviside(s, eps):
    return np.where(s < -eps, 0.0, np.where(s > eps, 1.0,
                    0.5 * (1.0 + s / eps + np.sin(math.pi * s / eps) / math.pi)))


def _case(seed, nmodes=6, vmax=2.0):
    rng = np.random.default_rng(seed)
    params = inputs.stream_modes(rng, nmodes, NC, vmax)
    phi, psi = inputs.sdf_union(inputs.node_grid(NC), [[0.45, 0.5], [0.7, 0.3]], [0.2, 0.12])
    tgt, _ = inputs.sdf_union(inputs.node_grid(NC), [[0.5, 0.52]], [0.22])
    return params, phi, psi, tgt


def _with_extra(params, m, n, delta):
    return np.concatenate([params, [delta, m, n]])


def _real_functional(params, phi0, psi0, t0, dt, steps, period, lam, tgt, eps, mixed, bc):
    phi, psi = oracle.advance(2, NC, LO, HI, oracle.STREAM_SIN, params, period, phi0, psi0, t0,
                              dt, steps, mixed_mode=mixed, bc=bc)
    if lam is not None:
        N = phi.size
        return float(lam[:N] @ phi + lam[N:2 * N] @ psi[:N] + lam[2 * N:] @ psi[N:])
    h = [(HI[a] - LO[a]) / NC[a] for a in range(2)]
    d = _heaviside(phi, eps) - _heaviside(tgt, eps)
    return float(h[0] * h[1] * np.sum(d * d))


@pytest.mark.parametrize("functional", ["loss", "linear"])
@pytest.mark.parametrize("mixed,bc,period", [(oracle.MIXED_CENTRAL, oracle.BC_NEUMANN, 0.0),
                                             (oracle.MIXED_ZERO, oracle.BC_NEUMANN, 1.7),
                                             (oracle.MIXED_CENTRAL, oracle.BC_EXTRAPOLATE, 0.0)])
def test_complex_step_matches_finite_differences(functional, mixed, bc, period):
    params, phi0, psi0, tgt = _case(3)
    N = phi0.size
    lam = np.random.default_rng(9).normal(size=3 * N) if functional == "linear" else None
    eps = 1.5 / NC[0]
    t0, dt, steps = 0.05, 0.012, 6
    val, g = oracle.grad_cs(NC, LO, HI, params, period, phi0, psi0, t0, dt, steps, lam=lam,
                            phi_target=tgt, eps=eps, mixed_mode=mixed, bc=bc)
    ref = _real_functional(params, phi0, psi0, t0, dt, steps, period, lam, tgt, eps, mixed, bc)
    # the real part is the real advance's functional
    assert abs(val - ref) <= 1e-13 * max(abs(ref), 1e-300) + 1e-15
    fd = np.zeros((4, 4))
    delta = 1e-6
    for m in range(1, 5):
        for n in range(1, 5):
            fp = _real_functional(_with_extra(params, m, n, delta), phi0, psi0, t0, dt, steps,
                                  period, lam, tgt, eps, mixed, bc)
            fm = _real_functional(_with_extra(params, m, n, -delta), phi0, psi0, t0, dt, steps,
                                  period, lam, tgt, eps, mixed, bc)
            fd[m - 1, n - 1] = (fp - fm) / (2 * delta)
    scale = np.max(np.abs(g))
    print(f"{functional}: max|g| {scale:.3e}, max |cs - fd| {np.max(np.abs(g - fd)):.2e}")
    assert scale > 0
    assert np.max(np.abs(g - fd)) <= 1e-6 * scale


def test_zero_steps_have_zero_derivative():
    params, phi0, psi0, tgt = _case(4)
    val, g = oracle.grad_cs(NC, LO, HI, params, 0.0, phi0, psi0, 0.0, 0.01, 0, phi_target=tgt,
                            eps=0.1)
    assert np.all(g == 0.0)
    d = _heaviside(phi0, 0.1) - _heaviside(tgt, 0.1)
    assert abs(val - np.sum(d * d) / (NC[0] * NC[1])) < 1e-15


def test_derivative_is_linear_in_the_weights():
    """For the linear functional, d/dS sum(lam . u_T) is linear in lam."""
    params, phi0, psi0, _ = _case(5)
    N = phi0.size
    rng = np.random.default_rng(2)
    l1, l2 = rng.normal(size=3 * N), rng.normal(size=3 * N)
    args = (NC, LO, HI, params, 0.0, phi0, psi0, 0.0, 0.01, 4)
    _, g1 = oracle.grad_cs(*args, lam=l1)
    _, g2 = oracle.grad_cs(*args, lam=l2)
    _, g12 = oracle.grad_cs(*args, lam=2.0 * l1 - 3.0 * l2)
    assert np.max(np.abs(g12 - (2.0 * g1 - 3.0 * g2))) <= 1e-12 * np.max(np.abs(g12))


def test_modes_sharing_a_wavenumber_pair_share_a_derivative():
    """dF/da_k = dF/dS[m_k][n_k]: splitting a mode into two of the same (m, n)
    leaves the advance, the functional and the derivative table unchanged."""
    params, phi0, psi0, tgt = _case(6, nmodes=3)
    split = np.concatenate([params, params])
    split[0::3] *= 0.5
    args = (NC, LO, HI)
    rest = (0.0, phi0, psi0, 0.0, 0.01, 3)
    v1, g1 = oracle.grad_cs(*args, params, *rest, phi_target=tgt, eps=0.1)
    v2, g2 = oracle.grad_cs(*args, split, *rest, phi_target=tgt, eps=0.1)
    assert abs(v1 - v2) <= 1e-14
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g1))
