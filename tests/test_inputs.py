"""Checks of the seeded input generators that need no GPU."""
import numpy as np

from paper_0905_3409_amd import inputs


def test_box_signed_distance_matches_brute_force():
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, (2000, 3))
    coords = [pts[:, a] for a in range(3)]
    c, half = (0.35, 0.35, 0.35), (0.15, 0.15, 0.15)
    phi, psi = inputs.sdf_box(coords, c, half)
    # distance to the box: clamp each point to the box
    clamped = np.clip(pts, np.array(c) - half, np.array(c) + half)
    outside = np.linalg.norm(pts - clamped, axis=1)
    inside_depth = np.min(np.array(half) - np.abs(pts - c), axis=1)
    want = np.where(outside > 0, outside, -inside_depth)
    assert np.abs(phi - want).max() < 1e-14
    # the gradient is the derivative of phi (away from the box's ridges)
    eps = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        fp = inputs.sdf_box([pts[:, b] + e[b] for b in range(3)], c, half)[0]
        fm = inputs.sdf_box([pts[:, b] - e[b] for b in range(3)], c, half)[0]
        assert np.median(np.abs((fp - fm) / (2 * eps) - psi[a * 2000:(a + 1) * 2000])) < 1e-8


def test_leveque_shapes():
    w = inputs.leveque_shape("sphere", 40)
    assert w["steps"] == 100 and w["dt"] == 1 / 40 and w["period"] == 2.5
    assert w["phi0"].min() < 0 < w["phi0"].max()


def test_separable_sines_gradient_is_exact():
    """psi of the separable state is the gradient of phi: central differences
    of the analytic factors on a fine axis agree to O(h^2)."""
    for dim in (2, 3):
        ncell = (4000,) + (7,) * (dim - 1)
        F, dF = inputs.separable_sines(5, ncell)
        h = 1.0 / 4000
        fd = (F[0][2:] - F[0][:-2]) / (2 * h)
        assert np.max(np.abs(fd - dF[0][1:-1])) <= 1e-4 * np.max(np.abs(dF[0]))
        phi, psi = inputs.separable_dense(F, dF)
        n = [c + 1 for c in ncell]
        P = phi.reshape(tuple(reversed(n)))
        G = psi.reshape((dim,) + tuple(reversed(n)))
        # x is the last array axis: psi_x = dF_x times the other factors
        other = F[1][:, None] if dim == 2 else F[2][:, None, None] * F[1][None, :, None]
        np.testing.assert_allclose(G[0], other * dF[0], rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(P, other * F[0], rtol=1e-15, atol=1e-15)
