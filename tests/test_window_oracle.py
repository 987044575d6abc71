"""The reduction the largest-grid GPU tests rest on: one or two steps of the
oracle on a window of a grid (same node coordinates, the window's data) equal
the steps on the whole grid at every window node farther than a margin from
the window's sides inside the domain. Sides on the domain boundary keep
their nodes. Checked here at sizes where the oracle runs on the whole grid."""
import numpy as np
import pytest

import oracle
from gpu_util import rel, rel_psi
from helpers import interior_mask, windows
from paper_0905_3409_amd import inputs


def _check(dim, n, kind, params, period, dt, steps, m, margin, seed):
    ncell = (n,) * dim
    F, dF = inputs.separable_sines(seed, ncell)
    axes = inputs.node_axes(ncell)
    phi, psi = inputs.separable_dense(F, dF)
    fp, fg = oracle.advance(dim, ncell, (0.0,) * dim, (1.0,) * dim, kind, params, period, phi,
                            psi, 0.0, dt, steps)
    shape = (n + 1,) * dim
    FP, FG = fp.reshape(shape), fg.reshape((dim,) + shape)
    for win in windows(n + 1, m, dim):
        sl = tuple(slice(*w) for w in reversed(win))
        pw, gw = inputs.separable_dense(F, dF, win)
        assert np.array_equal(pw, phi.reshape(shape)[sl].ravel())
        assert np.array_equal(gw, np.concatenate([psi.reshape((dim,) + shape)[a][sl].ravel()
                                                  for a in range(dim)]))
        lo = [axes[a][win[a][0]] for a in range(dim)]
        hi = [axes[a][win[a][1] - 1] for a in range(dim)]
        op, og = oracle.advance(dim, (m,) * dim, lo, hi, kind, params, period, pw, gw, 0.0, dt,
                                steps)
        keep = interior_mask(win, n + 1, margin)
        kp = np.tile(keep, dim)
        gp = FP[sl].ravel()
        gg = np.concatenate([FG[a][sl].ravel() for a in range(dim)])
        # node coordinates lo_w + i h_w and lo + (i0 + i) h differ by rounding only
        assert rel(gp[keep], op[keep]) <= 1e-13, win
        assert rel_psi(gg[kp], og[kp], op[keep], 1.0 / n) <= 1e-13, win


def test_stream_function_window_equals_whole_grid():
    params = inputs.stream_modes(np.random.default_rng(11), 8, (256, 256), 1.0)
    _check(2, 400, inputs.STREAM_SIN, params, 2.0, 0.8 / 400, 2, 48, 8, 12)


def test_vector_potential_window_equals_whole_grid():
    params = inputs.vecpot_modes(np.random.default_rng(13), 6, (32, 32, 32), 1.0)
    _check(3, 60, inputs.VECPOT_SIN, params, 3.0, 0.9 / 60, 1, 16, 4, 14)


def test_window_margin_is_needed():
    """Without the margin the window's own boundary shows: the comparison
    above is not vacuous."""
    n, m = 400, 48
    params = inputs.stream_modes(np.random.default_rng(11), 8, (256, 256), 1.0)
    F, dF = inputs.separable_sines(12, (n, n))
    axes = inputs.node_axes((n, n))
    phi, psi = inputs.separable_dense(F, dF)
    fp, _ = oracle.advance(2, (n, n), (0.0, 0.0), (1.0, 1.0), inputs.STREAM_SIN, params, 2.0,
                           phi, psi, 0.0, 0.8 / n, 2)
    win = windows(n + 1, m, 2)[4]  # the centre window: every side inside the domain
    pw, gw = inputs.separable_dense(F, dF, win)
    op, _ = oracle.advance(2, (m, m), [axes[a][win[a][0]] for a in range(2)],
                           [axes[a][win[a][1] - 1] for a in range(2)], inputs.STREAM_SIN, params,
                           2.0, pw, gw, 0.0, 0.8 / n, 2)
    sl = tuple(slice(*w) for w in reversed(win))
    assert rel(fp.reshape(n + 1, n + 1)[sl].ravel(), op) > 1e-8
