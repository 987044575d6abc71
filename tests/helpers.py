"""Test-only helpers: exact polynomials and small numeric utilities.

Nothing here implements the GA-CIR scheme; these are independent closed forms
used to pin the oracle (exact reproduction, translation, affine flows).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


class Poly:
    """Polynomial sum c_e x^e over exponent tuples e, evaluated exactly."""

    def __init__(self, terms):
        self.terms = {tuple(e): float(c) for e, c in terms.items() if c != 0.0}
        self.dim = len(next(iter(terms)))

    @staticmethod
    def random_total_degree(rng, dim, deg=3):
        terms = {}
        for e in itertools.product(range(deg + 1), repeat=dim):
            if sum(e) <= deg:
                terms[e] = rng.normal()
        return Poly(terms)

    @staticmethod
    def random_pcubic(rng, dim):
        terms = {e: rng.normal() for e in itertools.product(range(4), repeat=dim)}
        return Poly(terms)

    def deriv(self, order):
        out = {}
        for e, c in self.terms.items():
            ne = list(e)
            k = c
            ok = True
            for a, o in enumerate(order):
                for _ in range(o):
                    if ne[a] == 0:
                        ok = False
                        break
                    k *= ne[a]
                    ne[a] -= 1
                if not ok:
                    break
            if ok:
                out[tuple(ne)] = out.get(tuple(ne), 0.0) + k
        if not out:
            out = {(0,) * self.dim: 0.0}
        p = Poly.__new__(Poly)
        p.terms = out
        p.dim = self.dim
        return p

    def __call__(self, *coords):
        coords = [np.asarray(c, dtype=np.float64) for c in coords]
        val = np.zeros(np.broadcast(*coords).shape)
        for e, c in self.terms.items():
            t = c
            for a in range(self.dim):
                t = t * coords[a] ** e[a]
            val = val + t
        return val

    def __mul__(self, other):
        out = {}
        for e1, c1 in self.terms.items():
            for e2, c2 in other.terms.items():
                e = tuple(a + b for a, b in zip(e1, e2))
                out[e] = out.get(e, 0.0) + c1 * c2
        return Poly(out)

    def compose_affine(self, M, c):
        """Return a callable x -> p(c + M (x - c)) (not expanded)."""
        M = np.asarray(M, dtype=np.float64)
        c = np.asarray(c, dtype=np.float64)

        def f(*coords):
            y = [coords[a] - c[a] for a in range(self.dim)]
            z = [c[i] + sum(M[i, j] * y[j] for j in range(self.dim)) for i in range(self.dim)]
            return self(*z)
        return f


def unit(dim, a):
    return tuple(1 if b == a else 0 for b in range(dim))


def poly_state(p, coords):
    """Exact phi and psi planes of polynomial p at node coordinates."""
    dim = p.dim
    phi = p(*coords)
    psi = np.concatenate([p.deriv(unit(dim, a))(*coords) for a in range(dim)])
    return phi, psi


def poly_mixed(p, coords):
    """Exact cross-derivative planes in the oracle's order
    (2D: xy; 3D: xy, xz, yz, xyz)."""
    if p.dim == 2:
        return p.deriv((1, 1))(*coords)
    return np.concatenate([p.deriv(o)(*coords) for o in
                           ((1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1))])


def observed_orders(hs, errs):
    hs = np.asarray(hs, dtype=np.float64)
    errs = np.asarray(errs, dtype=np.float64)
    return np.log(errs[:-1] / errs[1:]) / np.log(hs[:-1] / hs[1:])


def rel_err(a, b):
    """max |a-b| / max |b| (normwise relative error)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


PI = math.pi


# ---------------------------------------------------------------------------
# Grids at the size limit and windows of them
# ---------------------------------------------------------------------------
PLANE_LIMIT = 2 ** 31  # bytes: a plane must stay below this


def largest_ncell(dim, elem_bytes):
    """Largest N such that the (N+1)^dim-node grid's plane fits the limit."""
    n = int((PLANE_LIMIT / elem_bytes) ** (1.0 / dim)) + 64
    while True:
        pitch = -(-n // 64) * 64
        if pitch * n ** (dim - 1) * elem_bytes < PLANE_LIMIT:
            return n - 1
        n -= 1


def windows(n_nodes, m, dim):
    """Node ranges of windows of m cells: all corners' extremes and the centre."""
    lo, mid, hi = 0, (n_nodes - m) // 2, n_nodes - 1 - m
    if dim == 2:
        starts = [(lo, lo), (hi, lo), (lo, hi), (hi, hi), (mid, mid)]
    else:
        starts = [(lo, lo, lo), (hi, hi, hi), (hi, lo, hi), (lo, hi, lo), (mid, mid, mid)]
    return [[(s, s + m + 1) for s in st] for st in starts]


def interior_mask(win, n_nodes, margin):
    """Nodes of the window at least margin away from its sides inside the domain."""
    keep = []
    for s, e in win:
        idx = np.arange(s, e)
        ok = np.ones(e - s, dtype=bool)
        if s > 0:
            ok &= idx >= s + margin
        if e < n_nodes:
            ok &= idx < e - 1 - margin
        keep.append(ok)
    mask = keep[1][:, None] & keep[0][None, :]
    if len(win) == 3:
        mask = keep[2][:, None, None] & mask[None, :, :]
    return mask.ravel()
