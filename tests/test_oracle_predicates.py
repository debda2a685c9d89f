"""Pins for the oracle's exact orientation predicates and its symbolic
perturbation (Simulation of Simplicity), checked against exact rational
arithmetic (Python ``fractions``) and a brute-force symbolic expansion."""
import itertools
from fractions import Fraction

import numpy as np
import pytest


def frac_orient(p):
    a, b, c, d = [[Fraction(x) for x in r] for r in p]
    u = [b[i] - a[i] for i in range(3)]
    v = [c[i] - a[i] for i in range(3)]
    w = [d[i] - a[i] for i in range(3)]
    det = (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0])
           + u[2] * (v[0] * w[1] - v[1] * w[0]))
    return (det > 0) - (det < 0)


def frac_det3(p):
    a, b, c = [[Fraction(x) for x in r] for r in p]
    det = (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
           + a[2] * (b[0] * c[1] - b[1] * c[0]))
    return (det > 0) - (det < 0)


def symbolic_sos_orient(p, idx):
    """Sign of the perturbed orientation by brute-force expansion.

    The perturbed 4x4 matrix has entries x + e(r, j) in the coordinate columns
    and 1 in the last.  Expanding the determinant over all column
    permutations and all choices (value or epsilon) per row gives the
    coefficient of every epsilon monomial; monomials are ordered by the
    perturbation exponents (lowest index point, z before y before x, is the
    largest).  The sign of the first non-zero coefficient is the answer.
    """
    order = sorted(range(4), key=lambda r: idx[r])
    rows = [[Fraction(x) for x in p[r]] + [Fraction(1)] for r in order]
    perm_sign = 1
    for i in range(4):
        for j in range(i + 1, 4):
            if order[i] > order[j]:
                perm_sign = -perm_sign
    coef = {}
    for sigma in itertools.permutations(range(4)):
        inv = sum(1 for i in range(4) for j in range(i + 1, 4) if sigma[i] > sigma[j])
        sgn = -1 if inv % 2 else 1
        for choice in itertools.product((0, 1), repeat=4):
            term = Fraction(sgn)
            mono = 0
            ok = True
            for r in range(4):
                c = sigma[r]
                if choice[r]:
                    if c == 3:
                        ok = False
                        break
                    mono |= 1 << (3 * r + (2 - c))
                else:
                    term *= rows[r][c]
            if ok:
                coef[mono] = coef.get(mono, Fraction(0)) + term
    for mono in sorted(coef):
        if coef[mono] != 0:
            det_sorted = (coef[mono] > 0) - (coef[mono] < 0)
            return -perm_sign * det_sorted   # orient = -det[L]
    raise AssertionError("all coefficients vanish")


def test_orient_random_matches_fractions(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(3000):
        p = rng.normal(size=(4, 3)) * rng.choice([1e-3, 1.0, 1e3])
        assert oracle_lib.orient(p, sos=False) == frac_orient(p)


def test_orient_near_degenerate_matches_fractions(oracle_lib):
    """Points nudged off a common plane by a few ulps: the filter must defer
    to exact arithmetic and still get the sign right."""
    rng = np.random.default_rng(2)
    hits = 0
    for _ in range(3000):
        a, b, c = rng.normal(size=(3, 3)) * 3
        s, t = rng.random(2)
        d = a + s * (b - a) + t * (c - a)
        d = d + rng.integers(-3, 4, size=3) * np.spacing(d)
        p = np.array([a, b, c, d])
        e = frac_orient(p)
        hits += e == 0
        assert oracle_lib.orient(p, sos=False) == e
    # also exactly representable coplanar sets
    for _ in range(500):
        q = rng.integers(-4, 5, size=(3, 3)).astype(float)
        d = q[0] + 2 * (q[1] - q[0]) - (q[2] - q[0])
        p = np.vstack([q, d])
        assert frac_orient(p) == 0
        assert oracle_lib.orient(p, sos=False) == 0


def test_det3_matches_fractions(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(2000):
        p = rng.normal(size=(3, 3))
        if rng.random() < 0.3:
            p[2] = p[0] * rng.integers(-2, 3) + p[1] * rng.integers(-2, 3)
        assert oracle_lib.det3(p) == frac_det3(p)


def test_sos_equals_exact_when_nonzero(oracle_lib):
    rng = np.random.default_rng(4)
    for _ in range(1000):
        p = rng.normal(size=(4, 3))
        idx = rng.permutation(10)[:4]
        assert oracle_lib.orient(p, idx, sos=True) == frac_orient(p)


@pytest.mark.parametrize("seed", range(6))
def test_sos_degenerate_matches_symbolic_expansion(oracle_lib, seed):
    """Coplanar, collinear and coincident integer point sets."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(60):
        kind = rng.integers(0, 4)
        q = rng.integers(-2, 3, size=(4, 3)).astype(float)
        if kind == 1:       # coplanar
            q[3] = q[0] + rng.integers(-2, 3) * (q[1] - q[0]) + rng.integers(-2, 3) * (q[2] - q[0])
        elif kind == 2:     # collinear triple
            q[2] = q[0] + 2 * (q[1] - q[0])
            q[3] = q[0] + rng.integers(-2, 3) * (q[1] - q[0])
        elif kind == 3:     # coincident points, all on one axis plane
            q[:, 2] = 0
            q[1] = q[0]
        idx = list(rng.permutation(20)[:4])
        got = oracle_lib.orient(q, idx, sos=True)
        assert got in (-1, 1)
        assert got == symbolic_sos_orient(q, idx)


def test_sos_antisymmetric_under_swaps(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(300):
        q = rng.integers(-1, 2, size=(4, 3)).astype(float)
        idx = list(rng.permutation(8)[:4])
        s = oracle_lib.orient(q, idx, sos=True)
        for i, j in itertools.combinations(range(4), 2):
            q2 = q.copy()
            q2[[i, j]] = q2[[j, i]]
            idx2 = list(idx)
            idx2[i], idx2[j] = idx2[j], idx2[i]
            assert oracle_lib.orient(q2, idx2, sos=True) == -s
