"""Pins for the oracle's superposition (eqs. 1-4 of the paper): closed form
vs direct numerical minimisation, Kabsch SVD, planted rotations/scales."""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

from paper_1603_05143_amd.synthetic import quat_to_matrix, random_rotations


def normalise(p):
    c = p - p.mean(axis=0)
    return c / np.linalg.norm(c, axis=1).mean()


def eq3_numeric(obs, tpl):
    """min over s, Q of eq. (3) by direct numerical optimisation over the
    rotation vector (s eliminated in closed form at each step)."""
    a = obs - obs.mean(axis=0)
    b = normalise(tpl)
    N = len(a)

    def f(rv):
        R = Rotation.from_rotvec(rv).as_matrix()
        rb = b @ R.T
        s = max(np.sum(a * rb) / np.sum(a * a), 0.0)
        return np.sum((s * a - rb) ** 2) / N

    best = None
    rng = np.random.default_rng(0)
    for _ in range(12):
        res = minimize(f, rng.normal(size=3), method="BFGS", options={"gtol": 1e-13})
        if best is None or res.fun < best.fun:
            best = res
    return np.sqrt(best.fun)


def kabsch_lambda(a, b):
    M = b.T @ a
    U, S, Vt = np.linalg.svd(M)
    return S[0] + S[1] + np.sign(np.linalg.det(M)) * S[2]


@pytest.mark.parametrize("N", [7, 13, 15])
def test_rmsd_equals_numerical_minimum(oracle_lib, N):
    rng = np.random.default_rng(N)
    for _ in range(5):
        tpl = rng.normal(size=(N, 3))
        obs = tpl @ random_rotations(rng, 1)[0].T * 2.3 + rng.normal(scale=0.3, size=(N, 3)) + 5
        r, s, q, lam = oracle_lib.superpose(obs, tpl)
        assert abs(r - eq3_numeric(obs, tpl)) < 1e-7


def test_lambda_equals_kabsch(oracle_lib):
    rng = np.random.default_rng(2)
    for _ in range(200):
        N = rng.integers(4, 16)
        tpl = rng.normal(size=(N, 3))
        obs = rng.normal(size=(N, 3))
        r, s, q, lam = oracle_lib.superpose(obs, tpl)
        a = obs - obs.mean(0)
        b = normalise(tpl)
        lk = kabsch_lambda(a, b)
        assert abs(lam - lk) <= 1e-12 * max(1.0, abs(lk))
        # eq.(3) minimum in closed form: (G_b - lambda^2 / G_a) / N
        Ga, Gb = np.sum(a * a), np.sum(b * b)
        assert abs(r * r - (Gb - lk * lk / Ga) / N) < 1e-12


def test_planted_rotation_scale_translation(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(100):
        N = 13
        tpl = rng.normal(size=(N, 3))
        R = random_rotations(rng, 1)[0]
        c = rng.uniform(0.2, 5.0)
        obs = (tpl @ R.T) * c + rng.normal(size=3) * 10
        r, s, q, lam = oracle_lib.superpose(obs, tpl)
        assert r < 1e-12
        # s maps the observed set onto the unit-mean-distance template
        l_obs = np.linalg.norm(obs - obs.mean(0), axis=1).mean()
        assert abs(s - 1.0 / l_obs) < 1e-12 * s
        assert np.allclose(quat_to_matrix(q), R, atol=1e-10)


def test_scale_invariance_of_template(oracle_lib):
    """eq.(4): scaling or translating the template does not change RMSD."""
    rng = np.random.default_rng(4)
    tpl = rng.normal(size=(15, 3))
    obs = rng.normal(size=(15, 3))
    r0 = oracle_lib.superpose(obs, tpl)[0]
    for f in (1e-3, 0.7, 42.0):
        assert abs(oracle_lib.superpose(obs, tpl * f + rng.normal(size=3))[0] - r0) < 1e-13
