"""Pins of the post-hoc cut-off and RMSD-histogram oracle (oracle/posthoc.py,
Sec. 5.1): the cut-off applied afterwards to the best matches equals the
oracle pipeline run with that cut-off (an independent code path, the C
oracle's own decision), and the histograms agree with numpy.histogram away
from bin edges, put edges, overflow and non-finite values where the
definition says, and conserve the atom count of every type."""
import numpy as np
import pytest

from paper_1603_05143_amd import synthetic as S


@pytest.fixture(scope="module")
def P(oracle_lib):
    from oracle import posthoc
    return posthoc


@pytest.fixture(scope="module")
def noisy(oracle_lib):
    rng = np.random.default_rng(21)
    f = S.perfect_crystal("fcc", reps=(5, 5, 5), a=3.615)
    pos = f.positions + rng.normal(scale=0.12, size=f.positions.shape)
    res = oracle_lib.classify(pos, f.box)
    return pos, f.box, res


def test_cutoff_afterwards_equals_pipeline_cutoff(oracle_lib, P, noisy):
    pos, box, res = noisy
    r = res["rmsd"]
    finite = np.sort(r[np.isfinite(r)])
    assert len(finite) > 400 and np.unique(res["type"]).size >= 2  # noise spreads the matches
    # cut-offs between values, and exactly on an atom's RMSD (the rule is <=)
    cuts = [np.quantile(finite, q) for q in (0.1, 0.5, 0.9)] + [finite[37], finite[-3], 0.0]
    for c in cuts:
        want = oracle_lib.classify(pos, box, cutoff=float(c))["type"]
        got = P.apply_cutoff(res["type"], r, float(c))
        assert np.array_equal(got, want), c
    assert np.sum(P.apply_cutoff(res["type"], r, float(finite[37])) > 0) >= 38


def test_histogram_matches_numpy_away_from_edges(P):
    rng = np.random.default_rng(4)
    n, nbins, rmax = 20000, 37, 0.3
    t = rng.integers(0, 6, n).astype(np.int8)
    r = rng.uniform(0, rmax, n)
    frac = r * (nbins / rmax)
    keep = np.abs(frac - np.round(frac)) > 1e-6
    t, r = t[keep], r[keep]
    got = P.rmsd_histograms(t, r, nbins, rmax)
    for ty in range(6):
        want, _ = np.histogram(r[t == ty], bins=nbins, range=(0.0, rmax))
        assert np.array_equal(got[ty], want), ty
    assert np.array_equal(got.sum(axis=1), np.bincount(t, minlength=6))


def test_histogram_edges_overflow_nonfinite(P):
    nbins, rmax = 8, 0.5  # nbins / rmax = 16 exactly: edges are k / 16
    r = np.array([0.0, 1 / 16, np.nextafter(2 / 16, 0.0), 7 / 16, 0.5, 0.75, np.inf, np.nan, -1e-3])
    t = np.array([1, 1, 1, 1, 1, 2, 0, 3, 4], np.int8)
    h = P.rmsd_histograms(t, r, nbins, rmax)
    assert h[1].tolist() == [1, 2, 0, 0, 0, 0, 0, 2]  # 0; 1/16 and just below 2/16 in bin 1; 7/16, 0.5 last
    assert h[2, 7] == 1 and h[0, 7] == 1 and h[3, 7] == 1 and h[4, 0] == 1
    assert h.sum() == len(r)
    assert np.array_equal(P.rmsd_histograms(t, r, 1, rmax)[:, 0], np.bincount(t, minlength=6))


def test_perfect_lattice_histogram(oracle_lib, P):
    f = S.perfect_crystal("bcc", reps=(4, 4, 4), a=2.87)
    res = oracle_lib.classify(f.positions, f.box)
    h = P.rmsd_histograms(res["type"], res["rmsd"], 50, 0.25)
    assert h[5, 0] == f.n and h.sum() == f.n
