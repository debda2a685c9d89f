"""Pins of the oracle's topological neighbour ordering (Sec. 3): Voronoi
interface areas against closed forms of the perfect lattices' cells, the
cell volume and the closed-surface identity, and scipy's Qhull Voronoi
diagram on random neighbourhoods; the ordering itself on perfect lattices,
a planted swap of shells and an unbounded cell; and the paper's finding that
topological ordering finds more FCC in a hot crystal (Sec. 5.2)."""
import math

import numpy as np
import pytest

from paper_1603_05143_amd import synthetic as S


def _shell(oracle_lib, kind, a, i=0):
    f = S.perfect_crystal(kind, reps=(4, 3, 3) if kind == "hcp" else (4, 4, 4), a=a)
    ids, rel, d2 = oracle_lib.knn(f.positions, f.box, i, 18)
    return rel


@pytest.mark.parametrize("kind,a,areas", [
    ("fcc", 3.615, [3.615 ** 2 * math.sqrt(2) / 8] * 12 + [0.0] * 6),            # rhombic dodecahedron
    ("bcc", 2.87, [3 * math.sqrt(3) * 2.87 ** 2 / 16] * 8 + [2.87 ** 2 / 8] * 6 + [0.0] * 4),  # truncated octahedron
    ("sc", 2.6, [2.6 ** 2] * 6 + [0.0] * 12),                                      # cube
])
def test_closed_form_areas(oracle_lib, kind, a, areas):
    ok, area, order, tm = oracle_lib.voronoi(_shell(oracle_lib, kind, a))
    assert ok
    assert np.allclose(area, areas, rtol=1e-12, atol=1e-12)
    # equal areas tie on the grid, so the order is the Euclidean one
    assert order.tolist() == list(range(18))


@pytest.mark.parametrize("kind,a,vol", [("fcc", 3.615, 3.615 ** 3 / 4), ("bcc", 2.87, 2.87 ** 3 / 2),
                                        ("sc", 2.6, 2.6 ** 3), ("hcp", 2.51, 2.51 ** 3 / math.sqrt(2))])
def test_cell_volume_and_closed_surface(oracle_lib, kind, a, vol):
    rel = _shell(oracle_lib, kind, a)
    ok, area, order, tm = oracle_lib.voronoi(rel)
    d = np.linalg.norm(rel, axis=1)
    # the cell is the union of pyramids over its faces, apex at the centre,
    # height d_j / 2: its volume is the volume per atom of the lattice
    assert np.sum(area * d) / 6 == pytest.approx(vol, rel=1e-12)
    # a closed surface has zero vector area
    assert np.max(np.abs(np.sum(area[:, None] * rel / d[:, None], axis=0))) < 1e-12 * np.sum(area)


def _qhull_areas(rel):
    """Interface areas of point 0 (the origin) from scipy's Qhull Voronoi."""
    from scipy.spatial import ConvexHull, Voronoi
    pts = np.vstack([np.zeros(3), rel])
    vor = Voronoi(pts)
    out = np.zeros(len(rel))
    for (p, q), rv in zip(vor.ridge_points, vor.ridge_vertices):
        if 0 not in (p, q):
            continue
        j = (q if p == 0 else p) - 1
        assert -1 not in rv, "cell of the origin must be bounded"
        V = vor.vertices[rv]
        n = rel[j] / np.linalg.norm(rel[j])
        u = np.cross(n, [1.0, 0, 0] if abs(n[0]) < 0.9 else [0, 1.0, 0])
        u /= np.linalg.norm(u)
        w = np.cross(n, u)
        P = np.stack([(V - V.mean(0)) @ u, (V - V.mean(0)) @ w], axis=1)
        out[j] = ConvexHull(P).volume if len(V) >= 3 else 0.0  # 2-D hull "volume" is its area
    return out


def test_areas_match_qhull(oracle_lib):
    rng = np.random.default_rng(8)
    base = _shell(oracle_lib, "fcc", 3.615)
    bcc = _shell(oracle_lib, "bcc", 2.87)
    for trial in range(40):
        src = base if trial % 2 == 0 else bcc
        rel = src + rng.normal(scale=0.12 + 0.1 * (trial % 3), size=src.shape)
        rel = rel[np.argsort(np.einsum("ij,ij->i", rel, rel))]
        ok, area, order, tm = oracle_lib.voronoi(rel)
        assert ok
        want = _qhull_areas(rel)
        assert np.allclose(area, want, rtol=1e-9, atol=1e-9 * want.max()), (trial, area, want)


def test_planted_shell_swap(oracle_lib):
    """A first-shell FCC neighbour pushed out beyond a second-shell one that
    is pulled in: the Euclidean first 12 take the intruder, the topological
    first 12 keep the first shell (larger interface)."""
    rel = _shell(oracle_lib, "fcc", 3.615).copy()
    rel[5] *= 1.15   # first shell, now at 2.94 A
    rel[14] *= 0.80  # second shell, now at 2.89 A
    o = np.argsort(np.einsum("ij,ij->i", rel, rel), kind="stable")
    rel = rel[o]
    assert 14 in o[:12] and 5 not in o[:12]
    ok, area, order, tm = oracle_lib.voronoi(rel)
    assert ok
    topo12 = set(o[order[:12]].tolist())
    assert topo12 == set(range(12))
    # the order is by area (on the grid), larger first
    q = np.floor(area / area.sum() * 2 ** 20)
    assert np.all(np.diff(q[order]) <= 0)


def test_unbounded_cell_keeps_euclidean_order(oracle_lib):
    rng = np.random.default_rng(2)
    rel = rng.normal(size=(18, 3))
    rel[:, 2] = np.abs(rel[:, 2]) + 0.1  # every neighbour above the centre
    rel = rel[np.argsort(np.einsum("ij,ij->i", rel, rel))]
    ok, area, order, tm = oracle_lib.voronoi(rel)
    assert not ok and order.tolist() == list(range(18)) and tm == math.inf


def test_hot_crystal_more_fcc_topological(oracle_lib):
    """Sec. 5.2: near melting, topological ordering identifies more FCC
    atoms than distance ordering; on a perfect crystal the two agree."""
    f = S.perfect_crystal("fcc", reps=(6, 6, 6), a=3.615)
    ref_e = oracle_lib.classify(f.positions, f.box)
    ref_t = oracle_lib.classify(f.positions, f.box, ordering="topological")
    for k in ("type", "neighbours", "rmsd"):
        assert np.array_equal(ref_e[k], ref_t[k])
    rng = np.random.default_rng(13)
    pos = f.positions + rng.normal(scale=0.26, size=f.positions.shape)
    e = oracle_lib.classify(pos, f.box)
    t = oracle_lib.classify(pos, f.box, ordering="topological")
    n_e, n_t = int(np.sum(e["type"] == 2)), int(np.sum(t["type"] == 2))
    assert n_t > n_e * 1.03, (n_e, n_t)
    assert np.all(np.isfinite(t["tmargin"]) | (t["type"] == 0))


def test_coincident_neighbours_keep_euclidean_order(oracle_lib):
    """Two coincident neighbours share one bisector plane: the reading keeps
    the Euclidean order (and reports no area grid margin)."""
    rng = np.random.default_rng(4)
    rel = _shell(oracle_lib, "bcc", 2.87) + rng.normal(scale=0.1, size=(18, 3))
    rel[9] = rel[4]
    rel = rel[np.argsort(np.einsum("ij,ij->i", rel, rel), kind="stable")]
    ok, area, order, tm = oracle_lib.voronoi(rel)
    assert not ok and order.tolist() == list(range(18)) and tm == math.inf
    j = next(j for j in range(17) if np.array_equal(rel[j], rel[j + 1]))
    rel[j + 1] = rel[j + 1] * (1 + 1e-9)  # no longer coincident: ordered by area
    ok, area, order, tm = oracle_lib.voronoi(rel)
    assert ok


def test_neighbour_at_the_centre_keeps_euclidean_order(oracle_lib):
    """A neighbour coinciding with the centre has no bisector plane: the
    Euclidean order is kept."""
    rng = np.random.default_rng(6)
    rel = _shell(oracle_lib, "bcc", 2.87)[:17] + rng.normal(scale=0.1, size=(17, 3))
    rel = np.vstack([np.zeros(3), rel[np.argsort(np.einsum("ij,ij->i", rel, rel))]])
    ok, area, order, tm = oracle_lib.voronoi(rel)
    assert not ok and order.tolist() == list(range(18)) and tm == math.inf
