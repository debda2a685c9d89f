"""Pins for the oracle's convex hull (all triples + SoS) and its
orientation-preserving canonical form (Sec. 4 of the paper)."""
import itertools

import numpy as np
import pytest
from scipy.spatial import ConvexHull


def sphere_points(rng, k):
    p = rng.normal(size=(k, 3))
    return p / np.linalg.norm(p, axis=1, keepdims=True) * rng.uniform(2.0, 3.0)


def oriented_scipy_facets(p):
    h = ConvexHull(p)
    out = set()
    for simp, eq in zip(h.simplices, h.equations):
        a, b, c = simp
        n = np.cross(p[b] - p[a], p[c] - p[a])
        if np.dot(n, eq[:3]) < 0:
            b, c = c, b
        out.add(canon_tri((a, b, c)))
    return out


def canon_tri(t):
    a, b, c = (int(x) for x in t)
    r = [(a, b, c), (b, c, a), (c, a, b)]
    return min(r)


@pytest.mark.parametrize("k", [6, 12, 14])
def test_hull_matches_scipy_on_generic_points(oracle_lib, k):
    rng = np.random.default_rng(k)
    for _ in range(40):
        p = sphere_points(rng, k)
        ok, tris = oracle_lib.hull(p)
        assert len(tris) == 2 * k - 4
        assert {canon_tri(t) for t in tris} == oriented_scipy_facets(p)
        # valid iff the origin (central atom) is strictly inside
        inside = bool(np.all(ConvexHull(p).equations[:, 3] < -1e-9))
        assert ok == inside


def test_hull_rejects_interior_point_and_outside_centre(oracle_lib):
    rng = np.random.default_rng(5)
    p = sphere_points(rng, 12)
    p[3] *= 0.2                      # pull one neighbour deep inside
    ok, _ = oracle_lib.hull(p)
    assert not ok
    q = sphere_points(rng, 12) + np.array([5.0, 0, 0])   # centre outside
    ok, tris = oracle_lib.hull(q)
    assert not ok and len(tris) == 20


def test_hull_centre_on_facet_plane_fails(oracle_lib):
    """The central atom must be strictly inside: on the boundary fails."""
    p = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    ok, _ = oracle_lib.hull(p)
    assert ok
    # shifted so that the origin is the midpoint of the edge (1,0,0)-(0,1,0)
    ok2, tris = oracle_lib.hull(p + np.array([-0.5, -0.5, 0.0]))
    assert len(tris) == 8 and not ok2
    # a shift keeping the origin strictly inside stays valid
    ok3, _ = oracle_lib.hull(p + np.array([-0.25, -0.25, 0.1]))
    assert ok3


def supporting(p, t):
    a, b, c = p[t[0]], p[t[1]], p[t[2]]
    n = np.cross(b - a, c - a)
    s = (p - a) @ n
    return np.all(s <= 1e-9 * np.abs(n).sum())


@pytest.mark.parametrize("shell", ["sc", "fcc", "bcc"])
def test_hull_of_degenerate_lattice_shell_is_valid_triangulation(oracle_lib, shell):
    """Exactly coplanar square/rhombus facets: SoS must pick one diagonal per
    face, giving 2k-4 outward triangles that each lie on a supporting plane."""
    if shell == "sc":
        p = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    elif shell == "fcc":
        p = np.array([v for v in itertools.product((-1, 0, 1), repeat=3)
                      if sum(abs(x) for x in v) == 2], float)
    else:
        p = np.array([v for v in itertools.product((-1, 1), repeat=3)]
                     + [[2, 0, 0], [-2, 0, 0], [0, 2, 0], [0, -2, 0], [0, 0, 2], [0, 0, -2]], float)
    rng = np.random.default_rng(0)
    for _ in range(5):
        perm = rng.permutation(len(p))
        q = p[perm] * 1.5
        ok, tris = oracle_lib.hull(q)
        k = len(q)
        assert ok and len(tris) == 2 * k - 4
        for t in tris:
            assert supporting(q, t)
        # every undirected edge shared by exactly two triangles, opposite directions
        darts = [(t[i], t[(i + 1) % 3]) for t in tris for i in range(3)]
        assert len(set(darts)) == len(darts)
        assert all((b, a) in set(darts) for a, b in darts)


# ---------------------------------------------------------------- canonical
def rotation_system(k, tris):
    nxt = {}
    for a, b, c in tris:
        nxt[(a, b)] = c
        nxt[(b, c)] = a
        nxt[(c, a)] = b
    return nxt


def op_isomorphisms(k, tg, th):
    """All orientation-preserving isomorphisms G -> H by brute force: fix one
    dart of G, try every dart of H, propagate through the rotation systems."""
    ng, nh = rotation_system(k, tg), rotation_system(k, th)
    d0 = next(iter(ng))
    found = []
    for e0 in nh:
        f = {d0[0]: e0[0], d0[1]: e0[1]}
        stack = [d0]
        seen = {d0}
        ok = True
        while stack and ok:
            u, v = stack.pop()
            fu, fv = f[u], f[v]
            if (fu, fv) not in nh:
                ok = False
                break
            w, fw = ng[(u, v)], nh[(fu, fv)]
            if f.setdefault(w, fw) != fw:
                ok = False
                break
            for d in ((v, u), (u, w), (w, u), (v, w), (w, v)):
                if d in ng and d not in seen:
                    seen.add(d)
                    stack.append(d)
        if ok and len(set(f.values())) == k and len(f) == k:
            if all((f[a], f[b]) in nh for a, b in ng):
                found.append(dict(f))
    return found


def noisy_template_triangulations(oracle_lib, t, count, rng, sigma=0.05):
    w = oracle_lib.template(t)["w"]
    out = []
    while len(out) < count:
        p = w + rng.normal(scale=sigma, size=w.shape)
        ok, tris = oracle_lib.hull(p)
        if ok:
            out.append(tris)
    return out


def test_canonical_code_invariant_under_relabelling(oracle_lib):
    rng = np.random.default_rng(11)
    for t in range(5):
        for tris in noisy_template_triangulations(oracle_lib, t, 6, rng):
            k = oracle_lib.TEMPLATE_K[t]
            code, na, _ = oracle_lib.canonical(k, tris)
            for _ in range(3):
                perm = rng.permutation(k)
                t2 = perm[tris]
                t2 = t2[rng.permutation(len(t2))]
                t2 = np.array([np.roll(x, rng.integers(3)) for x in t2])
                code2, na2, _ = oracle_lib.canonical(k, t2)
                assert code2 == code and na2 == na


def test_canonical_code_complete_against_brute_force_isomorphism(oracle_lib):
    """Equal codes <=> an orientation-preserving isomorphism exists; the
    automorphism count equals the brute-force count."""
    rng = np.random.default_rng(12)
    graphs = []
    for t in (1, 2, 3):
        graphs += noisy_template_triangulations(oracle_lib, t, 10, rng, sigma=0.08)
    graphs.append(np.array([[a, c, b] for a, b, c in graphs[0]]))   # a mirror image
    for _ in range(6):
        ok, tris = oracle_lib.hull(sphere_points(rng, 12))
        graphs.append(tris)
    codes = [oracle_lib.canonical(12, g) for g in graphs]
    for i in range(len(graphs)):
        auts = op_isomorphisms(12, graphs[i], graphs[i])
        assert len(auts) == codes[i][1]
        for j in range(i + 1, len(graphs)):
            iso = len(op_isomorphisms(12, graphs[i], graphs[j])) > 0
            assert iso == (codes[i][0] == codes[j][0])


def test_canonical_labelling_is_an_isomorphism(oracle_lib):
    """vertex_of_label maps equal-code graphs onto each other."""
    rng = np.random.default_rng(13)
    for tris in noisy_template_triangulations(oracle_lib, 4, 5, rng):
        k = 14
        code, _, vl = oracle_lib.canonical(k, tris)
        perm = rng.permutation(k)
        t2 = perm[tris]
        code2, _, vl2 = oracle_lib.canonical(k, t2)
        assert code2 == code
        f = {int(vl[i]): int(vl2[i]) for i in range(k)}
        d1 = {(a, b) for a, b, c in tris for (a, b) in ((a, b), (b, c), (c, a))}
        d2 = {(a, b) for a, b, c in t2 for (a, b) in ((a, b), (b, c), (c, a))}
        assert {(f[a], f[b]) for a, b in d1} == d2
