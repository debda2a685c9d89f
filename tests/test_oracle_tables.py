"""Pins for the oracle's template tables against the facts the paper states
(Table 1, Sec. 4, App. A) and counts fixed by Burnside's lemma."""
import json
import os

import numpy as np
import pytest
from scipy.spatial import ConvexHull

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
NAMES = ("SC", "FCC", "HCP", "ICO", "BCC")


@pytest.mark.parametrize("t", range(5))
def test_template_counts_match_paper(oracle_lib, t):
    d = oracle_lib.template(t)
    name = NAMES[t]
    assert d["k"] == GOLD["neighbours_required"][name]
    assert d["group_order"] == GOLD["symmetry_order"][name]
    assert d["triangulations"] == GOLD["triangulations"][name]
    assert d["orbits"] == GOLD["orbits_under_rotations"][name]


@pytest.mark.parametrize("t", range(5))
def test_group_elements_are_proper_rotations_of_the_template(oracle_lib, t):
    d = oracle_lib.template(t)
    w = d["w"]
    for perm, R in zip(d["gperm"], d["grot"]):
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1) < 1e-12
        assert np.allclose(w @ R.T, w[perm], atol=1e-12)
    assert len({tuple(p) for p in d["gperm"]}) == d["group_order"]


def faces_from_scipy(w):
    """Hull faces of the ideal template, coplanar triangles merged."""
    h = ConvexHull(w)
    groups = {}
    for simp, eq in zip(h.simplices, h.equations):
        key = tuple(np.round(eq, 6))
        groups.setdefault(key, set()).update(int(x) for x in simp)
    return [sorted(v) for v in groups.values()]


def burnside_orbits(w, gperm):
    faces = faces_from_scipy(w)
    quads = [f for f in faces if len(f) == 4]
    # the two diagonals of each quad: the pairs of non-adjacent vertices
    diag = []
    for q in quads:
        pts = w[q]
        d = np.linalg.norm(pts[:, None] - pts[None], axis=-1)
        pairs = []
        for i in range(4):
            j = int(np.argmax(d[i]))
            pair = tuple(sorted((q[i], q[j])))
            if pair not in pairs:
                pairs.append(pair)
        assert len(pairs) == 2
        diag.append(pairs)
    where = {}
    for qi, pairs in enumerate(diag):
        for di, pr in enumerate(pairs):
            where[pr] = (qi, di)
    total = 0
    for perm in gperm:
        # map (quad, diagonal) -> (quad, diagonal)
        img = {}
        for qi, pairs in enumerate(diag):
            for di, (a, b) in enumerate(pairs):
                img[(qi, di)] = where[tuple(sorted((perm[a], perm[b])))]
        seen, fix = set(), 1
        for qi in range(len(diag)):
            if qi in seen:
                continue
            # follow the cycle of quad qi, tracking whether diagonal 0 returns to 0
            cur = (qi, 0)
            while True:
                seen.add(cur[0])
                cur = img[cur]
                if cur[0] == qi:
                    break
            fix *= 2 if cur[1] == 0 else 0
        total += fix
    assert total % len(gperm) == 0
    return len(faces) - len(quads), len(quads), total // len(gperm)


@pytest.mark.parametrize("t", range(5))
def test_face_structure_and_burnside_orbit_count(oracle_lib, t):
    d = oracle_lib.template(t)
    ntri, nquad, orbits = burnside_orbits(d["w"], d["gperm"])
    name = NAMES[t]
    assert ntri == GOLD["hull_faces"][name]["triangles"]
    assert nquad == GOLD["hull_faces"][name]["quads"]
    assert 2 ** nquad == d["triangulations"]
    assert orbits == d["orbits"] == GOLD["orbits_under_rotations"][name]


def test_sc_and_ico_automorphisms(oracle_lib):
    """App. A: the unique SC and ICO triangulations have 24 and 60
    orientation-preserving automorphisms, all symmetrically equivalent."""
    for t, expect in ((0, 24), (3, 60)):
        d = oracle_lib.template(t)
        ok, tris = oracle_lib.hull(d["w"])
        assert ok
        _, naut, _ = oracle_lib.canonical(d["k"], tris)
        assert naut == expect == d["group_order"]


def test_fcc_hcp_ico_codes_overlap(oracle_lib):
    """Sec. 4: some FCC and HCP triangulations are isomorphic, and both can be
    isomorphic to the icosahedral graph."""
    codes = {}
    for t in (1, 2, 3):
        n = oracle_lib.template(t)["triangulations"]
        codes[t] = {oracle_lib.template_code(t, s)[0] for s in range(n)}
    assert codes[1] & codes[2]
    assert codes[1] & codes[3]
    assert codes[2] & codes[3]


def test_each_template_triangulation_code_is_its_own_hull_code(oracle_lib):
    """The stored code of a triangulation equals the code of the hull of a
    slightly perturbed template whose SoS/noise picks that triangulation."""
    rng = np.random.default_rng(3)
    for t in range(5):
        d = oracle_lib.template(t)
        n = d["triangulations"]
        stored = {oracle_lib.template_code(t, s)[0] for s in range(n)}
        for _ in range(20):
            ok, tris = oracle_lib.hull(d["w"] + rng.normal(scale=0.02, size=d["w"].shape))
            assert ok
            assert oracle_lib.canonical(d["k"], tris)[0] in stored
