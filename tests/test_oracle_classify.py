"""Pins for the oracle's per-atom classification (Alg. 1 and Secs. 5-8 of the
paper): perfect lattices, invariances, planted correspondences with brute
force, strain of planted deformations, alloy rules, cut-off and masks."""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1603_05143_amd import synthetic as S

OPEN = np.zeros(3)


def rot_angle(q1, q2):
    d = abs(float(np.dot(q1, q2)))
    return 2 * math.acos(min(1.0, d))


def misorientation_mod_group(q1, q2, group_rots):
    """Smallest rotation angle between R1 and R2 g over the template group."""
    R1, R2 = S.quat_to_matrix(q1), S.quat_to_matrix(q2)
    best = 10.0
    for G in group_rots:
        M = R1.T @ R2 @ G
        c = (np.trace(M) - 1) / 2
        best = min(best, math.acos(max(-1.0, min(1.0, c))))
    return best


@pytest.mark.parametrize("kind,a,tpl", [("fcc", 3.615, 2), ("bcc", 2.87, 5), ("sc", 2.6, 1),
                                        ("hcp", 2.51, 3)])
def test_perfect_crystals(oracle_lib, kind, a, tpl):
    f = S.perfect_crystal(kind, (4, 4, 4), a=a)
    o = oracle_lib.classify(f.positions, f.box)
    assert np.all(o["type"] == tpl)
    assert o["rmsd"].max() < 1e-12
    assert np.abs(o["strain"] - np.eye(3).reshape(-1)).max() < 1e-12
    k = oracle_lib.TEMPLATE_K[tpl - 1]
    d = np.linalg.norm(f.positions[o["neighbours"][0, :k]] - f.positions[0], axis=1)
    d = np.minimum(d, np.linalg.norm(np.mod(f.positions[o["neighbours"][0, :k]] - f.positions[0]
                                            + f.box / 2, f.box) - f.box / 2, axis=1))
    l_v = d.sum() / (k + 1)
    assert np.allclose(o["scale"], 1.0 / l_v, rtol=1e-12)
    # every atom's neighbour list is a permutation of its k nearest atoms
    assert np.all(np.sort(o["neighbours"][:, :k], 1) == np.sort(o["knn"][:, :k], 1))


def test_mackay_icosahedron_centre_is_ico(oracle_lib):
    p = S.mackay_icosahedron(2, nn=2.55)
    o = oracle_lib.classify(p, OPEN, atoms=[0])
    assert o["type"][0] == 4 and o["rmsd"][0] < 1e-12


def test_config0_all_fcc(oracle_lib):
    f = S.config0()
    o = oracle_lib.classify(f.positions, f.box)
    assert np.all(o["type"] == 2)
    assert 0.01 < o["rmsd"].mean() < 0.06


def test_knn_matches_kdtree(oracle_lib):
    f = S.config0()
    tree = cKDTree(f.positions, boxsize=f.box)
    d, j = tree.query(f.positions, k=15)
    o = oracle_lib.classify(f.positions, f.box, mask=0)
    assert np.array_equal(o["knn"], j[:, 1:].astype(np.int32))
    for i in (0, 17, 255):
        ids, rel, d2 = oracle_lib.knn(f.positions, f.box, i)
        assert np.allclose(np.sqrt(d2), d[i, 1:], atol=1e-12)


def test_rigid_motion_and_relabelling_invariance(oracle_lib):
    """Rotating, translating and relabelling a noisy crystal leaves type and
    RMSD unchanged and rotates the orientation by the applied rotation."""
    f = S.perfect_crystal("fcc", (3, 3, 3), a=3.615)
    rng = np.random.default_rng(5)
    pos = f.positions + rng.normal(scale=0.04, size=f.positions.shape)
    # open cluster: classify interior atoms only
    ctr = pos.mean(0)
    inner = np.nonzero(np.linalg.norm(pos - ctr, axis=1) < 3.0)[0]
    o1 = oracle_lib.classify(pos, OPEN, atoms=inner, mask=0x6)
    R = S.random_rotations(rng, 1)[0]
    perm = rng.permutation(len(pos))
    inv = np.argsort(perm)
    pos2 = (pos @ R.T + rng.normal(size=3) * 7)[perm]
    o2 = oracle_lib.classify(pos2, OPEN, atoms=inv[inner], mask=0x6)
    assert np.array_equal(o1["type"], o2["type"])
    assert np.allclose(o1["rmsd"], o2["rmsd"], atol=1e-12)
    assert np.allclose(o1["scale"], o2["scale"], rtol=1e-12)
    g = oracle_lib.template(1)["grot"]
    qR = S.quat_to_matrix  # noqa
    for a in range(len(inner)):
        # the representative neighbour list maps atom ids through the relabelling
        assert np.array_equal(inv[o1["neighbours"][a, :12]], o2["neighbours"][a, :12])
        R1 = S.quat_to_matrix(o1["quat"][a])
        R2 = S.quat_to_matrix(o2["quat"][a])
        assert np.allclose(R2, R @ R1, atol=1e-9)
        # strain rotates as a tensor
        P1 = o1["strain"][a].reshape(3, 3)
        P2 = o2["strain"][a].reshape(3, 3)
        assert np.allclose(P2, R @ P1 @ R.T, atol=1e-10)
    del g


def eq3_rmsd_svd(obs, tpl):
    a = obs - obs.mean(0)
    b = tpl - tpl.mean(0)
    b = b / np.linalg.norm(b, axis=1).mean()
    M = b.T @ a
    U, Sv, Vt = np.linalg.svd(M)
    lam = Sv[0] + Sv[1] + np.sign(np.linalg.det(M)) * Sv[2]
    N = len(a)
    return math.sqrt(max(0.0, (np.sum(b * b) - lam * lam / np.sum(a * a)) / N))


def test_sc_brute_force_over_all_permutations(oracle_lib):
    """Sec. 2: with the correspondence unknown, the best match is the minimum
    over all neighbour permutations; PTM's graph candidates must reach it."""
    rng = np.random.default_rng(6)
    w = oracle_lib.template(0)["w"] * 2.6
    for _ in range(10):
        R = S.random_rotations(rng, 1)[0]
        nb = w @ R.T + rng.normal(scale=0.05, size=w.shape)
        pts = np.vstack([np.zeros(3), nb]) + 3.0
        o = oracle_lib.classify(pts, OPEN, atoms=[0], mask=0x1)
        tpl = np.vstack([np.zeros(3), w])
        best = min(eq3_rmsd_svd(np.vstack([np.zeros(3), nb[list(p)]]), tpl)
                   for p in itertools.permutations(range(6)))
        assert o["type"][0] == 1
        assert abs(o["rmsd"][0] - best) < 1e-9


@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_planted_correspondence(oracle_lib, t):
    """Template + planted permutation, rotation, scale and small noise: the
    PTM minimum equals the eq.(3) RMSD under the planted map, and the
    orientation equals the planted rotation modulo the template group."""
    rng = np.random.default_rng(10 + t)
    d = oracle_lib.template(t)
    w, k = d["w"], d["k"]
    nn = np.linalg.norm(w, axis=1).min()
    for _ in range(8):
        R = S.random_rotations(rng, 1)[0]
        c = rng.uniform(2.0, 3.0) / nn
        noisy = (w @ R.T) * c + rng.normal(scale=0.02 * nn * c, size=w.shape)
        perm = rng.permutation(k)
        nb = np.empty_like(noisy)
        nb[perm] = noisy                 # observed atom perm[j] is template vertex j
        pts = np.vstack([np.zeros(3), nb])
        o = oracle_lib.classify(pts, OPEN, atoms=[0], mask=1 << t)
        planted = eq3_rmsd_svd(np.vstack([np.zeros(3), noisy]), np.vstack([np.zeros(3), w]))
        assert o["type"][0] == t + 1
        assert abs(o["rmsd"][0] - planted) < 1e-9
        q = o["quat"][0]
        ang = misorientation_mod_group(q, S_rot_to_quat(R), d["grot"])
        assert ang < 0.1


def S_rot_to_quat(R):
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])


@pytest.mark.parametrize("t", [1, 4])
def test_planted_affine_strain(oracle_lib, t):
    """Sec. 8: for x' = F x applied to a perfect template the residual is zero
    and P is the left stretch of F times l(x)/l(Fx) (both sets normalised)."""
    rng = np.random.default_rng(20 + t)
    d = oracle_lib.template(t)
    w, k = d["w"], d["k"]
    for _ in range(5):
        eps = rng.uniform(-0.04, 0.04, size=(3, 3))
        eps = (eps + eps.T) / 2
        F = S.random_rotations(rng, 1)[0] @ (np.eye(3) + eps)
        nb = (w * 2.0) @ F.T
        pts = np.vstack([np.zeros(3), nb])
        o = oracle_lib.classify(pts, OPEN, atoms=[0], mask=1 << t)
        assert o["type"][0] == t + 1
        x = np.vstack([np.zeros(3), w * 2.0])
        fx = x @ F.T
        lx = np.linalg.norm(x - x.mean(0), axis=1).mean()
        lfx = np.linalg.norm(fx - fx.mean(0), axis=1).mean()
        ev, V = np.linalg.eigh(F @ F.T)
        VF = V @ np.diag(np.sqrt(ev)) @ V.T
        assert np.allclose(o["strain"][0].reshape(3, 3), VF * lx / lfx, atol=1e-12)


@pytest.mark.parametrize("kind,expect", [("l12", {3, 4}), ("l10", {2}), ("a1", {1}),
                                         ("b2", {7}), ("a2", {6})])
def test_alloy_rules(oracle_lib, kind, expect):
    a = 2.88 if kind in ("b2", "a2") else 3.6
    f = S.perfect_crystal(kind, (3, 3, 3), a=a)
    rng = np.random.default_rng(1)
    pos = S.wrap(f.positions + rng.normal(scale=0.03, size=f.positions.shape), f.box)
    o = oracle_lib.classify(pos, f.box, species=f.species)
    assert set(np.unique(o["alloy"]).tolist()) == expect
    if kind == "l12":
        # minority (B) atoms sit at cube corners; all others are majority sites
        assert np.all(o["alloy"][f.species == 1] == 4)
        assert np.all(o["alloy"][f.species == 0] == 3)


def test_cutoff_keeps_geometry(oracle_lib):
    f = S.config0()
    o1 = oracle_lib.classify(f.positions, f.box)
    cut = float(np.median(o1["rmsd"]))
    o2 = oracle_lib.classify(f.positions, f.box, cutoff=cut)
    assert np.array_equal(o2["type"] == 2, o1["rmsd"] <= cut)
    assert np.all(o2["type"][o1["rmsd"] > cut] == 0)
    for key in ("rmsd", "scale", "quat", "neighbours", "strain"):
        assert np.array_equal(o1[key], o2[key])


def test_template_mask(oracle_lib):
    f = S.config0()
    o = oracle_lib.classify(f.positions, f.box, mask=0x1D)   # no FCC
    assert not np.any(o["type"] == 2)
    o = oracle_lib.classify(f.positions, f.box, mask=0)
    assert np.all(o["type"] == 0) and np.all(np.isinf(o["rmsd"]))
    assert np.all(o["quat"] == np.array([1, 0, 0, 0]))


def test_too_few_neighbours(oracle_lib):
    pts = np.random.default_rng(0).normal(size=(9, 3)) * 2
    o = oracle_lib.classify(pts, OPEN)
    assert np.all(o["knn"][:, 8:] == -1)
    assert np.all(o["neighbours"][:, 6:] == -1)
    assert np.all(o["type"] <= 1)


def polar_left_proper(A):
    """A = P U with U a proper rotation (det +1), from numpy's SVD: the sign
    of det A goes to the smallest singular value."""
    X, sv, Yt = np.linalg.svd(A)
    d = np.sign(np.linalg.det(X @ Yt))
    U = X @ np.diag([1.0, 1.0, d]) @ Yt
    return A @ U.T, U


@pytest.mark.parametrize("t", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("flip", [False, True])
def test_strain_right_handed_rotation(oracle_lib, t, flip):
    """Sec. 8: A = P U with U orthogonal and right-handed.  For an exact
    affine image x' = F x of a template (centre at the origin) eq.(6) gives
    A = F l(x) / l(Fx); P then equals A U^T for the proper rotation U of
    the SVD polar decomposition, which for det F < 0 carries a negative
    eigenvalue (the smallest singular value, negated)."""
    rng = np.random.default_rng(40 + t)
    d = oracle_lib.template(t)
    w = d["w"]
    for _ in range(6):
        eps = rng.uniform(-0.2, 0.2, size=(3, 3))
        F = S.random_rotations(rng, 1)[0] @ (np.eye(3) + eps)
        if flip:
            F = F @ np.diag([1.0, 1.0, -1.0])
        assert (np.linalg.det(F) < 0) == flip
        x = np.vstack([np.zeros(3), w * 2.3])
        fx = x @ F.T
        lx = np.linalg.norm(x - x.mean(0), axis=1).mean()
        lfx = np.linalg.norm(fx - fx.mean(0), axis=1).mean()
        A = F * lx / lfx
        P_ref, U = polar_left_proper(A)
        assert np.linalg.det(U) > 0 and np.allclose(P_ref, P_ref.T, atol=1e-12)
        P = oracle_lib.strain(t, fx)
        assert np.allclose(P, P_ref, atol=1e-12), (P, P_ref)
        assert (np.linalg.det(P) < 0) == flip
        # U = P^-1 A is a proper rotation
        Uo = np.linalg.solve(P, A)
        assert np.allclose(Uo @ Uo.T, np.eye(3), atol=1e-10) and np.linalg.det(Uo) > 0


def test_strain_hook_matches_classification(oracle_lib):
    """The strain entry point is the function the classification uses (on
    the representative's neighbour order, which differs from the winning
    correspondence by a template rotation that leaves P unchanged)."""
    f = S.polycrystal(L=30.0, n_grains=3, sigma=0.1, seed=41)
    atoms = np.arange(0, f.n, 7)[:200]
    o = oracle_lib.classify(f.positions, f.box, atoms=atoms)
    for s, i in enumerate(atoms):
        t = int(o["type"][s]) - 1
        if t < 0:
            continue
        k = oracle_lib.TEMPLATE_K[t]
        nb = o["neighbours"][s, :k]
        dv = f.positions[nb] - f.positions[i]
        dv = dv - np.rint(dv * (1.0 / f.box)) * f.box
        P = oracle_lib.strain(t, np.vstack([np.zeros(3), dv]))
        assert np.allclose(P.reshape(-1), o["strain"][s], rtol=0, atol=1e-13)
