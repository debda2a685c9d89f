"""Pin of the oracle's orientation representative (Alg. 1 output Q, Sec. 7):
the quaternion, the scale and the ordered neighbour list describe one and
the same superposition.  Rebuilding the eq.(3) residual from the outputs
alone -- observed points taken in the order of ``neighbours`` (template
vertex m <- atom neighbours[m]), template points of eq.(4) in vertex order,
rotation R(quat) -- must give back N * rmsd^2 for every matched atom.  A
representative whose rotation were composed the wrong way (Q R_g instead of
Q R_g^T for a group element g of order above two) or whose neighbour order
were permuted without the rotation would break the identity."""

import numpy as np
import pytest

from paper_1603_05143_amd import synthetic as S

OPEN = np.zeros(3)


def min_image(d, box):
    """Minimum image as the oracle defines it: s = rint(d * (1/L)), d - s L."""
    d = np.array(d, dtype=np.float64)
    for a in range(3):
        if box[a] > 0:
            d[..., a] = d[..., a] - np.rint(d[..., a] * (1.0 / box[a])) * box[a]
    return d


def residual_from_outputs(oracle, positions, box, atoms, out):
    """N * RMSD^2 recomputed from (quat, scale, neighbours) of each atom, and
    the template index used (from the type of the best match)."""
    T = [oracle.template(t) for t in range(5)]
    res = np.full(len(atoms), np.nan)
    for s, i in enumerate(atoms):
        if not np.isfinite(out["rmsd"][s]):
            continue
        t = int(out["type"][s]) - 1
        assert t >= 0, "run with an infinite cut-off: every match keeps its type"
        k = T[t]["k"]
        nb = out["neighbours"][s, :k]
        assert np.all(nb >= 0) and np.all(out["neighbours"][s, k:] == -1)
        obs = np.vstack([np.zeros(3), min_image(positions[nb] - positions[i], box)])
        a = obs - obs.mean(0)
        b = T[t]["b"]
        R = S.quat_to_matrix(out["quat"][s])
        d = out["scale"][s] * a - b @ R.T
        res[s] = float(np.sum(d * d))
    return res


def check_identity(oracle, positions, box, atoms, out, tol=1e-12):
    res = residual_from_outputs(oracle, positions, box, atoms, out)
    fin = np.isfinite(out["rmsd"])
    assert fin.sum() > 0
    N = np.array([oracle.TEMPLATE_K[int(t) - 1] + 1 if t > 0 else 0 for t in out["type"]])
    err = np.abs(res[fin] - N[fin] * out["rmsd"][fin] ** 2)
    assert np.max(err) <= tol, (np.max(err), np.argmax(err))
    # the quaternion is a unit quaternion with the stated sign convention
    q = out["quat"][fin]
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    first = np.array([row[np.nonzero(row)[0][0]] for row in q])
    assert np.all(first > 0)
    return err


def test_identity_on_noisy_polycrystal(oracle_lib):
    """FCC, HCP and BCC grains (and their boundaries) at 0.1 A noise."""
    f = S.polycrystal(L=36.0, n_grains=4, sigma=0.1, seed=31)
    rng = np.random.default_rng(31)
    atoms = np.sort(rng.choice(f.n, min(f.n, 1500), replace=False))
    o = oracle_lib.classify(f.positions, f.box, atoms=atoms)
    assert len(set(o["type"].tolist()) - {0}) >= 3
    check_identity(oracle_lib, f.positions, f.box, atoms, o)


@pytest.mark.parametrize("t", [0, 1, 2, 3, 4])
def test_identity_on_planted_rotations(oracle_lib, t):
    """Each template under random rotations (every group element's
    representative appears), planted neighbour permutations, scale and
    0.03 x nn noise; open boundaries, centre atom classified."""
    rng = np.random.default_rng(100 + t)
    T = oracle_lib.template(t)
    w = T["w"] / np.linalg.norm(T["w"][0]) * 2.7
    blocks, atoms = [], []
    for c in range(60):
        R = S.random_rotations(rng, 1)[0]
        nb = (w @ R.T) * rng.uniform(0.8, 1.3)
        nb = nb[rng.permutation(len(nb))] + rng.normal(scale=0.03 * 2.7, size=nb.shape)
        base = np.array([30.0 * c, 0.0, 0.0])
        atoms.append(len(blocks) * (len(w) + 1))
        blocks.append(np.vstack([base, base + nb]))
    pos = np.vstack(blocks)
    o = oracle_lib.classify(pos, OPEN, atoms=np.array(atoms), mask=1 << t)
    assert np.all(o["type"] == t + 1)
    check_identity(oracle_lib, pos, OPEN, np.array(atoms), o)
