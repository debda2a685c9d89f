"""FP64 oracle of the quantities derived from a match (test infrastructure).

Only ``tests/`` may import this module.  Plain numpy, written from the
paper's definitions, independent of the HIP library:

* von Mises shear strain of the strain matrix P (Sec. 8);
* the residual of the least-squares fit of eq.(6) (Falk-Langer D^2_min,
  Sec. 8), by ``numpy.linalg.lstsq``;
* the nearest-neighbour distance implied by the fit, i.e. the hydrostatic
  part recovered from the scale (Sec. 8): the distance of template vertex 0
  from the centre in the units of eq.(4), divided by the scale s;
* the orientation in the fundamental zone (Sec. 7): of the orientations
  equivalent under the template's proper rotations, the one of largest w;
* the misorientation angle of two orientations of the same template:
  the smallest rotation angle of conj(q1) q2 q_h over the group.

Readings: eq.(6) uses the N = k + 1 points (centre included), both sets
centred on their barycentre and divided by their own l(.) (eq. 4); the
residual is the sum of squares (D^2_min is a sum of squared residuals).
"""
from __future__ import annotations

import numpy as np

from . import TEMPLATE_K, template


def _min_image(d, box):
    d = np.array(d, dtype=np.float64)
    for a in range(3):
        if box[a] > 0:
            d[..., a] -= box[a] * np.round(d[..., a] / box[a])
    return d


def _normalised(points):
    """eq.(4): centred on the barycentre, divided by the mean distance from it."""
    c = points - points.mean(axis=0)
    return c / np.mean(np.linalg.norm(c, axis=1))


def matrix_to_quat(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix (largest-pivot method)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    cand = [tr, R[0, 0], R[1, 1], R[2, 2]]
    k = int(np.argmax(cand))
    if k == 0:
        w = np.sqrt(1.0 + tr) / 2
        q = [w, (R[2, 1] - R[1, 2]) / (4 * w), (R[0, 2] - R[2, 0]) / (4 * w), (R[1, 0] - R[0, 1]) / (4 * w)]
    elif k == 1:
        x = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) / 2
        q = [(R[2, 1] - R[1, 2]) / (4 * x), x, (R[0, 1] + R[1, 0]) / (4 * x), (R[0, 2] + R[2, 0]) / (4 * x)]
    elif k == 2:
        y = np.sqrt(1.0 - R[0, 0] + R[1, 1] - R[2, 2]) / 2
        q = [(R[0, 2] - R[2, 0]) / (4 * y), (R[0, 1] + R[1, 0]) / (4 * y), y, (R[1, 2] + R[2, 1]) / (4 * y)]
    else:
        z = np.sqrt(1.0 - R[0, 0] - R[1, 1] + R[2, 2]) / 2
        q = [(R[1, 0] - R[0, 1]) / (4 * z), (R[0, 2] + R[2, 0]) / (4 * z), (R[1, 2] + R[2, 1]) / (4 * z), z]
    q = np.array(q)
    return q / np.linalg.norm(q)


def quat_mul(a, b):
    """Hamilton product of quaternions (w, x, y, z), broadcasting."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def conj(q):
    q = np.array(q, dtype=np.float64)
    q[..., 1:] *= -1
    return q


def group_quaternions(t: int) -> np.ndarray:
    """Quaternions of the proper rotations of template t (Sec. 4)."""
    return np.array([matrix_to_quat(R) for R in template(t)["grot"]])


def von_mises(P):
    """Sec. 8: sqrt(3/2 sum P_ij^2 - 1/2 (tr P)^2)."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 3, 3)
    v = 1.5 * np.sum(P * P, axis=(1, 2)) - 0.5 * np.trace(P, axis1=1, axis2=2) ** 2
    return np.sqrt(np.maximum(v, 0.0))


def fz_quaternion(q, t: int):
    """Sec. 7: the equivalent orientation q conj(q_h) of largest |w|, w >= 0;
    also returns the gap between the two largest |w| (0 on a tie)."""
    G = group_quaternions(t)
    cands = quat_mul(np.asarray(q)[None, :], conj(G))
    ws = np.abs(cands[:, 0])
    order = np.argsort(-ws, kind="stable")
    best = cands[order[0]]
    gap = ws[order[0]] - ws[order[1]] if len(ws) > 1 else np.inf
    s = np.sign(best[np.nonzero(best)[0][0]])
    return best * s, gap


def misorientation(q1, q2, t: int) -> float:
    """Smallest rotation angle of conj(q1) q2 q_h over the template's group."""
    G = group_quaternions(t)
    m = quat_mul(quat_mul(conj(q1), q2)[None, :], G)
    return float(2.0 * np.arccos(np.clip(np.max(np.abs(m[:, 0])), 0.0, 1.0)))


def derived(positions, box, res, atoms=None):
    """Derived outputs of oracle.classify results ``res`` (for the atoms
    ``atoms``, default all; the best match must be the type, i.e. results
    computed without an RMSD cut-off).  Returns vm_strain, strain_residual,
    nn_distance, quat_fz and fz_gap (the |w| gap of quat_fz, 0 on ties)."""
    pos = np.asarray(positions, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    m = len(res["type"])
    idx = np.arange(m) if atoms is None else np.asarray(atoms)
    out = {"vm_strain": np.zeros(m), "strain_residual": np.zeros(m), "nn_distance": np.zeros(m),
           "quat_fz": np.tile([1.0, 0.0, 0.0, 0.0], (m, 1)), "fz_gap": np.full(m, np.inf)}
    tpl = {}
    for j in range(m):
        ty = int(res["type"][j])
        if ty == 0:
            assert not np.isfinite(res["rmsd"][j]), "derived() needs results without a cut-off"
            continue
        t = ty - 1
        if t not in tpl:
            info = template(t)
            V = _normalised(np.vstack([np.zeros(3), info["w"]]))
            tpl[t] = (info["k"], V)
        k, V = tpl[t]
        nb = res["neighbours"][j][:k]
        i = idx[j]
        W = np.vstack([np.zeros(3), _min_image(pos[nb] - pos[i], box)])
        Wn = _normalised(W)
        At, resid, _, _ = np.linalg.lstsq(V, Wn, rcond=None)
        out["strain_residual"][j] = float(np.sum((V @ At - Wn) ** 2))
        out["vm_strain"][j] = von_mises(res["strain"][j])[0]
        out["nn_distance"][j] = np.linalg.norm(V[1]) / res["scale"][j]
        out["quat_fz"][j], out["fz_gap"][j] = fz_quaternion(res["quat"][j], t)
    return out
