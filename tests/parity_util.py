"""Comparison of HIP-path outputs with the oracle's (shared by GPU tests)."""
import math

import numpy as np

# FP64 plain path vs the FP64 oracle: decisions bit-exact; reals differ only
# by algorithm (QCP Newton/adjugate vs Jacobi; explicit residuals)
TOL64 = {"rmsd": 1e-12, "scale_rel": 1e-12, "angle": 1e-9, "strain": 1e-10}
# FP32-mixed path: decisions bit-exact; reals within the stated tolerances
TOL32 = {"rmsd": 1e-5, "scale_rel": 1e-6, "angle": 1e-4, "strain": 1e-5}


def quat_angle(q1, q2):
    """Rotation angle between unit quaternions (sign-invariant), in the
    well-conditioned form 4 asin(|q1 - q2| / 2) after aligning signs."""
    q1, q2 = np.asarray(q1, float), np.asarray(q2, float)
    sgn = np.where(np.sum(q1 * q2, axis=-1) < 0, -1.0, 1.0)[..., None]
    d = np.linalg.norm(q1 - sgn * q2, axis=-1)
    return 4 * np.arcsin(np.clip(d / 2, 0.0, 1.0))


def compare(got, ref, tol=TOL64, check_alloy=True, check_knn=True, label=""):
    """Assert parity; returns a dict of observed maxima."""
    n = len(ref["type"])
    for key in ("type", "neighbours") + (("alloy",) if check_alloy else ()) + (("knn",) if check_knn else ()):
        g, r = np.asarray(got[key]), np.asarray(ref[key])
        bad = np.nonzero(np.any((g != r).reshape(n, -1), axis=1))[0]
        assert len(bad) == 0, f"{label}{key} differs at {len(bad)} atoms, first {bad[:5]}: got {g[bad[:2]]} ref {r[bad[:2]]}"
    r_g, r_r = got["rmsd"], ref["rmsd"]
    fin = np.isfinite(r_r)
    assert np.array_equal(np.isfinite(r_g), fin), f"{label}rmsd finiteness differs"
    stats = {}
    if fin.any():
        stats["rmsd"] = float(np.max(np.abs(r_g[fin] - r_r[fin])))
        stats["scale_rel"] = float(np.max(np.abs(got["scale"][fin] - ref["scale"][fin]) / np.abs(ref["scale"][fin])))
        stats["angle"] = float(np.max(quat_angle(got["quat"][fin], ref["quat"][fin])))
        stats["strain"] = float(np.max(np.abs(got["strain"][fin] - ref["strain"][fin])))
        for k, v in stats.items():
            assert v <= tol[k], f"{label}{k} max error {v:.3e} > {tol[k]:.1e}"
    nf = ~fin
    if nf.any():
        assert np.all(got["scale"][nf] == 0) and np.all(got["quat"][nf] == np.array([1, 0, 0, 0]))
        assert np.all(got["strain"][nf] == 0) and np.all(got["neighbours"][nf] == -1)
    return stats
