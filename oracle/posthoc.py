"""FP64 oracle of the post-hoc cut-off and the per-type RMSD histograms
(test infrastructure: only ``tests/`` may import this module).

Sec. 5.1 recommends choosing the RMSD cut-off after the analysis, from the
distribution of RMSD values of each identified structure.  Both operations
take the best match of every atom, found without a cut-off: ``best_type``
(template + 1, 0 when the atom has no candidate) and its RMSD.

* apply_cutoff: the structure type under a cut-off c is the best match when
  its RMSD is at most c, otherwise none (the rule of Sec. 5.1 applied to
  the stored minimum).
* rmsd_histograms: counts[t][b] = number of atoms whose best match is t and
  whose RMSD falls in bin b of nbins equal bins over [0, rmax).  The bin of
  r is floor(r * (nbins / rmax)) with the factor nbins / rmax formed first
  in FP64, clamped to 0 .. nbins - 1; r >= rmax, +inf and NaN fall in the
  last bin.  (The definition fixes the arithmetic so that an r on a bin
  edge is binned the same way by any implementation of it.)
"""
from __future__ import annotations

import math

import numpy as np


def apply_cutoff(best_type, rmsd, cutoff: float) -> np.ndarray:
    best_type = np.asarray(best_type, dtype=np.int8)
    rmsd = np.asarray(rmsd, dtype=np.float64)
    out = np.zeros(len(best_type), np.int8)
    for i in range(len(best_type)):
        out[i] = best_type[i] if rmsd[i] <= cutoff else 0
    return out


def bin_of(r: float, nbins: int, rmax: float) -> int:
    if not (r < rmax):
        return nbins - 1
    return min(nbins - 1, max(0, math.floor(r * (nbins / rmax))))


def rmsd_histograms(best_type, rmsd, nbins: int, rmax: float) -> np.ndarray:
    """(6, nbins) int64 counts, rows indexed by best_type (0 = no candidate)."""
    counts = np.zeros((6, nbins), np.int64)
    for t, r in zip(np.asarray(best_type).tolist(), np.asarray(rmsd, dtype=np.float64).tolist()):
        if 0 <= t <= 5:
            counts[t, bin_of(r, nbins, rmax)] += 1
    return counts
