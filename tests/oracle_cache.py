"""Oracle results for the full-size parity tests, kept in memory for the
session and on disk between sessions.

A result is keyed by a digest of: the frame's positions, box and species
(so a change to the input generator is a new key), the selected atoms, the
classification arguments, and the oracle's own source (a change to the
oracle invalidates every entry).  The directory is $PTM_ORACLE_CACHE, else
tests/.oracle_cache (not part of the repository).  Entries are plain .npz
files written by this module from oracle.classify; nothing else writes
them.  A full 4 M-atom result is about 1 GB, so entries are written only
when the disk has room for them.
"""
from __future__ import annotations

import hashlib
import os
import shutil

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE_DIR = os.environ.get("PTM_ORACLE_CACHE", os.path.join(ROOT, "tests", ".oracle_cache"))
FIELDS = ("type", "alloy", "rmsd", "scale", "quat", "neighbours", "strain", "knn", "margin", "tmargin")

_memory: dict[str, dict] = {}


def _digest_arrays(h, *arrays):
    for a in arrays:
        if a is None:
            h.update(b"none")
            continue
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(memoryview(a).cast("B"))


def oracle_digest() -> str:
    h = hashlib.sha256()
    for name in ("ptm_oracle.c", "__init__.py"):
        with open(os.path.join(ROOT, "oracle", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def key_of(frame, atoms, kw) -> str:
    h = hashlib.sha256(oracle_digest().encode())
    _digest_arrays(h, frame.positions, frame.box, frame.species, atoms)
    h.update(repr(sorted(kw.items())).encode())
    return h.hexdigest()[:32]


def classify(oracle, frame, atoms=None, **kw) -> dict:
    """oracle.classify(frame.positions, frame.box, species=frame.species,
    atoms=atoms, **kw), from the cache when the same call was made before."""
    key = key_of(frame, atoms, kw)
    if key in _memory:
        return _memory[key]
    path = os.path.join(CACHE_DIR, key + ".npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            res = {k: z[k] for k in z.files}
        res["box_ok"] = bool(res["box_ok"])
        _memory[key] = res
        return res
    res = oracle.classify(frame.positions, frame.box, species=frame.species, atoms=atoms, **kw)
    _memory[key] = res
    need = sum(res[k].nbytes for k in FIELDS) * 2
    try:
        os.makedirs(CACHE_DIR, exist_ok=True)
        if shutil.disk_usage(CACHE_DIR).free > need + (8 << 30):
            tmp = path + ".tmp.npz"
            np.savez(tmp, box_ok=np.array(res["box_ok"]), **{k: res[k] for k in FIELDS})
            os.replace(tmp, path)
    except OSError:
        pass
    return res
