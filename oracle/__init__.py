"""FP64 CPU reference of Polyhedral Template Matching -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP product path never touches
it.  The C source (``ptm_oracle.c``) is a plain, slow FP64 implementation of
the method, written step by step from the paper; see its header for the
section each step follows.  ``build()`` compiles it with gcc.

Parity pins: every function here is checked in ``tests/test_oracle_*.py``
against values fixed by the paper or by mathematics (exact rational
arithmetic, closed forms, brute force on tiny inputs, planted rotations and
deformations, template group orders and triangulation counts).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ptm_oracle.c")
LIB = os.path.join(HERE, "libptm_oracle.so")

TEMPLATES = ("SC", "FCC", "HCP", "ICO", "BCC")
TEMPLATE_K = (6, 12, 12, 12, 14)
MASK_ALL = 0x1F
ORDER_TOPOLOGICAL = 0x100  # mask bit of the C oracle: topological neighbour ordering (Sec. 3)


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        L.ptm_oracle_classify.restype = C.c_int
        L.ptm_oracle_classify.argtypes = [p, p, p, C.c_int64, C.c_uint32, C.c_double, p, C.c_int64,
                                          C.c_int, p, p, p, p, p, p, p, p, p, p, p, p]
        L.ptm_oracle_voronoi.restype = C.c_int
        L.ptm_oracle_voronoi.argtypes = [p, p, p, p]
        L.ptm_oracle_voronoi_areas.argtypes = [C.c_int, p, p]
        L.ptm_oracle_orient.argtypes = [p, p, C.c_int]
        L.ptm_oracle_det3.argtypes = [p]
        L.ptm_oracle_hull.argtypes = [C.c_int, p, p, p]
        L.ptm_oracle_canonical.argtypes = [C.c_int, p, C.c_int, p, p, p]
        L.ptm_oracle_template.argtypes = [C.c_int, p, p, p, p, p, p]
        L.ptm_oracle_template_code.argtypes = [C.c_int, C.c_int, p, p]
        L.ptm_oracle_superpose.argtypes = [C.c_int, p, p, p, p, p, p]
        L.ptm_oracle_knn.argtypes = [p, C.c_int64, p, C.c_int64, C.c_int, p, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def classify(positions, box, species=None, mask=MASK_ALL, cutoff=float("inf"), atoms=None,
             threads=None, counters=False, ordering="euclidean"):
    """Classify atoms (all, or the indices in ``atoms``).  Returns a dict of
    numpy arrays: type, alloy, rmsd, scale, quat (w,x,y,z), neighbours
    (template-vertex order), strain (3x3 row-major P), knn (distance order),
    margin, ncand, tmargin (topological ordering: distance of the nearest
    area grid value to a rounding boundary); plus ``counters`` when
    requested.  ``ordering``: "euclidean" or "topological" (Sec. 3)."""
    if ordering not in ("euclidean", "topological"):
        raise ValueError(ordering)
    if ordering == "topological":
        mask = mask | ORDER_TOPOLOGICAL
    pos = np.ascontiguousarray(positions, dtype=np.float64)
    n = pos.shape[0]
    bx = np.ascontiguousarray(box, dtype=np.float64)
    spc = None if species is None else np.ascontiguousarray(species, dtype=np.int8)
    sel = None if atoms is None else np.ascontiguousarray(atoms, dtype=np.int64)
    m = n if sel is None else len(sel)
    out = {
        "type": np.zeros(m, np.int8), "alloy": np.zeros(m, np.int8),
        "rmsd": np.zeros(m), "scale": np.zeros(m), "quat": np.zeros((m, 4)),
        "neighbours": np.zeros((m, 14), np.int32), "strain": np.zeros((m, 9)),
        "knn": np.zeros((m, 14), np.int32), "margin": np.zeros(m), "ncand": np.zeros(m, np.int32),
        "tmargin": np.zeros(m),
    }
    cnt = np.zeros(5, np.int64)
    if threads is None:
        threads = min(os.cpu_count() or 1, 16)
    rc = lib().ptm_oracle_classify(_ptr(pos), _ptr(spc), _ptr(bx), n, mask, cutoff, _ptr(sel),
                                   m, threads, _ptr(out["type"]), _ptr(out["alloy"]),
                                   _ptr(out["rmsd"]), _ptr(out["scale"]), _ptr(out["quat"]),
                                   _ptr(out["neighbours"]), _ptr(out["strain"]), _ptr(out["knn"]),
                                   _ptr(out["margin"]), _ptr(out["ncand"]), _ptr(out["tmargin"]), _ptr(cnt))
    if rc != 0:
        raise RuntimeError("oracle initialisation failed")
    if counters:
        out["counters"] = dict(zip(("hulls", "codes", "candidates", "orient_tests", "orient_exact"),
                                   cnt.tolist()))
    return out


def orient(p4, idx=None, sos=True) -> int:
    """Sign of det[b-a, c-a, d-a] for rows a,b,c,d of p4 (exact, optionally SoS)."""
    p = np.ascontiguousarray(p4, dtype=np.float64).reshape(4, 3)
    ids = np.ascontiguousarray([0, 1, 2, 3] if idx is None else idx, dtype=np.int32)
    return int(lib().ptm_oracle_orient(_ptr(p), _ptr(ids), 1 if sos else 0))


def det3(p3) -> int:
    p = np.ascontiguousarray(p3, dtype=np.float64).reshape(3, 3)
    return int(lib().ptm_oracle_det3(_ptr(p)))


def hull(points):
    """(valid, triangles) for k points (outward counter-clockwise triangles)."""
    p = np.ascontiguousarray(points, dtype=np.float64)
    k = p.shape[0]
    tris = np.zeros((64, 3), np.int32)
    nt = C.c_int(0)
    ok = lib().ptm_oracle_hull(k, _ptr(p), _ptr(tris), C.byref(nt))
    return ok == 1, tris[:nt.value].copy()


def canonical(k, tris):
    """(code, n_automorphisms, vertex_of_label) of a triangulated sphere."""
    t = np.ascontiguousarray(tris, dtype=np.int32)
    code = np.zeros(2 * (3 * 14 - 6) + 1, np.int32)
    ln = C.c_int(0)
    vl = np.zeros(k, np.int32)
    na = lib().ptm_oracle_canonical(k, _ptr(t), len(t), _ptr(code), C.byref(ln), _ptr(vl))
    if na < 0:
        raise ValueError("not a triangulated sphere")
    return tuple(code[:ln.value].tolist()), na, vl


def template(t: int):
    """Facts about template t: k, group order, triangulations, orbits, points."""
    info = np.zeros(4, np.int32)
    w = np.zeros((14, 3))
    b = np.zeros((15, 3))
    gperm = np.zeros((60, 14), np.int32)
    grot = np.zeros((60, 9))
    vp = np.zeros((3, 15))
    if lib().ptm_oracle_template(t, _ptr(info), _ptr(w), _ptr(b), _ptr(gperm), _ptr(grot), _ptr(vp)) != 0:
        raise RuntimeError("oracle initialisation failed")
    k, ng, ntri, norb = info.tolist()
    vp_k = vp.reshape(-1)[: 3 * (k + 1)].reshape(3, k + 1)
    gp = gperm.reshape(-1)[: ng * k].reshape(ng, k)
    return {"k": k, "group_order": ng, "triangulations": ntri, "orbits": norb,
            "w": w[:k].copy(), "b": b[: k + 1].copy(), "gperm": gp.copy(),
            "grot": grot[:ng].reshape(ng, 3, 3).copy(), "vpinv": vp_k.copy()}


def template_code(t: int, s: int):
    code = np.zeros(2 * (3 * 14 - 6) + 1, np.int32)
    vl = np.zeros(14, np.int32)
    ln = lib().ptm_oracle_template_code(t, s, _ptr(code), _ptr(vl))
    if ln < 0:
        raise IndexError(s)
    k = TEMPLATE_K[t]
    return tuple(code[:ln].tolist()), vl[:k].copy()


def superpose(obs, tpl):
    """eq.(3) for a fixed correspondence: (rmsd, scale, quat, lambda)."""
    a = np.ascontiguousarray(obs, dtype=np.float64)
    b = np.ascontiguousarray(tpl, dtype=np.float64)
    r, s, lam = C.c_double(), C.c_double(), C.c_double()
    q = np.zeros(4)
    lib().ptm_oracle_superpose(a.shape[0], _ptr(a), _ptr(b), C.byref(r), C.byref(s), _ptr(q), C.byref(lam))
    return r.value, s.value, q, lam.value


def knn(positions, box, i, K=14):
    pos = np.ascontiguousarray(positions, dtype=np.float64)
    bx = np.ascontiguousarray(box, dtype=np.float64)
    ids = np.zeros(K, np.int32)
    rel = np.zeros((K, 3))
    d2 = np.zeros(K)
    cnt = lib().ptm_oracle_knn(_ptr(pos), pos.shape[0], _ptr(bx), i, K, _ptr(ids), _ptr(rel), _ptr(d2))
    return ids[:cnt], rel[:cnt], d2[:cnt]


def voronoi(rel18):
    """(bounded, areas[18], order[18], tmargin) of the Voronoi cell of the
    origin with 18 neighbour vectors in Euclidean order (Sec. 3)."""
    r = np.ascontiguousarray(rel18, dtype=np.float64).reshape(18, 3)
    area = np.zeros(18)
    order = np.zeros(18, np.int32)
    tm = np.zeros(1)
    ok = lib().ptm_oracle_voronoi(_ptr(r), _ptr(area), _ptr(order), _ptr(tm))
    return ok == 1, area, order, float(tm[0])


def voronoi_areas(rel):
    """Interface areas of the (bounded) Voronoi cell of the origin with the
    k <= 18 neighbour vectors ``rel``."""
    r = np.ascontiguousarray(rel, dtype=np.float64)
    area = np.zeros(r.shape[0])
    lib().ptm_oracle_voronoi_areas(r.shape[0], _ptr(r), _ptr(area))
    return area
