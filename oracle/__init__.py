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
KNN_FORCE_GRID = 0x200     # mask bit: certified cell search whatever the frame size
KNN_FORCE_BRUTE = 0x400    # mask bit: brute-force neighbours whatever the frame size
BRUTE_MAX = 200000         # frames above this size use the cell search by default


class BoxError(ValueError):
    """A periodic box too short for the neighbour shell: some atom's K-th
    minimum-image neighbour (K = 14, or 18 for the topological ordering) is
    not strictly closer than half a periodic box length, so other periodic
    images could belong to its shell (Sec. 5 periodic samples)."""


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
        L.ptm_oracle_neighbours.restype = C.c_int
        L.ptm_oracle_neighbours.argtypes = [p, p, C.c_int64, p, C.c_int64, C.c_int, C.c_int, C.c_int, p, p, p, p]
        L.ptm_oracle_classify_given.restype = C.c_int
        L.ptm_oracle_classify_given.argtypes = [p, p, C.c_uint32, C.c_double, p, C.c_int64, p, p, p, p, C.c_int,
                                                p, p, p, p, p, p, p, p]
        L.ptm_oracle_strain.restype = C.c_int
        L.ptm_oracle_strain.argtypes = [C.c_int, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def classify(positions, box, species=None, mask=MASK_ALL, cutoff=float("inf"), atoms=None,
             threads=None, counters=False, ordering="euclidean", knn_search="auto", allow_box=False):
    """Classify atoms (all, or the indices in ``atoms``).  Returns a dict of
    numpy arrays: type, alloy, rmsd, scale, quat (w,x,y,z), neighbours
    (template-vertex order), strain (3x3 row-major P), knn (distance order),
    margin, ncand, tmargin (topological ordering: distance of the nearest
    area grid value to a rounding boundary), box_ok; plus ``counters`` when
    requested.  ``ordering``: "euclidean" or "topological" (Sec. 3).
    ``knn_search``: "auto" (brute force up to BRUTE_MAX atoms, else the
    certified cell search), "grid" or "brute".  A periodic frame whose box
    is too short for some listed atom's neighbour shell raises BoxError
    unless ``allow_box`` (then ``box_ok`` is False)."""
    if ordering not in ("euclidean", "topological"):
        raise ValueError(ordering)
    if ordering == "topological":
        mask = mask | ORDER_TOPOLOGICAL
    mask |= {"auto": 0, "grid": KNN_FORCE_GRID, "brute": KNN_FORCE_BRUTE}[knn_search]
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
        threads = default_threads()
    rc = lib().ptm_oracle_classify(_ptr(pos), _ptr(spc), _ptr(bx), n, mask, cutoff, _ptr(sel),
                                   m, threads, _ptr(out["type"]), _ptr(out["alloy"]),
                                   _ptr(out["rmsd"]), _ptr(out["scale"]), _ptr(out["quat"]),
                                   _ptr(out["neighbours"]), _ptr(out["strain"]), _ptr(out["knn"]),
                                   _ptr(out["margin"]), _ptr(out["ncand"]), _ptr(out["tmargin"]), _ptr(cnt))
    if rc == 1:
        raise RuntimeError("oracle initialisation failed")
    if rc == 2 and not allow_box:
        raise BoxError("periodic box shorter than twice the neighbour shell")
    out["box_ok"] = rc == 0
    if counters:
        out["counters"] = dict(zip(("hulls", "codes", "candidates", "orient_tests", "orient_exact"),
                                   cnt.tolist()))
    return out


def default_threads() -> int:
    """Threads for the oracle: the CPUs this process may run on, at most 16
    (the host share of one GPU on the machines the GPU tests run on)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def neighbours(positions, box, atoms=None, K=14, knn_search="auto", threads=None):
    """The neighbour search alone (Sec. 3 Euclidean order) for the atoms in
    ``atoms`` (or all): (ids[m][K], rel[m][K][3], d2[m][K], cnt[m], box_ok)."""
    pos = np.ascontiguousarray(positions, dtype=np.float64)
    n = pos.shape[0]
    bx = np.ascontiguousarray(box, dtype=np.float64)
    sel = None if atoms is None else np.ascontiguousarray(atoms, dtype=np.int64)
    m = n if sel is None else len(sel)
    ids = np.full((m, K), -1, np.int32)
    rel = np.zeros((m, K, 3))
    d2 = np.zeros((m, K))
    cnt = np.zeros(m, np.int32)
    force = {"auto": 0, "grid": 1, "brute": 2}[knn_search]
    rc = lib().ptm_oracle_neighbours(_ptr(pos), _ptr(bx), n, _ptr(sel), m, K, force,
                                     threads or default_threads(), _ptr(ids), _ptr(rel), _ptr(d2), _ptr(cnt))
    if rc == 1:
        raise RuntimeError("oracle neighbour search failed")
    return ids, rel, d2, cnt, rc == 0


def classify_given(nbrs, atoms, box, species=None, mask=MASK_ALL, cutoff=float("inf"), threads=None,
                   ordering="euclidean"):
    """classify() with the neighbours already found by neighbours() for the
    same atoms: the classification alone (the paper's timing excludes
    neighbour-list generation, Table 2)."""
    ids, rel, d2, cnt, _ = nbrs
    if ordering == "topological":
        mask = mask | ORDER_TOPOLOGICAL
    sel = np.ascontiguousarray(atoms, dtype=np.int64)
    m = len(sel)
    bx = np.ascontiguousarray(box, dtype=np.float64)
    spc = None if species is None else np.ascontiguousarray(species, dtype=np.int8)
    out = {"type": np.zeros(m, np.int8), "alloy": np.zeros(m, np.int8), "rmsd": np.zeros(m),
           "scale": np.zeros(m), "quat": np.zeros((m, 4)), "neighbours": np.zeros((m, 14), np.int32),
           "strain": np.zeros((m, 9)), "knn": np.zeros((m, 14), np.int32)}
    rc = lib().ptm_oracle_classify_given(_ptr(spc), _ptr(bx), mask, cutoff, _ptr(sel), m, _ptr(ids), _ptr(rel),
                                         _ptr(d2), _ptr(cnt), threads or default_threads(), _ptr(out["type"]),
                                         _ptr(out["alloy"]), _ptr(out["rmsd"]), _ptr(out["scale"]),
                                         _ptr(out["quat"]), _ptr(out["neighbours"]), _ptr(out["strain"]),
                                         _ptr(out["knn"]))
    if rc == 1:
        raise RuntimeError("oracle initialisation failed")
    out["box_ok"] = rc == 0
    return out


def strain(t: int, obs):
    """Sec. 8 strain P (3x3) of template t for the k+1 observed points in
    template-vertex order, centre first."""
    o = np.ascontiguousarray(obs, dtype=np.float64)
    P = np.zeros(9)
    if lib().ptm_oracle_strain(t, _ptr(o), _ptr(P)) != 0:
        raise ValueError(t)
    return P.reshape(3, 3)


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
