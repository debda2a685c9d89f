"""GPU parity of both HIP forms against the FP64 oracle, through the C ABI:
decisions (type, neighbour orders, alloy) bit-exact; reals within
parity_util.TOL64 (FP64 plain) or TOL32 (FP32-mixed)."""
import math
import sys

import numpy as np
import pytest

from paper_1603_05143_amd import ptm, synthetic as S
from parity_util import TOL32, TOL64, compare as _compare, quat_angle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module", params=[ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def clf(torch_cuda, request):
    c = ptm.Classifier(device=0, precision=request.param)
    c.tol = TOL64 if request.param == ptm.PTM_FP64 else TOL32
    yield c
    c.close()


_current_tol = [TOL64]


def compare(got, ref, **kw):
    return _compare(got, ref, tol=_current_tol[0], **kw)


def run_gpu(torch, clf, frame, mask=ptm.PTM_ALL, cutoff=math.inf):
    _current_tol[0] = clf.tol
    print(f"[gpu] n={frame.n} box={frame.box.tolist()} mask={mask}", flush=True)
    pos = torch.from_numpy(np.ascontiguousarray(frame.positions)).to("cuda:0")
    sp = None if frame.species is None else torch.from_numpy(frame.species).to("cuda:0")
    out = clf.classify(pos, frame.box, species=sp, mask=mask, cutoff=cutoff, knn=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def run_ref(oracle, frame, mask=ptm.PTM_ALL, cutoff=math.inf, atoms=None):
    return oracle.classify(frame.positions, frame.box, species=frame.species, mask=mask, cutoff=cutoff,
                           atoms=atoms)


def test_config0(torch_cuda, clf, oracle_lib):
    f = S.config0()
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    st = compare(got, ref)
    assert np.all(got["type"] == 2)
    print("config0", st)


@pytest.mark.parametrize("kind,a", [("fcc", 3.615), ("bcc", 2.87), ("sc", 2.6), ("hcp", 2.51),
                                    ("fcc", 2.0), ("bcc", 2.0)])
def test_perfect_lattices_degenerate(torch_cuda, clf, oracle_lib, kind, a):
    """Exactly or nearly coplanar facets everywhere: exact predicates + SoS."""
    f = S.perfect_crystal(kind, (4, 4, 4), a=a)
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    compare(got, ref)


@pytest.mark.parametrize("kind", ["l12", "l10", "b2", "a1", "a2"])
def test_alloys(torch_cuda, clf, oracle_lib, kind):
    a = 2.88 if kind in ("b2", "a2") else 3.6
    f = S.perfect_crystal(kind, (3, 3, 3), a=a)
    rng = np.random.default_rng(3)
    f.positions = S.wrap(f.positions + rng.normal(scale=0.05, size=f.positions.shape), f.box)
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    compare(got, ref)


def test_small_polycrystal(torch_cuda, clf, oracle_lib):
    f = S.polycrystal(L=40.0, n_grains=4, sigma=0.1, seed=11)
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    st = compare(got, ref)
    print("polycrystal", f.n, np.bincount(got["type"], minlength=6), st)


def test_small_alloy_slabs(torch_cuda, clf, oracle_lib):
    f = S.alloy_slabs(n_cells=12, seed=12)
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    compare(got, ref)


@pytest.mark.parametrize("mask,cutoff", [(ptm.PTM_FCC | ptm.PTM_HCP, math.inf), (ptm.PTM_BCC, math.inf),
                                         (ptm.PTM_SC | ptm.PTM_ICO, 0.3), (ptm.PTM_ALL, 0.06), (0, math.inf)])
def test_mask_and_cutoff(torch_cuda, clf, oracle_lib, mask, cutoff):
    f = S.polycrystal(L=30.0, n_grains=3, sigma=0.15, seed=13)
    got = run_gpu(torch_cuda, clf, f, mask=mask, cutoff=cutoff)
    ref = run_ref(oracle_lib, f, mask=mask, cutoff=cutoff)
    compare(got, ref)


def test_open_boundaries_icosahedron(torch_cuda, clf, oracle_lib):
    p = S.mackay_icosahedron(3, nn=2.55)
    rng = np.random.default_rng(5)
    p = p + rng.normal(scale=0.02, size=p.shape)
    f = S.Frame(positions=p, box=np.zeros(3))
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    compare(got, ref)
    assert got["type"][0] == 4


def test_mixed_periodic_open_axes(torch_cuda, clf, oracle_lib):
    f = S.polycrystal(L=30.0, n_grains=2, sigma=0.1, seed=14)
    f.box = np.array([f.box[0], 0.0, f.box[2]])
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    compare(got, ref)


@pytest.mark.parametrize("n", [1023, 1024, 1025, 2049])
def test_pair_tile_boundaries(torch_cuda, clf, oracle_lib, n):
    """Frames whose atom counts end just before, on and after a multiple of
    the candidate pair list's 1024-atom tile, against the oracle atom by
    atom: a perturbed FCC crystal of 8 x 8 x 4 cells (1024 sites) with sites
    removed or interstitials added, and of 8 x 8 x 8 cells for 2049."""
    rng = np.random.default_rng(n)
    reps = (8, 8, 8) if n > 1025 else (8, 8, 4)
    f = S.perfect_crystal("fcc", reps, a=3.615)
    pos = f.positions + rng.normal(scale=0.08, size=f.positions.shape)
    if n < len(pos):
        pos = np.delete(pos, rng.choice(len(pos), len(pos) - n, replace=False), axis=0)
    while len(pos) < n:  # an interstitial at an octahedral site
        c = rng.integers(0, np.array(reps)) * 3.615 + 0.5 * 3.615
        pos = np.vstack([pos, c[None, :]])
    g = S.Frame(positions=S.wrap(pos, f.box), box=f.box)
    assert g.n == n
    got = run_gpu(torch_cuda, clf, g)
    ref = run_ref(oracle_lib, g)
    compare(got, ref)


def expect_box_error(torch, clf, frame, **kw):
    """The frame's periodic box is too short for its neighbour shell: the
    call fails with PTM_E_BOX and leaves every output untouched."""
    pos = torch.from_numpy(np.ascontiguousarray(frame.positions)).to("cuda:0")
    out = clf.alloc_outputs(frame.n, "cuda:0", knn=True, derived=True)
    for v in out.values():
        v.fill_(7)
    torch.cuda.synchronize()
    with pytest.raises(ptm.PTMError) as e:
        clf.classify(pos, frame.box, out=out, **kw)
    assert e.value.status == ptm.PTM_E_BOX, e.value
    torch.cuda.synchronize()
    for k, v in out.items():
        assert bool((v == 7).all()), f"{k} written on PTM_E_BOX"


@pytest.mark.parametrize("n", [1, 2, 7, 13, 15, 40])
def test_tiny_periodic_systems_rejected(torch_cuda, clf, oracle_lib, n):
    """Periodic boxes holding too few atoms for a 14-neighbour shell within
    half a box length: the oracle rejects them, and so does the library."""
    rng = np.random.default_rng(n)
    f = S.Frame(positions=rng.random((n, 3)) * 6.0, box=np.array([6.0, 6.0, 6.0]))
    with pytest.raises(oracle_lib.BoxError):
        run_ref(oracle_lib, f)
    expect_box_error(torch_cuda, clf, f)


@pytest.mark.parametrize("n", [1, 2, 7, 13, 15])
def test_tiny_open_systems(torch_cuda, clf, oracle_lib, n):
    rng = np.random.default_rng(n)
    f = S.Frame(positions=rng.random((n, 3)) * 6.0, box=np.zeros(3))
    got = run_gpu(torch_cuda, clf, f)
    ref = run_ref(oracle_lib, f)
    compare(got, ref)


@pytest.mark.parametrize("ordering", ["euclidean", "topological"])
def test_box_rule_matches_oracle(torch_cuda, oracle_lib, ordering):
    """Small periodic gases and crystals around the limit: the library
    rejects a frame exactly when the oracle's rule (14th, or 18th,
    neighbour strictly inside half of every periodic length) fails, and
    otherwise classifies it as the oracle does."""
    torch = torch_cuda
    rng = np.random.default_rng(5 if ordering == "euclidean" else 6)
    frames = []
    for n in (20, 24, 28, 32, 40, 60):
        L = (n / 0.085) ** (1 / 3)
        frames.append(S.Frame(positions=rng.random((n, 3)) * L, box=np.array([L, L, L])))
    for kind, reps, a in (("sc", (2, 2, 2), 2.6), ("sc", (3, 3, 3), 2.6), ("bcc", (3, 3, 3), 2.87),
                          ("fcc", (3, 3, 3), 3.615)):
        f = S.perfect_crystal(kind, reps, a=a)
        f.positions = f.positions + rng.normal(scale=0.1, size=f.positions.shape)
        frames.append(f)
    seen = set()
    for prec in (ptm.PTM_FP64, ptm.PTM_FP32_MIXED):
        c = ptm.Classifier(device=0, precision=prec, topological=ordering == "topological")
        try:
            for f in frames:
                print(f"[box] n={f.n} box={f.box.tolist()} {ordering} prec={prec}", flush=True)
                ref = oracle_lib.classify(f.positions, f.box, ordering=ordering, allow_box=True)
                seen.add(ref["box_ok"])
                if ref["box_ok"]:
                    pos = torch.from_numpy(np.ascontiguousarray(f.positions)).to("cuda:0")
                    out = c.classify(pos, f.box, knn=True)
                    torch.cuda.synchronize()
                    got = {k: v.cpu().numpy() for k, v in out.items()}
                    sure = ~(ref["tmargin"] < 1e-6)
                    _compare({k: v[sure] for k, v in got.items()}, {k: ref[k][sure] for k in got},
                             tol=TOL64 if prec == ptm.PTM_FP64 else TOL32)
                else:
                    expect_box_error(torch, c, f)
        finally:
            c.close()
    assert seen == {True, False}


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_strain_right_handed_on_device(torch_cuda, oracle_lib, precision):
    """Sec. 8 strain by the decision kernels' device code (eq. (6) fit, polar
    factor with U right-handed) against the oracle, on planted deformations
    of every template, reflected ones (det A < 0, P with a negative
    eigenvalue) included.  No classified atom of the synthetic inputs has
    det A <= 0 (orientation-preserving hull correspondences keep the fit's
    handedness), so the branch is driven through this entry point."""
    import ctypes as C
    L = ptm.lib()
    L.ptm_selftest_strain_device.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    tol = 1e-11 if precision == ptm.PTM_FP64 else 5e-6
    ctx = ptm.ptm_create(0, precision)
    try:
        rng = np.random.default_rng(62)
        for t in range(5):
            w = oracle_lib.template(t)["w"]
            for flip in (False, True):
                for _ in range(3):
                    F = np.linalg.qr(rng.normal(size=(3, 3)))[0]
                    F = F * np.sign(np.linalg.det(F)) @ (np.eye(3) + rng.uniform(-0.2, 0.2, (3, 3)))
                    if flip:
                        F = F @ np.diag([1.0, 1.0, -1.0])
                    obs = np.ascontiguousarray(np.vstack([np.zeros(3), w * 2.4]) @ F.T + rng.normal(size=3))
                    P = np.zeros(9)
                    st = L.ptm_selftest_strain_device(ctx, t, obs.ctypes.data, P.ctypes.data)
                    assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
                    ref = oracle_lib.strain(t, obs)
                    assert np.max(np.abs(P.reshape(3, 3) - ref)) <= tol, (t, flip)
                    assert (np.linalg.det(P.reshape(3, 3)) < 0) == flip
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
@pytest.mark.parametrize("mask", [ptm.PTM_ALL, ptm.PTM_FCC | ptm.PTM_HCP | ptm.PTM_BCC], ids=["all", "fcc-hcp-bcc"])
def test_full_rule_for_every_atom(torch_cuda, oracle_lib, precision, mask):
    """Every atom with a candidate decided by the full rule (the test-only
    context flag PTM_F_FULL_RULE): each wave runs it for all its atoms in
    turn, every candidate superposed in FP64 with the tie rule of Alg. 1.
    The outputs equal the oracle's to the FP64 tolerance in both forms (the
    full rule is FP64 throughout)."""
    torch = torch_cuda
    f = S.polycrystal(L=34.0, n_grains=4, sigma=0.12, seed=71)
    ref = oracle_lib.classify(f.positions, f.box, mask=mask)
    ctx = ptm.ptm_create(0, precision, None, 0, ptm.PTM_F_PROFILE | ptm.PTM_F_FULL_RULE)
    try:
        pos = torch.from_numpy(f.positions).to("cuda:0")
        out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True)
        st = ptm.ptm_classify(ctx, pos.data_ptr(), None, f.box, f.n, mask, math.inf,
                              ptm.Classifier.outputs_struct(out))
        assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        torch.cuda.synchronize()
        info = ptm.ptm_frame_info(ctx)
        got = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        ptm.ptm_destroy(ctx)
    print("full rule", f.n, info, flush=True)
    assert info["decide_full"] == int(np.sum(np.isfinite(ref["rmsd"]))) > 0.5 * f.n
    _compare(got, ref, tol=TOL64)


def test_inputs_written_by_torch_just_before(torch_cuda, oracle_lib):
    """Positions produced by a torch kernel queued on the caller's stream
    right before the call (behind a long matrix product): the library's
    work waits for them."""
    torch = torch_cuda
    f = S.polycrystal(L=30.0, n_grains=3, sigma=0.1, seed=72)
    ref = oracle_lib.classify(f.positions, f.box)
    c = ptm.Classifier(device=0, precision=ptm.PTM_FP64)
    try:
        base = torch.from_numpy(f.positions).to("cuda:0")
        big = torch.randn(4096, 4096, device="cuda:0")
        torch.cuda.synchronize()
        for _ in range(3):
            big = big @ big
            big = big / big.norm()
        pos = (base * 2.0 - base).contiguous()  # the same values, written by a kernel behind the products
        out = c.classify(pos, f.box, knn=True)
        got = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        c.close()
    compare(got, ref)


def test_empty_frame(torch_cuda, clf):
    pos = torch_cuda.zeros((0, 3), dtype=torch_cuda.float64, device="cuda:0")
    out = clf.classify(pos, [10.0, 10.0, 10.0])
    assert out["type"].numel() == 0


def test_invalid_inputs(torch_cuda, clf):
    f = S.config0()
    p = f.positions.copy()
    p[7, 1] = np.nan
    pos = torch_cuda.from_numpy(p).to("cuda:0")
    with pytest.raises(ptm.PTMError) as e:
        clf.classify(pos, f.box)
    assert e.value.status == ptm.PTM_E_INVALID
    pos = torch_cuda.from_numpy(f.positions).to("cuda:0")
    for box in ([-1.0, 10, 10], [math.inf, 10, 10], [math.nan, 10, 10]):
        with pytest.raises(ptm.PTMError) as e:
            clf.classify(pos, box)
        assert e.value.status == ptm.PTM_E_INVALID
    with pytest.raises(ptm.PTMError):
        clf.classify(pos, f.box, cutoff=math.nan)


def test_deterministic_and_translation_invariant(torch_cuda, clf):
    f = S.polycrystal(L=30.0, n_grains=3, sigma=0.1, seed=15)
    a = run_gpu(torch_cuda, clf, f)
    b = run_gpu(torch_cuda, clf, f)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    g = S.Frame(positions=f.positions + f.box * np.array([2.0, -3.0, 1.0]), box=f.box)
    c = run_gpu(torch_cuda, clf, g)
    for k in ("type", "knn", "neighbours"):
        assert np.array_equal(a[k], c[k]), k


def test_misaligned_device_outputs_refused(torch_cuda, clf):
    """quat / quat_fz records are written as 16-byte pairs and neighbours as
    8-byte pairs: device arrays that are not aligned for that are refused
    before any work, and aligned views of the same buffers are accepted."""
    torch = torch_cuda
    f = S.polycrystal(L=30.0, n_grains=3, sigma=0.1, seed=16)
    pos = torch.from_numpy(f.positions).to("cuda:0")
    n = f.n
    ref = clf.classify(pos, f.box, derived=True)
    torch.cuda.synchronize()
    for key, width, dtype in (("quat", 4, torch.float64), ("quat_fz", 4, torch.float64),
                              ("neighbours", 14, torch.int32)):
        flat = torch.empty(n * width + 2, dtype=dtype, device="cuda:0")
        out = ptm.Classifier.alloc_outputs(n, "cuda:0", derived=True)
        out[key] = flat[1:1 + n * width].view(n, width)  # one element past an aligned base
        with pytest.raises(ptm.PTMError) as e:
            clf.classify(pos, f.box, out=out, derived=True)
        assert e.value.status == ptm.PTM_E_INVALID, key
        out[key] = flat[2:2 + n * width].view(n, width) if dtype == torch.int32 else flat[:n * width].view(n, width)
        got = clf.classify(pos, f.box, out=out, derived=True)
        torch.cuda.synchronize()
        assert torch.equal(got[key].cpu(), ref[key].cpu()), key


def test_host_pointer_context(torch_cuda, oracle_lib):
    import ctypes as C
    f = S.config0()
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, ptm.PTM_F_HOST_POINTERS)
    try:
        n = f.n
        pos = np.ascontiguousarray(f.positions)
        out = {"type": np.zeros(n, np.int8), "alloy": np.zeros(n, np.int8), "rmsd": np.zeros(n),
               "scale": np.zeros(n), "quat": np.zeros((n, 4)), "neighbours": np.zeros((n, 14), np.int32),
               "strain": np.zeros((n, 9)), "knn": np.zeros((n, 14), np.int32)}
        o = ptm.ptm_outputs(*[out[k].ctypes.data for k in ("type", "alloy", "rmsd", "scale", "quat",
                                                         "neighbours", "strain", "knn")])
        st = ptm.ptm_classify(ctx, pos.ctypes.data, None, f.box, n, ptm.PTM_ALL, math.inf, o)
        assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        compare(out, oracle_lib.classify(f.positions, f.box))
    finally:
        ptm.ptm_destroy(ctx)


def test_config1_fp32_decisions_equal_fp64(torch_cuda):
    """Whole 0.92 M-atom polycrystal: every decision of the FP32-mixed form
    (type, alloy, ordered neighbours) equals the FP64 form's, and the reals
    agree within the FP32 tolerances.  The atoms whose FP32 margins were too
    small are decided by the full rule (checked to occur)."""
    torch = torch_cuda
    f = S.polycrystal()
    pos = torch.from_numpy(f.positions).to("cuda:0")
    res, full = {}, {}
    for prec in (ptm.PTM_FP64, ptm.PTM_FP32_MIXED):
        ctx = ptm.ptm_create(0, prec, None, 0, ptm.PTM_F_PROFILE)
        try:
            out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True)
            st = ptm.ptm_classify(ctx, pos.data_ptr(), None, f.box, f.n, ptm.PTM_ALL, math.inf,
                                  ptm.Classifier.outputs_struct(out))
            assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
            torch.cuda.synchronize()
            res[prec] = {k: v.cpu().numpy() for k, v in out.items()}
            full[prec] = ptm.ptm_frame_info(ctx)["decide_full"]
        finally:
            ptm.ptm_destroy(ctx)
    st = _compare(res[ptm.PTM_FP32_MIXED], res[ptm.PTM_FP64], tol=TOL32, label="fp32 vs fp64 ")
    print("fp32 vs fp64 on", f.n, "atoms:", st, "full-rule atoms:", full)
    assert full[ptm.PTM_FP32_MIXED] > 0


@pytest.mark.parametrize("case", ["config0", "fcc", "bcc", "sc", "hcp", "polycrystal"])
def test_derived_outputs(torch_cuda, clf, oracle_lib, case):
    """von Mises strain, eq.(6) residual, nearest-neighbour distance and the
    fundamental-zone orientation (Sec. 7, Sec. 8) against oracle/derived.py."""
    from oracle import derived as OD
    torch = torch_cuda
    if case == "config0":
        f = S.config0()
    elif case == "polycrystal":
        f = S.polycrystal(L=40.0, n_grains=3, sigma=0.1, seed=77)
    else:
        a = {"fcc": 3.615, "bcc": 2.87, "sc": 2.6, "hcp": 2.51}[case]
        f = S.perfect_crystal(case, reps=(4, 4, 4) if case != "hcp" else (4, 3, 3), a=a)
        f.positions = f.positions + np.random.default_rng(1).normal(0, 0.04, f.positions.shape)
        f.positions = np.mod(f.positions, f.box)
    pos = torch.from_numpy(np.ascontiguousarray(f.positions)).to("cuda:0")
    out = clf.classify(pos, f.box, derived=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    atoms = np.arange(f.n) if f.n <= 600 else np.sort(np.random.default_rng(2).choice(f.n, 600, replace=False))
    ref = oracle_lib.classify(f.positions, f.box, atoms=atoms)
    d = OD.derived(f.positions, f.box, ref, atoms=atoms)
    tol = clf.tol
    fin = np.isfinite(ref["rmsd"])
    assert np.array_equal(got["type"][atoms], ref["type"])
    for k, t in (("vm_strain", tol["strain"] * 10), ("strain_residual", tol["strain"])):
        err = np.max(np.abs(got[k][atoms][fin] - d[k][fin]), initial=0.0)
        assert err <= t, (k, err)
    rel = np.max(np.abs(got["nn_distance"][atoms][fin] / d["nn_distance"][fin] - 1), initial=0.0)
    assert rel <= tol["scale_rel"] * 10, rel
    # the fundamental-zone representative is unique where its |w| leads by a margin
    uniq = fin & (d["fz_gap"] > 1e-6)
    ang = quat_angle(got["quat_fz"][atoms][uniq], d["quat_fz"][uniq])
    assert np.max(ang, initial=0.0) <= tol["angle"], np.max(ang)
    dw = np.abs(got["quat_fz"][atoms][fin][:, 0] - d["quat_fz"][fin][:, 0])
    assert np.max(dw, initial=0.0) <= tol["angle"]
    nf = ~fin
    assert np.all(got["vm_strain"][atoms][nf] == 0) and np.all(got["nn_distance"][atoms][nf] == 0)
    print(case, f.n, "vm", float(np.max(got["vm_strain"])), "nn", float(np.median(got["nn_distance"][atoms][fin])))


def test_misorientation(torch_cuda, oracle_lib):
    """ptm_misorientation against oracle/derived.py: random orientation pairs
    of every type (NONE: no symmetry), device and host pointers."""
    import ctypes as C
    from oracle import derived as OD
    torch = torch_cuda
    rng = np.random.default_rng(21)
    n = 600
    q = rng.normal(size=(2, n, 4))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    # include equivalent pairs (zero misorientation) and near-identical ones
    types = (np.arange(n) % 6).astype(np.int8)
    for t in range(1, 6):  # atom 60 + t has type t
        G = OD.group_quaternions(t - 1)
        q[1, 60 + t] = OD.quat_mul(q[0, 60 + t], G[len(G) // 2])
    q[1, 5] = q[0, 5] + 1e-9
    q[1, 5] /= np.linalg.norm(q[1, 5])
    want = np.array([OD.misorientation(q[0, i], q[1, i], t - 1) if t > 0 else
                     2 * np.arccos(min(1.0, abs(OD.quat_mul(OD.conj(q[0, i]), q[1, i])[0])))
                     for i, t in enumerate(types)])
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, 0)
    try:
        dq1 = torch.from_numpy(np.ascontiguousarray(q[0])).to("cuda:0")
        dq2 = torch.from_numpy(np.ascontiguousarray(q[1])).to("cuda:0")
        dt = torch.from_numpy(types).to("cuda:0")
        da = torch.empty(n, dtype=torch.float64, device="cuda:0")
        st = ptm.ptm_misorientation(ctx, dt.data_ptr(), dq1.data_ptr(), dq2.data_ptr(), n, da.data_ptr())
        assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        got = da.cpu().numpy()
        # the oracle's arccos loses accuracy only near zero angle
        assert np.max(np.abs(got - want)) < 1e-7
        for t in range(1, 6):
            assert got[60 + t] < 1e-7
        cubic = types[:] == 2
        assert np.max(got[cubic]) <= np.radians(62.81)
        bad = torch.tensor([7], dtype=torch.int8, device="cuda:0")
        st = ptm.ptm_misorientation(ctx, bad.data_ptr(), dq1.data_ptr(), dq2.data_ptr(), 1, da.data_ptr())
        assert st == ptm.PTM_OK and np.isnan(da[0].item())
        # out-of-range types among valid ones (device arrays are not checked
        # on the host): NaN there, every other angle unchanged
        mixed = types.copy()
        mixed[3::7] = 7
        mixed[5::11] = -2
        dm = torch.from_numpy(mixed).to("cuda:0")
        st = ptm.ptm_misorientation(ctx, dm.data_ptr(), dq1.data_ptr(), dq2.data_ptr(), n, da.data_ptr())
        assert st == ptm.PTM_OK
        gm = da.cpu().numpy()
        inv = (mixed < 0) | (mixed > 5)
        assert np.all(np.isnan(gm[inv])) and np.array_equal(gm[~inv], got[~inv])
    finally:
        ptm.ptm_destroy(ctx)
    hctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, ptm.PTM_F_HOST_POINTERS)
    try:
        h1, h2 = np.ascontiguousarray(q[0]), np.ascontiguousarray(q[1])
        ha = np.zeros(n)
        st = ptm.ptm_misorientation(hctx, types.ctypes.data, h1.ctypes.data, h2.ctypes.data, n, ha.ctypes.data)
        assert st == ptm.PTM_OK
        assert np.array_equal(ha, got)
        bt = np.full(n, 9, np.int8)
        assert ptm.ptm_misorientation(hctx, bt.ctypes.data, h1.ctypes.data, h2.ctypes.data, n,
                                      ha.ctypes.data) == ptm.PTM_E_INVALID
    finally:
        ptm.ptm_destroy(hctx)


def _pyritohedral_shell(s, nn=2.55):
    """The 12 points (0, +-1, +-s) and their cyclic permutations, at distance
    nn: the cuboctahedron at s = 1, the icosahedron at s = golden ratio, and
    in between a shell whose hull graph is the icosahedron's, a code that
    the FCC and ICO tables share (Sec. 4)."""
    v = []
    for a in (1.0, -1.0):
        for b in (1.0, -1.0):
            base = np.array([0.0, a, b * s])
            v += [base, np.roll(base, 1), np.roll(base, 2)]
    v = np.array(v)
    return v / np.linalg.norm(v[0]) * nn


def _fcc_minus_ico(oracle_lib, s):
    pts = np.vstack([np.zeros(3), _pyritohedral_shell(s)])
    rf = oracle_lib.classify(pts, np.zeros(3), atoms=[0], mask=ptm.PTM_FCC)["rmsd"][0]
    ri = oracle_lib.classify(pts, np.zeros(3), atoms=[0], mask=ptm.PTM_ICO)["rmsd"][0]
    return rf - ri, ri


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_candidate_gaps_straddling_the_fp32_bound(torch_cuda, oracle_lib, precision):
    """Atoms whose two best candidates (FCC and ICO of one shared hull code)
    differ by planted RMSD gaps from 1e-8 to 2e-5 either way -- inside,
    around and beyond twice the FP32-mixed decision bound -- and atoms whose
    RMSD straddles the cut-off: the shells move along the
    cuboctahedron-icosahedron path, rotated at random, and every decision
    equals the oracle's.  In the FP32-mixed form the close ones are decided
    by the FP64 full rule."""
    torch = torch_cuda
    lo, hi = 1.2318, 1.309  # r_FCC - r_ICO changes sign in between
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if _fcc_minus_ico(oracle_lib, mid)[0] < 0:
            lo = mid
        else:
            hi = mid
    s_star = 0.5 * (lo + hi)
    slope = (_fcc_minus_ico(oracle_lib, s_star + 1e-4)[0] - _fcc_minus_ico(oracle_lib, s_star - 1e-4)[0]) / 2e-4
    gaps = [g * sgn for g in (1e-8, 3e-7, 1e-6, 2e-6, 4e-6, 8e-6, 2e-5) for sgn in (-1, 1)]
    rng = np.random.default_rng(91)
    blocks, centres, planted = [], [], []
    for k, g in enumerate(gaps * 3):
        s = s_star + g / slope
        planted.append(_fcc_minus_ico(oracle_lib, s)[0])
        R = S.random_rotations(rng, 1)[0]
        base = 12.0 * np.array([k % 5, (k // 5) % 5, k // 25], dtype=float)
        centres.append(len(blocks) * 13)
        blocks.append(np.vstack([base, base + _pyritohedral_shell(s) @ R.T]))
    f = S.Frame(positions=np.vstack(blocks), box=np.zeros(3))
    planted = np.array(planted)
    assert np.sum(np.abs(planted) < 3e-6) >= 6 and np.sum(np.abs(planted) > 1e-5) >= 6
    r_star = _fcc_minus_ico(oracle_lib, s_star)[1]
    for cutoff in (math.inf, r_star - 1e-7, r_star - 1e-6, r_star - 3e-6):
        ref = oracle_lib.classify(f.positions, f.box, cutoff=cutoff)
        ctx = ptm.ptm_create(0, precision, None, 0, ptm.PTM_F_PROFILE)
        try:
            pos = torch.from_numpy(f.positions).to("cuda:0")
            out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True)
            st = ptm.ptm_classify(ctx, pos.data_ptr(), None, f.box, f.n, ptm.PTM_ALL, cutoff,
                                  ptm.Classifier.outputs_struct(out))
            assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
            info = ptm.ptm_frame_info(ctx)
            got = {k: v.cpu().numpy() for k, v in out.items()}
        finally:
            ptm.ptm_destroy(ctx)
        _compare(got, ref, tol=TOL64 if precision == ptm.PTM_FP64 else TOL32, label=f"cutoff {cutoff} ")
        types = got["type"][centres]
        if cutoff == math.inf:
            assert set(types.tolist()) == {2, 4}, types
        else:
            assert 0 in types and (2 in types or 4 in types), types
        if precision == ptm.PTM_FP32_MIXED:
            close = int(np.sum(np.abs(planted) < 2e-6))
            assert info["decide_full"] >= close, (info, close)
        print(f"[gaps] cutoff={cutoff} types={np.bincount(types, minlength=6).tolist()} info={info}", flush=True)
