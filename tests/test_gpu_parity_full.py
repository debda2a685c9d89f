"""GPU parity at full size, through the C ABI, in the launch configuration
the benchmark uses (whole frames on the device, default context):

* the 918,996-atom periodic polycrystal and the ~4.03 M-atom ordered-alloy
  slabs (with species): every atom against the FP64 oracle;
* the ~31.7 M-atom mixed frame (BCC matrix, Mackay icosahedra, simple-cubic
  cubes, adsorbed liquid slab): a seeded sample of 2 x 10^6 atoms plus every
  icosahedron centre and 150 atoms of each region kind;
* with the topological ordering: samples of the polycrystal and the mixed
  frame.

Decisions (type, ordered neighbours, Euclidean neighbours, alloy) bit-exact,
reals within the form's tolerance.  The oracle runs with its certified cell
search for these frame sizes; its results are cached (tests/oracle_cache.py)
so both precision forms compare against one oracle run."""
import numpy as np
import pytest

import oracle_cache
from paper_1603_05143_amd import ptm, synthetic as S
from parity_util import TOL32, TOL64, compare

pytestmark = pytest.mark.gpu

FIELDS = ("type", "alloy", "rmsd", "scale", "quat", "neighbours", "strain", "knn")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu(torch, precision, f, atoms=None, topological=False):
    """Classify the whole frame on the GPU; return the outputs of the listed
    atoms (all when atoms is None) and the type counts of the frame."""
    m = f.n if atoms is None else len(atoms)
    print(f"[full] n={f.n} precision={precision} compared={m} topological={topological}", flush=True)
    c = ptm.Classifier(device=0, precision=precision, topological=topological)
    try:
        pos = torch.from_numpy(np.ascontiguousarray(f.positions)).to("cuda:0")
        sp = None if f.species is None else torch.from_numpy(f.species).to("cuda:0")
        out = c.classify(pos, f.box, species=sp, knn=True, best_type=True)
        if atoms is None:
            res = {k: out[k].cpu().numpy() for k in FIELDS}
        else:
            idx = torch.from_numpy(np.asarray(atoms, dtype=np.int64)).to("cuda:0")
            res = {k: out[k].index_select(0, idx).cpu().numpy() for k in FIELDS}
        types = torch.bincount(out["type"].long(), minlength=6).cpu().numpy()
        # post-hoc outputs over the whole frame (properties that hold at any
        # size): without a cut-off the best match is the type, and the RMSD
        # histograms hold every atom under its type
        assert torch.equal(out["best_type"], out["type"])
        hist = c.rmsd_histogram(out, 200, 0.5)
        assert np.array_equal(hist.sum(axis=1), types), (hist.sum(axis=1), types)
        half = c.apply_cutoff(out, 0.1)
        assert torch.equal(half, torch.where(out["rmsd"] <= 0.1, out["type"], torch.zeros_like(half)))
        del out, pos, sp
        torch.cuda.synchronize()
    finally:
        c.close()
    return res, types


def _oracle(oracle_lib, f, atoms=None, **kw):
    print(f"[full] oracle n={f.n} atoms={'all' if atoms is None else len(atoms)} {kw}", flush=True)
    return oracle_cache.classify(oracle_lib, f, atoms=atoms, **kw)


@pytest.fixture(scope="module")
def poly():
    return S.polycrystal()


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_polycrystal_every_atom(torch_cuda, oracle_lib, poly, precision):
    """All 918,996 atoms of the polycrystal."""
    f = poly
    got, types = _gpu(torch_cuda, precision, f)
    ref = _oracle(oracle_lib, f)
    st = compare(got, ref, tol=TOL64 if precision == ptm.PTM_FP64 else TOL32, check_alloy=False,
                 label="polycrystal ")
    assert np.array_equal(types, np.bincount(ref["type"], minlength=6))
    near = int(np.sum(ref["margin"] < 1e-9))
    print("polycrystal", f.n, types.tolist(), st, "near ties", near, flush=True)


@pytest.fixture(scope="module")
def alloy_frame():
    return S.alloy_slabs()


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_alloy_slabs_every_atom(torch_cuda, oracle_lib, alloy_frame, precision):
    """All ~4.03 M atoms of the alloy slabs, species included."""
    f = alloy_frame
    got, types = _gpu(torch_cuda, precision, f)
    ref = _oracle(oracle_lib, f)
    tol = TOL64 if precision == ptm.PTM_FP64 else TOL32
    st = compare(got, ref, tol=tol, label="alloy-slabs ")
    # the slabs hold L1_0, both L1_2 sites and B2
    assert set(np.unique(ref["alloy"])) >= {2, 3, 4, 7}, np.unique(ref["alloy"])
    print("alloy slabs", f.n, types.tolist(), st, flush=True)


@pytest.fixture(scope="module")
def mixed():
    f = S.mixed_frame()
    rng = np.random.default_rng(12)
    kind = f.labels["kind"]
    # inclusions follow the matrix, one after another: the icosahedra (first
    # half 55 atoms, second half 147), then the cubes; each cluster starts
    # with its centre atom
    n_ico = int(np.sum(f.labels["inclusion_kind"] == 1))
    sizes = np.array([55] * (n_ico // 2) + [147] * (n_ico - n_ico // 2))
    centres = int(np.nonzero(kind == 1)[0][0]) + np.concatenate([[0], np.cumsum(sizes)[:-1]])
    assert np.all(kind[centres] == 1)
    picks = [rng.choice(f.n, 2_000_000, replace=False), centres]
    for k in (1, 2, 3):
        picks.append(rng.choice(np.nonzero(kind == k)[0], 150, replace=False))
    return f, np.unique(np.concatenate(picks)), centres


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_mixed_frame_2M_sample(torch_cuda, oracle_lib, mixed, precision):
    f, atoms, centres = mixed
    got, types = _gpu(torch_cuda, precision, f, atoms)
    ref = _oracle(oracle_lib, f, atoms)
    tol = TOL64 if precision == ptm.PTM_FP64 else TOL32
    st = compare(got, ref, tol=tol, check_alloy=False, label="mixed ")
    # every structure of the frame is found: BCC matrix, SC cubes,
    # icosahedral centres, and disorder in the slab
    kind = f.labels["kind"]
    assert types[5] > 0.7 * np.sum(kind == 0) and types[1] > 0 and types[4] > 0 and types[0] > 0, types
    at_centres = ref["type"][np.searchsorted(atoms, centres)]
    assert np.mean(at_centres == 4) > 0.9, np.bincount(at_centres, minlength=6)
    print("mixed frame", f.n, "compared", len(atoms), types.tolist(), st, flush=True)


@pytest.fixture(scope="module")
def poly_sample(poly):
    rng = np.random.default_rng(13)
    return poly, np.unique(rng.choice(poly.n, 20000, replace=False))


def _sure(ref, got):
    """Atoms whose topological order cannot round differently (tmargin)."""
    sure = ~(ref["tmargin"] < 1e-6)
    assert np.sum(~sure) <= 2, np.sum(~sure)
    return ({k: v[sure] for k, v in got.items()}, {k: v[sure] for k, v in ref.items() if k in got})


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_polycrystal_topological_sampled(torch_cuda, oracle_lib, poly_sample, precision):
    """The 918,996-atom polycrystal with topological ordering (Sec. 3):
    20,000 seeded atoms."""
    f, atoms = poly_sample
    got, types = _gpu(torch_cuda, precision, f, atoms, topological=True)
    ref = _oracle(oracle_lib, f, atoms, ordering="topological")
    g, r = _sure(ref, got)
    st = compare(g, r, tol=TOL64 if precision == ptm.PTM_FP64 else TOL32, check_alloy=False, label="poly topo ")
    print("polycrystal topological", f.n, types.tolist(), st)


@pytest.mark.parametrize("precision", [ptm.PTM_FP32_MIXED], ids=["fp32mixed"])
def test_mixed_frame_topological_sampled(torch_cuda, oracle_lib, mixed, precision):
    """The ~32 M-atom mixed frame with topological ordering: 20,000 seeded
    atoms plus the icosahedron centres and region picks."""
    f, atoms, centres = mixed
    rng = np.random.default_rng(14)
    atoms = np.unique(np.concatenate([rng.choice(atoms, 20000, replace=False), centres]))
    got, types = _gpu(torch_cuda, precision, f, atoms, topological=True)
    ref = _oracle(oracle_lib, f, atoms, ordering="topological")
    g, r = _sure(ref, got)
    st = compare(g, r, tol=TOL32, check_alloy=False, label="mixed topo ")
    print("mixed frame topological", f.n, types.tolist(), st)
