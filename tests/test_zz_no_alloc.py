"""ptm_classify_noalloc, the entry point that allocates nothing, through the
C ABI: its outputs equal ptm_classify's on the same inputs, bit for bit (the
same kernels on the same inputs), for two calls in a row with the second
frame smaller than the first (the static scratch keeps the previous call's
contents), in both precision forms and both neighbour orderings, and for a
frame of exactly the largest size.  Sizes beyond the limit and host-pointer
contexts are refused before any device work; a periodic box too short for
the neighbour shell gives PTM_E_BOX with no output written."""
import math

import numpy as np
import pytest

from paper_1603_05143_amd import ptm, synthetic as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _run(torch, ctx, f, noalloc, fill=None):
    pos = torch.from_numpy(np.ascontiguousarray(f.positions)).to("cuda:0")
    sp = None if f.species is None else torch.from_numpy(f.species).to("cuda:0")
    out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True, derived=True)
    if fill is not None:
        for v in out.values():
            v.fill_(fill)
    torch.cuda.synchronize()
    call = ptm.ptm_classify_noalloc if noalloc else ptm.ptm_classify
    st = call(ctx, pos.data_ptr(), None if sp is None else sp.data_ptr(), f.box, f.n, ptm.PTM_ALL, math.inf,
              ptm.Classifier.outputs_struct(out))
    torch.cuda.synchronize()
    return st, {k: v.cpu().numpy() for k, v in out.items()}


def _frames():
    big = S.polycrystal(L=88.0, n_grains=5, sigma=0.1, seed=81)
    small = S.serving_frame(9000, seed=82)
    edge = S.perfect_crystal("fcc", (32, 32, 16), a=3.615)
    edge.positions = S.wrap(edge.positions + np.random.default_rng(83).normal(scale=0.05, size=edge.positions.shape),
                            edge.box)
    assert small.n < big.n <= ptm.PTM_NOALLOC_MAX_ATOMS and edge.n == ptm.PTM_NOALLOC_MAX_ATOMS
    return [big, small, edge]


@pytest.mark.parametrize("topological", [False, True], ids=["euclidean", "topological"])
@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_noalloc_equals_classify(torch_cuda, precision, topological):
    torch = torch_cuda
    flags = ptm.PTM_F_TOPOLOGICAL if topological else 0
    a = ptm.ptm_create(0, precision, None, 0, flags)
    b = ptm.ptm_create(0, precision, None, 0, flags)
    try:
        for f in _frames():  # the second call is smaller than the first
            print(f"[noalloc] n={f.n} precision={precision} topological={topological}", flush=True)
            st, ref = _run(torch, a, f, noalloc=False)
            assert st == ptm.PTM_OK, ptm.ptm_last_error(a)
            st, got = _run(torch, b, f, noalloc=True, fill=3)
            assert st == ptm.PTM_OK, ptm.ptm_last_error(b)
            for k in ref:
                assert np.array_equal(got[k], ref[k], equal_nan=True), (f.n, k)
    finally:
        ptm.ptm_destroy(a)
        ptm.ptm_destroy(b)


def test_noalloc_limits(torch_cuda):
    torch = torch_cuda
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, 0)
    try:
        n = ptm.PTM_NOALLOC_MAX_ATOMS + 1
        pos = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
        out = ptm.Classifier.alloc_outputs(n, "cuda:0")
        st = ptm.ptm_classify_noalloc(ctx, pos.data_ptr(), None, (50.0, 50.0, 50.0), n, ptm.PTM_ALL, math.inf,
                                      ptm.Classifier.outputs_struct(out))
        assert st == ptm.PTM_E_TOO_LARGE
        assert "PTM_NOALLOC_MAX_ATOMS" in ptm.ptm_last_error(ctx)
        # a periodic box too short for the shell: PTM_E_BOX, outputs untouched
        rng = np.random.default_rng(84)
        bad = S.Frame(positions=rng.random((30, 3)) * 6.0, box=np.array([6.0, 6.0, 6.0]))
        st, got = _run(torch, ctx, bad, noalloc=True, fill=7)
        assert st == ptm.PTM_E_BOX
        for k, v in got.items():
            assert np.all(v == 7), k
        # empty frame
        o = ptm.ptm_outputs()
        assert ptm.ptm_classify_noalloc(ctx, None, None, (10.0, 10.0, 10.0), 0, ptm.PTM_ALL, math.inf, o) == ptm.PTM_OK
    finally:
        ptm.ptm_destroy(ctx)
    hctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, ptm.PTM_F_HOST_POINTERS)
    try:
        f = S.config0()
        p = np.ascontiguousarray(f.positions)
        t = np.zeros(f.n, np.int8)
        o = ptm.ptm_outputs(type=t.ctypes.data)
        st = ptm.ptm_classify_noalloc(hctx, p.ctypes.data, None, f.box, f.n, ptm.PTM_ALL, math.inf, o)
        assert st == ptm.PTM_E_INVALID
    finally:
        ptm.ptm_destroy(hctx)
