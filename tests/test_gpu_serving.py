"""Serving loop (ptm_submit / ptm_wait) on the GPU, through the C ABI, in
both of its forms: frames on a pool of streams, and frames drained by one
persistent kernel (PTM_F_PERSISTENT).

Frames of uneven size are submitted back to back so that their work
overlaps on the device; each result must equal the result of the same frame
classified alone (the pipeline is deterministic, so equality is exact), in
both precision forms.  Admission by HBM budget and the timeout path are
checked as well.
"""
import math

import numpy as np
import pytest

from paper_1603_05143_amd import ptm, synthetic as S

pytestmark = pytest.mark.gpu

FIELDS = ("type", "alloy", "rmsd", "scale", "quat", "neighbours", "strain", "knn")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


MODES = [0, ptm.PTM_F_PERSISTENT]
MODE_IDS = ["streams", "persistent"]


def _open_cluster(shells, seed):
    """An open-boundary frame: a thermally displaced Mackay icosahedron."""
    rng = np.random.default_rng(seed)
    pos = S.mackay_icosahedron(shells)
    return S.Frame(positions=pos + rng.normal(0.0, 0.05, pos.shape), box=np.zeros(3))


@pytest.fixture(scope="module")
def frames():
    sizes = [1200, 40000, 3000, 150000, 700, 12000, 90000, 5000]
    fr = [S.serving_frame(int(n), seed=1000 + k) for k, n in enumerate(sizes)]
    fr.insert(3, _open_cluster(5, 7))  # open axes: the grid follows from the bounds
    return fr


def _device_frame(torch, f):
    pos = torch.from_numpy(np.ascontiguousarray(f.positions)).to("cuda:0")
    sp = None if f.species is None else torch.from_numpy(f.species).to("cuda:0")
    return pos, sp


def _alone(torch, precision, frames):
    c = ptm.Classifier(device=0, precision=precision)
    res = []
    for f in frames:
        pos, sp = _device_frame(torch, f)
        out = c.classify(pos, f.box, species=sp, knn=True, derived=True)
        torch.cuda.synchronize()
        res.append({k: v.cpu().numpy() for k, v in out.items()})
    c.close()
    return res


def _submit_all(torch, ctx, frames):
    keep, tickets = [], []
    for f in frames:
        pos, sp = _device_frame(torch, f)
        out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True, derived=True)
        o = ptm.Classifier.outputs_struct(out)
        st, t = ptm.ptm_submit(ctx, pos.data_ptr(), None if sp is None else sp.data_ptr(), f.box, f.n,
                               ptm.PTM_ALL, math.inf, o)
        assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        keep.append((pos, sp, out, o))
        tickets.append(t)
    return keep, tickets


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_mixed_equals_alone(torch_cuda, frames, precision, mode):
    torch = torch_cuda
    ref = _alone(torch, precision, frames)
    ctx = ptm.ptm_create(0, precision, None, 0, mode)
    try:
        for rep in range(2):  # the second pass reuses pooled scratch
            keep, tickets = _submit_all(torch, ctx, frames)
            stats = []
            for t in reversed(tickets):  # any completion order
                st, s = ptm.ptm_wait(ctx, t, -1)
                assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
                stats.append((s.submit_time_us, s.start_time_us, s.complete_time_us, s.n_atoms))
            for (pos, sp, out, o), r, f in zip(keep, ref, frames):
                got = {k: v.cpu().numpy() for k, v in out.items()}
                assert set(got) == set(FIELDS) | {"vm_strain", "strain_residual", "nn_distance", "quat_fz",
                                                  "best_type"}
                for k in got:
                    assert np.array_equal(got[k], r[k], equal_nan=True), (rep, f.n, k)
            for sub, start, done, n in stats:
                assert sub <= start <= done + 1e3, (sub, start, done)
                assert n in [f.n for f in frames]
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_budget_admission(torch_cuda, frames, mode):
    torch = torch_cuda
    big = max(frames, key=lambda f: f.n)
    # a budget that holds one frame of this size but not two
    probe = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, mode)
    keep, (t,) = _submit_all(torch, probe, [big])
    st, s = ptm.ptm_wait(probe, t, -1)
    assert st == ptm.PTM_OK
    ptm.ptm_destroy(probe)
    cls = s.scratch_bytes
    assert cls >= 24 * big.n and cls & (cls - 1) == 0
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, cls + cls // 2, mode)
    try:
        pos, sp = _device_frame(torch, big)
        outs = [ptm.Classifier.alloc_outputs(big.n, "cuda:0") for _ in range(2)]
        o1, o2 = (ptm.Classifier.outputs_struct(o) for o in outs)
        st1, t1 = ptm.ptm_submit(ctx, pos.data_ptr(), None, big.box, big.n, ptm.PTM_ALL, math.inf, o1)
        assert st1 == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        st2, _ = ptm.ptm_submit(ctx, pos.data_ptr(), None, big.box, big.n, ptm.PTM_ALL, math.inf, o2)
        assert st2 == ptm.PTM_E_BUSY
        assert ptm.ptm_wait(ctx, t1, -1)[0] == ptm.PTM_OK
        st2, t2 = ptm.ptm_submit(ctx, pos.data_ptr(), None, big.box, big.n, ptm.PTM_ALL, math.inf, o2)
        assert st2 == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        assert ptm.ptm_wait(ctx, t2, -1)[0] == ptm.PTM_OK
        torch.cuda.synchronize()
        for k in ("type", "rmsd", "neighbours"):
            assert torch.equal(outs[0][k], outs[1][k])
        # a budget smaller than one frame's class is a hard error
        tiny = ptm.ptm_create(0, ptm.PTM_FP64, None, 1 << 20, mode)
        st3, _ = ptm.ptm_submit(tiny, pos.data_ptr(), None, big.box, big.n, ptm.PTM_ALL, math.inf, o1)
        assert st3 == ptm.PTM_E_NOMEM
        ptm.ptm_destroy(tiny)
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_wait_timeout_and_unknown_ticket(torch_cuda, frames, mode):
    torch = torch_cuda
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, mode)
    try:
        big = max(frames, key=lambda f: f.n)
        keep, (t,) = _submit_all(torch, ctx, [big])
        st, _ = ptm.ptm_wait(ctx, t, 0)
        assert st in (ptm.PTM_OK, ptm.PTM_E_TIMEOUT)
        if st == ptm.PTM_E_TIMEOUT:  # the ticket stays valid
            assert ptm.ptm_wait(ctx, t, -1)[0] == ptm.PTM_OK
        assert ptm.ptm_wait(ctx, t, -1)[0] == ptm.PTM_E_INVALID  # already retired
        assert ptm.ptm_wait(ctx, 987654321, 0)[0] == ptm.PTM_E_INVALID
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_empty_frame_ticket(torch_cuda, mode):
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, mode)
    try:
        o = ptm.ptm_outputs()
        st, t = ptm.ptm_submit(ctx, None, None, (10.0, 10.0, 10.0), 0, ptm.PTM_ALL, math.inf, o)
        assert st == ptm.PTM_OK
        st, s = ptm.ptm_wait(ctx, t, 0)
        assert st == ptm.PTM_OK and s.n_atoms == 0
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_mixed_equals_oracle(torch_cuda, oracle_lib, frames, precision, mode):
    """The frames submitted together, overlapping on the device, against the
    FP64 oracle frame by frame: decisions bit-exact, reals within the form's
    tolerance."""
    from parity_util import TOL32, TOL64, compare
    torch = torch_cuda
    ctx = ptm.ptm_create(0, precision, None, 0, mode)
    try:
        keep, tickets = _submit_all(torch, ctx, frames)
        for t in tickets:
            st, _ = ptm.ptm_wait(ctx, t, -1)
            assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
        for (pos, sp, out, o), f in zip(keep, frames):
            print(f"[serve-oracle] n={f.n} precision={precision}", flush=True)
            got = {k: out[k].cpu().numpy() for k in FIELDS}
            ref = oracle_lib.classify(f.positions, f.box, species=f.species)
            compare(got, {k: ref[k] for k in FIELDS}, tol=TOL64 if precision == ptm.PTM_FP64 else TOL32,
                    check_alloy=f.species is not None, label=f"serving n={f.n} ")
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_box_error_in_the_stream(torch_cuda, oracle_lib, frames, mode):
    """A frame whose periodic box is too short for its neighbour shell,
    submitted between others: its ticket reports PTM_E_BOX and its outputs
    stay untouched; the frames around it are unaffected."""
    torch = torch_cuda
    rng = np.random.default_rng(5)
    bad = S.Frame(positions=rng.random((20, 3)) * 6.0, box=np.array([6.0, 6.0, 6.0]))
    with pytest.raises(oracle_lib.BoxError):
        oracle_lib.classify(bad.positions, bad.box)
    mix = [frames[0], bad, frames[2]]
    ref = _alone(torch, ptm.PTM_FP64, [frames[0], frames[2]])
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, mode)
    try:
        keep, tickets = [], []
        for f in mix:
            pos, sp = _device_frame(torch, f)
            out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True, derived=True)
            for v in out.values():
                v.fill_(7)
            torch.cuda.synchronize()
            o = ptm.Classifier.outputs_struct(out)
            st, t = ptm.ptm_submit(ctx, pos.data_ptr(), None if sp is None else sp.data_ptr(), f.box, f.n,
                                   ptm.PTM_ALL, math.inf, o)
            assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
            keep.append((pos, sp, out, o))
            tickets.append(t)
        status = [ptm.ptm_wait(ctx, t, -1)[0] for t in tickets]
        assert status == [ptm.PTM_OK, ptm.PTM_E_BOX, ptm.PTM_OK]
        torch.cuda.synchronize()
        for k, v in keep[1][2].items():
            assert bool((v == 7).all()), k
        for (pos, sp, out, o), r in zip((keep[0], keep[2]), ref):
            for k in out:
                assert np.array_equal(out[k].cpu().numpy(), r[k], equal_nan=True), k
    finally:
        ptm.ptm_destroy(ctx)


def test_persistent_nonfinite_frame(torch_cuda, frames):
    """A non-finite coordinate in a frame handed to the persistent kernel:
    ptm_submit accepts it (nothing is checked on the host), ptm_wait reports
    PTM_E_INVALID, the outputs stay untouched and the next frame is served."""
    torch = torch_cuda
    f = frames[0]
    bad = f.positions.copy()
    bad[17, 1] = np.nan
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, None, 0, ptm.PTM_F_PERSISTENT)
    try:
        pos = torch.from_numpy(bad).to("cuda:0")
        out = ptm.Classifier.alloc_outputs(f.n, "cuda:0")
        for v in out.values():
            v.fill_(7)
        torch.cuda.synchronize()
        st, t = ptm.ptm_submit(ctx, pos.data_ptr(), None, f.box, f.n, ptm.PTM_ALL, math.inf,
                               ptm.Classifier.outputs_struct(out))
        assert st == ptm.PTM_OK
        assert ptm.ptm_wait(ctx, t, -1)[0] == ptm.PTM_E_INVALID
        assert "non-finite" in ptm.ptm_last_error(ctx)
        torch.cuda.synchronize()
        for k, v in out.items():
            assert bool((v == 7).all()), k
        keep, (t2,) = _submit_all(torch, ctx, [f])
        assert ptm.ptm_wait(ctx, t2, -1)[0] == ptm.PTM_OK
    finally:
        ptm.ptm_destroy(ctx)


@pytest.mark.parametrize("precision", [ptm.PTM_FP64, ptm.PTM_FP32_MIXED], ids=["fp64", "fp32mixed"])
def test_persistent_many_frames(torch_cuda, precision):
    """300 frames of 64 to 6000 atoms (periodic and open) through the
    persistent kernel, more than its 256 slots: submissions past the slots
    return PTM_E_BUSY and are retried after waiting for the oldest ticket;
    every frame equals the same frame classified alone."""
    torch = torch_cuda
    rng = np.random.default_rng(31)
    fr = []
    for k in range(300):
        if k % 7 == 3:
            fr.append(_open_cluster(int(rng.integers(2, 5)), 100 + k))
        else:
            fr.append(S.serving_frame(int(rng.integers(64, 6000)), seed=2000 + k))
    ref = _alone(torch, precision, fr)
    ctx = ptm.ptm_create(0, precision, None, 0, ptm.PTM_F_PERSISTENT)
    try:
        pending, done, busy = [], {}, 0
        for k, f in enumerate(fr):
            pos, sp = _device_frame(torch, f)
            out = ptm.Classifier.alloc_outputs(f.n, "cuda:0", knn=True, derived=True)
            o = ptm.Classifier.outputs_struct(out)
            while True:
                st, t = ptm.ptm_submit(ctx, pos.data_ptr(), None if sp is None else sp.data_ptr(), f.box, f.n,
                                       ptm.PTM_ALL, math.inf, o)
                if st != ptm.PTM_E_BUSY:
                    break
                busy += 1
                j, t0, keep0 = pending.pop(0)
                assert ptm.ptm_wait(ctx, t0, -1)[0] == ptm.PTM_OK, ptm.ptm_last_error(ctx)
                done[j] = keep0
            assert st == ptm.PTM_OK, ptm.ptm_last_error(ctx)
            pending.append((k, t, (pos, sp, out, o)))
        for j, t0, keep0 in pending:
            assert ptm.ptm_wait(ctx, t0, -1)[0] == ptm.PTM_OK, ptm.ptm_last_error(ctx)
            done[j] = keep0
        assert busy > 0
        for k, f in enumerate(fr):
            out = done[k][2]
            for key, v in out.items():
                assert np.array_equal(v.cpu().numpy(), ref[k][key], equal_nan=True), (k, f.n, key)
        print("persistent frames", len(fr), "busy retries", busy, flush=True)
    finally:
        ptm.ptm_destroy(ctx)


def test_persistent_with_topological_is_refused():
    with pytest.raises(ptm.PTMError):
        ptm.ptm_create(0, ptm.PTM_FP64, None, 0, ptm.PTM_F_PERSISTENT | ptm.PTM_F_TOPOLOGICAL)
