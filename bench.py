#!/usr/bin/env python3
"""Throughput of the PTM classification pass on one MI355X.

One step = one ptm_classify call over the whole frame (bounds, binning,
k-NN, three hulls + canonical codes, candidate superposition, decision,
strain, alloy, write-back) with inputs and outputs resident in HBM, all five
templates enabled.  The headline workload is the single ~31.7 M-atom frame:
a periodic BCC matrix (a = 2.87 A, L = 256 a, 1 % vacancies) with 200 Mackay
icosahedra, 10 simple-cubic cubes and a liquid-like slab of 15 % of the
volume, sigma = 0.15 A.  ``value`` is the FP64 plain form (the paper's
method as it computes it); the FP32-mixed form is reported beside it.  The
~4.03 M-atom ordered-alloy slabs (species) and the 0.92 M-atom polycrystal
are measured as extra lines.

Prints one JSON line.  ``roofline`` covers the dominant kernel of the
headline run, timed with HIP events on the stream its kernels run on;
``cpu_baseline`` times the FP64 reference implementation on bounded samples
of the same frame (all host threads of the GPU's share and one thread, each
with and without the neighbour search); ``serving`` reports the serving loop
(ptm_submit / ptm_wait) on a stream of frames of uneven size: throughput when
saturated and p50/p99 frame latency under Poisson arrivals at 0.7 x the FP64
plain capacity.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atoms/s (PTM, all templates) FP32-mixed vs FP64 plain; p50/p99 frame latency"
STAGES = ("bounds", "bin", "knn", "topo", "match")

# MI355X published peaks: HBM3E bandwidth; vector FP64, which equals vector
# FP32 without packed instructions (the library is built without them)
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TFLOPS = 78.6

def orient_tests(K: int) -> int:
    """Orientation tests of the incremental hull of K points: the first
    tetrahedron, every facet of the current hull against each later point
    (2m - 4 facets when m points are in), and the centre against the 2K - 4
    final facets (counted separately)."""
    return 1 + sum(2 * m - 4 for m in range(4, K))


def work_model(stage: str, n: int, info: dict) -> tuple[str, float, str]:
    """Algorithmic work of one launch of a stage: (bound, amount, unit).

    Counted from the method, not from the kernels' instruction mix: FP
    operations for the arithmetic stages, HBM bytes for binning.
      knn     18 in-sphere distances per atom (the minimum any search must
              evaluate) x 11 FLOP (difference, minimum image, squared norm)
      topo    one incremental hull of the 14 neighbours (orient3d from
              differences = 23 FLOP per test) read off at 6, 12 and 14 points,
              each checked for the centre (14 FLOP per facet: the centre is
              the origin)
      match   per superposed candidate with N = 13 points: covariance 18N,
              G_b 6N, residual 27N, key matrix + characteristic polynomial +
              Newton + adjugate eigenvector + rotation ~290 FLOP; per atom
              the winner's outputs: quaternion (30) + strain (A^T = V+ W'
              234, A A^T 54, Jacobi 540, P 90) ~ 950 FLOP
      bin     104 B per atom (positions read twice, cell/slot/sorted writes)
              + 8 B per cell (histogram scan)
    """
    if stage == "bin":
        return "hbm", 104.0 * n + 8.0 * info.get("cells", 0), "bytes"
    if stage == "knn":
        return "alu", 18 * 11.0 * n, "flop"
    if stage == "topo":
        inside = sum(2 * K - 4 for K in (6, 12, 14))
        return "alu", (23.0 * orient_tests(14) + 14.0 * inside) * n, "flop"
    if stage == "match":
        N = 13
        return "alu", (51.0 * N + 290.0) * info.get("pairs", 0) + 950.0 * n, "flop"
    raise KeyError(stage)


def kernel_source_digest() -> str:
    """Digest of the kernel sources without their comments and blank lines;
    HBM traffic measured on other code is stale."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("ptm_kernels.hip", "ptm_device.hpp", "ptm_kernels.hpp", "ptm_tables.hpp"):
        with open(os.path.join(ROOT, "paper_1603_05143_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _profile_rows(name: str):
    """Rows of a summary table under profiles/ whose last column is the
    kernel source digest of this tree (numbers taken on other code are
    stale and ignored)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return []
    digest = kernel_source_digest()
    rows = []
    for line in open(path):
        cols = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cols) >= 4 and cols[-1] == digest:
            rows.append(cols)
    return rows


def measured_traffic(workload: str, stage: str, precision: str):
    """HBM bytes per launch of a stage's kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary under profiles/ (scaled by the copy-kernel
    calibration recorded there), or None if absent or taken on other sources."""
    for cols in _profile_rows(f"hbm_traffic_{workload}.md"):
        if len(cols) >= 6 and cols[0] == stage and cols[1] in (precision, "both"):
            try:
                return float(cols[2]) + float(cols[3])
            except ValueError:
                return None
    return None


def measured_valu_issue(workload: str, stage: str, precision: str):
    """Share of the vector units' issue slots the stage's kernel used
    (SQ_INSTS_VALU per wave x waves / (SIMDs x clock x kernel time)) from the
    rocprofv3 counter summary under profiles/, or None."""
    for cols in _profile_rows(f"valu_issue_{workload}.md"):
        if len(cols) >= 4 and cols[0] == stage and cols[1] in (precision, "both"):
            try:
                return float(cols[2])
            except ValueError:
                return None
    return None


# workloads: (key used by profiles/, description, generator)
WORKLOADS = {
    "mixed_31.7m": ("single periodic frame: BCC matrix a=2.87 A (L=256a, 1% vacancies), 200 Mackay icosahedra "
                    "(55/147 atoms, nn 2.55 A), 10 simple-cubic cubes (a=2.6 A), 15%-volume liquid-like slab "
                    "(2.2 A minimum distance), sigma 0.15 A, all templates", "mixed_frame"),
    "alloy_slabs_4.0m": ("ordered-alloy slabs with int8 species: L1_2 A3B (3.57 A), L1_0 AB (3.85 A, c/a 0.97), "
                         "B2 AB (2.88 A), random FCC; 2% antisites, 1% vacancies, sigma 0.25 A, all templates",
                         "alloy_slabs"),
    "polycrystal_919k": ("periodic Voronoi polycrystal, L=220 A, 16 grains FCC 3.615/BCC 2.87/HCP 2.51 "
                         "(c/a 1.633), sigma 0.10 A, all templates", "polycrystal"),
}


def build_frame(key: str):
    from paper_1603_05143_amd import synthetic as S
    t = time.time()
    f = getattr(S, WORKLOADS[key][1])()
    print(f"[bench] {key}: n={f.n} generated in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    return f


def run_gpu(frame, precision, steps, warmup, flags=0):
    import torch
    from paper_1603_05143_amd import ptm
    pos = torch.from_numpy(frame.positions).to("cuda:0")
    spc = None if frame.species is None else torch.from_numpy(frame.species).to("cuda:0")
    ctx = ptm.ptm_create(0, precision, None, 0, ptm.PTM_F_PROFILE | flags)
    out = ptm.Classifier.alloc_outputs(frame.n, "cuda:0")
    o = ptm.Classifier.outputs_struct(out)

    def step():
        st = ptm.ptm_classify(ctx, pos.data_ptr(), None if spc is None else spc.data_ptr(), frame.box, frame.n,
                              ptm.PTM_ALL, math.inf, o)
        if st != ptm.PTM_OK:
            raise RuntimeError(ptm.ptm_last_error(ctx))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    acc = [0.0] * len(STAGES)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        st_ms = ptm.ptm_stage_times(ctx)
        for i, s in enumerate(STAGES):
            acc[i] += st_ms[s]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = ptm.ptm_frame_info(ctx)
    types = torch.bincount(out["type"].long(), minlength=6).cpu().tolist()
    ptm.ptm_destroy(ctx)
    del out, pos, spc
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    return {"ms_per_step": ms, "atoms_per_s": frame.n / (ms / 1e3),
            "stage_ms": {s: acc[i] / steps for i, s in enumerate(STAGES)}, "types": types, "info": info}


def derived_overhead(frame, steps, warmup):
    """FP32-mixed frame time with every output of the widened rows requested
    (von Mises strain, eq.(6) residual, implied nearest-neighbour distance,
    fundamental-zone orientation, best match for the post-hoc cut-off)."""
    import torch
    from paper_1603_05143_amd import ptm
    pos = torch.from_numpy(frame.positions).to("cuda:0")
    ctx = ptm.ptm_create(0, ptm.PTM_FP32_MIXED, None, 0, 0)
    out = ptm.Classifier.alloc_outputs(frame.n, "cuda:0", derived=True)
    o = ptm.Classifier.outputs_struct(out)
    try:
        for k in range(warmup + steps):
            if k == warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            st = ptm.ptm_classify(ctx, pos.data_ptr(), None, frame.box, frame.n, ptm.PTM_ALL, math.inf, o)
            if st != ptm.PTM_OK:
                raise RuntimeError(ptm.ptm_last_error(ctx))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    finally:
        ptm.ptm_destroy(ctx)
    return ms


def posthoc_bench(n, reps=10):
    """Device time of the post-hoc entry points (HIP events on the stream the
    library launches on) over n seeded synthetic best matches with RMSDs
    spread like a thermal frame, and of ptm_misorientation over n / 4 pairs.
    All three are HBM-bound: bytes are the arrays read and written once."""
    import torch
    from paper_1603_05143_amd import ptm
    stream = torch.cuda.Stream()  # default priority; the library launches on it
    ctx = ptm.ptm_create(0, ptm.PTM_FP64, stream.cuda_stream, 0, 0)
    res = {}

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    def entry(name, ms, nbytes, count):
        gbs = nbytes / (ms / 1e3) / 1e9
        res[name] = {"n": count, "ms": round(ms, 4), "GB_s": round(gbs, 1),
                     "frac_of_hbm": round(gbs / PEAK_HBM_GBS, 3)}

    try:
        with torch.cuda.stream(stream):
            g = torch.Generator(device="cuda:0")
            g.manual_seed(160305143)
            bt = torch.randint(0, 6, (n,), dtype=torch.int8, device="cuda:0", generator=g)
            r = 0.02 + 0.08 * torch.rand(n, dtype=torch.float64, device="cuda:0", generator=g)
            ty = torch.empty(n, dtype=torch.int8, device="cuda:0")
            stream.synchronize()
            entry("apply_cutoff", timed(lambda: _ok(ptm.ptm_apply_cutoff(ctx, bt.data_ptr(), r.data_ptr(), n, 0.06,
                                                                         ty.data_ptr()))), 10 * n, n)
            entry("rmsd_histogram", timed(lambda: _ok(ptm.ptm_rmsd_histogram(ctx, bt.data_ptr(), r.data_ptr(), n,
                                                                             100, 0.3)[0])), 9 * n, n)
            del bt, r, ty
            m = n // 4
            q = torch.randn((2, m, 4), dtype=torch.float64, device="cuda:0", generator=g)
            q = q / q.norm(dim=-1, keepdim=True)
            q1, q2 = q[0].contiguous(), q[1].contiguous()
            tm = torch.randint(1, 6, (m,), dtype=torch.int8, device="cuda:0", generator=g)
            ang = torch.empty(m, dtype=torch.float64, device="cuda:0")
            stream.synchronize()
            entry("misorientation", timed(lambda: _ok(ptm.ptm_misorientation(ctx, tm.data_ptr(), q1.data_ptr(),
                                                                             q2.data_ptr(), m, ang.data_ptr()))),
                  73 * m, m)
    finally:
        stream.synchronize()
        ptm.ptm_destroy(ctx)
    return res


def _ok(status):
    if status != 0:
        raise RuntimeError(f"post-hoc entry point failed with status {status}")


def _mono_us():
    return time.clock_gettime(time.CLOCK_MONOTONIC) * 1e6  # the clock of ptm_frame_stats


def _pool_frame(arg):
    from threadpoolctl import threadpool_limits

    from paper_1603_05143_amd import synthetic as S
    n, seed = arg
    with threadpool_limits(1):  # one BLAS thread per worker process
        return S.serving_frame(n, seed=seed)


def serving_pool(pool_levels):
    """The distinct frames the serving stream draws from: log-spaced sizes in
    [1e3, 2e6], each its own seeded polycrystal (grain count, phases from the
    polycrystal and alloy workloads, noise U[0.02, 0.3] A).  Generated by
    worker processes before this process touches the GPU."""
    import multiprocessing as mp

    import numpy as np
    from paper_1603_05143_amd import synthetic as S
    levels = np.exp(np.linspace(math.log(1e3), math.log(2e6), pool_levels))
    jobs = [(int(round(n)), S.BASE_SEED + 300 + k) for k, n in enumerate(levels)]
    t = time.time()
    # largest first, so the long ones do not finish last
    order = sorted(range(len(jobs)), key=lambda k: -jobs[k][0])
    with mp.get_context("fork").Pool(processes=min(cpu_threads(), 16)) as pl:
        made = pl.map(_pool_frame, [jobs[k] for k in order], chunksize=1)
    pool = [None] * len(jobs)
    for k, f in zip(order, made):
        pool[k] = f
    print(f"[serve] pool of {len(pool)} frames ({sum(f.n for f in pool)} atoms) in {time.time() - t:.1f}s",
          file=sys.stderr, flush=True)
    return pool


def serving_bench(pool, n_frames, ring, budget_gb, seed_shift=0):
    """Serving loop on a stream of frames with log-uniform sizes in [1e3, 2e6],
    in both serving forms: the persistent kernel (PTM_F_PERSISTENT, first:
    the headline p50/p99) and the pool of streams.

    Each stream frame is the pool frame nearest to its size in log scale
    (the pool of distinct frames is resident on the device).  ``ring``
    output sets bound the frames in flight on the client side; admission on
    the library side is by the HBM budget.  Per form and precision: the
    saturated rate (every frame submitted as soon as an output set is free),
    then latency at one Poisson arrival rate for all runs, 0.7 x the
    persistent FP64 saturated frame rate.  Latency = completion time on the
    host clock - scheduled arrival time.
    """
    import collections

    import numpy as np
    import torch
    from paper_1603_05143_amd import ptm, synthetic as S

    sizes, _ = S.serving_stream(n_frames)
    pick = np.argmin(np.abs(np.log(sizes)[:, None] - np.log([f.n for f in pool])[None, :]), axis=1)
    dev = [(torch.from_numpy(f.positions).to("cuda:0"), torch.from_numpy(f.species).to("cuda:0"), f)
           for f in pool]
    nmax = max(f.n for f in pool)
    outs = [ptm.Classifier.alloc_outputs(nmax, "cuda:0") for _ in range(ring)]
    structs = [ptm.Classifier.outputs_struct(o) for o in outs]
    rng = np.random.default_rng(S.BASE_SEED + 3 + seed_shift)
    gaps = rng.exponential(1.0, n_frames)  # unit-rate Poisson process, scaled below
    atoms = np.array([pool[i].n for i in pick], dtype=np.float64)

    def run(ctx, rate_hz):
        free = collections.deque(range(ring))
        pending = collections.deque()
        done = np.zeros(n_frames)

        def reap(block):
            while pending:
                tk, k, slot = pending[0]
                st, s = ptm.ptm_wait(ctx, tk, -1 if block else 0)
                if st == ptm.PTM_E_TIMEOUT:
                    return
                if st != ptm.PTM_OK:
                    raise RuntimeError(ptm.ptm_last_error(ctx))
                pending.popleft()
                free.append(slot)
                done[k] = s.complete_time_us
                if block:
                    return

        arrive = None if rate_hz is None else np.cumsum(gaps) / rate_hz * 1e6
        t0 = _mono_us()
        for k in range(n_frames):
            if arrive is not None:
                while _mono_us() < t0 + arrive[k]:
                    reap(False)
            while not free:
                reap(True)
            slot = free.popleft()
            pos, spc, f = dev[pick[k]]
            while True:
                st, tk = ptm.ptm_submit(ctx, pos.data_ptr(), spc.data_ptr(), f.box, f.n, ptm.PTM_ALL, math.inf,
                                        structs[slot])
                if st != ptm.PTM_E_BUSY:
                    break
                reap(True)
            if st != ptm.PTM_OK:
                raise RuntimeError(ptm.ptm_last_error(ctx))
            pending.append((tk, k, slot))
        while pending:
            reap(True)
        return t0, arrive, done

    res = {}
    rate = None
    for mode, flags in (("persistent", ptm.PTM_F_PERSISTENT), ("streams", 0)):
        for name, prec in (("fp64", ptm.PTM_FP64), ("fp32_mixed", ptm.PTM_FP32_MIXED)):
            ctx = ptm.ptm_create(0, prec, None, int(budget_gb * 1e9), flags)
            # warm the scratch pool: every pool frame twice, in flight together
            keep = []
            for rep in range(2):
                for j, (pos, spc, f) in enumerate(dev):
                    while True:
                        st, tk = ptm.ptm_submit(ctx, pos.data_ptr(), spc.data_ptr(), f.box, f.n, ptm.PTM_ALL,
                                                math.inf, structs[(rep * len(dev) + j) % ring])
                        if st != ptm.PTM_E_BUSY or not keep:
                            break
                        ptm.ptm_wait(ctx, keep.pop(0), -1)
                    if st != ptm.PTM_OK:
                        raise RuntimeError(ptm.ptm_last_error(ctx))
                    keep.append(tk)
            for tk in keep:
                ptm.ptm_wait(ctx, tk, -1)
            t0, _, done = run(ctx, None)
            span_s = (done.max() - t0) / 1e6
            r = {"atoms_per_s": atoms.sum() / span_s, "frames_per_s": n_frames / span_s}
            if rate is None:
                rate = 0.7 * r["frames_per_s"]  # same arrival rate for both forms
            t0, arrive, done = run(ctx, rate)
            lat_ms = (done - (t0 + arrive)) / 1e3
            lat = lat_ms[50:] if n_frames > 100 else lat_ms
            r.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "mean_ms": float(lat.mean())})
            ptm.ptm_destroy(ctx)
            print(f"[serve] {mode} {name}: {r}", file=sys.stderr, flush=True)
            res.setdefault(mode, {})[name] = r
    del outs, dev
    return {"frames": n_frames, "sizes": "log-uniform in [1e3, 2e6] atoms",
            "pool_frames": len(pool), "pool_atoms": int(sum(f.n for f in pool)),
            "distinct_frames_used": int(len(np.unique(pick))),
            "rate_hz": rate, "budget_gb": budget_gb, "client_ring": ring,
            "latency_over": f"frames 51-{n_frames}" if n_frames > 100 else "all frames",
            "form": "persistent kernel (PTM_F_PERSISTENT)",
            "fp64": res["persistent"]["fp64"], "fp32_mixed": res["persistent"]["fp32_mixed"],
            "streams": res["streams"]}


def cpu_threads() -> int:
    """Host threads: the CPUs this process may use, at most 16 (the host
    share of one GPU on the machines this runs on)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(frame, label, sample_all, sample_one):
    """The FP64 oracle as it stands on the GPU machine's host: all threads
    of the share and one thread, each with its neighbour search timed and
    without it (neighbours found first, untimed: the paper's Table 2 timing
    excludes neighbour-list generation).  Seeded atom samples of the frame."""
    import numpy as np
    import oracle
    threads = cpu_threads()
    rng = np.random.default_rng(2024)
    big = np.sort(rng.choice(frame.n, sample_all, replace=False))
    small = np.sort(rng.choice(big, sample_one, replace=False))
    oracle.lib()
    res = {}
    for name, atoms, th in (("all_threads", big, threads), ("single_thread", small, 1)):
        t = time.perf_counter()
        oracle.classify(frame.positions, frame.box, species=frame.species, atoms=atoms, threads=th)
        dt = time.perf_counter() - t
        nb = oracle.neighbours(frame.positions, frame.box, atoms=atoms, threads=threads)
        t = time.perf_counter()
        oracle.classify_given(nb, atoms, frame.box, species=frame.species, threads=th)
        dt2 = time.perf_counter() - t
        res[name] = {"atoms_per_s": len(atoms) / dt, "atoms_per_s_without_knn": len(atoms) / dt2,
                     "threads": th, "sample_atoms": int(len(atoms)), "wall_s": round(dt, 2),
                     "wall_s_without_knn": round(dt2, 2)}
        print(f"[bench] cpu oracle {name}: {res[name]}", file=sys.stderr, flush=True)
    nproc = os.cpu_count()
    return {"value": res["all_threads"]["atoms_per_s"], "unit": "atoms/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample_all} seeded atoms of the {frame.n}-atom {label} on {threads} threads "
                      f"({res['all_threads']['wall_s']} s wall; neighbours by the oracle's certified cell "
                      f"search, brute force below 2e5 atoms); also {sample_one} of them on one thread, "
                      f"and both without the neighbour search",
            "host_cpus_visible": nproc,
            "all_threads_without_knn": res["all_threads"]["atoms_per_s_without_knn"],
            "single_thread": res["single_thread"]["atoms_per_s"],
            "single_thread_without_knn": res["single_thread"]["atoms_per_s_without_knn"],
            "detail": res}


def roofline(run, n, stage_kernel, workload, precision):
    """Roofline object of the stage with the largest device time."""
    stage_ms = run["stage_ms"]
    dom = max(stage_kernel, key=lambda st: stage_ms[st])
    bound, work, unit = work_model(dom, n, run["info"])
    t = stage_ms[dom] / 1e3
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": work / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": work / t / 1e12, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(workload, dom, precision)
    roof["valu_issue_frac"] = measured_valu_issue(workload, dom, precision)
    roof["kernel"] = stage_kernel[dom]
    roof["kernel_ms"] = stage_ms[dom]
    roof["work_per_launch"] = work
    roof["work_unit"] = unit
    return roof


def line_of(run):
    return {"atoms_per_s": run["atoms_per_s"], "ms_per_step": round(run["ms_per_step"], 4),
            "stage_ms": {k: round(v, 4) for k, v in run["stage_ms"].items()}, "work_counts": run["info"]}


def polycrystal_extras(args):
    """The 0.92 M-atom polycrystal in both forms, with and without the
    topological ordering and with every derived output; then the post-hoc
    entry points."""
    from paper_1603_05143_amd import ptm
    extra = {}
    poly = build_frame("polycrystal_919k")
    p64 = run_gpu(poly, ptm.PTM_FP64, args.steps * 2, args.warmup)
    p32 = run_gpu(poly, ptm.PTM_FP32_MIXED, args.steps * 2, args.warmup)
    print(f"[bench] polycrystal fp64 {p64['ms_per_step']:.2f} fp32-mixed {p32['ms_per_step']:.2f} ms/step",
          file=sys.stderr, flush=True)
    # topological neighbour ordering (Sec. 3): the same frame, both forms;
    # its Voronoi kernels run inside the k-NN stage
    t64 = run_gpu(poly, ptm.PTM_FP64, args.steps * 2, args.warmup, ptm.PTM_F_TOPOLOGICAL)
    t32 = run_gpu(poly, ptm.PTM_FP32_MIXED, args.steps * 2, args.warmup, ptm.PTM_F_TOPOLOGICAL)
    print(f"[bench] topological fp32-mixed {t32['ms_per_step']:.2f} ms/step, fp64 {t64['ms_per_step']:.2f}",
          file=sys.stderr, flush=True)
    extra["polycrystal_919k"] = {
        "workload": WORKLOADS["polycrystal_919k"][0], "n_atoms": poly.n,
        "fp32_mixed": line_of(p32), "fp64": line_of(p64),
        "fp32_mixed_over_fp64": p32["atoms_per_s"] / p64["atoms_per_s"],
        "types": dict(zip(ptm.TYPE_NAMES, p32["types"])),
        "topological": {
            "fp32_mixed_atoms_per_s": t32["atoms_per_s"], "fp64_atoms_per_s": t64["atoms_per_s"],
            "fp32_mixed_ms_per_step": round(t32["ms_per_step"], 4), "fp64_ms_per_step": round(t64["ms_per_step"], 4),
            "fp32_mixed_stage_ms": {k: round(v, 4) for k, v in t32["stage_ms"].items()},
            "cost_over_euclidean": round(t32["ms_per_step"] / p32["ms_per_step"], 3),
            "types": dict(zip(ptm.TYPE_NAMES, t32["types"])),
        },
    }
    derived_ms = derived_overhead(poly, args.steps * 2, args.warmup)
    extra["polycrystal_919k"]["derived_outputs_ms_per_step"] = round(derived_ms, 4)
    del poly
    posthoc = posthoc_bench(1 << 27)
    print(f"[bench] derived outputs {derived_ms:.2f} ms/step; post-hoc {posthoc}", file=sys.stderr, flush=True)
    return extra["polycrystal_919k"], posthoc


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", choices=("all", "headline", "fp64", "fp32", "polycrystal"), default="all",
                    help="headline: the 31.7 M-atom frame alone (both forms, or one with fp64 / fp32); "
                         "polycrystal: the 0.92 M-atom frame's lines and the post-hoc entry points alone; "
                         "for profiling runs")
    ap.add_argument("--cpu-sample", type=int, default=100000, help="atoms of the all-threads CPU sample")
    ap.add_argument("--cpu-sample-1t", type=int, default=6000, help="atoms of the one-thread CPU sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-frames", type=int, default=2000)
    ap.add_argument("--serve-pool", type=int, default=200)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy a 256 MiB device buffer (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    pool = None
    if args.only == "all" and not args.no_serve:
        pool = serving_pool(args.serve_pool)
    import torch  # (loads the HIP runtime shared with libptm)
    from paper_1603_05143_amd import ptm

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only == "polycrystal":
        poly_line, posthoc = polycrystal_extras(args)
        print(json.dumps({"polycrystal_919k": poly_line, "posthoc": posthoc}))
        return

    # ---- headline: the 31.7 M-atom frame, FP64 plain (value) and FP32-mixed
    head = "mixed_31.7m"
    frame = build_frame(head)
    r64 = r32 = None
    if args.only in ("all", "headline", "fp64"):
        r64 = run_gpu(frame, ptm.PTM_FP64, args.steps, args.warmup)
        print(f"[bench] {head} fp64 {r64['ms_per_step']:.2f} ms/step {r64['stage_ms']}", file=sys.stderr, flush=True)
    if args.only in ("all", "headline", "fp32"):
        r32 = run_gpu(frame, ptm.PTM_FP32_MIXED, args.steps, args.warmup)
        print(f"[bench] {head} fp32-mixed {r32['ms_per_step']:.2f} ms/step {r32['stage_ms']}", file=sys.stderr,
              flush=True)
    main_run = r64 if r64 is not None else r32
    dtype = "f64" if r64 is not None else "f32-mixed"
    stage_kernel = {"knn": "k_knn_fast<14> + k_knn_exact<14>", "topo": "k_topo",
                    "match": "k_match<double>" if r64 is not None else "k_match<float>"}
    roof = roofline(main_run, frame.n, stage_kernel, head, "fp64" if r64 is not None else "fp32_mixed")
    roof["kernel"] += " in the " + ("FP64" if r64 is not None else "FP32-mixed") + " frame"

    line = {
        "metric": METRIC, "value": main_run["atoms_per_s"], "unit": "atoms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[head][0], "n_atoms": frame.n, "template_mask": "SC|FCC|HCP|ICO|BCC",
                   "rmsd_cutoff": "inf", "form": "FP64 plain" if r64 is not None else "FP32-mixed"},
        "fp64_atoms_per_s": None if r64 is None else r64["atoms_per_s"],
        "fp32_mixed_atoms_per_s": None if r32 is None else r32["atoms_per_s"],
        "fp32_mixed_over_fp64": None if (r64 is None or r32 is None) else r32["atoms_per_s"] / r64["atoms_per_s"],
        "fp32_mixed_over_fp64_target": 2.0,
        "stage_ms": {k: round(v, 4) for k, v in main_run["stage_ms"].items()},
        "fp32_mixed_stage_ms": None if r32 is None else {k: round(v, 4) for k, v in r32["stage_ms"].items()},
        "work_counts": main_run["info"],
        "types": dict(zip(ptm.TYPE_NAMES, main_run["types"])),
        "roofline": roof,
    }
    if args.only != "all":
        print(json.dumps(line))
        return

    # ---- the other full-size workloads (extra lines)
    extra = {}
    alloy = build_frame("alloy_slabs_4.0m")
    a64 = run_gpu(alloy, ptm.PTM_FP64, args.steps, args.warmup)
    a32 = run_gpu(alloy, ptm.PTM_FP32_MIXED, args.steps, args.warmup)
    print(f"[bench] alloy slabs fp64 {a64['ms_per_step']:.2f} fp32-mixed {a32['ms_per_step']:.2f} ms/step",
          file=sys.stderr, flush=True)
    extra["alloy_slabs_4.0m"] = {"workload": WORKLOADS["alloy_slabs_4.0m"][0], "n_atoms": alloy.n,
                                 "fp32_mixed": line_of(a32), "fp64": line_of(a64),
                                 "fp32_mixed_over_fp64": a32["atoms_per_s"] / a64["atoms_per_s"],
                                 "types": dict(zip(ptm.TYPE_NAMES, a32["types"]))}
    del alloy
    extra["polycrystal_919k"], posthoc = polycrystal_extras(args)

    serving = None
    if not args.no_serve:
        serving = serving_bench(pool, args.serve_frames, ring=24, budget_gb=200.0)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(frame, "mixed frame", args.cpu_sample, args.cpu_sample_1t)
        cpu["paper_single_core_context"] = ("1.08e5 atoms/s: the paper's one laptop core (i7-4770HQ, 2014) on an "
                                            "88,737-atom system, neighbour lists excluded (Table 2, Sec. 9)")

    line.update({"extra_workloads": extra, "posthoc": posthoc, "serving": serving, "cpu_baseline": cpu})
    print(json.dumps(line))


if __name__ == "__main__":
    main()
