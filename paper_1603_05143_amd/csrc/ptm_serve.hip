// ptm_serve.hip -- table upload, host-pointer staging and the serving loop
// (ptm_submit / ptm_wait).
//
// Serving is continuous batching over a pool of HIP streams (default
// priority): each admitted frame gets its own scratch and runs its whole
// pipeline on the next stream of the pool, so frames that arrive while
// others are on the device overlap with them.  Scratch comes from a
// grow-only pool of power-of-two size classes (no device free, hence no
// implicit device synchronisation, while serving).  Admission is by bytes:
// a frame is admitted when the pool memory it needs fits within the
// context's HBM budget next to that of all in-flight frames; otherwise
// ptm_submit returns PTM_E_BUSY and the caller retries after a ptm_wait.
// Completion times are read from timing events on the device timeline.
//
// With PTM_F_PERSISTENT the frames go to one persistent kernel instead
// (k_serve): ptm_submit writes the frame's request (inputs, outputs and
// its pooled scratch) into a pinned block and returns; the kernel pulls it
// and runs every stage as work items; ptm_wait polls the completion word
// the kernel writes back, relaunching the kernel if it has exited idle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "ptm_internal.hpp"

using namespace ptm;

namespace ptm {

static constexpr int SERVE_STREAMS = 4;

ptm_status upload_tables(ptm_ctx *ctx) {
    auto up = [&](const void *src, size_t bytes, void **dst) -> ptm_status {
        if (bytes == 0) bytes = 8;
        PTM_HIP(ctx, hipMalloc(dst, bytes));
        ctx->table_buffers.push_back(*dst);
        if (src) PTM_HIP(ctx, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return PTM_OK;
    };
    void *p;
    ptm_status st;
    if ((st = up(ctx->host.tpl, sizeof(TemplateDev) * NT, &p)) != PTM_OK) return st;
    ctx->view.tpl = (const TemplateDev *)p;
    for (int g = 0; g < NGRP; g++) {
        HostTables &H = ctx->host;
        if ((st = up(H.codes[g].data(), H.codes[g].size() * 8, &p)) != PTM_OK) return st;
        ctx->view.codes[g] = (const uint64_t *)p;
        if ((st = up(H.slots[g].data(), H.slots[g].size() * 4, &p)) != PTM_OK) return st;
        ctx->view.slots[g] = (const int32_t *)p;
        if ((st = up(H.cstart[g].data(), H.cstart[g].size() * 4, &p)) != PTM_OK) return st;
        ctx->view.cstart[g] = (const int32_t *)p;
        if ((st = up(H.cand[g].data(), H.cand[g].size() * sizeof(Candidate), &p)) != PTM_OK) return st;
        ctx->view.cand[g] = (const Candidate *)p;
        ctx->view.hmask[g] = H.hmask[g];
        ctx->view.ncodes[g] = H.ncodes[g];
    }
    return PTM_OK;
}

static size_t staging_bytes(int64_t n) {
    size_t a = 0;
    auto add = [&](size_t s) { a += (s + 255) & ~(size_t)255; };
    add(24 * (size_t)n);   // positions
    add((size_t)n);        // species
    add((size_t)n);        // type
    add((size_t)n);        // alloy
    add(8 * (size_t)n);    // rmsd
    add(8 * (size_t)n);    // scale
    add(32 * (size_t)n);   // quat
    add(56 * (size_t)n);   // neighbours
    add(72 * (size_t)n);   // strain
    add(56 * (size_t)n);   // knn
    add(8 * (size_t)n);    // vm_strain
    add(8 * (size_t)n);    // strain_residual
    add(8 * (size_t)n);    // nn_distance
    add(32 * (size_t)n);   // quat_fz
    add((size_t)n);        // best_type
    return a;
}

ptm_status stage_in_buffers(ptm_ctx *ctx, StagingBuffers &B, const double *positions, const int8_t *species,
                            const ptm_outputs *out, int64_t n, FrameJob &J, HostStage &H, hipStream_t st) {
    if (!(ctx->flags & PTM_F_HOST_POINTERS)) {
        J.pos = positions;
        J.species = species;
        J.out = *out;
        H.active = false;
        return PTM_OK;
    }
    size_t need = staging_bytes(n);
    if (need > B.bytes) {
        B.release();
        if (hipMalloc(&B.base, need) != hipSuccess) {
            (void)hipGetLastError();
            ctx->err = "staging allocation failed";
            return PTM_E_NOMEM;
        }
        B.bytes = need;
    }
    char *p = (char *)B.base;
    auto take = [&](size_t s) {
        char *r = p;
        p += (s + 255) & ~(size_t)255;
        return (void *)r;
    };
    double *dpos = (double *)take(24 * (size_t)n);
    int8_t *dspc = (int8_t *)take((size_t)n);
    ptm_outputs d;
    d.type = (int8_t *)take((size_t)n);
    d.alloy = (int8_t *)take((size_t)n);
    d.rmsd = (double *)take(8 * (size_t)n);
    d.scale = (double *)take(8 * (size_t)n);
    d.quat = (double *)take(32 * (size_t)n);
    d.neighbours = (int32_t *)take(56 * (size_t)n);
    d.strain = (double *)take(72 * (size_t)n);
    d.knn = (int32_t *)take(56 * (size_t)n);
    d.vm_strain = (double *)take(8 * (size_t)n);
    d.strain_residual = (double *)take(8 * (size_t)n);
    d.nn_distance = (double *)take(8 * (size_t)n);
    d.quat_fz = (double *)take(32 * (size_t)n);
    d.best_type = (int8_t *)take((size_t)n);
    if (!out->alloy) d.alloy = nullptr;
    if (!out->rmsd) d.rmsd = nullptr;
    if (!out->scale) d.scale = nullptr;
    if (!out->quat) d.quat = nullptr;
    if (!out->neighbours) d.neighbours = nullptr;
    if (!out->strain) d.strain = nullptr;
    if (!out->knn) d.knn = nullptr;
    if (!out->vm_strain) d.vm_strain = nullptr;
    if (!out->strain_residual) d.strain_residual = nullptr;
    if (!out->nn_distance) d.nn_distance = nullptr;
    if (!out->quat_fz) d.quat_fz = nullptr;
    if (!out->best_type) d.best_type = nullptr;
    PTM_HIP(ctx, hipMemcpyAsync(dpos, positions, 24 * (size_t)n, hipMemcpyHostToDevice, st));
    if (species) PTM_HIP(ctx, hipMemcpyAsync(dspc, species, (size_t)n, hipMemcpyHostToDevice, st));
    J.pos = dpos;
    J.species = species ? dspc : nullptr;
    J.out = d;
    H.active = true;
    H.host_out = *out;
    return PTM_OK;
}

ptm_status stage_in(ptm_ctx *ctx, const double *positions, const int8_t *species, const ptm_outputs *out, int64_t n,
                    FrameJob &J, HostStage &H) {
    return stage_in_buffers(ctx, ctx->staging, positions, species, out, n, J, H, ctx->stream);
}

ptm_status stage_out(ptm_ctx *ctx, const ptm_outputs *out, int64_t n, const FrameJob &J, const HostStage &H,
                     hipStream_t st) {
    (void)out;
    if (!H.active) return PTM_OK;
    const ptm_outputs &h = H.host_out, &d = J.out;
    auto cp = [&](void *dst, const void *src, size_t bytes) -> ptm_status {
        if (dst && src) PTM_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        return PTM_OK;
    };
    ptm_status s;
    if ((s = cp(h.type, d.type, (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.alloy, d.alloy, (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.rmsd, d.rmsd, 8 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.scale, d.scale, 8 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.quat, d.quat, 32 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.neighbours, d.neighbours, 56 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.strain, d.strain, 72 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.knn, d.knn, 56 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.vm_strain, d.vm_strain, 8 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.strain_residual, d.strain_residual, 8 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.nn_distance, d.nn_distance, 8 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.quat_fz, d.quat_fz, 32 * (size_t)n)) != PTM_OK) return s;
    if ((s = cp(h.best_type, d.best_type, (size_t)n)) != PTM_OK) return s;
    return PTM_OK;
}

static ptm_status serve_init(ptm_ctx *ctx) {
    if (ctx->bounds_stream) return PTM_OK;
    // (persistent serving runs no per-frame work on streams)
    for (int s = 0; s < ((ctx->flags & PTM_F_PERSISTENT) ? 0 : SERVE_STREAMS); s++) {
        hipStream_t h;
        PTM_HIP(ctx, hipStreamCreateWithFlags(&h, hipStreamNonBlocking));
        ctx->serve_streams.push_back(h);
    }
    PTM_HIP(ctx, hipStreamCreateWithFlags(&ctx->bounds_stream, hipStreamNonBlocking));
    PTM_HIP(ctx, hipMalloc(&ctx->bounds_part, 8 * 7 * (size_t)bounds_blocks(PTM_MAX_ATOMS)));
    // reference point of the device timeline on the host clock
    PTM_HIP(ctx, hipEventCreateWithFlags(&ctx->order_event, hipEventDisableTiming));
    PTM_HIP(ctx, hipEventCreate(&ctx->ref_event));
    PTM_HIP(ctx, hipEventRecord(ctx->ref_event, ctx->bounds_stream));
    PTM_HIP(ctx, hipEventSynchronize(ctx->ref_event));
    ctx->ref_time_us = now_us();
    return PTM_OK;
}

// Size class of a frame's scratch: the next power of two (at least 1 MiB)
// of an upper bound of its bytes that holds for any cell grid make_grid
// may choose (at most 4n + 4096 cells).
static size_t scratch_class(int64_t n, bool topo) {
    int64_t cells = 4 * n + 4096;
    size_t need = frame_bytes(n, cells, bounds_blocks(n), topo);
    size_t c = (size_t)1 << 20;
    while (c < need) c <<= 1;
    return c;
}

// Take a pooled scratch of class c (allocating one if none is free and the
// budget allows).  Returns PTM_E_BUSY / PTM_E_NOMEM when it does not fit.
static ptm_status take_scratch(ptm_ctx *ctx, size_t c, FrameScratch &out) {
    for (size_t i = 0; i < ctx->free_scratch.size(); i++)
        if (ctx->free_scratch[i].bytes == c) {
            out = ctx->free_scratch[i];
            ctx->free_scratch.erase(ctx->free_scratch.begin() + i);
            return PTM_OK;
        }
    if (ctx->budget) {
        if (c > ctx->budget) {
            ctx->err = "frame larger than the HBM budget";
            return PTM_E_NOMEM;
        }
        // idle buffers of other classes give their memory back first
        while (ctx->pool_bytes + c > ctx->budget && !ctx->free_scratch.empty()) {
            ctx->pool_bytes -= ctx->free_scratch.back().bytes;
            ctx->free_scratch.back().release();
            ctx->free_scratch.pop_back();
        }
        if (ctx->pool_bytes + c > ctx->budget) {
            ctx->err = "HBM budget full";
            return PTM_E_BUSY;
        }
    }
    if (hipMalloc(&out.base, c) != hipSuccess) {
        (void)hipGetLastError();
        out.base = nullptr;
        ctx->err = "device allocation of " + std::to_string(c) + " bytes failed";
        return PTM_E_NOMEM;
    }
    out.bytes = c;
    out.pooled = true;
    ctx->pool_bytes += c;
    return PTM_OK;
}

static void retire(ptm_ctx *ctx, Ticket *T) {
    ctx->inflight_bytes -= T->footprint;
    if (T->slot >= 0) ctx->sv_free.push_back(T->slot);
    T->slot = -1;
    if (T->done) (void)hipEventDestroy(T->done);
    T->done = nullptr;
    if (T->scratch.base) ctx->free_scratch.push_back(T->scratch);
    T->scratch = FrameScratch();
    T->staging.release();
}

// ------------------------------------------------ persistent serving
// (PTM_F_PERSISTENT; the kernel is k_serve in ptm_kernels.hip).  The host
// side: a pinned block shared with the kernel (requests in, completions
// out), a free list of slots, and the kernel's launch state.
static constexpr double SERVE_IDLE_MS = 20.0;

static ptm_status persistent_init(ptm_ctx *ctx) {
    if (ctx->sv_dev) return PTM_OK;
    PTM_HIP(ctx, hipMalloc(&ctx->sv_dev, sizeof(ServeDev)));
    PTM_HIP(ctx, hipMemset(ctx->sv_dev, 0, sizeof(ServeDev)));
    PTM_HIP(ctx, hipHostMalloc((void **)&ctx->sv_host, sizeof(ServeHost), hipHostMallocCoherent));
    std::memset((void *)ctx->sv_host, 0, sizeof(ServeHost));
    PTM_HIP(ctx, hipHostMalloc((void **)&ctx->sv_clock, sizeof(long long), hipHostMallocCoherent));
    // The kernel's stream gets a hardware queue of its own: a stream with a
    // CU mask (here every CU) is not multiplexed with other streams, so work
    // the application queues on its streams never waits behind the
    // long-running kernel.
    int cus = 0;
    PTM_HIP(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    std::vector<uint32_t> cu_mask((size_t)(cus + 31) / 32, 0u);
    for (int c = 0; c < cus; c++) cu_mask[(size_t)c / 32] |= 1u << (c % 32);
    if (hipExtStreamCreateWithCUMask(&ctx->sv_stream, (uint32_t)cu_mask.size(), cu_mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        PTM_HIP(ctx, hipStreamCreateWithFlags(&ctx->sv_stream, hipStreamNonBlocking));
    }
    PTM_HIP(ctx, hipEventCreateWithFlags(&ctx->sv_exit, hipEventDisableTiming));
    int khz = 0;
    PTM_HIP(ctx, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
    ctx->sv_clock_khz = khz > 0 ? (double)khz : 1e5;
    // the device wall clock against the host clock: a kernel that reads it,
    // bracketed by host times (the tightest of three)
    double best = 1e300;
    for (int k = 0; k < 3; k++) {
        *ctx->sv_clock = 0;
        const double t0 = now_us();
        launch_wall_clock(ctx->sv_clock, ctx->sv_stream);
        PTM_HIP(ctx, hipStreamSynchronize(ctx->sv_stream));
        const double t1 = now_us();
        if (t1 - t0 < best) {
            best = t1 - t0;
            ctx->sv_ref_host_us = 0.5 * (t0 + t1);
            ctx->sv_ref_dev = *ctx->sv_clock;
        }
    }
    ctx->sv_free.clear();
    for (int k = SERVE_SLOTS - 1; k >= 0; k--) ctx->sv_free.push_back(k);
    return PTM_OK;
}

// (re)launch the persistent kernel unless it is running
static ptm_status persistent_run(ptm_ctx *ctx) {
    if (ctx->sv_launched) {
        const hipError_t q = hipEventQuery(ctx->sv_exit);
        if (q == hipErrorNotReady) return PTM_OK;
        if (q != hipSuccess) {
            ctx->err = std::string("persistent serving kernel failed: ") + hipGetErrorString(q);
            return PTM_E_DEVICE;
        }
    }
    const long long idle = (long long)(SERVE_IDLE_MS * ctx->sv_clock_khz);
    if (launch_serve(ctx->precision == PTM_FP32_MIXED, ctx->view, ctx->sv_dev, ctx->sv_host, idle,
                     ctx->sv_stream) <= 0) {
        ctx->err = "launch of the persistent serving kernel failed";
        return PTM_E_DEVICE;
    }
    PTM_HIP(ctx, hipEventRecord(ctx->sv_exit, ctx->sv_stream));
    ctx->sv_launched = true;
    return PTM_OK;
}

static bool persistent_done(const ptm_ctx *ctx, const Ticket *T) {
    return __atomic_load_n(&ctx->sv_host->done[T->slot], __ATOMIC_ACQUIRE) == T->gen;
}

// hand the frame of ticket T over to the kernel
static ptm_status persistent_submit(ptm_ctx *ctx, const double *positions, const int8_t *species,
                                    const double *box, const ptm_outputs *out, Ticket *T) {
    ptm_status st;
    if ((st = persistent_init(ctx)) != PTM_OK) return st;
    if (ctx->sv_free.empty()) {
        ctx->err = "every serving slot is in flight";
        return PTM_E_BUSY;
    }
    const int64_t n = T->job.n;
    // the frame's inputs may be written by work queued on the context stream
    PTM_HIP(ctx, hipEventRecord(ctx->order_event, ctx->stream));
    PTM_HIP(ctx, hipEventSynchronize(ctx->order_event));
    st = stage_in_buffers(ctx, T->staging, positions, species, out, n, T->job, T->stage, ctx->bounds_stream);
    if (st == PTM_OK && T->stage.active) PTM_HIP(ctx, hipStreamSynchronize(ctx->bounds_stream));
    if (st != PTM_OK) return st;
    // scratch for the largest grid the kernel can choose
    T->footprint = scratch_class(n, false);
    st = take_scratch(ctx, T->footprint, T->scratch);
    if (st == PTM_OK && !T->scratch.reserve(n, 4 * n + 4096, false, ctx->err)) st = PTM_E_DEVICE;
    if (st != PTM_OK) {
        if (T->scratch.base) ctx->free_scratch.push_back(T->scratch);
        T->scratch = FrameScratch();
        T->staging.release();
        return st;
    }
    ctx->inflight_bytes += T->footprint;
    T->slot = ctx->sv_free.back();
    ctx->sv_free.pop_back();
    // generations count from 1 and stay below 2^36 (the claim counters'
    // field); a wrap would take 6.9e10 frames
    ctx->sv_gen = (ctx->sv_gen % ((1ull << 36) - 1)) + 1;
    T->gen = ctx->sv_gen;
    const uint32_t m = T->job.mask;
    const ptm_outputs &o = T->job.out;
    const FrameScratch &S = T->scratch;
    ServeRequest R;
    std::memset(&R, 0, sizeof(R));
    R.n = n;
    for (int a = 0; a < 3; a++) R.box[a] = box[a];
    R.cutoff = T->job.cutoff;
    R.mask = m;
    R.need = ((m & 0x1u) ? 1u : 0u) | ((m & 0xEu) ? 2u : 0u) | ((m & 0x10u) ? 4u : 0u);
    R.pos = T->job.pos;
    R.species = T->job.species;
    R.O = MatchOut{o.type, o.alloy, o.rmsd, o.scale, o.quat, o.neighbours, o.strain, o.vm_strain, o.strain_residual,
                   o.nn_distance, o.quat_fz, o.best_type};
    R.knn_out = o.knn;
    R.cell_of = S.cell_of;
    R.slot_of = S.slot_of;
    R.sid = S.sid;
    R.count = S.count;
    R.start = S.start;
    R.spos = S.spos;
    R.nbr_id = S.nbr_id;
    R.nbr_rel = S.nbr_rel;
    R.code = S.code;
    R.ord = S.ord;
    R.part = S.sv_part;
    R.bsum = S.sv_bsum;
    R.gen = T->gen;
    // request, then its ring entry, then the tail (the kernel reads them in
    // the opposite order with acquire loads)
    ServeHost *H = ctx->sv_host;
    std::memcpy((void *)&H->req[T->slot], &R, sizeof(R));
    const unsigned long long tail = __atomic_load_n(&H->tail, __ATOMIC_RELAXED);
    __atomic_store_n(&H->ring[tail % SERVE_SLOTS], T->slot, __ATOMIC_RELEASE);
    __atomic_store_n(&H->tail, tail + 1, __ATOMIC_RELEASE);
    T->t_start = now_us();
    return persistent_run(ctx);
}

// wait for a persistent ticket's completion (timeout_us < 0: forever)
static ptm_status persistent_wait(ptm_ctx *ctx, Ticket *T, int64_t timeout_us) {
    const double t0 = now_us();
    while (!persistent_done(ctx, T)) {
        if (timeout_us >= 0 && now_us() - t0 >= (double)timeout_us) return PTM_E_TIMEOUT;
        ptm_status rs = persistent_run(ctx);  // relaunch if the kernel has exited
        if (rs != PTM_OK) return rs;
    }
    const ServeHost *H = ctx->sv_host;
    const int status = __atomic_load_n(&H->status[T->slot], __ATOMIC_RELAXED);
    const long long td = __atomic_load_n(&H->t_done[T->slot], __ATOMIC_RELAXED);
    T->t_complete = ctx->sv_ref_host_us + (double)(td - ctx->sv_ref_dev) * 1e3 / ctx->sv_clock_khz;
    T->complete = true;
    T->box_fail = status == SERVE_BOX;
    T->nonfinite = status == SERVE_NONFINITE;
    if (status == SERVE_OK && T->stage.active) {
        ptm_status so = stage_out(ctx, &T->stage.host_out, T->job.n, T->job, T->stage, ctx->bounds_stream);
        if (so != PTM_OK) return so;
        PTM_HIP(ctx, hipStreamSynchronize(ctx->bounds_stream));
        T->t_complete = now_us();  // the outputs are in host memory only now
    }
    return PTM_OK;
}

static void persistent_shutdown(ptm_ctx *ctx) {
    if (!ctx->sv_dev) return;
    if (ctx->sv_host) __atomic_store_n(&ctx->sv_host->stop, 1, __ATOMIC_RELEASE);
    if (ctx->sv_stream) (void)hipStreamSynchronize(ctx->sv_stream);
    (void)hipFree(ctx->sv_dev);
    ctx->sv_dev = nullptr;
    if (ctx->sv_host) (void)hipHostFree((void *)ctx->sv_host);
    ctx->sv_host = nullptr;
    if (ctx->sv_clock) (void)hipHostFree(ctx->sv_clock);
    ctx->sv_clock = nullptr;
    if (ctx->sv_exit) (void)hipEventDestroy(ctx->sv_exit);
    ctx->sv_exit = nullptr;
    if (ctx->sv_stream) (void)hipStreamDestroy(ctx->sv_stream);
    ctx->sv_stream = nullptr;
    ctx->sv_launched = false;
}

void serve_shutdown(ptm_ctx *ctx) {
    for (auto &kv : ctx->tickets) {
        Ticket *T = kv.second;
        if (T->done) (void)hipEventSynchronize(T->done);
        // a persistent frame still in flight: its scratch is in use until
        // it completes (bounded wait: 60 s)
        if (T->slot >= 0 && !T->complete) (void)persistent_wait(ctx, T, 60000000);
        retire(ctx, T);
        delete T;
    }
    persistent_shutdown(ctx);
    ctx->tickets.clear();
    for (auto &s : ctx->free_scratch) s.release();
    ctx->free_scratch.clear();
    ctx->pool_bytes = 0;
    if (ctx->bounds_part) (void)hipFree(ctx->bounds_part);
    ctx->bounds_part = nullptr;
    if (ctx->ref_event) (void)hipEventDestroy(ctx->ref_event);
    ctx->ref_event = nullptr;
    if (ctx->order_event) (void)hipEventDestroy(ctx->order_event);
    ctx->order_event = nullptr;
    for (auto s : ctx->serve_streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    ctx->serve_streams.clear();
    if (ctx->bounds_stream) (void)hipStreamDestroy(ctx->bounds_stream);
    ctx->bounds_stream = nullptr;
}

}  // namespace ptm

extern "C" {

ptm_status ptm_submit(ptm_ctx *ctx, const double *positions, const int8_t *species, const double *box,
                      int64_t n_atoms, uint32_t template_mask, double rmsd_cutoff, const ptm_outputs *out,
                      uint64_t *ticket) {
    ptm_status st = validate(ctx, positions, box, n_atoms, rmsd_cutoff, out);
    if (st != PTM_OK) return st;
    if (!ticket) {
        ctx->err = "ticket must not be NULL";
        return PTM_E_INVALID;
    }
    ctx->err.clear();
    PTM_HIP(ctx, hipSetDevice(ctx->device));
    if ((st = serve_init(ctx)) != PTM_OK) return st;
    double t_submit = now_us();
    Ticket *T = new Ticket();
    T->t_submit = t_submit;
    T->job.n = n_atoms;
    T->job.mask = template_mask & PTM_ALL;
    T->job.cutoff = rmsd_cutoff;
    T->job.topo = (ctx->flags & PTM_F_TOPOLOGICAL) != 0;
    if (n_atoms > 0 && (ctx->flags & PTM_F_PERSISTENT)) {
        st = persistent_submit(ctx, positions, species, box, out, T);
        if (st != PTM_OK) {
            if (T->slot >= 0) {
                // handed over already (only the launch failed): it stays a ticket
                uint64_t id = ctx->next_ticket++;
                ctx->tickets[id] = T;
                *ticket = id;
            } else {
                delete T;
            }
            return st;
        }
    } else if (n_atoms > 0) {
        hipStream_t bst = ctx->bounds_stream;
        // the frame starts after the work already queued on the context's
        // stream (which may have written its inputs)
        PTM_HIP(ctx, hipEventRecord(ctx->order_event, ctx->stream));
        PTM_HIP(ctx, hipStreamWaitEvent(bst, ctx->order_event, 0));
        // bounds first (synchronous on the bounds stream): the grid depends on them
        st = stage_in_buffers(ctx, T->staging, positions, species, out, n_atoms, T->job, T->stage, bst);
        double mn[3], mx[3];
        bool bad = false;
        FrameScratch bs;
        bs.part = ctx->bounds_part;
        if (st == PTM_OK) st = frame_bounds(ctx, bs, T->job.pos, n_atoms, mn, mx, bad, bst);
        if (st == PTM_OK && bad) {
            ctx->err = "non-finite coordinate";
            st = PTM_E_INVALID;
        }
        int64_t cells = 1;
        if (st == PTM_OK) {
            T->job.grid = make_grid(box, mn, mx, n_atoms, T->job.topo ? VK : KMAX);
            cells = (int64_t)T->job.grid.nc[0] * T->job.grid.nc[1] * T->job.grid.nc[2];
            T->footprint = scratch_class(n_atoms, T->job.topo);
            st = take_scratch(ctx, T->footprint, T->scratch);
            if (st == PTM_OK && !T->scratch.reserve(n_atoms, cells, T->job.topo, ctx->err)) st = PTM_E_DEVICE;
        }
        if (st != PTM_OK) {
            if (T->scratch.base) ctx->free_scratch.push_back(T->scratch);
            T->staging.release();
            delete T;
            return st;
        }
        ctx->inflight_bytes += T->footprint;
        T->stream = ctx->next_stream;
        ctx->next_stream = (ctx->next_stream + 1) % (int)ctx->serve_streams.size();
        hipStream_t s = ctx->serve_streams[T->stream];
        T->t_start = now_us();
        st = enqueue_frame(ctx, T->scratch, T->job, s);
        // (host outputs are copied back by ptm_wait once the box flag is
        // known to be clear: nothing is written for a rejected frame)
        if (st == PTM_OK && hipEventCreate(&T->done) != hipSuccess) st = PTM_E_DEVICE;
        if (st == PTM_OK && hipEventRecord(T->done, s) != hipSuccess) st = PTM_E_DEVICE;
        if (st != PTM_OK) {
            (void)hipStreamSynchronize(s);
            retire(ctx, T);
            delete T;
            return st;
        }
    } else {
        T->t_start = T->t_complete = now_us();
        T->complete = true;
    }
    uint64_t id = ctx->next_ticket++;
    ctx->tickets[id] = T;
    *ticket = id;
    return PTM_OK;
}

ptm_status ptm_wait(ptm_ctx *ctx, uint64_t ticket, int64_t timeout_us, ptm_frame_stats *stats) {
    if (!ctx) return PTM_E_INVALID;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) {
        ctx->err = "unknown ticket";
        return PTM_E_INVALID;
    }
    Ticket *T = it->second;
    if (!T->complete && T->slot >= 0) {
        PTM_HIP(ctx, hipSetDevice(ctx->device));
        ptm_status ws = persistent_wait(ctx, T, timeout_us);
        if (ws != PTM_OK) return ws;
    } else if (!T->complete) {
        PTM_HIP(ctx, hipSetDevice(ctx->device));
        double t0 = now_us();
        for (;;) {
            hipError_t q = hipEventQuery(T->done);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) {
                ctx->err = std::string("frame failed: ") + hipGetErrorString(q);
                return PTM_E_DEVICE;
            }
            if (timeout_us >= 0 && now_us() - t0 >= (double)timeout_us) return PTM_E_TIMEOUT;
        }
        // completion on the device timeline, mapped to the host clock
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->ref_event, T->done) == hipSuccess)
            T->t_complete = ctx->ref_time_us + 1e3 * (double)ms;
        else
            T->t_complete = now_us();
        T->complete = true;
        // the frame's box flag (its kernels are done; read on the side stream)
        *ctx->pinned = 0;
        PTM_HIP(ctx, hipMemcpyAsync(ctx->pinned, box_flag(T->scratch, T->job.grid), 4, hipMemcpyDeviceToHost,
                                    ctx->bounds_stream));
        PTM_HIP(ctx, hipStreamSynchronize(ctx->bounds_stream));
        T->box_fail = *ctx->pinned != 0;
        if (!T->box_fail && T->stage.active) {
            hipStream_t s = ctx->serve_streams[T->stream];
            ptm_status so = stage_out(ctx, &T->stage.host_out, T->job.n, T->job, T->stage, s);
            if (so == PTM_OK) PTM_HIP(ctx, hipStreamSynchronize(s));
            if (so != PTM_OK) return so;
            T->t_complete = now_us();  // the outputs are in host memory only now
        }
    }
    const bool box_fail = T->box_fail, nonfinite = T->nonfinite;
    const bool topo = T->job.topo;
    if (stats) {
        stats->submit_time_us = T->t_submit;
        stats->start_time_us = T->t_start;
        stats->complete_time_us = T->t_complete;
        stats->n_atoms = T->job.n;
        stats->scratch_bytes = T->footprint;
    }
    retire(ctx, T);
    delete T;
    ctx->tickets.erase(it);
    if (box_fail) {
        ctx->err = box_message(topo);
        return PTM_E_BOX;
    }
    if (nonfinite) {
        ctx->err = "non-finite coordinate";
        return PTM_E_INVALID;
    }
    return PTM_OK;
}

}  // extern "C"
