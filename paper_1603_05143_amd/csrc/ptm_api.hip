// ptm_api.hip -- C ABI of the PTM library (declared in include/ptm.h).
//
// A context owns the device copy of the template tables, one stream and the
// scratch of the synchronous path; ptm_classify validates the arguments,
// sizes the cell grid from the frame's density, runs the kernel pipeline
// and synchronises.  ptm_submit / ptm_wait run frames on a pool of streams
// with per-frame scratch, admitted against the HBM budget (see
// ptm_serve.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/ptm.h"
#include "ptm_internal.hpp"
#include "ptm_kernels.hpp"
#include "ptm_tables.hpp"

using namespace ptm;

namespace ptm {

// ------------------------------------------------------------ scratch
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t frame_bytes(int64_t n, int64_t cells, int nbounds, bool topo) {
    size_t b = 0;
    b += align_up(4 * (size_t)n) * 3;         // cell_of, slot_of, sid
    // count (+ the frame's counters and the box flag), start
    b += align_up(4 * (size_t)(cells + FRAME_COUNTERS)) * 2;
    b += align_up(24 * (size_t)n);           // sorted positions
    b += align_up(4 * (size_t)n * KMAX);      // neighbour ids
    b += align_up(8 * (size_t)n * KMAX * 3);  // neighbour vectors
    b += align_up(4 * (size_t)n * NGRP);      // code ids
    b += align_up(8 * (size_t)n * NGRP);      // labellings
    b += align_up(8 * 7 * (size_t)nbounds);   // bounds partials
    b += align_up(8 * 7 * (size_t)serve_bounds_items(n));  // persistent serving: per-item bounds
    b += align_up(4 * (size_t)(serve_scan_items(n) + 1));  // per-item totals of the cell-start scan
    if (topo) {
        b += align_up(4 * (size_t)n * VK);      // the 18 Euclidean neighbours' ids
        b += align_up(8 * (size_t)n * VK * 3);  // and vectors
        b += align_up(4 * (size_t)n * (2 * VK - 4));  // facets of their Voronoi hull
        b += align_up(4 * (size_t)n);                 // and its facet masks
    }
    return b;
}

bool FrameScratch::reserve(int64_t n, int64_t cells, bool topo, std::string &err) {
    int nb = bounds_blocks(n);
    if (scan_items(cells) > serve_scan_items(n)) {  // make_grid keeps cells <= 4n + 4096
        err = "cell grid larger than the scratch layout allows";
        return false;
    }
    size_t need = frame_bytes(n, cells, nb, topo);
    if (need > bytes) {
        if (pooled) {
            // a pooled buffer is sized for its class and never reallocated
            err = "pooled scratch of " + std::to_string(bytes) + " bytes is too small for " + std::to_string(need);
            return false;
        }
        if (base) (void)hipFree(base);
        base = nullptr;
        bytes = 0;
        if (hipMalloc(&base, need) != hipSuccess) {
            (void)hipGetLastError();
            err = "device allocation of " + std::to_string(need) + " bytes failed";
            return false;
        }
        bytes = need;
    }
    char *p = (char *)base;
    auto take = [&](size_t sz) {
        char *r = p;
        p += align_up(sz);
        return (void *)r;
    };
    cell_of = (int32_t *)take(4 * (size_t)n);
    slot_of = (int32_t *)take(4 * (size_t)n);
    sid = (int32_t *)take(4 * (size_t)n);
    count = (int32_t *)take(4 * (size_t)(cells + FRAME_COUNTERS));
    start = (int32_t *)take(4 * (size_t)(cells + FRAME_COUNTERS));
    spos = (double *)take(24 * (size_t)n);
    nbr_id = (int32_t *)take(4 * (size_t)n * KMAX);
    nbr_rel = (double *)take(8 * (size_t)n * KMAX * 3);
    code = (int32_t *)take(4 * (size_t)n * NGRP);
    ord = (uint64_t *)take(8 * (size_t)n * NGRP);
    part = (double *)take(8 * 7 * (size_t)nb);
    sv_part = (double *)take(8 * 7 * (size_t)serve_bounds_items(n));
    sv_bsum = (int32_t *)take(4 * (size_t)(serve_scan_items(n) + 1));
    id18 = topo ? (int32_t *)take(4 * (size_t)n * VK) : nullptr;
    rel18 = topo ? (double *)take(8 * (size_t)n * VK * 3) : nullptr;
    vf = topo ? (uint32_t *)take(4 * (size_t)n * (2 * VK - 4)) : nullptr;
    vlive = topo ? (uint32_t *)take(4 * (size_t)n) : nullptr;
    return true;
}

void FrameScratch::release() {
    if (base) (void)hipFree(base);
    base = nullptr;
    bytes = 0;
}

int bounds_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

// Choose the cell grid: cell edge 0.6 x the expected distance of the kn-th
// neighbour (kn = 14, or 18 for the topological ordering), so that shells
// 0..2 of cells around an atom (5x5x5 block) usually certify its kn nearest
// neighbours; at least 3 cells on periodic axes.  The grid affects only
// speed: the search is certified exact.
Grid make_grid(const double box[3], const double mn[3], const double mx[3], int64_t n, int kn) {
    Grid g;
    double ext[3], vol = 1.0;
    int flat = 0;
    for (int a = 0; a < 3; a++) {
        g.periodic[a] = box[a] > 0;
        ext[a] = g.periodic[a] ? box[a] : std::fmax(mx[a] - mn[a], 0.0);
        if (ext[a] > 0) vol *= ext[a];
        else flat++;
    }
    double h;
    if (flat == 0 && vol > 0) {
        double rho = (double)n / vol;
        h = 0.6 * std::cbrt((double)kn / (4.1887902047863905 * rho));
    } else {
        h = 1.0;
        for (int a = 0; a < 3; a++) h = std::fmax(h, ext[a] / 16.0);
    }
    for (int iter = 0; iter < 200; iter++) {
        double cells = 1;
        for (int a = 0; a < 3; a++) {
            int nc;
            if (g.periodic[a]) nc = (int)std::fmin(std::floor(ext[a] / h), 1 << 20);
            else nc = ext[a] > 0 ? (int)std::fmin(std::floor(ext[a] / h), 1 << 20) : 1;
            if (g.periodic[a] && nc < 3) nc = 3;
            if (nc < 1) nc = 1;
            g.nc[a] = nc;
            cells *= nc;
        }
        if (cells <= (double)(1 << 30) && cells <= 4.0 * (double)n + 4096.0) break;
        h *= 1.25;
    }
    double hmax = 0;
    for (int a = 0; a < 3; a++) {
        if (g.periodic[a]) {
            g.L[a] = box[a];
            g.invL[a] = 1.0 / box[a];
            g.lo[a] = 0.0;
            g.h[a] = box[a] / g.nc[a];
            g.inv_h[a] = g.nc[a] / box[a];
        } else {
            g.L[a] = 0.0;
            g.invL[a] = 0.0;
            g.lo[a] = mn[a];
            g.h[a] = ext[a] > 0 ? ext[a] / g.nc[a] : 1.0;
            g.inv_h[a] = ext[a] > 0 ? g.nc[a] / ext[a] : 1.0;
        }
        hmax = std::fmax(hmax, g.h[a]);
    }
    g.margin = 1e-9 * hmax;
    g.canonical = 1;
    for (int a = 0; a < 3; a++)
        if (g.periodic[a] && !(mn[a] >= 0.0 && mx[a] < box[a])) g.canonical = 0;
    return g;
}

// Enqueue the whole pipeline for one frame whose bounds are known.
ptm_status enqueue_frame(ptm_ctx *ctx, FrameScratch &S, const FrameJob &J, hipStream_t st, bool prof) {
    const int64_t n = J.n;
    auto mark = [&](int e) -> ptm_status {
        if (prof) PTM_HIP(ctx, hipEventRecord(ctx->prof_ev[e], st));
        return PTM_OK;
    };
    ptm_status ps;
    const Grid &g = J.grid;
    if ((ps = mark(PTM_STAGE_BIN)) != PTM_OK) return ps;
    int64_t cells = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    // count[cells + 1] and count[cells + 2] count the atoms the fast k-NN
    // search leaves over and those the full rule decides; count[cells + 3]
    // is the box flag (set by the k-NN kernels, read by every later stage);
    // job_counter() the candidates superposed
    launch_zero(S.count, cells + FRAME_COUNTERS, st);
    const int32_t *box_fail = S.count + cells + 3;
    launch_bin_count(J.pos, n, g, S.cell_of, S.slot_of, S.count, st);
    launch_cell_starts(S.count, cells, S.sv_bsum, S.start, st);
    launch_bin_scatter(J.pos, n, S.cell_of, S.slot_of, S.start, S.spos, S.sid, st);
    if ((ps = mark(PTM_STAGE_KNN)) != PTM_OK) return ps;
    // slot_of is free once the atoms are scattered: it holds the leftover list
    if (J.topo) {
        // the 18 Euclidean neighbours, then their topological order (Sec. 3)
        launch_knn(n, g, VK, S.spos, S.sid, S.start, S.id18, S.rel18, S.slot_of, S.count + cells + 1,
                   S.count + cells + 3, st);
        launch_voronoi(n, S.rel18, S.id18, S.vf, S.vlive, S.nbr_rel, S.nbr_id, box_fail, st);
    } else {
        launch_knn(n, g, KMAX, S.spos, S.sid, S.start, S.nbr_id, S.nbr_rel, S.slot_of, S.count + cells + 1,
                   S.count + cells + 3, st);
    }
    if ((ps = mark(PTM_STAGE_TOPO)) != PTM_OK) return ps;
    const uint32_t m = J.mask;
    const uint32_t need = ((m & 0x1u) ? 1u : 0u) | ((m & 0xEu) ? 2u : 0u) | ((m & 0x10u) ? 4u : 0u);
    launch_topo(n, S.nbr_rel, S.nbr_id, ctx->view, need, S.code, S.ord, box_fail, st);
    if ((ps = mark(PTM_STAGE_MATCH)) != PTM_OK) return ps;
    MatchOut O = {J.out.type,       J.out.alloy,     J.out.rmsd,
                  J.out.scale,      J.out.quat,      J.out.neighbours,
                  J.out.strain,     J.out.vm_strain, J.out.strain_residual,
                  J.out.nn_distance, J.out.quat_fz, J.out.best_type};
    const bool f32 = ctx->precision == PTM_FP32_MIXED;
    // the knn output is the Euclidean order (the 18-neighbour list of the
    // topological ordering starts with it)
    launch_match(n, S.nbr_rel, S.nbr_id, S.sid, J.species, ctx->view, S.code, S.ord, m, J.cutoff,
                 (ctx->flags & PTM_F_FULL_RULE) != 0, O, S.count + cells + 2, job_counter(S.count, cells),
                 J.topo ? S.id18 : S.nbr_id, J.out.knn, box_fail, f32, st);
    if ((ps = mark(PTM_NSTAGES)) != PTM_OK) return ps;
    PTM_HIP(ctx, hipGetLastError());
    return PTM_OK;
}

// Bounds of the frame: finite check and per-axis extent (synchronous on st).
ptm_status frame_bounds(ptm_ctx *ctx, FrameScratch &S, const double *pos, int64_t n, double mn[3], double mx[3],
                        bool &bad, hipStream_t st) {
    int nb = bounds_blocks(n);
    launch_bounds(pos, n, S.part, nb, st);
    PTM_HIP(ctx, hipGetLastError());
    double *h = ctx->pinned_bounds;  // pinned host space for 7 x 1024 partials
    PTM_HIP(ctx, hipMemcpyAsync(h, S.part, (size_t)nb * 7 * 8, hipMemcpyDeviceToHost, st));
    PTM_HIP(ctx, hipStreamSynchronize(st));
    bad = false;
    for (int a = 0; a < 3; a++) {
        mn[a] = 1e308;
        mx[a] = -1e308;
    }
    for (int b = 0; b < nb; b++) {
        for (int a = 0; a < 3; a++) {
            mn[a] = std::fmin(mn[a], h[7 * b + a]);
            mx[a] = std::fmax(mx[a], h[7 * b + 3 + a]);
        }
        if (h[7 * b + 6] != 0.0) bad = true;
    }
    return PTM_OK;
}

const char *box_message(bool topo) {
    return topo ? "a periodic box length is not more than twice some atom's 18th-neighbour distance"
                : "a periodic box length is not more than twice some atom's 14th-neighbour distance";
}

ptm_status validate(ptm_ctx *ctx, const double *positions, const double *box, int64_t n, double cutoff,
                    const ptm_outputs *out) {
    if (!ctx) return PTM_E_INVALID;
    if (!box || !out || (n > 0 && !out->type)) {
        ctx->err = "box, out and (for n > 0) out->type must not be NULL";
        return PTM_E_INVALID;
    }
    if (n < 0) {
        ctx->err = "n_atoms < 0";
        return PTM_E_INVALID;
    }
    if (n > PTM_MAX_ATOMS) {
        ctx->err = "n_atoms exceeds PTM_MAX_ATOMS";
        return PTM_E_TOO_LARGE;
    }
    if (n > 0 && !positions) {
        ctx->err = "positions must not be NULL";
        return PTM_E_INVALID;
    }
    for (int a = 0; a < 3; a++)
        if (!(box[a] >= 0.0) || std::isinf(box[a])) {
            ctx->err = "box lengths must be finite and >= 0";
            return PTM_E_INVALID;
        }
    if (std::isnan(cutoff)) {
        ctx->err = "rmsd_cutoff is NaN";
        return PTM_E_INVALID;
    }
    // the match kernel writes these records as 16- and 8-byte pairs
    if (!(ctx->flags & PTM_F_HOST_POINTERS) &&
        (((uintptr_t)out->quat & 15) || ((uintptr_t)out->quat_fz & 15) || ((uintptr_t)out->neighbours & 7))) {
        ctx->err = "device outputs: quat and quat_fz must be 16-byte aligned, neighbours 8-byte aligned";
        return PTM_E_INVALID;
    }
    return PTM_OK;
}

// ------------------------------------------------------ static scratch
// Device scratch of ptm_classify_noalloc: a file-scope array in every
// device's memory for the life of the process, sized for PTM_NOALLOC_MAX_ATOMS
// atoms with either neighbour ordering.  Host code reaches it only through
// the address hipGetSymbolAddress returns for the current device (the
// array's name on the host is not a device address).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)104 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// this device's address of the array, looked up once per device (the device
// must be current)
hipError_t noalloc_scratch_of(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[256] = {};
    if (device < 0 || device >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

// One frame through the pipeline with the scratch S (the context's own,
// grown on demand, or a fixed buffer when noalloc: then nothing is
// allocated and a frame that does not fit is PTM_E_TOO_LARGE).
ptm_status classify_frame(ptm_ctx *ctx, FrameScratch &S, bool noalloc, const double *positions,
                          const int8_t *species, const double *box, int64_t n_atoms, uint32_t template_mask,
                          double rmsd_cutoff, const ptm_outputs *out) {
    ctx->err.clear();
    if (n_atoms == 0) return PTM_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->err = "hipSetDevice failed";
        return PTM_E_DEVICE;
    }
    FrameJob J;
    J.n = n_atoms;
    J.mask = template_mask & PTM_ALL;
    J.cutoff = rmsd_cutoff;
    J.topo = (ctx->flags & PTM_F_TOPOLOGICAL) != 0;
    HostStage H;
    ptm_status st = stage_in(ctx, positions, species, out, n_atoms, J, H);
    if (st != PTM_OK) return st;
    auto reserve = [&](int64_t cells) -> ptm_status {
        if (S.reserve(n_atoms, cells, J.topo, ctx->err)) return PTM_OK;
        return noalloc ? PTM_E_TOO_LARGE : PTM_E_NOMEM;
    };
    // bounds first (needs scratch for the partials): reserve with a tiny grid
    if ((st = reserve(1)) != PTM_OK) return st;
    double mn[3], mx[3];
    bool bad = false;
    const bool prof = (ctx->flags & PTM_F_PROFILE) != 0;
    ctx->prof_valid = false;
    if (prof) PTM_HIP(ctx, hipEventRecord(ctx->prof_ev[PTM_STAGE_BOUNDS], ctx->stream));
    st = frame_bounds(ctx, S, J.pos, n_atoms, mn, mx, bad, ctx->stream);
    if (st != PTM_OK) return st;
    if (bad) {
        ctx->err = "non-finite coordinate";
        return PTM_E_INVALID;
    }
    J.grid = make_grid(box, mn, mx, n_atoms, J.topo ? VK : KMAX);
    int64_t cells = (int64_t)J.grid.nc[0] * J.grid.nc[1] * J.grid.nc[2];
    if (ctx->budget && frame_bytes(n_atoms, cells, bounds_blocks(n_atoms), J.topo) > ctx->budget) {
        ctx->err = "frame scratch exceeds the HBM budget";
        return PTM_E_NOMEM;
    }
    if ((st = reserve(cells)) != PTM_OK) return st;
    st = enqueue_frame(ctx, S, J, ctx->stream, prof);
    if (st != PTM_OK) return st;
    // the box flag comes back with the frame; host outputs are copied only
    // once it is known to be clear (nothing is written on an error)
    *ctx->pinned = 0;
    PTM_HIP(ctx, hipMemcpyAsync(ctx->pinned, box_flag(S, J.grid), 4, hipMemcpyDeviceToHost, ctx->stream));
    if (H.active) {
        PTM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (*ctx->pinned) {
            ctx->err = box_message(J.topo);
            return PTM_E_BOX;
        }
        st = stage_out(ctx, out, n_atoms, J, H, ctx->stream);
        if (st != PTM_OK) return st;
    }
    PTM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (*ctx->pinned) {
        ctx->err = box_message(J.topo);
        return PTM_E_BOX;
    }
    if (prof) {
        int32_t left[2] = {0, 0};
        unsigned long long pairs = 0;
        PTM_HIP(ctx, hipMemcpy(left, S.count + cells + 1, 8, hipMemcpyDeviceToHost));
        PTM_HIP(ctx, hipMemcpy(&pairs, job_counter(S.count, cells), 8, hipMemcpyDeviceToHost));
        ctx->prof_info[PTM_INFO_CELLS] = cells;
        ctx->prof_info[PTM_INFO_KNN_EXACT] = knn_fast_applies(J.grid) ? left[0] : n_atoms;
        ctx->prof_info[PTM_INFO_PAIRS] = (int64_t)pairs;
        ctx->prof_info[PTM_INFO_DECIDE_FULL] = left[1];
    }
    ctx->prof_valid = prof;
    return PTM_OK;
}

}  // namespace ptm

// ============================================================== C ABI
extern "C" {

const char *ptm_status_string(ptm_status s) {
    switch (s) {
        case PTM_OK: return "ok";
        case PTM_E_INVALID: return "invalid argument";
        case PTM_E_NOMEM: return "out of device memory or HBM budget";
        case PTM_E_DEVICE: return "HIP runtime error";
        case PTM_E_BOX: return "box unusable for the neighbour search";
        case PTM_E_TOO_LARGE: return "too many atoms";
        case PTM_E_BUSY: return "serving queue full";
        case PTM_E_TIMEOUT: return "timed out";
    }
    return "unknown status";
}

const char *ptm_last_error(const ptm_ctx *ctx) {
    if (!ctx) return "";
    return ctx->err.c_str();
}

ptm_status ptm_template_info(int t, int64_t info[5]) {
    if (t < 0 || t >= NT || !info) return PTM_E_INVALID;
    static std::once_flag once;
    static HostTables *T = nullptr;
    static bool ok = false;
    std::call_once(once, [] {
        T = new (std::nothrow) HostTables();
        std::string err;
        ok = T && build_tables(*T, err);
    });
    if (!ok) return PTM_E_NOMEM;
    info[0] = T->tpl[t].k;
    info[1] = T->tpl[t].ngroup;
    info[2] = T->ntri[t];
    info[3] = T->ncodes_t[t];
    info[4] = T->ncand_kept[t];
    return PTM_OK;
}

ptm_status ptm_create(const ptm_config *cfg, ptm_ctx **out) {
    if (!cfg || !out) return PTM_E_INVALID;
    *out = nullptr;
    if (cfg->precision != PTM_FP64 && cfg->precision != PTM_FP32_MIXED) return PTM_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
        (void)hipGetLastError();
        return PTM_E_DEVICE;
    }
    ptm_ctx *ctx = new (std::nothrow) ptm_ctx();
    if (!ctx) return PTM_E_NOMEM;
    ctx->device = cfg->device;
    ctx->precision = cfg->precision;
    ctx->budget = cfg->hbm_budget_bytes;
    ctx->flags = cfg->flags;
    if ((ctx->flags & PTM_F_PERSISTENT) && (ctx->flags & PTM_F_TOPOLOGICAL)) {
        delete ctx;
        return PTM_E_INVALID;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        delete ctx;
        return PTM_E_DEVICE;
    }
    if (cfg->hip_stream) {
        ctx->stream = (hipStream_t)cfg->hip_stream;
        ctx->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return PTM_E_DEVICE;
        }
        ctx->own_stream = true;
    }
    // pinned host words: the box flag, then the per-block bounds partials
    if (hipHostMalloc((void **)&ctx->pinned, 256 + 8 * 7 * 1024, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ctx->pinned = nullptr;
        ptm_destroy(ctx);
        return PTM_E_NOMEM;
    }
    ctx->pinned_bounds = (double *)((char *)ctx->pinned + 256);
    if (noalloc_scratch_of(ctx->device, &ctx->noalloc_scratch) != hipSuccess) {
        ptm_destroy(ctx);
        return PTM_E_DEVICE;
    }
    if (ctx->flags & PTM_F_PROFILE)
        for (int e = 0; e <= PTM_NSTAGES; e++)
            if (hipEventCreate(&ctx->prof_ev[e]) != hipSuccess) {
                ptm_destroy(ctx);
                return PTM_E_DEVICE;
            }
    std::string err;
    if (!build_tables(ctx->host, err)) {
        ptm_destroy(ctx);
        return PTM_E_NOMEM;
    }
    ptm_status st = upload_tables(ctx);
    if (st != PTM_OK) {
        ptm_destroy(ctx);
        return st;
    }
    *out = ctx;
    return PTM_OK;
}

void ptm_destroy(ptm_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    serve_shutdown(ctx);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    ctx->main.release();
    ctx->staging.release();
    for (void *p : ctx->table_buffers) (void)hipFree(p);
    if (ctx->aux) (void)hipFree(ctx->aux);
    for (int e = 0; e <= PTM_NSTAGES; e++)
        if (ctx->prof_ev[e]) (void)hipEventDestroy(ctx->prof_ev[e]);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

ptm_status ptm_classify(ptm_ctx *ctx, const double *positions, const int8_t *species, const double *box,
                        int64_t n_atoms, uint32_t template_mask, double rmsd_cutoff, const ptm_outputs *out) {
    ptm_status st = validate(ctx, positions, box, n_atoms, rmsd_cutoff, out);
    if (st != PTM_OK) return st;
    return classify_frame(ctx, ctx->main, false, positions, species, box, n_atoms, template_mask, rmsd_cutoff, out);
}

ptm_status ptm_classify_noalloc(ptm_ctx *ctx, const double *positions, const int8_t *species, const double *box,
                                int64_t n_atoms, uint32_t template_mask, double rmsd_cutoff,
                                const ptm_outputs *out) {
    ptm_status st = validate(ctx, positions, box, n_atoms, rmsd_cutoff, out);
    if (st != PTM_OK) return st;
    if (ctx->flags & PTM_F_HOST_POINTERS) {
        ctx->err = "ptm_classify_noalloc: host-pointer contexts stage through allocated buffers";
        return PTM_E_INVALID;
    }
    if (n_atoms > PTM_NOALLOC_MAX_ATOMS) {
        ctx->err = "ptm_classify_noalloc: n_atoms exceeds PTM_NOALLOC_MAX_ATOMS";
        return PTM_E_TOO_LARGE;
    }
    // the device's static array, carved like a frame scratch (never reallocated)
    FrameScratch S;
    S.base = ctx->noalloc_scratch;
    S.bytes = NOALLOC_SCRATCH_BYTES;
    S.pooled = true;
    return classify_frame(ctx, S, true, positions, species, box, n_atoms, template_mask, rmsd_cutoff, out);
}

ptm_status ptm_stage_times(const ptm_ctx *ctx, double *ms, int n) {
    if (!ctx || !ms || n < 0 || !(ctx->flags & PTM_F_PROFILE)) return PTM_E_INVALID;
    for (int i = 0; i < n && i < PTM_NSTAGES; i++) {
        ms[i] = 0.0;
        if (!ctx->prof_valid) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, ctx->prof_ev[i], ctx->prof_ev[i + 1]) != hipSuccess) {
            (void)hipGetLastError();
            return PTM_E_DEVICE;
        }
        ms[i] = t;
    }
    return PTM_OK;
}

ptm_status ptm_frame_info(const ptm_ctx *ctx, int64_t *info, int n) {
    if (!ctx || !info || n < 0 || !(ctx->flags & PTM_F_PROFILE)) return PTM_E_INVALID;
    for (int i = 0; i < n && i < PTM_NINFO; i++) info[i] = ctx->prof_valid ? ctx->prof_info[i] : 0;
    return PTM_OK;
}

ptm_status ptm_misorientation(ptm_ctx *ctx, const int8_t *type, const double *q1, const double *q2, int64_t n,
                              double *angle) {
    if (!ctx) return PTM_E_INVALID;
    if (n < 0 || (n > 0 && (!type || !q1 || !q2 || !angle))) {
        ctx->err = "ptm_misorientation: NULL array or n < 0";
        return PTM_E_INVALID;
    }
    ctx->err.clear();
    if (n == 0) return PTM_OK;
    PTM_HIP(ctx, hipSetDevice(ctx->device));
    const int8_t *dt = type;
    const double *d1 = q1, *d2 = q2;
    double *da = angle;
    void *buf = nullptr;
    const bool host = (ctx->flags & PTM_F_HOST_POINTERS) != 0;
    if (host) {
        // types first: reject invalid ones before any device work
        for (int64_t i = 0; i < n; i++)
            if (type[i] < 0 || type[i] > 5) {
                ctx->err = "ptm_misorientation: type outside 0..5";
                return PTM_E_INVALID;
            }
        size_t bytes = (size_t)n * (1 + 32 + 32 + 8) + 256;
        if (hipMalloc(&buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            ctx->err = "ptm_misorientation: staging allocation failed";
            return PTM_E_NOMEM;
        }
        char *b = (char *)buf;
        double *h1 = (double *)b, *h2 = h1 + 4 * n, *ha = h2 + 4 * n;
        int8_t *ht = (int8_t *)(ha + n);
        ptm_status st = PTM_OK;
        if (hipMemcpyAsync(h1, q1, 32 * (size_t)n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(h2, q2, 32 * (size_t)n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(ht, type, (size_t)n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
            st = PTM_E_DEVICE;
        if (st == PTM_OK) {
            launch_misorientation(n, ctx->view, ht, h1, h2, ha, ctx->stream);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(angle, ha, 8 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess)
                st = PTM_E_DEVICE;
        }
        (void)hipFree(buf);
        if (st != PTM_OK) ctx->err = "ptm_misorientation: HIP error";
        return st;
    }
    launch_misorientation(n, ctx->view, dt, d1, d2, da, ctx->stream);
    PTM_HIP(ctx, hipGetLastError());
    PTM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PTM_OK;
}

// Copies host arrays to device scratch for the post-hoc entry points of a
// PTM_F_HOST_POINTERS context (one allocation, freed by the caller).
static ptm_status stage_pair(ptm_ctx *ctx, const int8_t *t, const double *r, int64_t n, void **buf, int8_t **dt,
                             double **dr, size_t extra) {
    size_t bytes = 8 * (size_t)n + (size_t)n + extra + 512;
    if (hipMalloc(buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        ctx->err = "staging allocation failed";
        return PTM_E_NOMEM;
    }
    *dr = (double *)*buf;
    *dt = (int8_t *)(*dr + n);
    if (hipMemcpyAsync(*dr, r, 8 * (size_t)n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(*dt, t, (size_t)n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
        ctx->err = "staging copy failed";
        return PTM_E_DEVICE;
    }
    return PTM_OK;
}

ptm_status ptm_apply_cutoff(ptm_ctx *ctx, const int8_t *best_type, const double *rmsd, int64_t n,
                            double rmsd_cutoff, int8_t *type) {
    if (!ctx) return PTM_E_INVALID;
    if (n < 0 || (n > 0 && (!best_type || !rmsd || !type))) {
        ctx->err = "ptm_apply_cutoff: NULL array or n < 0";
        return PTM_E_INVALID;
    }
    ctx->err.clear();
    if (n == 0) return PTM_OK;
    PTM_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->flags & PTM_F_HOST_POINTERS) {
        void *buf = nullptr;
        int8_t *dt;
        double *dr;
        ptm_status st = stage_pair(ctx, best_type, rmsd, n, &buf, &dt, &dr, (size_t)n + 256);
        if (st == PTM_OK) {
            int8_t *dout = (int8_t *)(((uintptr_t)(dt + n) + 255) & ~(uintptr_t)255);
            launch_apply_cutoff(n, dt, dr, rmsd_cutoff, dout, ctx->stream);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(type, dout, (size_t)n, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess) {
                ctx->err = "ptm_apply_cutoff: HIP error";
                st = PTM_E_DEVICE;
            }
        }
        if (buf) (void)hipFree(buf);
        return st;
    }
    launch_apply_cutoff(n, best_type, rmsd, rmsd_cutoff, type, ctx->stream);
    PTM_HIP(ctx, hipGetLastError());
    PTM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PTM_OK;
}

ptm_status ptm_rmsd_histogram(ptm_ctx *ctx, const int8_t *best_type, const double *rmsd, int64_t n, int nbins,
                              double rmax, int64_t *counts) {
    if (!ctx) return PTM_E_INVALID;
    if (n < 0 || (n > 0 && (!best_type || !rmsd)) || !counts || nbins < 1 || nbins > 65536 || !(rmax > 0)) {
        ctx->err = "ptm_rmsd_histogram: invalid argument";
        return PTM_E_INVALID;
    }
    ctx->err.clear();
    std::memset(counts, 0, sizeof(int64_t) * 6 * (size_t)nbins);
    if (n == 0) return PTM_OK;
    PTM_HIP(ctx, hipSetDevice(ctx->device));
    const size_t cbytes = 8 * 6 * (size_t)nbins;
    void *buf = nullptr;
    int8_t *dt = const_cast<int8_t *>(best_type);
    double *dr = const_cast<double *>(rmsd);
    unsigned long long *dc = nullptr;
    ptm_status st = PTM_OK;
    if (ctx->flags & PTM_F_HOST_POINTERS) {
        st = stage_pair(ctx, best_type, rmsd, n, &buf, &dt, &dr, cbytes + 256);
        if (st == PTM_OK) dc = (unsigned long long *)(((uintptr_t)(dt + n) + 255) & ~(uintptr_t)255);
    } else {
        if (ctx->aux_bytes < cbytes) {
            // grow-only: later calls of this size allocate nothing
            if (ctx->aux) (void)hipFree(ctx->aux);
            ctx->aux = nullptr;
            ctx->aux_bytes = 0;
            if (hipMalloc(&ctx->aux, cbytes) != hipSuccess) {
                (void)hipGetLastError();
                ctx->aux = nullptr;
                ctx->err = "ptm_rmsd_histogram: allocation failed";
                st = PTM_E_NOMEM;
            } else {
                ctx->aux_bytes = cbytes;
            }
        }
        dc = (unsigned long long *)ctx->aux;
    }
    if (st == PTM_OK) {
        if (hipMemsetAsync(dc, 0, cbytes, ctx->stream) != hipSuccess) st = PTM_E_DEVICE;
        if (st == PTM_OK) launch_rmsd_histogram(n, dt, dr, nbins, rmax, dc, ctx->stream);
        if (st == PTM_OK && (hipGetLastError() != hipSuccess ||
                             hipMemcpyAsync(counts, dc, cbytes, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
                             hipStreamSynchronize(ctx->stream) != hipSuccess))
            st = PTM_E_DEVICE;
        if (st != PTM_OK && ctx->err.empty()) ctx->err = "ptm_rmsd_histogram: HIP error";
    }
    if (buf) (void)hipFree(buf);
    return st;
}

}  // extern "C"

// ======================================================= self-check entry points
#include "../../include/ptm_selftest.h"
#include "ptm_device.hpp"

extern "C" {

int ptm_selftest_orient(const double *p, const int32_t *r) {
    if (r[0] == r[1] || r[0] == r[2] || r[0] == r[3] || r[1] == r[2] || r[1] == r[3] || r[2] == r[3]) return 0;
    double m = 0;
    for (int i = 0; i < 12; i++) m = fmax(m, fabs(p[i]));
    return orient_sos64b(p, p + 3, p + 6, p + 9, r[0], r[1], r[2], r[3], f64_orient_bound(m));
}

int ptm_selftest_det3(const double *p) {
    double m = 0;
    for (int i = 0; i < 9; i++) m = fmax(m, fabs(p[i]));
    return det3_sign64b(p, p + 3, p + 6, f64_det3_bound(m));
}

int ptm_selftest_codes(int k, const int32_t *tris, int ntri, uint64_t *codes, int max_codes, int32_t *n_codes) {
    if (k < 4 || k > KMAX || ntri != 2 * k - 4) return -1;
    uint64_t nxt[KMAX];
    int deg[KMAX] = {0};
    for (int x = 0; x < k; x++) nxt[x] = ~0ull;
    for (int t = 0; t < ntri; t++)
        for (int e = 0; e < 3; e++) {
            int a = tris[3 * t + e], b = tris[3 * t + (e + 1) % 3], c = tris[3 * t + (e + 2) % 3];
            if (a < 0 || a >= k || b < 0 || b >= k || c < 0 || c >= k) return -1;
            if (((nxt[a] >> (4 * b)) & 0xF) != 0xF) return -1;
            nxt[a] &= ~(0xFull << (4 * b));
            nxt[a] |= (uint64_t)c << (4 * b);
            deg[a]++;
        }
    auto darts = min_degree_darts(k, nxt, deg);
    int m = 0;
    for (auto &d : darts) {
        if (m >= max_codes) break;
        uint64_t ord;
        dart_code(k, nxt, deg, d.first, d.second, codes + (size_t)m * k, &ord);
        m++;
    }
    *n_codes = (int32_t)darts.size();
    return 0;
}

int ptm_selftest_superpose(int N, const double *obs, const double *tpl, double *rmsd, double *scale, double *q) {
    if (N < 1 || N > NMAX) return -1;
    double a[NMAX][3], b[NMAX][3], ca[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
    for (int i = 0; i < N; i++)
        for (int d = 0; d < 3; d++) {
            ca[d] += obs[3 * i + d] / N;
            cb[d] += tpl[3 * i + d] / N;
        }
    double lb = 0, Ga = 0, Gb = 0;
    for (int i = 0; i < N; i++) {
        double s = 0;
        for (int d = 0; d < 3; d++) {
            a[i][d] = obs[3 * i + d] - ca[d];
            b[i][d] = tpl[3 * i + d] - cb[d];
            s += b[i][d] * b[i][d];
        }
        lb += sqrt(s);
    }
    lb /= N;
    double S[3][3] = {{0}};
    for (int i = 0; i < N; i++) {
        for (int d = 0; d < 3; d++) b[i][d] /= lb;
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) S[x][y] += b[i][x] * a[i][y];
        for (int d = 0; d < 3; d++) {
            Ga += a[i][d] * a[i][d];
            Gb += b[i][d] * b[i][d];
        }
    }
    double lam = qcp_solve(S, Ga, Gb, q);
    double s = Ga > 0 ? lam / Ga : 0.0, R[3][3], res = 0;
    quat_rot(q, R);
    for (int i = 0; i < N; i++)
        for (int x = 0; x < 3; x++) {
            double d = s * a[i][x] - (R[x][0] * b[i][0] + R[x][1] * b[i][1] + R[x][2] * b[i][2]);
            res += d * d;
        }
    *rmsd = sqrt(res / N);
    *scale = s;
    return 0;
}

}  // extern "C"

// host tables for the self-check entry points that need a template
static const HostTables *selftest_tables() {
    static std::once_flag once;
    static HostTables *T = nullptr;
    std::call_once(once, [] {
        HostTables *h = new (std::nothrow) HostTables();
        std::string err;
        if (h && build_tables(*h, err)) T = h;
        else delete h;
    });
    return T;
}

template <int K, typename RT>
static void selftest_strain_k(const TemplateDev &D, const double *obs, double *P) {
    double v[K][3];
    uint64_t tv = 0;
    for (int r = 0; r < K; r++) {
        for (int d = 0; d < 3; d++) v[r][d] = obs[3 * (r + 1) + d] - obs[d];
        tv |= (uint64_t)r << (4 * r);
    }
    RT a0[3], At[3][3], l, Pm[3][3];
    strain_inputs<K, RT>(D, tv, v, a0, At, l);
    polar_p<RT>(At, l, Pm);
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) P[3 * x + y] = (double)Pm[x][y];
}

template <typename RT>
static void selftest_strain_rt(const TemplateDev &D, const double *obs, double *P) {
    if (D.k == 6) selftest_strain_k<6, RT>(D, obs, P);
    else if (D.k == 12) selftest_strain_k<12, RT>(D, obs, P);
    else selftest_strain_k<14, RT>(D, obs, P);
}

extern "C" {

int ptm_selftest_strain(int t, int precision, const double *obs, double *P) {
    const HostTables *T = selftest_tables();
    if (!T || t < 0 || t >= NT || (precision != PTM_FP64 && precision != PTM_FP32_MIXED) || !obs || !P) return -1;
    if (precision == PTM_FP32_MIXED) selftest_strain_rt<float>(T->tpl[t], obs, P);
    else selftest_strain_rt<double>(T->tpl[t], obs, P);
    return 0;
}

int ptm_selftest_strain_device(ptm_ctx *ctx, int t, const double *obs, double *P) {
    if (!ctx || t < 0 || t >= NT || !obs || !P) return PTM_E_INVALID;
    PTM_HIP(ctx, hipSetDevice(ctx->device));
    const int k = template_k(t);
    double rel[KMAX * 3];
    for (int r = 0; r < k; r++)
        for (int d = 0; d < 3; d++) rel[3 * r + d] = obs[3 * (r + 1) + d] - obs[d];
    double *buf = nullptr;
    PTM_HIP(ctx, hipMalloc((void **)&buf, 8 * (KMAX * 3 + 9)));
    ptm_status st = PTM_OK;
    if (hipMemcpyAsync(buf, rel, 8 * 3 * (size_t)k, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) st = PTM_E_DEVICE;
    if (st == PTM_OK) {
        launch_selftest_strain(ctx->view, t, ctx->precision == PTM_FP32_MIXED, buf, buf + KMAX * 3, ctx->stream);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(P, buf + KMAX * 3, 72, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            st = PTM_E_DEVICE;
    }
    (void)hipFree(buf);
    if (st != PTM_OK) ctx->err = "ptm_selftest_strain_device: HIP error";
    return st;
}

int ptm_selftest_orient_f32filter(const double *p) {
    float f[12];
    float m = 0;
    for (int i = 0; i < 12; i++) {
        f[i] = (float)p[i];
        m = fmaxf(m, fabsf(f[i]));
    }
    return orient_filter_f32in(f, f + 3, f + 6, f + 9, f32_orient_bound(m));
}

int ptm_selftest_det3_f32filter(const double *p) {
    float f[9];
    float m = 0;
    for (int i = 0; i < 9; i++) {
        f[i] = (float)p[i];
        m = fmaxf(m, fabsf(f[i]));
    }
    return det3_filter_f32in(f, f + 3, f + 6, f32_det3_bound(m));
}

int ptm_selftest_superpose_f32(int N, const double *obs, const double *tpl, double *rmsd, double *scale, double *q,
                               double *excess) {
    if (N < 1 || N > NMAX) return -1;
    double ca[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
    for (int i = 0; i < N; i++)
        for (int d = 0; d < 3; d++) {
            ca[d] += obs[3 * i + d] / N;
            cb[d] += tpl[3 * i + d] / N;
        }
    double lb = 0, Ga64 = 0;
    float a[NMAX][3], b[NMAX][3];
    double b64[NMAX][3];
    for (int i = 0; i < N; i++) {
        double s = 0;
        for (int d = 0; d < 3; d++) {
            double x = obs[3 * i + d] - ca[d];
            a[i][d] = (float)x;
            Ga64 += x * x;
            b64[i][d] = tpl[3 * i + d] - cb[d];
            s += b64[i][d] * b64[i][d];
        }
        lb += sqrt(s);
    }
    lb /= N;
    float S[3][3] = {{0}}, Gb = 0, Ga = (float)Ga64;
    for (int i = 0; i < N; i++) {
        for (int d = 0; d < 3; d++) b[i][d] = (float)(b64[i][d] / lb);
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) S[x][y] += b[i][x] * a[i][y];
        for (int d = 0; d < 3; d++) Gb += b[i][d] * b[i][d];
    }
    float qf[4], cf = 0.f;
    float lam = qcp_solve<float>(S, Ga, Gb, qf, &cf);
    if (excess) *excess = f32_excess_bound(lam, cf, Ga);
    float s = Ga > 0 ? lam / Ga : 0.f, R[3][3], res = 0;
    quat_rot<float>(qf, R);
    for (int i = 0; i < N; i++)
        for (int x = 0; x < 3; x++) {
            float d = s * a[i][x] - (R[x][0] * b[i][0] + R[x][1] * b[i][1] + R[x][2] * b[i][2]);
            res += d * d;
        }
    *rmsd = sqrtf(res / N);
    *scale = s;
    for (int i = 0; i < 4; i++) q[i] = qf[i];
    return 0;
}

}  // extern "C"
