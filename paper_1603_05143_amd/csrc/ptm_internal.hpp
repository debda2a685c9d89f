// ptm_internal.hpp -- context and per-frame state shared by the ABI sources.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/ptm.h"
#include "ptm_kernels.hpp"
#include "ptm_tables.hpp"

#define PTM_HIP(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            return PTM_E_DEVICE;                                                            \
        }                                                                                   \
    } while (0)

namespace ptm {

// Device scratch of one frame (one allocation, carved into arrays).
struct FrameScratch {
    void *base = nullptr;
    size_t bytes = 0;
    bool pooled = false;  // a serving-pool buffer of a fixed size class
    int32_t *cell_of = nullptr, *slot_of = nullptr, *sid = nullptr, *count = nullptr, *start = nullptr;
    double *spos = nullptr;  // sorted positions, x y z of each atom together
    int32_t *nbr_id = nullptr;
    double *nbr_rel = nullptr;
    int32_t *id18 = nullptr;    // topological ordering: the 18 Euclidean neighbours
    double *rel18 = nullptr;
    uint32_t *vf = nullptr;     // and the facets of their Voronoi hull, [32][n] + live masks [n]
    uint32_t *vlive = nullptr;
    int32_t *code = nullptr;
    uint64_t *ord = nullptr;
    double *part = nullptr;
    double *sv_part = nullptr;   // persistent serving: per-item bounds
    int32_t *sv_bsum = nullptr;  // per-item totals of the cell-start scan (every path)
    bool reserve(int64_t n, int64_t cells, bool topo, std::string &err);
    void release();
};

// Staging buffers for host-pointer contexts.
struct StagingBuffers {
    void *base = nullptr;
    size_t bytes = 0;
    void release() {
        if (base) (void)hipFree(base);
        base = nullptr;
        bytes = 0;
    }
};

// Everything a frame's kernels need (device pointers).
struct FrameJob {
    int64_t n = 0;
    const double *pos = nullptr;
    const int8_t *species = nullptr;
    uint32_t mask = 0;
    bool topo = false;  // topological neighbour ordering
    double cutoff = 0;
    Grid grid;
    ptm_outputs out;  // device pointers
};

// Host pointers to copy back to when the context uses host pointers.
struct HostStage {
    bool active = false;
    ptm_outputs host_out;
};

struct Ticket {
    FrameScratch scratch;
    StagingBuffers staging;
    HostStage stage;
    FrameJob job;
    hipEvent_t done = nullptr;
    int stream = 0;
    size_t footprint = 0;
    double t_submit = 0, t_start = 0, t_complete = 0;
    bool complete = false;
    bool box_fail = false;  // the frame's periodic box was too short (PTM_E_BOX)
    bool nonfinite = false; // (persistent serving) a coordinate was not finite
    int slot = -1;          // persistent serving: the frame's slot and generation
    uint64_t gen = 0;
};

size_t frame_bytes(int64_t n, int64_t cells, int nbounds, bool topo);
// the box flag of a frame whose kernels have been enqueued (count[cells + 3])
inline int32_t *box_flag(const FrameScratch &S, const Grid &g) {
    return S.count + (int64_t)g.nc[0] * g.nc[1] * g.nc[2] + 3;
}
int bounds_blocks(int64_t n);
Grid make_grid(const double box[3], const double mn[3], const double mx[3], int64_t n, int kn);
ptm_status enqueue_frame(struct ::ptm_ctx *ctx, FrameScratch &S, const FrameJob &J, hipStream_t st,
                         bool prof = false);
ptm_status frame_bounds(struct ::ptm_ctx *ctx, FrameScratch &S, const double *pos, int64_t n, double mn[3],
                        double mx[3], bool &bad, hipStream_t st);
const char *box_message(bool topo);
hipError_t noalloc_scratch_of(int device, void **ptr);
ptm_status classify_frame(struct ::ptm_ctx *ctx, FrameScratch &S, bool noalloc, const double *positions,
                          const int8_t *species, const double *box, int64_t n_atoms, uint32_t template_mask,
                          double rmsd_cutoff, const ptm_outputs *out);
ptm_status validate(struct ::ptm_ctx *ctx, const double *positions, const double *box, int64_t n, double cutoff,
                    const ptm_outputs *out);
ptm_status upload_tables(struct ::ptm_ctx *ctx);
ptm_status stage_in(struct ::ptm_ctx *ctx, const double *positions, const int8_t *species, const ptm_outputs *out,
                    int64_t n, FrameJob &J, HostStage &H);
ptm_status stage_in_buffers(struct ::ptm_ctx *ctx, StagingBuffers &B, const double *positions,
                            const int8_t *species, const ptm_outputs *out, int64_t n, FrameJob &J, HostStage &H,
                            hipStream_t st);
ptm_status stage_out(struct ::ptm_ctx *ctx, const ptm_outputs *out, int64_t n, const FrameJob &J, const HostStage &H,
                     hipStream_t st);
void serve_shutdown(struct ::ptm_ctx *ctx);

inline double now_us() {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace ptm

struct ptm_ctx {
    int device = 0;
    ptm_precision precision = PTM_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    uint32_t flags = 0;
    int32_t *pinned = nullptr;      // pinned host word: the box flag of the last ptm_classify
    double *pinned_bounds = nullptr;  // pinned host space: per-block bounds of the frame being set up
    void *noalloc_scratch = nullptr;  // this device's static scratch array (ptm_classify_noalloc)
    ptm::HostTables host;
    std::vector<void *> table_buffers;
    ptm::TablesView view;
    ptm::FrameScratch main;
    ptm::StagingBuffers staging;
    std::string err;
    // serving state
    std::vector<hipStream_t> serve_streams;
    hipStream_t bounds_stream = nullptr;
    std::map<uint64_t, ptm::Ticket *> tickets;
    std::vector<ptm::FrameScratch> free_scratch;
    uint64_t next_ticket = 1;
    size_t inflight_bytes = 0;  // scratch held by in-flight frames
    size_t pool_bytes = 0;      // scratch allocated by the pool (in flight + free)
    int next_stream = 0;
    double *bounds_part = nullptr;      // per-block bounds of the frame being admitted
    hipEvent_t order_event = nullptr;   // orders serving frames after the context stream's work
    hipEvent_t ref_event = nullptr;     // device-timeline reference ...
    double ref_time_us = 0;             // ... and its host-clock time
    // persistent serving (PTM_F_PERSISTENT)
    ptm::ServeDev *sv_dev = nullptr;    // device queue and slots
    ptm::ServeHost *sv_host = nullptr;  // pinned block shared with the kernel
    long long *sv_clock = nullptr;      // pinned word: device wall clock reference
    hipStream_t sv_stream = nullptr;    // the persistent kernel's stream
    hipEvent_t sv_exit = nullptr;       // recorded after the last launch of the kernel
    bool sv_launched = false;
    std::vector<int> sv_free;           // free slots
    uint64_t sv_gen = 0;
    double sv_clock_khz = 0;            // device wall clock rate
    double sv_ref_host_us = 0;          // host time of ...
    long long sv_ref_dev = 0;           // ... this device wall clock value
    // stage profiling (PTM_F_PROFILE)
    hipEvent_t prof_ev[PTM_NSTAGES + 1] = {};
    bool prof_valid = false;
    int64_t prof_info[PTM_NINFO] = {};
    // grow-only device buffer of the small per-call outputs (histogram counts)
    void *aux = nullptr;
    size_t aux_bytes = 0;
};
