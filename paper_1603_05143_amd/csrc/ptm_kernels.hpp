// ptm_kernels.hpp -- host-visible launch wrappers of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ptm_tables.hpp"

namespace ptm {

constexpr int VK = 18;  // neighbours of the Voronoi cell of the topological ordering (Sec. 9)

// Cell grid of one frame (counting-sort binning; see k_bin_count).
struct Grid {
    int nc[3];        // cells per axis
    int periodic[3];  // 1 if the axis is periodic
    double L[3];      // periodic box length (0 on open axes)
    double invL[3];   // 1/L, correctly rounded (minimum image uses d*(1/L))
    double lo[3];     // grid origin on open axes
    double h[3];      // cell edge
    double inv_h[3];  // cells per unit length
    double margin;    // safety margin of the neighbour-search certificate
    int canonical;    // every periodic coordinate already lies in [0, L)
};

struct MatchOut {
    int8_t *type;
    int8_t *alloy;
    double *rmsd;
    double *scale;
    double *quat;
    int32_t *neighbours;
    double *strain;
    double *vm_strain;
    double *strain_residual;
    double *nn_distance;
    double *quat_fz;
    int8_t *best_type;
};

void launch_zero(int32_t *p, int64_t n, hipStream_t st);
void launch_bounds(const double *pos, int64_t n, double *part, int nblocks, hipStream_t st);
void launch_bin_count(const double *pos, int64_t n, const Grid &g, int32_t *cell_of, int32_t *slot_of,
                      int32_t *count, hipStream_t st);
// start[0 .. cells] = exclusive scan of count[0 .. cells - 1] (start[cells]
// = the total); bsum: scan_items(cells) words of scratch
void launch_cell_starts(const int32_t *count, int64_t cells, int32_t *bsum, int32_t *start, hipStream_t st);
void launch_bin_scatter(const double *pos, int64_t n, const int32_t *cell_of, const int32_t *slot_of,
                        const int32_t *start, double *spos, int32_t *sid, hipStream_t st);
// k-NN: fast block search, then the exact shell search for the atoms it
// leaves in todo (n entries) / *todo_count (zeroed by the caller).
bool knn_fast_applies(const Grid &g);
// nk = 14 (Euclidean ordering) or VK = 18 (input of the topological
// ordering) nearest neighbours, rank-major [nk][n] / [nk][3][n].  *box_fail
// (zeroed by the caller) is set when the frame has a periodic axis and some
// atom's nk-th neighbour is not strictly closer than half a periodic length
// (or it has fewer than nk neighbours); every later stage then does nothing.
void launch_knn(int64_t n, const Grid &g, int nk, const double *spos,
                const int32_t *sid, const int32_t *start, int32_t *nbr_id, double *nbr_rel, int32_t *todo,
                int32_t *todo_count, int32_t *box_fail, hipStream_t st);
// topological order (Sec. 3) of the 18 neighbours in rel18 / id18: the first
// 14 go to nbr_rel / nbr_id
// (vf: [32][n] facet words, vlive: [n] facet masks, scratch between the two kernels)
void launch_voronoi(int64_t n, const double *rel18, const int32_t *id18, uint32_t *vf, uint32_t *vlive,
                    double *nbr_rel, int32_t *nbr_id, const int32_t *box_fail, hipStream_t st);
// hulls of the first 6 / 12 / 14 neighbours (need: bit g for group g);
// code ids and labellings into code / ord [group][n]
void launch_topo(int64_t n, const double *nbr_rel, const int32_t *nbr_id, const TablesView &T, uint32_t need,
                 int32_t *code, uint64_t *ord, const int32_t *box_fail, hipStream_t st);
// match stage: superposition of every candidate of the codes, decision
// (the full rule where the common one cannot decide, or for every atom with
// force_full), outputs in input order.  *full_count (int32) and *job_count
// (zeroed by the caller) count the atoms the full rule decided and the
// candidates superposed; knn_out (nullable, [n][14] in input order) receives
// the first 14 rows of knn_src (the Euclidean ids, rank-major).
void launch_match(int64_t n, const double *nbr_rel, const int32_t *nbr_id, const int32_t *sid,
                  const int8_t *species, const TablesView &T, const int32_t *code, const uint64_t *ord,
                  uint32_t mask, double cutoff, bool force_full, const MatchOut &O, int32_t *full_count,
                  unsigned long long *job_count, const int32_t *knn_src, int32_t *knn_out, const int32_t *box_fail,
                  bool f32, hipStream_t st);

// int32 entries after the cell counts of a frame's count array: the scan's
// end, the k-NN leftover counter, the full-rule counter, the box flag, then
// (at the first 8-byte aligned entry) the 64-bit count of superposed
// candidates
constexpr int64_t FRAME_COUNTERS = 7;
__host__ __device__ inline unsigned long long *job_counter(int32_t *count, int64_t cells) {
    return (unsigned long long *)(count + ((cells + 5) & ~(int64_t)1));
}

// ------------------------------------- serving through one persistent kernel
// The host hands frames over through pinned memory (ServeHost); one
// persistent kernel (k_serve) pulls them into its device queue and runs
// every stage of every frame as work items: bounds, grid, zeroing, cell
// counts, two-level scan, scatter, k-NN, hulls + match.  Completion is
// written back to the pinned block.
constexpr int SERVE_SLOTS = 256;              // frames in flight at most
constexpr int SERVE_FIFO = 4096;              // device queue of (frame, stage) entries
constexpr int SERVE_NPH = 9;                  // stages of a frame
// Items are small, so that a small frame's stage spreads over many waves
// (a stage of one item is as slow as one wave); a stage holds at most 2^28.
constexpr int64_t SERVE_ATOMS_LIGHT = 512;    // atoms per item: bounds, counts, scatter
constexpr int64_t SERVE_ATOMS = 64;           // atoms per item: k-NN, hulls + match
constexpr int64_t SERVE_ZERO_CELLS = 16384;   // cells per item: zeroing
constexpr int64_t SERVE_SCAN_CELLS = 2048;    // cells per item: scan
enum { SERVE_OK = 0, SERVE_BOX = 1, SERVE_NONFINITE = 2 };

// One frame as the host hands it over: inputs, outputs and the frame's
// device scratch, carved for the largest grid (4n + 4096 cells).
struct ServeRequest {
    int64_t n;
    double box[3];
    double cutoff;
    uint32_t mask, need;
    const double *pos;
    const int8_t *species;
    MatchOut O;
    int32_t *knn_out;
    int32_t *cell_of, *slot_of, *sid, *count, *start;
    double *spos;
    int32_t *nbr_id;
    double *nbr_rel;
    int32_t *code;
    uint64_t *ord;
    double *part;   // [7][bounds items] per-item bounds
    int32_t *bsum;  // scan: per-item totals, then their exclusive prefix
    uint64_t gen;   // ticket generation of the slot (below 2^36)
};

// Pinned host block shared by the host and the kernel.
struct ServeHost {
    unsigned long long tail;              // requests published (host)
    int32_t ring[SERVE_SLOTS];            // slot of request k at ring[k % SERVE_SLOTS] (host)
    ServeRequest req[SERVE_SLOTS];        // (host)
    unsigned long long done[SERVE_SLOTS]; // generation of the slot's last completed frame (kernel)
    long long t_done[SERVE_SLOTS];        // device wall clock at completion (kernel)
    int32_t status[SERVE_SLOTS];          // SERVE_* (kernel)
    int32_t stop;                         // set by the host: every wave exits (host)
};

// Device state of one slot and of the queue (device memory, zeroed once).
struct ServeSlot {
    ServeRequest r;
    Grid g;
    int64_t cells;
    int32_t fast, bad;
    unsigned long long next[SERVE_NPH];  // claim counters: generation << 28 | next item
    long long done[SERVE_NPH], nr[SERVE_NPH];
};
struct ServeDev {
    unsigned long long head, tail, pulled;
    int32_t poll_lock, pad;
    unsigned long long seq[SERVE_FIFO];
    unsigned long long entry[SERVE_FIFO];
    ServeSlot slot[SERVE_SLOTS];
};

// scratch of the serving stages beyond the stream path's, for n atoms
inline int64_t serve_bounds_items(int64_t n) { return (n + SERVE_ATOMS_LIGHT - 1) / SERVE_ATOMS_LIGHT; }
// items of the cell-start scan over cells + 1 entries
inline int64_t scan_items(int64_t cells) { return (cells + 1 + SERVE_SCAN_CELLS - 1) / SERVE_SCAN_CELLS; }
inline int64_t serve_scan_items(int64_t n) { return scan_items(4 * n + 4096); }

// Launch the persistent kernel (grid: what fits on the device at once);
// its waves exit after idle_ticks of the device wall clock without work,
// or when host->stop is set.  Returns the number of workgroups, 0 on error.
int launch_serve(bool f32, const TablesView &T, ServeDev *dev, ServeHost *host, long long idle_ticks,
                 hipStream_t st);
// device wall clock into *out (pinned), for the host's clock reference
void launch_wall_clock(long long *out, hipStream_t st);

// post-hoc cut-off and RMSD histograms (counts: device, 6 * nbins, zeroed by the caller)
void launch_apply_cutoff(int64_t n, const int8_t *best_type, const double *rmsd, double cutoff, int8_t *type,
                         hipStream_t st);
void launch_rmsd_histogram(int64_t n, const int8_t *best_type, const double *rmsd, int nbins, double rmax,
                           unsigned long long *counts, hipStream_t st);
// self-check: the strain of one match (template t, K relative vectors rel
// [K][3] in template-vertex order, device pointers) in the working precision
void launch_selftest_strain(const TablesView &T, int t, bool f32, const double *rel, double *P, hipStream_t st);
// misorientation angles of orientation pairs under each template's symmetry
void launch_misorientation(int64_t n, const TablesView &T, const int8_t *type, const double *q1, const double *q2,
                           double *angle, hipStream_t st);

}  // namespace ptm
