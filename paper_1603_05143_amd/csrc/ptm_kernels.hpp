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
void launch_bin_scatter(const double *pos, int64_t n, const int32_t *cell_of, const int32_t *slot_of,
                        const int32_t *start, double *sx, double *sy, double *sz, int32_t *sid, hipStream_t st);
// k-NN: fast block search, then the exact shell search for the atoms it
// leaves in todo (n entries) / *todo_count (zeroed by the caller).
bool knn_fast_applies(const Grid &g);
// nk = 14 (Euclidean ordering) or VK = 18 (input of the topological
// ordering) nearest neighbours, rank-major [nk][n] / [nk][3][n].  *box_fail
// (zeroed by the caller) is set when the frame has a periodic axis and some
// atom's nk-th neighbour is not strictly closer than half a periodic length
// (or it has fewer than nk neighbours); every later stage then does nothing.
void launch_knn(int64_t n, const Grid &g, int nk, const double *sx, const double *sy, const double *sz,
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
