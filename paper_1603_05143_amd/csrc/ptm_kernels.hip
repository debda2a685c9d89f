// ptm_kernels.hip -- HIP kernels of the PTM classification pass for gfx950.
//
// Pipeline for one frame (Polyhedral Template Matching, arXiv:1603.05143):
//   k_bounds          finite check + bounding box (open axes)
//   k_bin_count       cell id + per-cell counter (counting sort, pass 1)
//   (scan)            exclusive prefix sum of the counters
//   k_bin_scatter     sorted copy of the positions, x y z of an atom together
//                     (counting sort, pass 2)
//   k_knn_fast/exact  14 (or 18) nearest neighbours by (d^2, id), Sec. 3
//                     Euclidean order
//   k_voronoi_hull/   optional topological order (Sec. 3): Voronoi interface
//   k_voronoi_order   areas of the centre and its 18 nearest neighbours
//   k_topo            hulls of the innermost 6 / 12 / 14 neighbours with exact
//                     predicates (Sec. 4; Alg. 1 requires the centre strictly
//                     inside), start-edge codes, template table lookups
//   k_match           superposition of every candidate correspondence of
//                     the codes (eqs. 2-4, App. A), decision (Alg. 1; the
//                     full tie rule in FP64 where needed), representative,
//                     orientation, strain (eq. 6, Sec. 8), alloy (Sec. 6,
//                     Table 3), derived outputs, write-back in input order
//   k_apply_cutoff, k_rmsd_histogram, k_misorientation: post-hoc utilities
//                     (Sec. 5.1, Sec. 7)
// One lane owns one atom in every per-atom kernel (k_match also gives a
// lane one candidate of its wave's atoms); atoms are processed in cell
// order so the lanes of a wave read the same cells.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ptm_device.hpp"
#include "ptm_kernels.hpp"
#include "ptm_tables.hpp"

namespace ptm {

// --------------------------------------------------------------- helpers
__device__ inline uint32_t nib(uint64_t w, int i) { return (uint32_t)((w >> (4 * i)) & 0xF); }
__device__ inline uint64_t setnib(uint64_t w, int i, uint32_t v) {
    return (w & ~(0xFull << (4 * i))) | ((uint64_t)v << (4 * i));
}

__device__ inline int cell_coord(double x, const Grid &g, int d) {
    double u;
    if (g.periodic[d]) {
        u = x - g.L[d] * floor(x * g.invL[d]);
    } else {
        u = x - g.lo[d];
    }
    double f = floor(u * g.inv_h[d]);
    // NaN (a non-finite coordinate, refused later) also lands in cell 0
    int c = !(f >= 0.0) ? 0 : (f >= (double)(g.nc[d] - 1) ? g.nc[d] - 1 : (int)f);
    return c;
}

__device__ inline double wrapped(double x, const Grid &g, int d) {
    return g.periodic[d] ? x - g.L[d] * floor(x * g.invL[d]) : x - g.lo[d];
}

// ------------------------------------------------------------------ bounds
// Per-block min/max of each axis and a non-finite flag.
__global__ void k_bounds(const double *__restrict__ pos, int64_t n, double *__restrict__ part) {
    __shared__ double smin[3][256], smax[3][256];
    __shared__ int sbad[256];
    double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; d++) {
            double x = pos[3 * i + d];
            if (!isfinite(x)) bad = 1;
            mn[d] = fmin(mn[d], x);
            mx[d] = fmax(mx[d], x);
        }
    }
    int t = threadIdx.x;
    for (int d = 0; d < 3; d++) { smin[d][t] = mn[d]; smax[d][t] = mx[d]; }
    sbad[t] = bad;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
            for (int d = 0; d < 3; d++) {
                smin[d][t] = fmin(smin[d][t], smin[d][t + s]);
                smax[d][t] = fmax(smax[d][t], smax[d][t + s]);
            }
            sbad[t] |= sbad[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        double *o = part + 7 * blockIdx.x;
        for (int d = 0; d < 3; d++) { o[d] = smin[d][0]; o[3 + d] = smax[d][0]; }
        o[6] = (double)sbad[0];
    }
}

// ----------------------------------------------------------------- binning
__global__ void k_bin_count(const double *__restrict__ pos, int64_t n, Grid g, int32_t *__restrict__ cell_of,
                            int32_t *__restrict__ slot_of, int32_t *__restrict__ count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(pos[3 * i + 0], g, 0);
    int cy = cell_coord(pos[3 * i + 1], g, 1);
    int cz = cell_coord(pos[3 * i + 2], g, 2);
    int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
    cell_of[i] = c;
    slot_of[i] = atomicAdd(&count[c], 1);
}

// Cell starts: the exclusive scan of the counts over cells + 1 entries (the
// last start is the number of atoms), in items of SERVE_SCAN_CELLS cells --
// the items' totals, their exclusive scan, then each item's cells from its
// offset (three passes: every atomic count must be final before the first).
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER = (int)(SERVE_SCAN_CELLS / SCAN_THREADS);  // cells per thread
static_assert(SERVE_SCAN_CELLS % SCAN_THREADS == 0 && SCAN_PER % 4 == 0, "an item is whole threads' 16-byte runs");

// exclusive scan over a block of NT threads (ws: NT / 64 words of LDS);
// total: the block's sum
template <int NT>
__device__ inline int32_t block_excl_scan(int32_t v, int32_t &total, int32_t *ws) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; k++) {
        const int32_t t = ws[k];
        before += k < w ? t : 0;
        all += t;
    }
    total = all;
    return before + x - v;
}

// item totals: 16-byte reads interleaved across the block, so they
// coalesce (count is 256-byte aligned and items are multiples of 4 cells)
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_totals(const int32_t *__restrict__ count, int64_t cells,
                                                               int32_t *__restrict__ bsum) {
    __shared__ int32_t ws[SCAN_THREADS / 64];
    const int64_t b = (int64_t)blockIdx.x * SERVE_SCAN_CELLS + 4 * (int64_t)threadIdx.x;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER / 4; k++) {
        const int64_t c = b + (int64_t)k * 4 * SCAN_THREADS;
        if (c + 4 <= cells) {
            const int4 x = *reinterpret_cast<const int4 *>(count + c);
            s += (x.x + x.y) + (x.z + x.w);
        } else {
            for (int j = 0; j < 4; j++) s += c + j < cells ? count[c + j] : 0;
        }
    }
    int32_t total;
    (void)block_excl_scan<SCAN_THREADS>(s, total, ws);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// exclusive scan of the item totals in place, one block
__global__ void __launch_bounds__(1024) k_scan_top(int32_t *__restrict__ bsum, int64_t items) {
    __shared__ int32_t ws[1024 / 64];
    const int64_t per = (items + 1023) / 1024;
    const int64_t lb = threadIdx.x * per, le = min(items, lb + per);
    int32_t s = 0;
    for (int64_t k = lb; k < le; k++) s += bsum[k];
    int32_t total;
    int32_t run = block_excl_scan<1024>(s, total, ws);
    for (int64_t k = lb; k < le; k++) {
        const int32_t v = bsum[k];
        bsum[k] = run;
        run += v;
    }
}

// each item's cells: a run of SCAN_PER consecutive cells per thread
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_cells(const int32_t *__restrict__ count, int64_t cells,
                                                              const int32_t *__restrict__ bsum,
                                                              int32_t *__restrict__ start) {
    __shared__ int32_t ws[SCAN_THREADS / 64];
    const int64_t b = (int64_t)blockIdx.x * SERVE_SCAN_CELLS + (int64_t)threadIdx.x * SCAN_PER;
    int32_t v[SCAN_PER], s = 0;
    if (b + SCAN_PER <= cells) {  // whole run in range: 16-byte reads (b is a multiple of 8)
        const int4 *q = reinterpret_cast<const int4 *>(count + b);
#pragma unroll
        for (int k = 0; k < SCAN_PER / 4; k++) {
            const int4 x = q[k];
            v[4 * k] = x.x;
            v[4 * k + 1] = x.y;
            v[4 * k + 2] = x.z;
            v[4 * k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_PER; k++) v[k] = b + k < cells ? count[b + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) s += v[k];
    int32_t total;
    int32_t run = bsum[blockIdx.x] + block_excl_scan<SCAN_THREADS>(s, total, ws);
    int32_t o[SCAN_PER];
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        o[k] = run;
        run += v[k];
    }
    if (b + SCAN_PER <= cells + 1) {
        int4 *q = reinterpret_cast<int4 *>(start + b);
#pragma unroll
        for (int k = 0; k < SCAN_PER / 4; k++) q[k] = make_int4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_PER; k++)
            if (b + k <= cells) start[b + k] = o[k];
    }
}

__global__ void k_bin_scatter(const double *__restrict__ pos, int64_t n, const int32_t *__restrict__ cell_of,
                              const int32_t *__restrict__ slot_of, const int32_t *__restrict__ start,
                              double *__restrict__ spos,
                              int32_t *__restrict__ sid) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t p = (int64_t)start[cell_of[i]] + slot_of[i];
    spos[3 * (int64_t)p] = pos[3 * i + 0];
    spos[3 * (int64_t)p + 1] = pos[3 * i + 1];
    spos[3 * (int64_t)p + 2] = pos[3 * i + 2];
    sid[p] = (int32_t)i;
}

// ---------------------------------------------------------------- k-NN
// Minimum-image difference exactly as specified: s = rint(d * (1/L)),
// d - s*L, without contraction (the library is built with
// -ffp-contract=off), so d^2 matches the reference bit for bit.
__device__ inline double min_image(double d, const Grid &g, int a) {
    if (g.periodic[a]) {
        double s = rint(d * g.invL[a]);
        d = d - s * g.L[a];
    }
    return d;
}

// insert (d2, j) -- with j's position q in the sorted arrays -- into the
// list (kd, kj, kq) of length KN, ascending by (d2, j)
template <int KN>
__device__ inline void topk_insert(double (&kd)[KN], int32_t (&kj)[KN], int32_t (&kq)[KN], double d2, int32_t j,
                                   int32_t q) {
    bool done = false;
#pragma unroll
    for (int m = KN - 1; m > 0; m--) {
        bool lt = !done && (d2 < kd[m - 1] || (d2 == kd[m - 1] && j < kj[m - 1]));
        if (!done) {
            kd[m] = lt ? kd[m - 1] : d2;
            kj[m] = lt ? kj[m - 1] : j;
            kq[m] = lt ? kq[m - 1] : q;
        }
        done = done || !lt;
    }
    if (!done) {
        kd[0] = d2;
        kj[0] = j;
        kq[0] = q;
    }
}

__device__ inline void shell_range(const Grid &g, int a, int s, int &lo, int &hi) {
    if (g.periodic[a]) {
        int half = (g.nc[a] - 1) / 2;
        lo = -min(s, half);
        hi = min(s, g.nc[a] - 1 - half);
    } else {
        lo = -s;
        hi = s;
    }
}

// scan the atoms of cell c into the top-K list
template <int KN>
__device__ inline void scan_cell(int c, const Grid &g, double xi, double yi, double zi, int32_t i,
                                 const double *__restrict__ spos, const int32_t *__restrict__ sid,
                                 const int32_t *__restrict__ start, double (&kd)[KN], int32_t (&kj)[KN],
                                 int32_t (&kq)[KN], int &found) {
    int q1 = start[c + 1];
    for (int q = start[c]; q < q1; q++) {
        int32_t j = sid[q];
        if (j == i) continue;
        double dx = min_image(spos[3 * (int64_t)q] - xi, g, 0);
        double dy = min_image(spos[3 * (int64_t)q + 1] - yi, g, 1);
        double dz = min_image(spos[3 * (int64_t)q + 2] - zi, g, 2);
        double xx = dx * dx, yy = dy * dy, zz = dz * dz;
        double d2 = (xx + yy) + zz;
        found++;
        if (d2 < kd[KN - 1] || (d2 == kd[KN - 1] && j < kj[KN - 1])) topk_insert<KN>(kd, kj, kq, d2, j, q);
    }
}

// Is the block of offsets [lo, hi] per axis a certificate for the current
// K-th distance?  all = the block covers every cell.
__device__ inline bool certified(const Grid &g, const int (&cc)[3], const double (&u)[3], const int (&lo)[3],
                                 const int (&hi)[3], int found, int KN, double kth, bool &all) {
    double dmin = INFINITY;
    all = true;
    for (int a = 0; a < 3; a++) {
        bool sat_lo, sat_hi;
        if (g.periodic[a]) {
            sat_lo = sat_hi = (hi[a] - lo[a] + 1) >= g.nc[a];
        } else {
            sat_lo = cc[a] + lo[a] <= 0;
            sat_hi = cc[a] + hi[a] >= g.nc[a] - 1;
        }
        if (!sat_lo) dmin = fmin(dmin, u[a] - (cc[a] + lo[a]) * g.h[a]);
        if (!sat_hi) dmin = fmin(dmin, (cc[a] + hi[a] + 1) * g.h[a] - u[a]);
        all = all && sat_lo && sat_hi;
    }
    if (all) return true;
    dmin -= g.margin;
    return found >= KN && dmin > 0 && kth < dmin * dmin;
}

// Sec. 5 samples are periodic.  Every image of an atom other than its
// minimum image lies at least half a box length away along that axis, so
// the minimum-image shell is the periodic crystal's shell only when its
// K-th member is strictly closer than half of every periodic length
// (compared as 4 d^2 < L*L in FP64); a periodic frame whose atom has fewer
// than K neighbours fails as well.  True = the frame is rejected.
__device__ inline bool shell_exceeds_box(const Grid &g, int cnt, int K, double kth) {
    bool periodic = false, bad = false;
    for (int a = 0; a < 3; a++)
        if (g.periodic[a]) {
            periodic = true;
            bad = bad || !(4.0 * kth < g.L[a] * g.L[a]);
        }
    return periodic && (cnt < K || bad);
}

// Write the K nearest neighbours of sorted atom p: ids and
// minimum-image vectors in the component-major layout the hull kernels read.
// spos[3q .. 3q+2] is a copy of pos[3 sid[q] ..], so the vectors are those of the input.
template <int KN>
__device__ inline void write_knn(int64_t n, int64_t p, int cnt, const int32_t (&kq)[KN], const Grid &g,
                                 double xi, double yi, double zi, const double *__restrict__ spos,
                                 const int32_t *__restrict__ sid, int32_t *__restrict__ nbr_id,
                                 double *__restrict__ nbr_rel) {
#pragma unroll
    for (int m = 0; m < KN; m++) {
        int32_t j = -1;
        double r0 = 0, r1 = 0, r2 = 0;
        if (m < cnt) {
            int32_t q = kq[m];
            j = sid[q];
            r0 = min_image(spos[3 * (int64_t)q] - xi, g, 0);
            r1 = min_image(spos[3 * (int64_t)q + 1] - yi, g, 1);
            r2 = min_image(spos[3 * (int64_t)q + 2] - zi, g, 2);
        }
        nbr_id[(int64_t)m * n + p] = j;
        nbr_rel[((int64_t)m * 3 + 0) * n + p] = r0;
        nbr_rel[((int64_t)m * 3 + 1) * n + p] = r1;
        nbr_rel[((int64_t)m * 3 + 2) * n + p] = r2;
    }
}

// Packed search key of a candidate: high word = FP32 rounding of d^2 (its
// bit pattern, offset by 2^20 so that the word read as the high half of an
// FP64 number is a normal, finite value), low word = sorted index q.  Keys
// compare as FP64 numbers in the order (round(d^2), q); rounding to nearest
// is monotone, so round(a) < round(b) implies a < b.
__device__ inline double pack_key(double d2, int32_t q) {
    uint32_t hi = __float_as_uint(__double2float_rn(d2)) + 0x00100000u;
    return __hiloint2double((int)hi, q);
}
__device__ inline uint32_t key_hi(double k) { return (uint32_t)__double2hiint(k); }
__device__ inline int32_t key_q(double k) { return __double2loint(k); }
// upper bound of every d^2 whose rounding gives the key's high word
// (relative error 2^-24 of a normal float, absolute 2^-150 of a subnormal)
__device__ inline double key_d2_upper(double k) {
    return (double)__uint_as_float(key_hi(k) - 0x00100000u) * (1.0 + 0x1p-22) + 0x1p-148;
}

// One step of the insertion: (a, t) <- (min(a, t), max(a, t)).  Written as
// two VALU instructions that update a in place: the keys are finite, normal
// FP64 numbers (no NaN, no denormal), for which the instructions return one
// of their operands unchanged, and keeping each list entry in one register
// avoids copies of the whole list on every loop iteration.
__device__ inline void minmax_step(double &a, double &t) {
    double hi;
    asm("v_max_f64 %0, %1, %2\n\tv_min_f64 %1, %1, %2" : "=&v"(hi), "+v"(a) : "v"(t));
    t = hi;
}


// Fast search: the 5x5x5 block of cells around the atom, walked as 25
// x-rows nearest-first.  A row of cells is one contiguous range of the
// sorted atoms (two if it wraps), and each lane walks its ranges in one flat
// loop, so a wave pays about the per-lane candidate count rather than the
// per-cell maximum.  The running list holds the 15 smallest packed keys,
// kept by a branch-free min/max insertion.  Once 14 keys are known, rows and
// the x-extent of each row are trimmed to an upper bound of the current 14th
// distance.  The result is accepted when it is provably the exact ordered
// (d^2, id) list: the high words of the 15 keys strictly increase (then the
// rounded order is the exact order and no atom outside ties with the 14th)
// and the exact 14th distance is certified by the block.  Other atoms are
// appended to a list for k_knn_exact.  Requires every periodic axis to have
// at least 5 cells (no axis wraps onto itself within the block).
// Workgroups are dispatched to the 8 XCDs round-robin, and each XCD has its
// own L2.  With a grid padded to a multiple of 8, this bijection gives every
// XCD one contiguous range of blocks, so that blocks sharing cells (and
// their atoms) run behind the same L2.
constexpr int NXCD = 8;
__device__ inline int64_t xcd_block(int64_t i, int64_t nblocks_padded) {
    const int64_t per = nblocks_padded / NXCD;
    return (i % NXCD) * per + i / NXCD;
}
inline int64_t xcd_pad(int64_t nblocks) { return (nblocks + NXCD - 1) / NXCD * NXCD; }

// NK = 14 neighbours (Euclidean ordering), or 18 (the input of the
// topological ordering); the list holds NK + 1 keys, the last one certifies
// the boundary.  One atom (lane); false: not certified, nothing written
// (the exact search must take it).
template <int NK>
__device__ inline bool knn_fast_atom(int64_t p, int64_t n, const Grid &g, const double *__restrict__ spos,
                                     const int32_t *__restrict__ sid, const int32_t *__restrict__ start,
                                     int32_t *__restrict__ nbr_id, double *__restrict__ nbr_rel,
                                     int32_t *__restrict__ box_fail) {
    constexpr int KN = NK + 1;
    const double xi = spos[3 * (int64_t)p], yi = spos[3 * (int64_t)p + 1], zi = spos[3 * (int64_t)p + 2];
    const double xs[3] = {xi, yi, zi};
    int cc[3];
    double u[3];
    for (int a = 0; a < 3; a++) {
        cc[a] = cell_coord(xs[a], g, a);
        u[a] = wrapped(xs[a], g, a);
    }
    const double INF = __longlong_as_double(0x7ff0000000000000ll);
    double key[KN];
#pragma unroll
    for (int m = 0; m < KN; m++) key[m] = INF;
    // known minimum-image shifts: every periodic coordinate in [0, L) and at
    // least 7 cells per periodic axis, so a wrapped row is exactly one box
    // length away and the shifted difference equals the minimum image
    bool shifted = g.canonical != 0;
    for (int a = 0; a < 3; a++) shifted = shifted && (!g.periodic[a] || g.nc[a] >= 7);
    // (dy + 2) + 5 (dz + 2) of the 25 rows by increasing dy^2 + dz^2, 5 bits each
    const uint64_t rows_lo = 0x013952440D13B56Cull;  // rows 0..11
    const uint64_t rows_hi = 0x0250171D4334BCB6ull;  // rows 12..23
    const int row_last = 24;                          // row 24: (dy, dz) = (2, 2)
    const int nx = g.nc[0];
    int r = 0, q = 0, qend = 0, seg2_lo = 0, seg2_hi = -1;
    double shx = 0, shy = 0, shz = 0, shx2 = 0;
    int cyz = 0;
    // Each iteration first moves to the next segment if the current one is
    // exhausted, then takes at most one candidate; the insertion runs on
    // every iteration (an empty step inserts +inf), and the loop exits only
    // after it, so the list stays in the same registers across the loop.
    bool more = true;
    do {
        if (q >= qend) {
            if (seg2_lo <= seg2_hi) {  // second (wrapped) part of the row
                q = start[cyz + seg2_lo];
                qend = start[cyz + seg2_hi + 1];
                shx = shx2;
                seg2_hi = -1;
            } else if (r < 25) {
                int code = r < 12 ? (int)((rows_lo >> (5 * r)) & 31)
                                  : (r < 24 ? (int)((rows_hi >> (5 * (r - 12))) & 31) : row_last);
                r++;
                int dz = code / 5 - 2, dy = code - 5 * (code / 5) - 2;
                int cy = cc[1] + dy, cz = cc[2] + dz;
                bool skip = false;
                shy = shz = 0;
                if (g.periodic[1]) {
                    if (cy < 0) { cy += g.nc[1]; shy = g.L[1]; }
                    else if (cy >= g.nc[1]) { cy -= g.nc[1]; shy = -g.L[1]; }
                } else {
                    skip = cy < 0 || cy >= g.nc[1];
                }
                if (g.periodic[2]) {
                    if (cz < 0) { cz += g.nc[2]; shz = g.L[2]; }
                    else if (cz >= g.nc[2]) { cz -= g.nc[2]; shz = -g.L[2]; }
                } else {
                    skip = skip || cz < 0 || cz >= g.nc[2];
                }
                int xlo = -2, xhi = 2;
                if (!skip && key[NK - 1] != INF) {
                    double ly = (cc[1] + dy) * g.h[1] - u[1], hy = ly + g.h[1];
                    double lz = (cc[2] + dz) * g.h[2] - u[2], hz = lz + g.h[2];
                    double gy = ly > 0 ? ly : (hy < 0 ? -hy : 0.0);
                    double gz = lz > 0 ? lz : (hz < 0 ? -hz : 0.0);
                    gy = gy > g.margin ? gy - g.margin : 0.0;
                    gz = gz > g.margin ? gz - g.margin : 0.0;
                    double rem = key_d2_upper(key[NK - 1]) - (gy * gy + gz * gz);
                    if (rem < 0) {
                        skip = true;
                    } else {
                        // cells whose x-gap less the margin exceeds sqrt(rem)
                        // cannot hold a better neighbour (compared squared)
                        const double x0 = u[0] - cc[0] * g.h[0];  // offset of the atom inside its cell
                        auto beyond = [&](double gap) {
                            const double e = gap - g.margin;
                            return e > 0 && e * e > rem;
                        };
                        while (xlo < 0 && beyond((-xlo - 1) * g.h[0] + x0)) xlo++;
                        while (xhi > 0 && beyond((xhi - 1) * g.h[0] + (g.h[0] - x0))) xhi--;
                    }
                }
                cyz = (cz * g.nc[1] + cy) * nx;
                int a0 = cc[0] + xlo, a1 = cc[0] + xhi;
                seg2_hi = -1;
                if (g.periodic[0]) {
                    if (a0 < 0) {  // wrapped part [a0 + nx, nx - 1] lies one box length up
                        seg2_lo = a0 + nx;
                        seg2_hi = nx - 1;
                        shx2 = g.L[0];
                        a0 = 0;
                    } else if (a1 >= nx) {
                        seg2_lo = 0;
                        seg2_hi = a1 - nx;
                        shx2 = -g.L[0];
                        a1 = nx - 1;
                    }
                } else {
                    a0 = max(a0, 0);
                    a1 = min(a1, nx - 1);
                    skip = skip || a0 > a1;
                }
                if (skip) {
                    q = qend = 0;
                    seg2_hi = -1;
                } else {
                    q = start[cyz + a0];
                    qend = start[cyz + a1 + 1];
                }
                shx = 0;
            } else {
                more = false;
            }
        }
        // up to two candidates per step: their loads are independent, so the
        // second one's latency hides behind the first's
        double t = INF, t2 = INF;
        if (q < qend) {
            const bool two = q + 1 < qend;
            const int q2 = two ? q + 1 : q;  // (a repeated, in-bounds load when there is no second)
            const double ax = spos[3 * (int64_t)q], ay = spos[3 * (int64_t)q + 1], az = spos[3 * (int64_t)q + 2];
            const double bx = spos[3 * (int64_t)q2], by = spos[3 * (int64_t)q2 + 1], bz = spos[3 * (int64_t)q2 + 2];
            double dx, dy, dz, ex, ey, ez;
            if (shifted) {
                dx = (ax - xi) - shx;
                dy = (ay - yi) - shy;
                dz = (az - zi) - shz;
                ex = (bx - xi) - shx;
                ey = (by - yi) - shy;
                ez = (bz - zi) - shz;
            } else {
                dx = min_image(ax - xi, g, 0);
                dy = min_image(ay - yi, g, 1);
                dz = min_image(az - zi, g, 2);
                ex = min_image(bx - xi, g, 0);
                ey = min_image(by - yi, g, 1);
                ez = min_image(bz - zi, g, 2);
            }
            const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
            const double d2 = (xx + yy) + zz;
            const double xx2 = ex * ex, yy2 = ey * ey, zz2 = ez * ez;
            const double e2 = (xx2 + yy2) + zz2;
            if (q != (int)p) t = pack_key(d2, q);
            if (two && q2 != (int)p) t2 = pack_key(e2, q2);
            q += two ? 2 : 1;
        }
        // the two insertions interleaved, the second one step behind the
        // first (step m of the second reads key[m] after step m of the
        // first): two independent dependency chains instead of one of twice
        // the length, with the result of inserting t, then t2
        minmax_step(key[0], t);
#pragma unroll
        for (int m = 1; m < KN; m++) {
            minmax_step(key[m], t);
            minmax_step(key[m - 1], t2);
        }
        minmax_step(key[KN - 1], t2);
    } while (more);
    bool ok = key[NK - 1] != INF;
#pragma unroll
    for (int m = 0; m < KN - 1; m++) ok = ok && key_hi(key[m]) < key_hi(key[m + 1]);
    int32_t kq[NK];
#pragma unroll
    for (int m = 0; m < NK; m++) kq[m] = key_q(key[m]);
    if (ok) {
        // certified on the key's upper bound of the K-th distance, so the
        // K-th neighbour's position is read only when the box check needs
        // the exact distance
        const double kth_up = key_d2_upper(key[NK - 1]);
        int lo[3] = {-2, -2, -2}, hi[3] = {2, 2, 2};
        bool all;
        ok = certified(g, cc, u, lo, hi, NK, NK, kth_up, all);
        if (ok && shell_exceeds_box(g, NK, NK, kth_up)) {
            const int32_t q13 = kq[NK - 1];
            const double ex = min_image(spos[3 * (int64_t)q13] - xi, g, 0);
            const double ey = min_image(spos[3 * (int64_t)q13 + 1] - yi, g, 1);
            const double ez = min_image(spos[3 * (int64_t)q13 + 2] - zi, g, 2);
            if (shell_exceeds_box(g, NK, NK, (ex * ex + ey * ey) + ez * ez)) atomicOr(box_fail, 1);
        }
    }
    if (!ok) return false;
    write_knn<NK>(n, p, NK, kq, g, xi, yi, zi, spos, sid, nbr_id, nbr_rel);
    return true;
}

template <int NK>
__global__ void __launch_bounds__(256) k_knn_fast(int64_t n, Grid g, const double *__restrict__ spos,
                                                  const int32_t *__restrict__ sid, const int32_t *__restrict__ start,
                                                  int32_t *__restrict__ nbr_id, double *__restrict__ nbr_rel,
                                                  int32_t *__restrict__ todo, int32_t *__restrict__ todo_count,
                                                  int32_t *__restrict__ box_fail) {
    int64_t p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (!knn_fast_atom<NK>(p, n, g, spos, sid, start, nbr_id, nbr_rel, box_fail))
        todo[atomicAdd(todo_count, 1)] = (int32_t)p;
}

// Exact search for the atoms the fast search left (or all atoms when todo
// is NULL), one wavefront per atom.  The lanes share the cells of the block
// of shells 0..2 (then of each further shell) and keep private lists
// ordered by the exact key (d^2, id); a 14-round wave-wide merge of the list
// heads gives the atom's ordered neighbours, and the shells grow until the
// searched block certifies the 14th distance.  A wave per atom keeps the
// latency of a few left-over atoms short: each lane scans one or two cells.
// One atom p (wave-uniform) by the whole wave.
template <int NK>
__device__ void knn_exact_atom(int64_t p, int64_t n, const Grid &g, const double *__restrict__ spos,
                               const int32_t *__restrict__ sid, const int32_t *__restrict__ start,
                               int32_t *__restrict__ nbr_id, double *__restrict__ nbr_rel,
                               int32_t *__restrict__ box_fail) {
    constexpr int KN = NK;
    const int lane = threadIdx.x & 63;
    {
        const double xi = spos[3 * (int64_t)p], yi = spos[3 * (int64_t)p + 1], zi = spos[3 * (int64_t)p + 2];
        const int32_t i = sid[p];
        const double xs[3] = {xi, yi, zi};
        int cc[3];
        double u[3];
        for (int a = 0; a < 3; a++) {
            cc[a] = cell_coord(xs[a], g, a);
            u[a] = wrapped(xs[a], g, a);
        }
        double kd[KN];
        int32_t kj[KN], kq[KN];
#pragma unroll
        for (int m = 0; m < KN; m++) { kd[m] = INFINITY; kj[m] = 0x7fffffff; kq[m] = 0; }
        int found = 0;
        // merged result: lane m < KN holds entry m
        double rd = INFINITY;
        int32_t rj = -1, rq = 0;
        int total = 0;
        double kth = INFINITY;
        int plo[3] = {1, 1, 1}, phi[3] = {0, 0, 0};  // block already searched (empty)
        for (int s = 2;; s++) {
            int lo[3], hi[3], ext[3];
            for (int a = 0; a < 3; a++) {
                shell_range(g, a, s, lo[a], hi[a]);
                ext[a] = hi[a] - lo[a] + 1;
            }
            const int ncell = ext[0] * ext[1] * ext[2];
            for (int c = lane; c < ncell; c += 64) {
                int ox = lo[0] + c % ext[0];
                int oy = lo[1] + (c / ext[0]) % ext[1];
                int oz = lo[2] + c / (ext[0] * ext[1]);
                bool inner = ox >= plo[0] && ox <= phi[0] && oy >= plo[1] && oy <= phi[1] && oz >= plo[2] &&
                             oz <= phi[2];
                if (inner) continue;
                int cx = cc[0] + ox, cy = cc[1] + oy, cz = cc[2] + oz;
                if (g.periodic[0]) cx = (cx % g.nc[0] + g.nc[0]) % g.nc[0];
                else if (cx < 0 || cx >= g.nc[0]) continue;
                if (g.periodic[1]) cy = (cy % g.nc[1] + g.nc[1]) % g.nc[1];
                else if (cy < 0 || cy >= g.nc[1]) continue;
                if (g.periodic[2]) cz = (cz % g.nc[2] + g.nc[2]) % g.nc[2];
                else if (cz < 0 || cz >= g.nc[2]) continue;
                scan_cell<KN>((cz * g.nc[1] + cy) * g.nc[0] + cx, g, xi, yi, zi, i, spos, sid, start, kd, kj,
                              kq, found);
            }
            // wave-wide merge of the list heads, smallest (d^2, id) first
            total = found;
            for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off);
#pragma unroll 1
            for (int m = 0; m < KN; m++) {
                double bd = kd[0];
                int32_t bj = kj[0];
                for (int off = 32; off > 0; off >>= 1) {
                    double od = __shfl_xor(bd, off);
                    int32_t oj = __shfl_xor(bj, off);
                    if (od < bd || (od == bd && oj < bj)) { bd = od; bj = oj; }
                }
                if (bd == INFINITY) break;  // every list is empty
                bool mine = kd[0] == bd && kj[0] == bj;
                uint64_t who = __ballot(mine);
                int src = __ffsll((unsigned long long)who) - 1;
                int32_t bq = __shfl(kq[0], src);
                if (lane == m) { rd = bd; rj = bj; rq = bq; }
                if (mine) {  // pop the head
#pragma unroll
                    for (int t = 0; t < KN - 1; t++) { kd[t] = kd[t + 1]; kj[t] = kj[t + 1]; kq[t] = kq[t + 1]; }
                    kd[KN - 1] = INFINITY;
                    kj[KN - 1] = 0x7fffffff;
                }
            }
            kth = __shfl(rd, KN - 1);
            bool all;
            bool done = certified(g, cc, u, lo, hi, total, KN, kth, all);
            for (int a = 0; a < 3; a++) { plo[a] = lo[a]; phi[a] = hi[a]; }
            if (done) break;
            // the merged entries seed lane 0's list for the next shell
#pragma unroll
            for (int m = 0; m < KN; m++) {
                double d = __shfl(rd, m);
                int32_t j = __shfl(rj, m), q = __shfl(rq, m);
                kd[m] = lane == 0 && j >= 0 ? d : INFINITY;
                kj[m] = lane == 0 && j >= 0 ? j : 0x7fffffff;
                kq[m] = q;
            }
            found = lane == 0 ? total : 0;
        }
        const int cnt = total < KN ? total : KN;
        if (lane == 0 && shell_exceeds_box(g, cnt, KN, kth)) atomicOr(box_fail, 1);
        if (lane < KN) {
            int32_t j = lane < cnt ? rj : -1;
            double r0 = 0, r1 = 0, r2 = 0;
            if (lane < cnt) {
                r0 = min_image(spos[3 * (int64_t)rq] - xi, g, 0);
                r1 = min_image(spos[3 * (int64_t)rq + 1] - yi, g, 1);
                r2 = min_image(spos[3 * (int64_t)rq + 2] - zi, g, 2);
            }
            nbr_id[(int64_t)lane * n + p] = j;
            nbr_rel[((int64_t)lane * 3 + 0) * n + p] = r0;
            nbr_rel[((int64_t)lane * 3 + 1) * n + p] = r1;
            nbr_rel[((int64_t)lane * 3 + 2) * n + p] = r2;
        }
    }
}

template <int NK>
__global__ void __launch_bounds__(256) k_knn_exact(int64_t n, Grid g, const double *__restrict__ spos,
                                                   const int32_t *__restrict__ sid, const int32_t *__restrict__ start,
                                                   int32_t *__restrict__ nbr_id, double *__restrict__ nbr_rel,
                                                   const int32_t *__restrict__ todo,
                                                   const int32_t *__restrict__ todo_count,
                                                   int32_t *__restrict__ box_fail) {
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t cnt_todo = todo ? (int64_t)*todo_count : n;
    for (int64_t w = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); w < cnt_todo; w += nwaves)
        knn_exact_atom<NK>(todo ? (int64_t)todo[w] : w, n, g, spos, sid, start, nbr_id, nbr_rel, box_fail);
}

// ------------------------------------------------- topological ordering
// Sec. 3: neighbours ordered by the area of the interface between the
// Voronoi cell of the centre and theirs, larger first, then by 1/d; the cell
// is that of the centre and its 18 nearest neighbours (Sec. 9).  The cell
// {x : x.n_j <= 1}, n_j = 2 d_j / |d_j|^2, is the polar of the convex hull
// of the points n_j: hull vertices are the cell's faces, each hull facet
// (a, b, c) is a cell vertex w (w.n_a = w.n_b = w.n_c = 1) and hull edges
// are cell edges.  Two kernels, one lane per atom in each:
//   k_voronoi_hull   builds the hull incrementally with exact predicates and
//                    Simulation of Simplicity by Euclidean rank (points
//                    inside the current hull are skipped; vertices that a
//                    later point swallows drop out of every facet) and
//                    writes its facets;
//   k_voronoi_order  reads them back, computes the area of face v as
//                    |sum over the facets f at v of (w_f x w_g) . n_v| /
//                    (2 |n_v|), g being the facet across f's edge that starts
//                    at v (consecutive vertices of the face polygon, in one
//                    direction), and writes the first 14 neighbours in the
//                    topological order.
// The hull keeps FP32 copies of the points in LDS (an exact filter, with the
// FP64 points recomputed from the neighbour vectors when it cannot decide),
// the areas need the FP64 points: splitting the two lets each kernel hold
// only what it reads.  Areas are compared on a grid of 2^-20 of the cell's
// surface, so that equal areas tie whatever their rounding; ties fall to the
// Euclidean rank, i.e. to 1/d.  Atoms with fewer than 18 neighbours, or an
// unbounded cell (the centre not strictly inside the hull), keep the
// Euclidean order: no hull of any subset of their neighbours can then hold
// the centre.
constexpr int VF = 2 * VK - 4;  // facets of a triangulated sphere on 18 vertices
constexpr int VB = 64;          // lanes per block
constexpr double AREA_GRID = 1048576.0;

// 24,320 bytes per 64-lane block: six blocks per CU
struct VHullShared {
    float P[3][VK][VB];  // the points n_j rounded to FP32, component-major, lane-minor
    uint32_t F[VF][VB];  // facets: vertices a | b << 5 | c << 10, link e at 15 + 5 e
    uint16_t H[VK][VB];  // horizon edges of the insertion in progress: a | b << 5 | g << 10
};
// 35,840 bytes per 64-lane block
struct VAreaShared {
    double P[3][VK][VB];  // the points n_j
    uint32_t F[VF][VB];
};

__device__ inline uint32_t vpack(int a, int b, int c, int g0, int g1, int g2) {
    return (uint32_t)a | ((uint32_t)b << 5) | ((uint32_t)c << 10) | ((uint32_t)g0 << 15) | ((uint32_t)g1 << 20) |
           ((uint32_t)g2 << 25);
}
__device__ inline int vv(uint32_t f, int e) { return (f >> (5 * e)) & 31; }
__device__ inline int vl(uint32_t f, int e) { return (f >> (15 + 5 * e)) & 31; }
// position of vertex x in facet f (f must hold x)
__device__ inline int vpos(uint32_t f, int x) { return vv(f, 0) == x ? 0 : (vv(f, 1) == x ? 1 : 2); }
__device__ inline int field5(uint64_t lo, uint64_t hi, int v) {
    return (int)((v < 12 ? lo >> (5 * v) : hi >> (5 * (v - 12))) & 31);
}
__device__ inline void set5(uint64_t &lo, uint64_t &hi, int v, int s) {
    if (v < 12) lo |= (uint64_t)s << (5 * v);
    else hi |= (uint64_t)s << (5 * (v - 12));
}

// n_j = d_j * (2 / |d_j|^2) from the neighbour vectors: the one definition
// of the FP64 points, used by both kernels
__device__ inline void dual_point(const double *__restrict__ rel18, int64_t n, int64_t p, int j, double (&x)[3]) {
    const double a = rel18[((int64_t)j * 3 + 0) * n + p], b = rel18[((int64_t)j * 3 + 1) * n + p],
                 c = rel18[((int64_t)j * 3 + 2) * n + p];
    const double sc = 2.0 / ((a * a + b * b) + c * c);
    x[0] = a * sc;
    x[1] = b * sc;
    x[2] = c * sc;
}

struct VLane {
    VHullShared &S;
    int t;
    const double *__restrict__ rel18;
    int64_t n, p;
    double bo, bd;      // FP32 filter bounds of this lane's points
    double bo64, bd64;  // FP64 filter bounds
    __device__ void load(int j, float (&x)[3]) const {
        x[0] = S.P[0][j][t];
        x[1] = S.P[1][j][t];
        x[2] = S.P[2][j][t];
    }
    // where the FP32 filter cannot decide: the FP64 filter, then exact
    // arithmetic with SoS
    __device__ int orient_exact(int a, int b, int c, int q) const {
        double da[3], db[3], dc[3], dq[3];
        dual_point(rel18, n, p, a, da);
        dual_point(rel18, n, p, b, db);
        dual_point(rel18, n, p, c, dc);
        dual_point(rel18, n, p, q, dq);
        return orient_sos64b(da, db, dc, dq, a, b, c, q, bo64);
    }
    __device__ int orient(int a, int b, int c, const float (&pq)[3], int q) const {
        float pa[3], pb[3], pc[3];
        load(a, pa);
        load(b, pb);
        load(c, pc);
        const int s = orient_filter_f32in(pa, pb, pc, pq, bo);
        return s ? s : orient_exact(a, b, c, q);
    }
    __device__ int det3(uint32_t f) const {
        float pa[3], pb[3], pc[3];
        load(vv(f, 0), pa);
        load(vv(f, 1), pb);
        load(vv(f, 2), pc);
        const int s = det3_filter_f32in(pa, pb, pc, bd);
        if (s) return s;
        double da[3], db[3], dc[3];
        dual_point(rel18, n, p, vv(f, 0), da);
        dual_point(rel18, n, p, vv(f, 1), db);
        dual_point(rel18, n, p, vv(f, 2), dc);
        return det3_sign64b(da, db, dc, bd64);
    }
};

// the cell vertex of the facet (a, b, c): w.n_a = w.n_b = w.n_c = 1, i.e.
// (n_b x n_c + n_c x n_a + n_a x n_b) / det[n_a; n_b; n_c]
__device__ inline void cell_vertex(const double (&a)[3], const double (&b)[3], const double (&c)[3], double (&w)[3]) {
#pragma clang fp contract(fast)
    const double bc0 = b[1] * c[2] - b[2] * c[1], bc1 = b[2] * c[0] - b[0] * c[2], bc2 = b[0] * c[1] - b[1] * c[0];
    const double ca0 = c[1] * a[2] - c[2] * a[1], ca1 = c[2] * a[0] - c[0] * a[2], ca2 = c[0] * a[1] - c[1] * a[0];
    const double ab0 = a[1] * b[2] - a[2] * b[1], ab1 = a[2] * b[0] - a[0] * b[2], ab2 = a[0] * b[1] - a[1] * b[0];
    const double inv = 1.0 / (a[0] * bc0 + a[1] * bc1 + a[2] * bc2);
    w[0] = (bc0 + ca0 + ab0) * inv;
    w[1] = (bc1 + ca1 + ab1) * inv;
    w[2] = (bc2 + ca2 + ab2) * inv;
}

// first tetrahedron of points 0..3, positively oriented; facets 0..3
__device__ inline void vhull_start(const VLane &L) {
    int a = 0, b = 1, c = 2;
    const int d = 3;
    float p3[3];
    L.load(3, p3);
    if (L.orient(0, 1, 2, p3, 3) > 0) { b = 2; c = 1; }
    L.S.F[0][L.t] = vpack(a, b, c, 1, 2, 3);
    L.S.F[1][L.t] = vpack(b, a, d, 0, 3, 2);
    L.S.F[2][L.t] = vpack(c, b, d, 0, 1, 3);
    L.S.F[3][L.t] = vpack(a, c, d, 0, 2, 1);
}

// Insert point p into the hull whose facets are the slots in `live`.  A
// point inside leaves the hull as it is.  New facets take the lowest free
// slots (the visible facets' included).  Returns false on an inconsistent
// hull, which exact predicates never produce.
__device__ inline bool vhull_insert(const VLane &L, int p, uint32_t &live) {
    VHullShared &S = L.S;
    const int t = L.t;
    float pp[3];
    L.load(p, pp);
    uint32_t vis = 0;
    const float bf = (float)L.bo;
    // two facets per step: both filters' loads are issued together.  A facet
    // is visible when its FP32 determinant lies below -bound; the rare one
    // within the bound (or NaN) takes the exact path.
    for (uint32_t m = live; m;) {
        const int f0 = __builtin_ctz(m);
        m &= m - 1;
        const bool two = m != 0;
        const int f1 = two ? __builtin_ctz(m) : f0;
        if (two) m &= m - 1;
        const uint32_t w0 = S.F[f0][t], w1 = S.F[f1][t];
        float a0[3], b0[3], c0[3], a1[3], b1[3], c1[3];
        L.load(vv(w0, 0), a0);
        L.load(vv(w0, 1), b0);
        L.load(vv(w0, 2), c0);
        L.load(vv(w1, 0), a1);
        L.load(vv(w1, 1), b1);
        L.load(vv(w1, 2), c1);
        const float d0 = orient_det_f32in(a0, b0, c0, pp), d1 = orient_det_f32in(a1, b1, c1, pp);
        bool v0 = d0 < -bf, v1 = d1 < -bf;
        if (!(fabsf(d0) > bf)) v0 = L.orient_exact(vv(w0, 0), vv(w0, 1), vv(w0, 2), p) > 0;
        if (two && !(fabsf(d1) > bf)) v1 = L.orient_exact(vv(w1, 0), vv(w1, 1), vv(w1, 2), p) > 0;
        vis |= (v0 ? 1u << f0 : 0u) | (two && v1 ? 1u << f1 : 0u);
    }
    if (!vis) return true;
    // horizon edges (a -> b) of the visible facets whose neighbour g is not
    // visible, one per start vertex: H[a] = b | g << 5.  Inner edges write
    // to row VK - 1, which is no start vertex (a < p <= VK - 1), so the loop
    // body has no branch.
    uint32_t hv = 0, he = 0;      // start and end vertices of the horizon
    uint64_t pr_lo = 0, pr_hi = 0;  // 5-bit field b: a of the horizon edge a -> b
    int nh = 0;
    bool bad = false;
    for (uint32_t m = vis; m; m &= m - 1) {
        const uint32_t w = S.F[__builtin_ctz(m)][t];
#pragma unroll
        for (int e = 0; e < 3; e++) {
            const int g = vl(w, e);
            bad |= !((live >> g) & 1);
            const bool hz = !((vis >> g) & 1);
            const int ha = vv(w, e), hb = vv(w, e == 2 ? 0 : e + 1);
            S.H[hz ? ha : VK - 1][t] = (uint16_t)(hb | (g << 5));
            hv |= (uint32_t)hz << ha;
            he |= (uint32_t)hz << hb;
            set5(pr_lo, pr_hi, hb, hz ? ha : 0);
            nh += hz;
        }
    }
    // the horizon is one cycle: an edge leaves and one enters every vertex
    if (bad || __builtin_popcount(hv) != nh || he != hv) return false;
    // slots in increasing order of the start vertex; the new facet (a, b, p)
    // links to g across a -> b, to the facet of b across b -> p and to the
    // facet of pred(a) across p -> a
    const uint32_t freeset = ~(live & ~vis);
    uint64_t sl_lo = 0, sl_hi = 0;  // 5-bit slot per start vertex
    uint32_t fr = freeset, added = 0;
    for (uint32_t m = hv; m; m &= m - 1) {
        if (!fr) return false;
        const int s = __builtin_ctz(fr);
        fr &= fr - 1;
        added |= 1u << s;
        set5(sl_lo, sl_hi, __builtin_ctz(m), s);
    }
    for (uint32_t m = hv; m; m &= m - 1) {
        const int a = __builtin_ctz(m);
        const uint32_t hw = S.H[a][t];
        const int b = hw & 31, g = (hw >> 5) & 31;
        const int sa = field5(sl_lo, sl_hi, a);
        S.F[sa][t] = vpack(a, b, p, g, field5(sl_lo, sl_hi, b), field5(sl_lo, sl_hi, field5(pr_lo, pr_hi, a)));
        // g holds the edge b -> a; its link there now points to sa
        const uint32_t gw = S.F[g][t];
        const int eg = vpos(gw, b);
        S.F[g][t] = (gw & ~(31u << (15 + 5 * eg))) | ((uint32_t)sa << (15 + 5 * eg));
    }
    live = (live & ~vis) | added;
    return true;
}

// Squared distance from the origin of the closest facet plane of a hull
// that holds the origin, from the FP64 points, lowered by a relative 1e-6
// (far above the rounding of the evaluation): a point closer to the origin
// than this is strictly inside the hull, and so inside every later (larger)
// hull.  -1 when the origin is not inside.
__device__ inline double vhull_inradius2(const VLane &L, uint32_t live) {
    double r2 = INFINITY;
    // four facets per step (the first one again where fewer are left), so
    // that their 36 loads are in flight together
    for (uint32_t m = live; m;) {
        int f[4];
        f[0] = __builtin_ctz(m);
        m &= m - 1;
#pragma unroll
        for (int k = 1; k < 4; k++) {
            f[k] = m ? __builtin_ctz(m) : f[0];
            m &= m - 1;
        }
        double a[4][3], b[4][3], c[4][3];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t w = L.S.F[f[k]][L.t];
            dual_point(L.rel18, L.n, L.p, vv(w, 0), a[k]);
            dual_point(L.rel18, L.n, L.p, vv(w, 1), b[k]);
            dual_point(L.rel18, L.n, L.p, vv(w, 2), c[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double u0 = b[k][0] - a[k][0], u1 = b[k][1] - a[k][1], u2 = b[k][2] - a[k][2];
            const double v0 = c[k][0] - a[k][0], v1 = c[k][1] - a[k][1], v2 = c[k][2] - a[k][2];
            const double n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
            const double h = n0 * a[k][0] + n1 * a[k][1] + n2 * a[k][2];
            if (!(h > 0)) return -1.0;  // the origin is not inside: no bound
            r2 = fmin(r2, h * h / ((n0 * n0 + n1 * n1) + n2 * n2));
        }
    }
    return r2 * (1.0 - 1e-6);
}

// Hull of the 18 points of each atom; facets to vf[f][n] (slots in the
// 32-bit mask vlive[n], 0 when the atom keeps its Euclidean order).
__global__ void __launch_bounds__(VB) k_voronoi_hull(int64_t n, const double *__restrict__ rel18,
                                                     const int32_t *__restrict__ id18, uint32_t *__restrict__ vf,
                                                     uint32_t *__restrict__ vlive,
                                                     const int32_t *__restrict__ box_fail) {
    __shared__ VHullShared S;
    const int t = threadIdx.x;
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * (int64_t)VB + t;
    if (p >= n || *box_fail) return;
    bool topo = id18[(int64_t)(VK - 1) * n + p] >= 0;
    float m = 0;
    uint32_t hk[VK];  // a mix of each point's FP32 bits: equal points have equal keys
    double nrm2[VK - 12];  // |n_q|^2 of points 12..17 (the inradius skip below)
#pragma unroll
    for (int v = 0; v < VK; v++) {
        double x[3];
        dual_point(rel18, n, p, v, x);
        if (v >= 12) nrm2[v - 12] = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
        // a neighbour at the centre has no bisector plane (its point is not
        // finite): the atom keeps its Euclidean order
        topo = topo && isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
        uint32_t h = 0;
        for (int d = 0; d < 3; d++) {
            const float xf = (float)x[d];
            S.P[d][v][t] = xf;
            m = fmaxf(m, fabsf(xf));
            h = h * 0x9E3779B1u + __float_as_uint(xf);
        }
        hk[v] = h;
    }
    // two coincident neighbours share one bisector plane: no interface
    // belongs to either alone, and the atom keeps its Euclidean order (equal
    // keys first, then the FP32 copies, then the FP64 vectors)
    bool maybe = false;
#pragma unroll
    for (int j = 0; j < VK - 1; j++)
#pragma unroll
        for (int k = j + 1; k < VK; k++) maybe = maybe || hk[j] == hk[k];
    if (maybe && topo)
        for (int j = 0; j < VK - 1 && topo; j++)
            for (int k = j + 1; k < VK && topo; k++)
                if (S.P[0][j][t] == S.P[0][k][t] && S.P[1][j][t] == S.P[1][k][t] && S.P[2][j][t] == S.P[2][k][t]) {
                    bool same = true;
                    for (int d = 0; d < 3; d++)
                        same = same && rel18[((int64_t)j * 3 + d) * n + p] == rel18[((int64_t)k * 3 + d) * n + p];
                    topo = !same;
                }
    uint32_t live = 0;
    if (topo) {
        double m64 = 0;
        for (int v = 0; v < VK; v++)
            for (int d = 0; d < 3; d++) m64 = fmax(m64, fabs((double)S.P[d][v][t]));
        // the FP64 bounds from the largest coordinate of the FP32 copies, widened to cover the rounding
        m64 *= 1.0 + 0x1p-22;
        VLane L{S, t, rel18, n, p, f32_orient_bound(m), f32_det3_bound(m), f64_orient_bound(m64),
                f64_det3_bound(m64)};
        vhull_start(L);
        live = 0xFu;
        double rin2 = -1.0;  // inradius bound of the 12-point hull
        for (int q = 4; q < VK && topo; q++) {
            if (q == 12) rin2 = vhull_inradius2(L, live);
            if (q >= 12 && rin2 > 0 && nrm2[q - 12] < rin2) continue;  // strictly inside
            topo = vhull_insert(L, q, live);
        }
        // the centre strictly inside every facet
        for (uint32_t mm = live; mm && topo; mm &= mm - 1) topo = L.det3(S.F[__builtin_ctz(mm)][t]) > 0;
        if (!topo) live = 0;
        for (uint32_t mm = live; mm; mm &= mm - 1) {
            const int f = __builtin_ctz(mm);
            vf[(int64_t)f * n + p] = S.F[f][t];
        }
    }
    vlive[p] = live;
}

// Areas, keys and the topological order from the facets of k_voronoi_hull.
__global__ void __launch_bounds__(VB) k_voronoi_order(int64_t n, const double *__restrict__ rel18,
                                                      const int32_t *__restrict__ id18,
                                                      const uint32_t *__restrict__ vf,
                                                      const uint32_t *__restrict__ vlive,
                                                      double *__restrict__ nbr_rel, int32_t *__restrict__ nbr_id,
                                                      const int32_t *__restrict__ box_fail) {
#pragma clang fp contract(fast)
    __shared__ VAreaShared S;
    const int t = threadIdx.x;
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * (int64_t)VB + t;
    if (p >= n || *box_fail) return;
    // Euclidean rank v goes to row pos(v); keys order (grid area descending, rank)
    uint32_t key[VK];
#pragma unroll
    for (int v = 0; v < VK; v++) key[v] = (uint32_t)v;
    const uint32_t live = vlive[p];
    if (live) {
        // every load is issued before any is used (one wave per SIMD: no
        // other wave hides a chain of round trips): all VF facet rows (each
        // exists; dead slots are read and ignored) and the points
        uint32_t fw[VF];
#pragma unroll
        for (int f = 0; f < VF; f++) fw[f] = vf[(int64_t)f * n + p];
#pragma unroll
        for (int v = 0; v < VK; v++) {
            double x[3];
            dual_point(rel18, n, p, v, x);
            S.P[0][v][t] = x[0];
            S.P[1][v][t] = x[1];
            S.P[2][v][t] = x[2];
        }
        // one facet at each vertex: 5-bit fields, 31 = not a vertex (a
        // vertex has at least three facets, so slot 31 is never needed)
        uint64_t at_lo = ~0ull, at_hi = ~0ull;
#pragma unroll
        for (int f = 0; f < VF; f++) {
            if (!((live >> f) & 1)) continue;
            const uint32_t w = fw[f];
            S.F[f][t] = w;
            if (f == 31) continue;
            for (int e = 0; e < 3; e++) {
                const int x = vv(w, e);
                if (x < 12) at_lo = (at_lo & ~(31ull << (5 * x))) | ((uint64_t)f << (5 * x));
                else at_hi = (at_hi & ~(31ull << (5 * (x - 12)))) | ((uint64_t)f << (5 * (x - 12)));
            }
        }
        auto load = [&](int j, double (&x)[3]) {
            x[0] = S.P[0][j][t];
            x[1] = S.P[1][j][t];
            x[2] = S.P[2][j][t];
        };
        // face v: walk the facets around v (each next one across the edge
        // that starts at v), summing w_f x w_next; every step brings one new
        // point, the facet's vertex after v
        double area[VK], tot = 0;
#pragma unroll
        for (int v = 0; v < VK; v++) {
            area[v] = 0;
            const int f0 = field5(at_lo, at_hi, v);
            if (f0 == 31) continue;
            double nv[3], a[3], b[3], w0[3], wp[3];
            load(v, nv);
            uint32_t w = S.F[f0][t];
            int e = vpos(w, v);
            load(vv(w, e == 2 ? 0 : e + 1), a);
            load(vv(w, e == 0 ? 2 : e - 1), b);
            cell_vertex(nv, a, b, w0);
            wp[0] = w0[0]; wp[1] = w0[1]; wp[2] = w0[2];
            double sx = 0, sy = 0, sz = 0;
            for (int step = 0; step < VF; step++) {
                const int g = vl(w, e);
                double wn[3];
                if (g == f0) {
                    wn[0] = w0[0]; wn[1] = w0[1]; wn[2] = w0[2];
                } else {
                    const uint32_t gw = S.F[g][t];
                    const int eg = vpos(gw, v);
                    // in g the edge v -> (previous successor) is reversed: the new point follows v
                    double c[3];
                    load(vv(gw, eg == 2 ? 0 : eg + 1), c);
                    cell_vertex(nv, c, a, wn);
                    a[0] = c[0]; a[1] = c[1]; a[2] = c[2];
                    w = gw;
                    e = eg;
                }
                sx += wp[1] * wn[2] - wp[2] * wn[1];
                sy += wp[2] * wn[0] - wp[0] * wn[2];
                sz += wp[0] * wn[1] - wp[1] * wn[0];
                wp[0] = wn[0]; wp[1] = wn[1]; wp[2] = wn[2];
                if (g == f0) break;
            }
            area[v] = fabs(sx * nv[0] + sy * nv[1] + sz * nv[2]) /
                      (2.0 * sqrt((nv[0] * nv[0] + nv[1] * nv[1]) + nv[2] * nv[2]));
            tot += area[v];
        }
        if (tot > 0) {
#pragma unroll
            for (int v = 0; v < VK; v++) {
                const double x = area[v] / tot * AREA_GRID;
                const uint32_t q = (uint32_t)fmin(fmax(floor(x), 0.0), AREA_GRID);
                key[v] = (((uint32_t)AREA_GRID - q) << 5) | (uint32_t)v;
            }
        }
    }
    int pos[VK];
#pragma unroll
    for (int v = 0; v < VK; v++) {
        pos[v] = 0;
#pragma unroll
        for (int u = 0; u < VK; u++) pos[v] += key[u] < key[v];
    }
    // output row by output row, so that the lanes of a wave write each row
    // together (whole cache lines); the source row differs per lane
    for (int m = 0; m < KMAX; m++) {
        int src = 0;
#pragma unroll
        for (int v = 0; v < VK; v++) src = pos[v] == m ? v : src;
        nbr_id[(int64_t)m * n + p] = id18[(int64_t)src * n + p];
#pragma unroll
        for (int c = 0; c < 3; c++) nbr_rel[((int64_t)m * 3 + c) * n + p] = rel18[((int64_t)src * 3 + c) * n + p];
    }
}

// --------------------------------------------------------------- topology
// One incremental convex hull per atom over its 14 nearest neighbours in
// rank order (every point must become a vertex and stay one), with facets
// and neighbour links.  The hull of the first k points is a state of that
// same construction, so the 6-, 12- and 14-point hulls are read off it
// after inserting points 5, 11 and 13: for each, the centre must lie
// strictly inside, then the rotation system and the canonical start-edge
// code are built and looked up.  Per-lane state lives in LDS, lane-minor,
// so dynamic indices never conflict across lanes.
constexpr int TB = 64;  // threads per block of the topology kernel

// LDS of one block.  P: the neighbour vectors rounded to FP32 (the input of
// the predicate filters; every predicate is decided exactly, so both
// precision forms use this kernel); F: facets; H: the horizon of the
// current insertion.  The rotation system of the 12-point hull, built
// between insertions, packs into H and the four facet slots that hull
// leaves free (F[20..23], which H follows in memory); the 14-point hull is
// the last, and its rotation system takes the space of P, which is no
// longer read.  20,480 bytes: eight blocks per CU.
struct TopoShared {
    float P[3][KMAX][TB];
    uint32_t F[2 * KMAX - 4][TB];
    uint32_t H[KMAX][TB];
};
static_assert(sizeof(float) * 3 * KMAX >= sizeof(uint64_t) * KMAX, "a 14-row rotation system fits in P");
static_assert(offsetof(TopoShared, H) == offsetof(TopoShared, F) + sizeof(uint32_t) * (2 * KMAX - 4) * TB,
              "H follows F");
static_assert(sizeof(TopoShared) == 20480, "eight blocks of the topology kernel per CU");

// A lane's rotation system: row x maps each neighbour y (nibble y) to the
// vertex after y counter-clockwise around x (0xF: not a neighbour).  Rows
// are kept complemented (0 = no neighbour), so they are built by atomic ORs
// that need no read-modify-write round trips.
// Rows of 16 nibbles, one 64-bit word each (the 14-point hull, in P):
struct RotSys {
    uint64_t (*w)[TB];
    int t;
    __device__ void clear(int k) const {
        for (int x = 0; x < k; x++) w[x][t] = 0;
    }
    __device__ void set_next(int x, int y, int z) const {
        atomicOr((unsigned long long *)&w[x][t], (unsigned long long)(z ^ 0xF) << (4 * y));
    }
    __device__ uint64_t get(int x) const { return ~w[x][t]; }
};
// Rows of 12 nibbles packed into 18 consecutive 32-bit words (the 12-point
// hull: row x starts at bit 48 x, so it spans two words and starts at bit
// 0 or 16 of the first):
struct RotSys12 {
    uint32_t (*w)[TB];
    int t;
    __device__ void clear(int) const {
        for (int i = 0; i < 18; i++) w[i][t] = 0;
    }
    __device__ void set_next(int x, int y, int z) const {
        const int bit = 48 * x + 4 * y;
        atomicOr(&w[bit >> 5][t], (uint32_t)(z ^ 0xF) << (bit & 31));
    }
    __device__ uint64_t get(int x) const {
        const int i = (48 * x) >> 5, sh = (48 * x) & 31;
        const uint64_t two = ((uint64_t)w[i + 1][t] << 32) | w[i][t];
        return ~((two >> sh) & 0xFFFFFFFFFFFFull);  // nibbles 12..15 read as no neighbour
    }
};

// facet word: v0 | v1<<4 | v2<<8 | nb0<<12 | nb1<<17 | nb2<<22
__device__ inline uint32_t fpack(int a, int b, int c, int n0, int n1, int n2) {
    return (uint32_t)a | ((uint32_t)b << 4) | ((uint32_t)c << 8) | ((uint32_t)n0 << 12) | ((uint32_t)n1 << 17) |
           ((uint32_t)n2 << 22);
}
__device__ inline int fv(uint32_t f, int e) { return (f >> (4 * e)) & 0xF; }
__device__ inline int fn(uint32_t f, int e) { return (f >> (12 + 5 * e)) & 0x1F; }
__device__ inline uint32_t fset_nb(uint32_t f, int e, int g) {
    int sh = 12 + 5 * e;
    return (f & ~(0x1Fu << sh)) | ((uint32_t)g << sh);
}

// Per-lane view of the hull inputs: LDS points plus the FP64 originals in
// global memory (used when an FP32 filter cannot decide), and the static
// filter bounds of the atom (from its largest neighbour coordinate).
struct Lane {
    TopoShared &S;
    int t;
    const double *__restrict__ rel;
    int64_t n, p;
    double bo, bd;        // FP32 filter bounds of orient and det3
    double bo64, bd64;    // FP64 filter bounds (the fallback)
    __device__ void load64(int r, double (&x)[3]) const {
        for (int d = 0; d < 3; d++) x[d] = rel[((int64_t)r * 3 + d) * n + p];
    }
    __device__ void load(int r, float (&x)[3]) const {
        for (int d = 0; d < 3; d++) x[d] = S.P[d][r][t];
    }
};

// orientation of facet (a,b,c) against point q where the FP32 filter
// cannot decide: the FP64 filter, then exact arithmetic with SoS
__device__ inline int lane_orient_exact(const Lane &L, int a, int b, int c, int q) {
    double da[3], db[3], dc[3], dq[3];
    L.load64(a, da);
    L.load64(b, db);
    L.load64(c, dc);
    L.load64(q, dq);
    return orient_sos64b(da, db, dc, dq, a, b, c, q, L.bo64);
}

// det[a; b; c] sign where the FP32 filter cannot decide
__device__ inline int lane_det3_exact(const Lane &L, int a, int b, int c) {
    double da[3], db[3], dc[3];
    L.load64(a, da);
    L.load64(b, db);
    L.load64(c, dc);
    return det3_sign64b(da, db, dc, L.bd64);
}

// orientation of facet (a,b,c) against point q (held in registers)
__device__ inline int lane_orient(const Lane &L, int a, int b, int c, const float (&pq)[3], int q) {
    float pa[3], pb[3], pc[3];
    L.load(a, pa);
    L.load(b, pb);
    L.load(c, pc);
    const int s = orient_filter_f32in(pa, pb, pc, pq, L.bo);
    return s ? s : lane_orient_exact(L, a, b, c, q);
}

// first tetrahedron of points 0..3, positively oriented; facets 0..3
__device__ inline void lane_hull_start(const Lane &L) {
    TopoShared &S = L.S;
    const int t = L.t;
    int a = 0, b = 1, c = 2, d = 3;
    float p3[3];
    L.load(3, p3);
    if (lane_orient(L, 0, 1, 2, p3, 3) > 0) { b = 2; c = 1; }
    S.F[0][t] = fpack(a, b, c, 1, 2, 3);
    S.F[1][t] = fpack(b, a, d, 0, 3, 2);
    S.F[2][t] = fpack(c, b, d, 0, 1, 3);
    S.F[3][t] = fpack(a, c, d, 0, 2, 1);
}

// Insert point p into the hull of points 0..p-1 (nf = 2p - 4 facets).
// Returns 0 if p lies inside (it never becomes a vertex) or swallows an
// earlier vertex: then no hull of p or more points is valid.  cv: facet
// slots whose centre test has passed; the slots rewritten here leave it.
__device__ int lane_insert(const Lane &L, int p, uint32_t &cv) {
    TopoShared &S = L.S;
    const int t = L.t;
    const int nf = 2 * p - 4;
    uint32_t vis = 0;
    float pp[3];
    L.load(p, pp);
    const float bf = (float)L.bo;
    // two facets per step (nf is even): both filters' loads are issued
    // together.  A facet is visible when its FP32 determinant lies below
    // -bound; the rare one within the bound (or NaN) takes the exact path.
    for (int f = 0; f < nf; f += 2) {
        const uint32_t w0 = S.F[f][t], w1 = S.F[f + 1][t];
        float a0[3], b0[3], c0[3], a1[3], b1[3], c1[3];
        L.load(fv(w0, 0), a0);
        L.load(fv(w0, 1), b0);
        L.load(fv(w0, 2), c0);
        L.load(fv(w1, 0), a1);
        L.load(fv(w1, 1), b1);
        L.load(fv(w1, 2), c1);
        const float d0 = orient_det_f32in(a0, b0, c0, pp), d1 = orient_det_f32in(a1, b1, c1, pp);
        bool v0 = d0 < -bf, v1 = d1 < -bf;
        if (!(fabsf(d0) > bf)) v0 = lane_orient_exact(L, fv(w0, 0), fv(w0, 1), fv(w0, 2), p) > 0;
        if (!(fabsf(d1) > bf)) v1 = lane_orient_exact(L, fv(w1, 0), fv(w1, 1), fv(w1, 2), p) > 0;
        vis |= (v0 ? 1u << f : 0u) | (v1 ? 2u << f : 0u);
    }
    if (vis == 0) return 0;  // p inside: never a vertex
    const int nvis = __builtin_popcount(vis);
    // horizon edges (a -> b) of the visible facets f whose neighbour g is
    // not visible, one per start vertex: H[a] = b | g << 4 | f << 9.  Inner
    // edges write to row KMAX - 1, which is no start vertex (a < p <=
    // KMAX - 1), so the loop body has no branch.
    uint32_t hv = 0, he = 0;  // start and end vertices of the horizon
    uint64_t pred = 0;        // nibble b: a of the horizon edge a -> b
    int nh = 0;
    bool bad = false;
    for (uint32_t vm = vis; vm; vm &= vm - 1) {  // visible facets only
        const int f = __builtin_ctz(vm);
        const uint32_t w = S.F[f][t];
#pragma unroll
        for (int e = 0; e < 3; e++) {
            const int g = fn(w, e);
            bad |= g >= nf;  // broken link (cannot happen with exact predicates)
            const bool hz = !((vis >> g) & 1);
            const int ha = fv(w, e), hb = fv(w, e == 2 ? 0 : e + 1);
            S.H[hz ? ha : KMAX - 1][t] = (uint32_t)hb | ((uint32_t)g << 4) | ((uint32_t)f << 9);
            hv |= (uint32_t)hz << ha;
            he |= (uint32_t)hz << hb;
            pred |= (uint64_t)(hz ? ha : 0) << (4 * hb);
            nh += hz;
        }
    }
    // a horizon of nvis+2 edges <=> no earlier vertex is swallowed; one
    // edge leaves and one enters every horizon vertex
    if (bad || nh != nvis + 2 || __builtin_popcount(hv) != nh || he != hv) return 0;
    // slots: freed visible facets first (increasing), then two new ones, in
    // increasing order of the start vertex; then the new facet (a, b, p)
    // links to g across a -> b, to the facet of b across b -> p and to the
    // facet of pred(a) across p -> a, and g's link turns from the visible
    // facet to the new one (an XOR: every link changes at most once, so no
    // read-modify-write is needed)
    uint64_t slo = 0, shi = 0;  // 5-bit slot per start vertex
    uint32_t freed = vis;
    int nf_new = nf;
    for (uint32_t m = hv; m; m &= m - 1) {
        int sl;
        if (freed) {
            sl = __builtin_ctz(freed);
            freed &= freed - 1;
        } else {
            sl = nf_new++;
        }
        set5(slo, shi, __builtin_ctz(m), sl);
    }
    for (uint32_t m = hv; m; m &= m - 1) {
        const int a = __builtin_ctz(m);
        const uint32_t hw = S.H[a][t];
        const int b = hw & 0xF, g = (hw >> 4) & 0x1F, f = (hw >> 9) & 0x1F;
        const int sa = field5(slo, shi, a);
        S.F[sa][t] = fpack(a, b, p, g, field5(slo, shi, b), field5(slo, shi, (int)nib(pred, a)));
        // g (not visible, so never a slot taken here) holds the edge b -> a
        // as its edge eg; only its links may have changed
        const uint32_t gw = S.F[g][t];
        const int eg = (fv(gw, 0) == b) ? 0 : ((fv(gw, 1) == b) ? 1 : 2);
        atomicXor(&S.F[g][t], (uint32_t)(f ^ sa) << (12 + 5 * eg));
    }
    cv &= ~vis;  // the freed slots hold new facets
    return 1;
}

// the centre lies strictly inside every facet of the K-point hull:
// det[a; b; c] > 0 exactly.  Facets in cv passed at a smaller hull and are
// not tested again; on success every facet joins cv.
__device__ inline int lane_centre_inside(const Lane &L, int K, uint32_t &cv) {
    const uint32_t all = (1u << (2 * K - 4)) - 1;
    const float bd = (float)L.bd;
    // two facets per step, as in the insertion
    for (uint32_t m = all & ~cv; m;) {
        const int f0 = __builtin_ctz(m);
        m &= m - 1;
        const int f1 = m ? __builtin_ctz(m) : f0;  // (f0 again when it is the last)
        m &= m - 1;
        const uint32_t w0 = L.S.F[f0][L.t], w1 = L.S.F[f1][L.t];
        float a0[3], b0[3], c0[3], a1[3], b1[3], c1[3];
        L.load(fv(w0, 0), a0);
        L.load(fv(w0, 1), b0);
        L.load(fv(w0, 2), c0);
        L.load(fv(w1, 0), a1);
        L.load(fv(w1, 1), b1);
        L.load(fv(w1, 2), c1);
        // outside below -bound; within the bound (or NaN) the exact path decides
        const float e0 = det3_f32in(a0, b0, c0), e1 = det3_f32in(a1, b1, c1);
        if (e0 < -bd || e1 < -bd) return 0;
        if (!(e0 > bd) && lane_det3_exact(L, fv(w0, 0), fv(w0, 1), fv(w0, 2)) <= 0) return 0;
        if (!(e1 > bd) && lane_det3_exact(L, fv(w1, 0), fv(w1, 1), fv(w1, 2)) <= 0) return 0;
    }
    cv |= all;
    return 1;
}

// Start-edge code (definition in ptm_tables.cpp) of the start edge u -> v
// with u the lowest-numbered vertex of minimum degree and v its
// lowest-numbered neighbour.  code[] receives the K words; the return value
// is the labelling (nibble l = vertex of label l).  One code per hull: the
// tables hold the codes of every start edge from a vertex of minimum degree
// of every template triangulation, so the choice among them needs no
// search.
template <int K, typename RS>
__device__ uint64_t lane_start_edge_code(const RS &NT, uint64_t degs, uint64_t (&code)[K]) {
    int mindeg = 15;
#pragma unroll
    for (int x = 0; x < K; x++) mindeg = min(mindeg, (int)nib(degs, x));
    uint32_t mdmask = 0;
#pragma unroll
    for (int x = 0; x < K; x++) mdmask |= (uint32_t)(nib(degs, x) == (uint32_t)mindeg) << x;
    const int bu = __builtin_ctz(mdmask);
    const uint64_t ntu = NT.get(bu);
    // lowest-numbered neighbour: first nibble of ntu that is not 0xF
    uint64_t z = ~ntu;
    z = (z | (z >> 1) | (z >> 2) | (z >> 3)) & 0x1111111111111111ull;
    const int bv = __builtin_ctzll(z) >> 2;
    // every nibble below is written once, from 0xF (lab) or 0 (ord, par, the
    // signature), so a single XOR or OR sets it
    uint64_t lab = ~0ull ^ (0xFull << (4 * bu)), ord = (uint64_t)bu, par = 0;
    uint64_t sig = (uint64_t)mindeg << 60;
    int y = bv;
    for (int j = 0; j < mindeg; j++) {
        lab ^= (uint64_t)(0xF ^ (j + 1)) << (4 * y);
        ord |= (uint64_t)y << (4 * (j + 1));
        par |= (uint64_t)bu << (4 * y);
        sig |= (uint64_t)nib(degs, y) << (56 - 4 * j);
        y = (int)nib(ntu, y);
    }
    code[0] = sig;
    uint32_t nl = mindeg + 1;
#pragma unroll
    for (int i = 1; i < K; i++) {
        int x = min((int)nib(ord, i), K - 1);
        int yy = (int)nib(par, x);
        uint64_t ntx = NT.get(x);
        int dx = (int)nib(degs, x);
        uint64_t row = (uint64_t)dx << 60;
        for (int j = 0; j < dx; j++) {
            uint32_t ly = nib(lab, yy);
            if (ly == 0xF) {
                ly = nl;
                lab ^= (uint64_t)(0xF ^ nl) << (4 * yy);
                ord |= (uint64_t)yy << (4 * nl);
                par |= (uint64_t)x << (4 * yy);
                nl++;
            }
            row |= (uint64_t)ly << (56 - 4 * j);
            yy = min((int)nib(ntx, yy), K - 1);
        }
        code[i] = row;
    }
    return ord;
}

// Rotation system and canonical code of the K-point hull now held in F: the
// K code words into best, the labelling into ordw; returns the code's hash
// (the table probe comes after the last insertion).
template <int K, typename RS>
__device__ uint64_t lane_code(const uint32_t (*F)[TB], const RS &NT, uint64_t (&best)[K], uint64_t &ordw) {
    const int t = NT.t;
    // every (x, y) nibble is written once
    uint64_t degs = 0;
    NT.clear(K);
    for (int f = 0; f < 2 * K - 4; f++) {
        uint32_t w = F[f][t];
        int a = fv(w, 0), b = fv(w, 1), c = fv(w, 2);
        NT.set_next(a, b, c);
        NT.set_next(b, c, a);
        NT.set_next(c, a, b);
        degs += (1ull << (4 * a)) + (1ull << (4 * b)) + (1ull << (4 * c));
    }
    ordw = lane_start_edge_code<K>(NT, degs, best);
    return code_hash(best, K);
}

// The 6-point hull: the only template triangulation of six points is the
// SC octahedron, and a triangulated sphere of six vertices is the
// octahedron exactly when every vertex has degree 4; the tables hold its one
// start-edge code (code 0 of the group; they refuse to build otherwise).  So
// the hull either is the octahedron -- code 0, with the labelling of the
// start edge from vertex 0 to its lowest-numbered neighbour read off the
// rotation around vertex 0: that neighbour, the next three counter-clockwise,
// then the one vertex not adjacent to 0 -- or has no candidate.  Only vertex
// 0's row of the rotation system is needed, built in a register.
__device__ inline bool lane_octahedron(const uint32_t (*F)[TB], int t, uint64_t &ordw) {
    uint64_t degs = 0, row = 0;  // row 0, complemented (0 = no neighbour)
#pragma unroll
    for (int f = 0; f < 8; f++) {
        const uint32_t w = F[f][t];
        const int a = fv(w, 0), b = fv(w, 1), c = fv(w, 2);
        degs += (1ull << (4 * a)) + (1ull << (4 * b)) + (1ull << (4 * c));
        if (a == 0) row |= (uint64_t)(c ^ 0xF) << (4 * b);
        if (b == 0) row |= (uint64_t)(a ^ 0xF) << (4 * c);
        if (c == 0) row |= (uint64_t)(b ^ 0xF) << (4 * a);
    }
    if (degs != 0x444444ull) return false;
    const uint64_t nt0 = ~row;
    uint64_t z = row;
    z = (z | (z >> 1) | (z >> 2) | (z >> 3)) & 0x1111111111111111ull;
    int y = __builtin_ctzll(z) >> 2;  // lowest-numbered neighbour of 0
    uint64_t ord = 0;
    int sum = 0;
#pragma unroll
    for (int j = 1; j <= 4; j++) {
        ord |= (uint64_t)y << (4 * j);
        sum += y;
        y = (int)nib(nt0, y);
    }
    ordw = ord | ((uint64_t)(15 - sum) << 20);  // the vertices 0..5 sum to 15
    return true;
}

// code row c of group grp equals best (all K words compared)
template <int K>
__device__ inline bool row_equal(const TablesView &T, int grp, int32_t c, const uint64_t (&best)[K]) {
    const uint64_t *cw = T.codes[grp] + (int64_t)c * K;
    uint64_t diff = 0;
#pragma unroll
    for (int i = 0; i < K; i++) diff |= cw[i] ^ best[i];
    return diff == 0;
}

// Table probe of a code of group grp whose first slot s held c: the code id
// (full-code verification), or -1 when no template triangulation has it.
template <int K>
__device__ int32_t probe_rest(const TablesView &T, int grp, const uint64_t (&best)[K], int s, int32_t c, bool hit) {
    const int mask = T.hmask[grp];
    for (int probe = 0; probe <= mask; probe++) {
        if (c < 0) return -1;
        if (hit) return c;
        s = (s + 1) & mask;
        c = T.slots[grp][s];
        hit = c >= 0 && row_equal<K>(T, grp, c, best);
    }
    return -1;
}

// One lane per atom: the hulls of the first 6, 12 and 14 neighbours (those
// enabled by need: bit g for hull group g), code ids and labellings into
// code_out / ord_out [group][n] (-1 / 0 for a group without a valid hull or
// not needed).
// One atom p per lane t of a 64-lane wave, with the wave's LDS S (always
// inlined: the LDS accesses must stay LDS instructions).
__device__ __attribute__((always_inline)) inline void topo_atom(TopoShared &S, int t, int64_t p, int64_t n, const double *__restrict__ nbr_rel,
                          const int32_t *__restrict__ nbr_id, const TablesView &T, uint32_t need,
                          int32_t *__restrict__ code_out, uint64_t *__restrict__ ord_out) {
    // the neighbour ids that say which hulls are possible (the K-th neighbour
    // exists) and all KMAX relative vectors are loaded in one round trip;
    // rows past the last wanted one are stored but never read
    int32_t kid[NGRP];
    for (int g = 0; g < NGRP; g++) kid[g] = nbr_id[(int64_t)(group_k(g) - 1) * n + p];
    double x[KMAX][3];
    for (int r = 0; r < KMAX; r++)
        for (int d = 0; d < 3; d++) x[r][d] = nbr_rel[((int64_t)r * 3 + d) * n + p];
    uint32_t want = 0;
    for (int g = 0; g < NGRP; g++)
        if (((need >> g) & 1) && kid[g] >= 0) want |= 1u << g;
    int32_t cid[NGRP] = {-1, -1, -1};
    uint64_t ordw[NGRP] = {0, 0, 0};
    if (want) {
        const int kl = (want & 4) ? 14 : ((want & 2) ? 12 : 6);  // last point to insert
        // The first six points go to LDS first: their loads were issued
        // first, so the 6-point hull is built while the others arrive.  The
        // filter bounds come from the largest coordinate (FP64, and of its
        // stored form) of the points inserted so far, which bounds every
        // predicate on them.
        double m64 = 0;
        float m32 = 0;
        for (int r = 0; r < 6; r++)
            for (int d = 0; d < 3; d++) {
                S.P[d][r][t] = (float)x[r][d];
                m64 = fmax(m64, fabs(x[r][d]));
                m32 = fmaxf(m32, fabsf((float)x[r][d]));
            }
        Lane L{S, t, nbr_rel, n, p, f32_orient_bound(m32), f32_det3_bound(m32), f64_orient_bound(m64),
               f64_det3_bound(m64)};
        lane_hull_start(L);
        const RotSys12 nt{&S.F[2 * 12 - 4], t};
        const RotSys nt14{reinterpret_cast<uint64_t (*)[TB]>(&S.P[0][0][0]), t};
        // codes of the valid hulls, probed together after the last insertion
        uint64_t c12[12] = {}, c14[14] = {}, h[NGRP] = {0, 0, 0};
        bool pend[NGRP] = {false, false, false};
        uint32_t cv = 0;  // facet slots whose centre test passed
        bool ok = lane_insert(L, 4, cv) && lane_insert(L, 5, cv);
        if (ok && (want & 1))
            pend[0] = lane_centre_inside(L, 6, cv) && lane_octahedron(S.F, t, ordw[0]);
        // the other points (rows past the last wanted one are stored but
        // never read)
        for (int r = 6; r < KMAX; r++)
            for (int d = 0; d < 3; d++) {
                S.P[d][r][t] = (float)x[r][d];
                if (r < kl) {
                    m64 = fmax(m64, fabs(x[r][d]));
                    m32 = fmaxf(m32, fabsf((float)x[r][d]));
                }
            }
        L.bo = f32_orient_bound(m32);
        L.bd = f32_det3_bound(m32);
        L.bo64 = f64_orient_bound(m64);
        L.bd64 = f64_det3_bound(m64);
        for (int q = 6; ok && q < kl; q++) {
            if (!lane_insert(L, q, cv)) break;
            const int K = q + 1;
            if (K == 12 && (want & 2)) {
                if ((pend[1] = lane_centre_inside(L, 12, cv))) h[1] = lane_code<12>(S.F, nt, c12, ordw[1]);
            } else if (K == 14) {
                if ((pend[2] = lane_centre_inside(L, 14, cv))) h[2] = lane_code<14>(S.F, nt14, c14, ordw[2]);
            }
        }
        cid[0] = pend[0] ? 0 : -1;  // the octahedron's code
        // first slots of the other two probes
        int sl[NGRP];
        int32_t c[NGRP];
        for (int g = 1; g < NGRP; g++) {
            sl[g] = (int)(h[g] & (uint64_t)T.hmask[g]);
            c[g] = pend[g] ? T.slots[g][sl[g]] : -1;
        }
        // every group has a code row 0 (the tables refuse to build
        // otherwise): it stands in for a missing hit, so the rows load
        // unconditionally, before any comparison waits
        const bool hit1 = row_equal<12>(T, 1, max(c[1], 0), c12) & (c[1] >= 0);
        const bool hit2 = row_equal<14>(T, 2, max(c[2], 0), c14) & (c[2] >= 0);
        cid[1] = probe_rest<12>(T, 1, c12, sl[1], c[1], hit1);
        cid[2] = probe_rest<14>(T, 2, c14, sl[2], c[2], hit2);
    }
    for (int g = 0; g < NGRP; g++) {
        code_out[(int64_t)g * n + p] = cid[g];
        ord_out[(int64_t)g * n + p] = cid[g] >= 0 ? ordw[g] : 0;
    }
}

__global__ void __launch_bounds__(TB) k_topo(int64_t n, const double *__restrict__ nbr_rel,
                                              const int32_t *__restrict__ nbr_id, TablesView T, uint32_t need,
                                              int32_t *__restrict__ code_out, uint64_t *__restrict__ ord_out,
                                              const int32_t *__restrict__ box_fail) {
    __shared__ TopoShared S;
    const int t = threadIdx.x;
    const int64_t p = blockIdx.x * (int64_t)TB + t;
    if (p >= n || *box_fail) return;
    topo_atom(S, t, p, n, nbr_rel, nbr_id, T, need, code_out, ord_out);
}

// ------------------------------------------------------------------ match
constexpr int MB = 256;  // threads per block of the match kernels

// What the match kernel keeps of each template in LDS: the normalised
// points b (eq. 4), the pseudoinverse V+ (eq. 6), the inverses of the
// rotation group's elements as vertex maps, k and the group order.  The
// group's quaternions are read from the device tables.
struct TemplateGeom {
    double b[NMAX][3];
    double vpinv[3][NMAX];
    uint64_t ginv[GMAX];
    int32_t k, ngroup;
};
struct MatchShared {
    TemplateGeom geo[NT];
};

// rank vector of the representative: min over g of (c(g^-1(m)))_m, packed
// with m = 0 in the most significant nibble.  Only the group elements whose
// first entry is minimal can win, so the full vectors are built for those
// alone (a vertex lies in the image of g^-1(0) for |G| / orbit elements).
__device__ inline uint64_t rep_vector(const TemplateGeom &D, uint64_t cmap, int &gbest) {
    uint32_t first = 16;
    uint64_t cand = 0;  // bit g: g attains the minimal first entry
    for (int g = 0; g < D.ngroup; g++) {
        uint32_t f = nib(cmap, (int)nib(D.ginv[g], 0));
        if (f < first) {
            first = f;
            cand = 0;
        }
        if (f == first) cand |= 1ull << g;
    }
    uint64_t best = ~0ull;
    gbest = 0;
    for (; cand; cand &= cand - 1) {
        int g = __builtin_ctzll(cand);
        uint64_t gi = D.ginv[g];
        uint64_t v = 0;
        for (int m = 0; m < D.k; m++) v |= (uint64_t)nib(cmap, (int)nib(gi, m)) << (4 * (15 - m));
        if (v < best) {
            best = v;
            gbest = g;
        }
    }
    return best;
}

template <typename T>
struct CandEval {
    T r, s, q[4];
    T c;  // FP32 form: bound on the eigen-solve's excess of RMSD^2 (f32_excess_bound)
};

// eq.(3) for one candidate of K = 6, 12 or 14 neighbours (observed rank r
// <-> template vertex tv(r); the template from the FP64 table) with the
// observed points streamed from the (cached) neighbour vectors instead of
// held in registers: covariance and G_a / G_b in one pass, the residual in
// a second, each recomputing the centred points from the barycentre cb
// (FP64, eq. 2).  K is a run-time value, so lanes of different hull sizes
// run one code path.  Moments (FP64 only): the residual at (s, q) is also
// G_b + s (s G_a - 2 rho), rho = sum_i a_i . R b_i = tr(R S^T); it is
// stationary in q and s at the optimum, and its rounding error, a few ulps
// of G_b ~ N, is at most 2e-13 in the RMSD once RMSD >= 0.01 (the
// difference cancels below that, where the explicit second pass runs).
template <typename T, bool Moments = false>
__device__ inline void eval_streamed(int K, const double *__restrict__ nbr_rel, int64_t n, int64_t p,
                                     const double (&cb)[3], const TemplateGeom &D, uint64_t tv, CandEval<T> &out) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    T S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    T Gb = 0;
    double g = 0;
    const T a0[3] = {(T)(-cb[0]), (T)(-cb[1]), (T)(-cb[2])};
    for (int d = 0; d < 3; d++) g += cb[d] * cb[d];
    {
        const T bb[3] = {(T)D.b[0][0], (T)D.b[0][1], (T)D.b[0][2]};
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) S[x][y] += bb[x] * a0[y];
        Gb += bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
    }
#pragma unroll 2
    for (int r = 0; r < K; r++) {
        T a[3];
        for (int d = 0; d < 3; d++) {
            double x = nbr_rel[((int64_t)r * 3 + d) * n + p] - cb[d];
            a[d] = (T)x;
            g += x * x;
        }
        const double *b64 = D.b[nib(tv, r) + 1];
        const T bb[3] = {(T)b64[0], (T)b64[1], (T)b64[2]};
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) S[x][y] += bb[x] * a[y];
        Gb += bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
    }
    const T Ga = (T)g;
    T cond = 0;
    T lam = qcp_solve<T>(S, Ga, Gb, out.q, sizeof(T) == 4 ? &cond : nullptr);
    if constexpr (sizeof(T) == 4) out.c = f32_excess_bound(lam, cond, Ga);
    T s = Ga > T(0) ? lam / Ga : T(0);
    T R[3][3];
    quat_rot<T>(out.q, R);
    if constexpr (Moments && sizeof(T) == 8) {
        T rho = 0;
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) rho += R[x][y] * S[y][x];
        const T rm = Gb + s * (s * Ga - T(2) * rho);
        if (rm >= T(1e-4) * T(K + 1)) {
            out.r = sqrt(rm / T(K + 1));
            out.s = s;
            return;
        }
    }
    T res = 0;
    {
        const T bb[3] = {(T)D.b[0][0], (T)D.b[0][1], (T)D.b[0][2]};
        for (int x = 0; x < 3; x++) {
            T d = s * a0[x] - (R[x][0] * bb[0] + R[x][1] * bb[1] + R[x][2] * bb[2]);
            res += d * d;
        }
    }
#pragma unroll 2
    for (int r = 0; r < K; r++) {
        T a[3];
        for (int d = 0; d < 3; d++) a[d] = (T)(nbr_rel[((int64_t)r * 3 + d) * n + p] - cb[d]);
        const double *b64 = D.b[nib(tv, r) + 1];
        const T bb[3] = {(T)b64[0], (T)b64[1], (T)b64[2]};
        for (int x = 0; x < 3; x++) {
            T d = s * a[x] - (R[x][0] * bb[0] + R[x][1] * bb[1] + R[x][2] * bb[2]);
            res += d * d;
        }
    }
    out.r = sqrt(res / T(K + 1));
    out.s = s;
}

// template vertex of each observed rank for candidate perm (label -> vertex)
// and labelling ord (label -> rank)
__device__ inline uint64_t tv_of_rank(uint64_t perm, uint64_t ord, int k) {
    uint64_t tv = 0;
    for (int l = 0; l < k; l++) tv |= (uint64_t)nib(perm, l) << (4 * nib(ord, l));
    return tv;
}

// observed rank at each template vertex
__device__ inline uint64_t rank_of_tv(uint64_t perm, uint64_t ord, int k) {
    uint64_t c = 0;
    for (int l = 0; l < k; l++) c |= (uint64_t)nib(ord, l) << (4 * nib(perm, l));
    return c;
}

// Outputs of the winning candidate from its superposition ev and the
// strain inputs A^T (sum over points of V+ columns times centred points, in
// template order) and l (mean point norm).
template <typename RT>
__device__ inline void finish_outputs(int K, const MatchShared &M, const TablesView &T, int grp, int c, uint64_t ord,
                                      const CandEval<RT> &ev, RT l, const RT (&At)[3][3], RT resid, double cutoff,
                                      int64_t p, int64_t n, int32_t i, const int32_t *__restrict__ nbr_id,
                                      const int8_t *__restrict__ species, const MatchOut &O) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    Candidate cd = T.cand[grp][c];
    const TemplateGeom &G = M.geo[cd.tmpl];
    const TemplateDev &D = T.tpl[cd.tmpl];  // the group's quaternions
    const uint64_t tv = tv_of_rank(cd.perm, ord, K);
    const int type = ((double)ev.r <= cutoff) ? cd.tmpl + 1 : 0;
    if (O.best_type) O.best_type[i] = (int8_t)(cd.tmpl + 1);
    int g;
    const uint64_t rep = rep_vector(G, rank_of_tv(cd.perm, ord, K), g);
    {
        // q' = q * conj(q_g), sign fixed so that the first non-zero component is positive
        const double *qg = D.gq[g];
        RT w1 = ev.q[0], x1 = ev.q[1], y1 = ev.q[2], z1 = ev.q[3];
        RT w2 = (RT)qg[0], x2 = -(RT)qg[1], y2 = -(RT)qg[2], z2 = -(RT)qg[3];
        RT q[4] = {w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                   w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2};
        RT qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        int flip = 0;
        for (int k = 0; k < 4; k++) {
            if (q[k] > 0) { flip = 1; break; }
            if (q[k] < 0) { flip = -1; break; }
        }
        RT sc = RT(flip < 0 ? -1 : 1) / qn;
        O.type[i] = (int8_t)type;
        if (O.rmsd) O.rmsd[i] = (double)ev.r;
        if (O.scale) O.scale[i] = (double)ev.s;
        if (O.quat) {
            // records as 16-byte pairs (the arrays are 16-byte aligned)
            double2 *qo = reinterpret_cast<double2 *>(O.quat + 4 * (int64_t)i);
            qo[0] = make_double2((double)(q[0] * sc), (double)(q[1] * sc));
            qo[1] = make_double2((double)(q[2] * sc), (double)(q[3] * sc));
        }
        if (O.quat_fz) {
            // Sec. 7: of the equivalent orientations q' x conj(q_h), the one
            // closest to the identity (largest |w|; the first on ties)
            const RT a0 = q[0] * sc, a1 = q[1] * sc, a2 = q[2] * sc, a3 = q[3] * sc;
            RT best[4] = {a0, a1, a2, a3};
            RT bw = RT(-1);
            for (int h = 0; h < G.ngroup; h++) {
                const double *qh = D.gq[h];
                const RT w2 = (RT)qh[0], x2 = -(RT)qh[1], y2 = -(RT)qh[2], z2 = -(RT)qh[3];
                const RT c0 = a0 * w2 - a1 * x2 - a2 * y2 - a3 * z2;
                if (fabs(c0) > bw) {
                    bw = fabs(c0);
                    best[0] = c0;
                    best[1] = a0 * x2 + a1 * w2 + a2 * z2 - a3 * y2;
                    best[2] = a0 * y2 - a1 * z2 + a2 * w2 + a3 * x2;
                    best[3] = a0 * z2 + a1 * y2 - a2 * x2 + a3 * w2;
                }
            }
            RT sg = best[0] < RT(0) ? RT(-1) : RT(1);
            if (best[0] == RT(0))
                for (int k = 1; k < 4; k++)
                    if (best[k] != RT(0)) {
                        sg = best[k] < RT(0) ? RT(-1) : RT(1);
                        break;
                    }
            double2 *qo = reinterpret_cast<double2 *>(O.quat_fz + 4 * (int64_t)i);
            qo[0] = make_double2((double)(sg * best[0]), (double)(sg * best[1]));
            qo[1] = make_double2((double)(sg * best[2]), (double)(sg * best[3]));
        }
        if (O.nn_distance) {
            // hydrostatic part (Sec. 8): template vertex 0 lies at |b_1| in eq.(4) units
            const double *b1 = G.b[1];
            O.nn_distance[i] = ev.s > RT(0) ? sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]) / (double)ev.s : 0.0;
        }
        if (O.strain_residual) O.strain_residual[i] = (double)resid;
    }
    if (O.neighbours) {
        int32_t ids[KMAX];
#pragma unroll
        for (int m = 0; m < KMAX; m++) {
            int32_t id = -1;
            if (m < K) {
                int rank = (int)((rep >> (4 * (15 - m))) & 0xF);
                id = nbr_id[(int64_t)rank * n + p];
            }
            ids[m] = id;
        }
        // as 8-byte pairs (the array is 8-byte aligned)
        int2 *no = reinterpret_cast<int2 *>(O.neighbours + (int64_t)i * KMAX);
#pragma unroll
        for (int m = 0; m < KMAX / 2; m++) no[m] = make_int2(ids[2 * m], ids[2 * m + 1]);
    }
    if (O.strain || O.vm_strain) {
        // Sec. 8: P of A = P U with U right-handed
        RT P[3][3];
        polar_p<RT>(At, l, P);
        RT sq = 0, tr = 0;
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) {
                const RT s = P[x][y];
                if (O.strain) O.strain[9 * (int64_t)i + 3 * x + y] = (double)s;
                sq += s * s;
                if (x == y) tr += s;
            }
        // Sec. 8: von Mises shear strain of P
        if (O.vm_strain) O.vm_strain[i] = (double)sqrt(fmax(RT(1.5) * sq - RT(0.5) * tr * tr, RT(0)));
    }
    if (O.alloy) {
        // alloy (Sec. 6, Table 3)
        int alloy = 0;
        if (species && type && (cd.tmpl == 1 || cd.tmpl == 4)) {
            const int8_t me = species[i];
            uint32_t cnt = 0;  // 8-bit counters: FCC groups 0..2, BCC inner/outer
#pragma unroll
            for (int r = 0; r < KMAX; r++) {
                if (r >= K) break;
                int32_t j = nbr_id[(int64_t)r * n + p];
                int other = species[j] != me;
                int tvx = (int)nib(tv, r);
                int grp2 = (cd.tmpl == 1) ? (tvx >> 2) : (tvx < 8 ? 0 : 1);
                cnt += (uint32_t)other << (8 * grp2);
            }
            if (cd.tmpl == 1) {
                int c0 = cnt & 0xFF, c1 = (cnt >> 8) & 0xFF, c2 = (cnt >> 16) & 0xFF;
                int lo = min(c0, min(c1, c2)), hi = max(c0, max(c1, c2)), mid = c0 + c1 + c2 - lo - hi;
                if (lo == 0 && mid == 0 && hi == 0) alloy = 1;
                else if (lo == 0 && mid == 4 && hi == 4) alloy = 2;
                else if (lo == 0 && mid == 0 && hi == 4) alloy = 3;
                else if (lo == 4 && mid == 4 && hi == 4) alloy = 4;
                else alloy = 5;
            } else {
                int inner = cnt & 0xFF, outer = (cnt >> 8) & 0xFF;
                if (inner == 0 && outer == 0) alloy = 6;
                else if (inner == 8 && outer == 0) alloy = 7;
                else alloy = 8;
            }
        }
        O.alloy[i] = (int8_t)alloy;
    }
}


// Outputs of the winning candidate from its superposition ev (r, q, s):
// the strain inputs are gathered from the points in one pass (the
// barycentre cb is known); the optional eq.(6) residual takes a second.
template <typename RT>
__device__ inline void finish(int K, const MatchShared &M, const TablesView &T, int grp, int c, uint64_t ord,
                              const CandEval<RT> &ev, const double (&cb)[3], const double *__restrict__ nbr_rel,
                              double cutoff, int64_t p, int64_t n, int32_t i, const int32_t *__restrict__ nbr_id,
                              const int8_t *__restrict__ species, const MatchOut &O) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    Candidate cd = T.cand[grp][c];
    const TemplateGeom &D = M.geo[cd.tmpl];
    const uint64_t tv = tv_of_rank(cd.perm, ord, K);
    RT a0[3], At[3][3], l;
    strain_begin<RT>(D, cb, a0, At, l);
#pragma unroll
    for (int rr = 0; rr < KMAX; rr++) {
        if (rr >= K) break;
        RT ar[3];
        for (int d = 0; d < 3; d++) ar[d] = (RT)(nbr_rel[((int64_t)rr * 3 + d) * n + p] - cb[d]);
        strain_add<RT>(D, (int)nib(tv, rr) + 1, ar, At, l);
    }
    l /= RT(K + 1);
    RT resid = 0;
    if (O.strain_residual) {
        // eq.(6) residual: sum over points of |V_i A^T - a_i|^2 / l^2
        for (int y = 0; y < 3; y++) {
            RT d = (RT)D.b[0][0] * At[0][y] + (RT)D.b[0][1] * At[1][y] + (RT)D.b[0][2] * At[2][y] - a0[y];
            resid += d * d;
        }
#pragma unroll 2
        for (int rr = 0; rr < K; rr++) {
            const double *v = D.b[(int)nib(tv, rr) + 1];
            for (int y = 0; y < 3; y++) {
                RT ay = (RT)(nbr_rel[((int64_t)rr * 3 + y) * n + p] - cb[y]);
                RT d = (RT)v[0] * At[0][y] + (RT)v[1] * At[1][y] + (RT)v[2] * At[2][y] - ay;
                resid += d * d;
            }
        }
        resid /= l * l;
    }
    finish_outputs<RT>(K, M, T, grp, c, ord, ev, l, At, resid, cutoff, p, n, i, nbr_id, species, O);
}

__device__ inline void write_none(const MatchOut &O, int32_t i) {
    O.type[i] = 0;
    if (O.alloy) O.alloy[i] = 0;
    if (O.rmsd) O.rmsd[i] = INFINITY;
    if (O.scale) O.scale[i] = 0.0;
    if (O.quat) {
        O.quat[4 * (int64_t)i] = 1.0;
        for (int k = 1; k < 4; k++) O.quat[4 * (int64_t)i + k] = 0.0;
    }
    if (O.strain)
        for (int k = 0; k < 9; k++) O.strain[9 * (int64_t)i + k] = 0.0;
    if (O.neighbours)
        for (int m = 0; m < KMAX; m++) O.neighbours[(int64_t)i * KMAX + m] = -1;
    if (O.best_type) O.best_type[i] = 0;
    if (O.vm_strain) O.vm_strain[i] = 0.0;
    if (O.strain_residual) O.strain_residual[i] = 0.0;
    if (O.nn_distance) O.nn_distance[i] = 0.0;
    if (O.quat_fz) {
        O.quat_fz[4 * (int64_t)i] = 1.0;
        for (int k = 1; k < 4; k++) O.quat_fz[4 * (int64_t)i + k] = 0.0;
    }
}

__device__ inline void load_templates(MatchShared &M, const TablesView &T) {
    constexpr int NB = NMAX * 3;  // doubles of b, and of vpinv
    for (int w = threadIdx.x; w < NT * 2 * NB; w += blockDim.x) {
        const int t = w / (2 * NB), e = w % (2 * NB);
        if (e < NB) (&M.geo[t].b[0][0])[e] = (&T.tpl[t].b[0][0])[e];
        else (&M.geo[t].vpinv[0][0])[e - NB] = (&T.tpl[t].vpinv[0][0])[e - NB];
    }
    for (int w = threadIdx.x; w < NT * GMAX; w += blockDim.x) M.geo[w / GMAX].ginv[w % GMAX] = T.tpl[w / GMAX].ginv[w % GMAX];
    if ((int)threadIdx.x < NT) {
        M.geo[threadIdx.x].k = T.tpl[threadIdx.x].k;
        M.geo[threadIdx.x].ngroup = T.tpl[threadIdx.x].ngroup;
    }
    __syncthreads();
}

// ------------------------------------------------------------ match stage
// One kernel superposes every candidate correspondence of the atoms' hull
// codes (eq. 3), takes the decision of Alg. 1 and writes the outputs of the
// winner.  A wave owns 64 consecutive atoms (cell order):
//  A. lane = atom: the Euclidean neighbour list is copied out, the
//     barycentres of the 6-, 12- and 14-neighbour groups (eq. 2, FP64) and
//     the first candidate of each code go to LDS, the enabled candidates
//     are counted;
//  B. the wave's candidates form one job list, atom after atom and within
//     an atom in (group, candidate) order, superposed 64 at a time with
//     lane = job (the superposition takes the hull size as a run-time
//     value, so a chunk mixing sizes runs one code path); after each chunk
//     every atom lane folds its jobs of the chunk, in order, into its
//     running minimum and marks itself as the owner of its jobs in the
//     next chunk;
//  C. an atom whose decision the common rule cannot take (a near tie, an
//     FP32 margin that the error bounds do not clear) is decided by the
//     full rule in FP64 by the whole wave; every other lane finishes its
//     own winner (the hull size is a run-time value there too, so a wave
//     mixing sizes runs one code path).
// Nothing per candidate leaves the chip: the neighbour vectors are read
// once per atom in A and again from the caches by the jobs and the finish.

// LDS of one wave
template <typename RT>
struct MatchWaveLds {
    double cb[NGRP][3][64];  // barycentre of each hull group of the wave's atoms
    int32_t k0[NGRP][64];    // first candidate of each atom's code in the group's list
    int32_t cnt[64];         // enabled candidates of each atom per group, 8 bits each
    int32_t off[64];         // each atom's first job
    int32_t owner[64];       // the atom of each job of the current chunk
    double r[64];            // the current chunk's results: RMSD,
    RT qs[5][64];            // quaternion and scale,
    float d2[64];            // FP32 form: excess bound (f32_excess_bound),
    int32_t cand[64];        // candidate index in the group's list
};
// working LDS of a block of NW waves
template <typename RT, int NW>
struct MatchWork {
    MatchWaveLds<RT> w[NW];
};
template <typename RT, int NW>
struct MatchLds {
    MatchShared M;
    // copies of the kernel's table view and output pointers for the full
    // rule, a call: arguments it takes by reference would otherwise be
    // copied to per-lane scratch memory by every lane
    TablesView T;
    MatchOut O;
    MatchWork<RT, NW> work;
};

// LDS written by some lanes of a wave and then read by others of the same
// wave: a wave's LDS instructions complete in issue order, so the only
// requirement is that the compiler keeps them on their side of this point.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one job: the candidate with tv of the atom at p, K neighbours, barycentre cb
template <typename RT>
__device__ inline void eval_job(int K, const double *__restrict__ nbr_rel, int64_t n, int64_t p,
                                const double (&cb)[3], const TemplateGeom &D, uint64_t tv, CandEval<RT> &ev) {
    // (FP64: the residual from the moments where that is exact enough)
    eval_streamed<RT, true>(K, nbr_rel, n, p, cb, D, tv, ev);
}

// The full rule of Alg. 1 for the wave's atom a (at p), in FP64, by the
// whole wave: lane j superposes the atom's j-th candidate (the codes of one
// atom hold at most 64 together, checked when the tables are built), the
// minimum r* is reduced over the wave, every enabled candidate within the
// tie tolerance of r* computes its representative vector, the (template,
// representative) minimum is reduced, and lane 0 finishes the winner.
// Wave-uniform arguments; cbw: the barycentres of the wave's atoms.
__device__ __noinline__ void full_rule(const MatchShared &M, const TablesView &T, int64_t n, int64_t p, int a,
                          const double (&cbw)[NGRP][3][64], const double *__restrict__ nbr_rel,
                          const int32_t *__restrict__ nbr_id, const int32_t *__restrict__ sid,
                          const int8_t *__restrict__ species, const int32_t *__restrict__ code,
                          const uint64_t *__restrict__ ords, uint32_t mask, double cutoff, const MatchOut &O) {
    const int lane = threadIdx.x & 63;
    const int32_t i = sid[p];
    int32_t c0[NGRP], nc[NGRP];
    uint64_t ord[NGRP];
    for (int g = 0; g < NGRP; g++) {
        const int32_t cid = code[(int64_t)g * n + p];
        ord[g] = ords[(int64_t)g * n + p];
        c0[g] = cid >= 0 ? T.cstart[g][cid] : 0;
        nc[g] = cid >= 0 ? T.cstart[g][cid + 1] - c0[g] : 0;
    }
    // this lane's candidate
    int g = -1, c = -1, tmpl = 99;
    double r = INFINITY;
    {
        int j = lane;
        for (int gg = 0; gg < NGRP && g < 0; gg++) {
            if (j < nc[gg]) {
                g = gg;
                c = c0[gg] + j;
            } else {
                j -= nc[gg];
            }
        }
    }
    Candidate cd = {0, 0, 0};
    CandEval<double> ev = {0, 0, {0, 0, 0, 0}};
    if (g >= 0) {
        cd = T.cand[g][c];
        if ((mask >> cd.tmpl) & 1) {
            tmpl = cd.tmpl;
            const double cb[3] = {cbw[g][0][a], cbw[g][1][a], cbw[g][2][a]};
            const int K = group_k(g);
            eval_streamed<double>(K, nbr_rel, n, p, cb, M.geo[cd.tmpl], tv_of_rank(cd.perm, ord[g], K), ev);
            r = ev.r;
        }
    }
    double m1 = r;
    for (int off = 32; off > 0; off >>= 1) m1 = fmin(m1, __shfl_xor(m1, off));
    if (m1 == INFINITY) {  // no candidate of an enabled template
        if (lane == 0) write_none(O, i);
        return;
    }
    // tie rule: earliest template, then the smallest representative vector
    int kt = 99;
    uint64_t krep = ~0ull;
    if (r <= m1 + 1e-12) {
        int gsel;
        kt = tmpl;
        krep = rep_vector(M.geo[tmpl], rank_of_tv(cd.perm, ord[g], group_k(g)), gsel);
    }
    int bt = kt, bl = lane;
    uint64_t brep = krep;
    for (int off = 32; off > 0; off >>= 1) {
        int ot = __shfl_xor(bt, off), ol = __shfl_xor(bl, off);
        uint64_t orep = __shfl_xor(brep, off);
        bool take = ot < bt || (ot == bt && (orep < brep || (orep == brep && ol < bl)));
        if (take) {
            bt = ot;
            brep = orep;
            bl = ol;
        }
    }
    const int wg = __shfl(g, bl), wc = __shfl(c, bl);
    // the winning lane's superposition, handed to the finishing lane
    CandEval<double> we;
    we.r = __shfl(ev.r, bl);
    we.s = __shfl(ev.s, bl);
    for (int k = 0; k < 4; k++) we.q[k] = __shfl(ev.q[k], bl);
    if (lane == 0) {
        const double cb[3] = {cbw[wg][0][a], cbw[wg][1][a], cbw[wg][2][a]};
        if (wg == 0) finish<double>(6, M, T, 0, wc, ord[0], we, cb, nbr_rel, cutoff, p, n, i, nbr_id, species, O);
        else if (wg == 1)
            finish<double>(12, M, T, 1, wc, ord[1], we, cb, nbr_rel, cutoff, p, n, i, nbr_id, species, O);
        else finish<double>(14, M, T, 2, wc, ord[2], we, cb, nbr_rel, cutoff, p, n, i, nbr_id, species, O);
    }
}

// Bound on |RMSD_FP32 - RMSD| of one candidate evaluated in FP32 from
// FP64-centred points (u = 2^-24; the terms are derived with the FP32-mixed
// form's description):
//   first order, u (72 + 25 r): rounding of the inputs (2.7 u), the
//     covariance sums seen as a perturbation of the inputs (36 u), the
//     rotation built from a unit quaternion rounded to FP32 (15 u), the
//     residual components (17 u), the 45-term sum of squares (23 u r), the
//     division and square root (2 u r);
//   the eigen-solve's excess d2 of RMSD^2 (f32_excess_bound; infinite for
//     an eigenpair FP32 cannot resolve): RMSD^2 + d2 has a square root
//     below RMSD + d2 / (RMSD + sqrt(d2)).
constexpr double RMSD_F32_U = 0x1p-24;
__device__ inline double rmsd_f32_bound(double r, double d2) {
    if (!(d2 < INFINITY)) return INFINITY;
    return RMSD_F32_U * (72.0 + 25.0 * r) + d2 / (r + sqrt(d2));
}

constexpr uint32_t ALL_TEMPLATES = (1u << NT) - 1;

// The match stage for the NW * 64 atoms from first (see the section head),
// by a block of NW waves: templates in M, the LDS copies Tl / Ol of the
// table view and outputs (for the full rule), working LDS Wk.  force_full:
// every atom with a candidate takes the full rule (a test of that path).
// full_count counts the atoms the full rule decides, job_count the
// superposed candidates.
template <typename RT, int NW>
__device__ void match_block(const MatchShared &M, const TablesView &Tl, const MatchOut &Ol, MatchWork<RT, NW> &Wk,
                            int64_t first, int64_t n, const double *__restrict__ nbr_rel,
                            const int32_t *__restrict__ nbr_id, const int32_t *__restrict__ sid,
                            const int8_t *__restrict__ species, const TablesView &T,
                            const int32_t *__restrict__ code, const uint64_t *__restrict__ ords, uint32_t mask,
                            double cutoff, int force_full, const MatchOut &O, int32_t *__restrict__ full_count,
                            unsigned long long *__restrict__ job_count, const int32_t *__restrict__ knn_src,
                            int32_t *__restrict__ knn_out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    MatchWaveLds<RT> &W = Wk.w[wv];
    const int64_t wbase = first + (int64_t)wv * 64;
    const int64_t p = wbase + lane;
    const bool live = p < n;

    // A. lane = atom
    int cnt[NGRP] = {0, 0, 0};
    if (live) {
        if (knn_out) {
            // the Euclidean order (Sec. 3) whatever the ordering of the hulls
            const int32_t i = sid[p];
#pragma unroll
            for (int m = 0; m < KMAX; m++) knn_out[(int64_t)i * KMAX + m] = knn_src[(int64_t)m * n + p];
        }
        // barycentres of the centre and the first 6, 12 and 14 neighbours
        double s[3] = {0, 0, 0};
#pragma unroll
        for (int r = 0; r < KMAX; r++) {
            for (int d = 0; d < 3; d++) s[d] += nbr_rel[((int64_t)r * 3 + d) * n + p];
#pragma unroll
            for (int g = 0; g < NGRP; g++)
                if (r + 1 == group_k(g))
                    for (int d = 0; d < 3; d++) W.cb[g][d][lane] = s[d] / (group_k(g) + 1);
        }
        for (int g = 0; g < NGRP; g++) {
            const int32_t cid = code[(int64_t)g * n + p];
            int k0 = 0;
            if (cid >= 0) {
                k0 = T.cstart[g][cid];
                const int k1 = T.cstart[g][cid + 1];
                if ((mask & ALL_TEMPLATES) == ALL_TEMPLATES) cnt[g] = k1 - k0;
                else
                    for (int k = k0; k < k1; k++) cnt[g] += (mask >> T.cand[g][k].tmpl) & 1;
            }
            W.k0[g][lane] = k0;
        }
        W.cnt[lane] = cnt[0] | (cnt[1] << 8) | (cnt[2] << 16);
    }
    // job offsets: exclusive scan over the wave
    const int mine = cnt[0] + cnt[1] + cnt[2];
    int my_off = mine;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(my_off, d);
        if (lane >= d) my_off += y;
    }
    const int jobs = __shfl(my_off, 63);
    my_off -= mine;
    W.off[lane] = my_off;
    if (lane == 0 && jobs > 0) atomicAdd(job_count, (unsigned long long)jobs);
    for (int t = my_off; t < min(my_off + mine, 64); t++) W.owner[t] = lane;  // owners of the first chunk
    wave_lds_sync();

    // B. jobs, 64 at a time
    double m1 = INFINITY, m2 = INFINITY, b1 = 0.0, lo2 = INFINITY;
    int arg_g = -1, arg_c = -1;
    RT wq[4] = {1, 0, 0, 0}, ws = 0;
    for (int c0 = 0; c0 < jobs; c0 += 64) {
        if (c0 + lane < jobs) {
            const int a = W.owner[lane];
            int j = c0 + lane - W.off[a];
            const int32_t cn = W.cnt[a];
            int g = 0;
            if (j >= (cn & 0xFF)) {
                j -= cn & 0xFF;
                g = 1;
                if (j >= ((cn >> 8) & 0xFF)) {
                    j -= (cn >> 8) & 0xFF;
                    g = 2;
                }
            }
            const int64_t pa = wbase + a;
            int k = W.k0[g][a];
            if ((mask & ALL_TEMPLATES) == ALL_TEMPLATES) {
                k += j;
            } else {
                // the j-th enabled candidate of the code
                for (;; k++)
                    if ((mask >> T.cand[g][k].tmpl) & 1) {
                        if (j == 0) break;
                        j--;
                    }
            }
            const Candidate cd = T.cand[g][k];
            const uint64_t ord = ords[(int64_t)g * n + pa];
            const double cb[3] = {W.cb[g][0][a], W.cb[g][1][a], W.cb[g][2][a]};
            const int K = group_k(g);
            CandEval<RT> ev;
            eval_job<RT>(K, nbr_rel, n, pa, cb, M.geo[cd.tmpl], tv_of_rank(cd.perm, ord, K), ev);
            W.r[lane] = (double)ev.r;
            for (int e = 0; e < 4; e++) W.qs[e][lane] = ev.q[e];
            W.qs[4][lane] = ev.s;
            if constexpr (sizeof(RT) == 4) W.d2[lane] = ev.c;
            W.cand[lane] = k;
        }
        wave_lds_sync();
        if (mine > 0) {
            // this atom's jobs of the chunk, in order (group, then
            // candidate); strict comparisons: ties go to the earlier job
            const int lo = max(my_off, c0), hi = min(my_off + mine, c0 + 64);
            for (int t = lo; t < hi; t++) {
                const int jj = t - my_off;
                const int g = jj < cnt[0] ? 0 : (jj < cnt[0] + cnt[1] ? 1 : 2);
                const int u = t - c0;
                const double r = W.r[u];
                double b = 0.0;
                if constexpr (sizeof(RT) == 4) b = rmsd_f32_bound(r, (double)W.d2[u]);
                if (r < m1) {
                    if constexpr (sizeof(RT) == 4) lo2 = fmin(lo2, m1 - b1);  // the previous winner joins the others
                    b1 = b;
                    m2 = m1;
                    m1 = r;
                    arg_g = g;
                    arg_c = W.cand[u];
                    for (int e = 0; e < 4; e++) wq[e] = W.qs[e][u];
                    ws = W.qs[4][u];
                } else {
                    if (r < m2) m2 = r;
                    if constexpr (sizeof(RT) == 4) lo2 = fmin(lo2, r - b);
                }
            }
            // owners of the next chunk (its jobs have read this one's)
            for (int t = max(my_off, c0 + 64); t < min(my_off + mine, c0 + 128); t++) W.owner[t - c0 - 64] = lane;
        }
        wave_lds_sync();
    }

    // C. decision.  The common case -- a unique winner by more than the tie
    // tolerance (FP32 form: by more than the two candidates' error bounds,
    // and clear of the cut-off by the winner's) -- is finished below in the
    // working precision; the others take the full rule.
    bool full = false;
    int cls = -1;  // hull group of the winner to finish below, -1 for none
    double cbw[3] = {0, 0, 0};
    if (live) {
        full = arg_c >= 0 && (force_full || !(m2 > m1 + 1e-12));
        if constexpr (sizeof(RT) == 4) {
            if (arg_c >= 0) full = full || !(lo2 - (m1 + b1) > 1e-12) || fabs(m1 - cutoff) <= b1;
        } else {
            // RMSDs from the moments carry up to 2e-13 each: near ties and
            // the cut-off get that much room (the full rule uses explicit
            // residuals)
            if (arg_c >= 0) full = full || !(m2 > m1 + 2e-12) || fabs(m1 - cutoff) <= 1e-12;
        }
        if (!full) {
            if (arg_c < 0) {
                write_none(O, sid[p]);
            } else {
                cls = arg_g;
                for (int d = 0; d < 3; d++) cbw[d] = W.cb[arg_g][d][lane];
            }
        }
    }
    uint64_t fb = __ballot(full);
    if (lane == 0 && fb) atomicAdd(full_count, (int32_t)__popcll(fb));
    while (fb) {
        const int a = __builtin_ctzll(fb);
        fb &= fb - 1;
        full_rule(M, Tl, n, wbase + a, a, W.cb, nbr_rel, nbr_id, sid, species, code, ords, mask, cutoff, Ol);
    }

    // every lane finishes its own winner, whatever its hull size
    if (cls >= 0) {
        const int32_t iw = sid[p];
        const uint64_t ord = ords[(int64_t)cls * n + p];
        CandEval<RT> ev;
        ev.r = (RT)m1;
        for (int e = 0; e < 4; e++) ev.q[e] = wq[e];
        ev.s = ws;
        finish<RT>(group_k(cls), M, T, cls, arg_c, ord, ev, cbw, nbr_rel, cutoff, p, n, iw, nbr_id, species, O);
    }
}

// The match kernel: blocks of four waves, 256 atoms each.  FP64: three
// blocks per CU (168 VGPRs at most) with the LDS of three; FP32: four (128
// VGPRs at most, the spills only around the rare full-rule call).
template <typename RT>
__global__ void __launch_bounds__(MB, sizeof(RT) == 4 ? 4 : 3) k_match(int64_t n, const double *__restrict__ nbr_rel,
                                                const int32_t *__restrict__ nbr_id, const int32_t *__restrict__ sid,
                                                const int8_t *__restrict__ species, TablesView T,
                                                const int32_t *__restrict__ code, const uint64_t *__restrict__ ords,
                                                uint32_t mask, double cutoff, int force_full, MatchOut O,
                                                int32_t *__restrict__ full_count,
                                                unsigned long long *__restrict__ job_count,
                                                const int32_t *__restrict__ knn_src, int32_t *__restrict__ knn_out,
                                                const int32_t *__restrict__ box_fail) {
    __shared__ MatchLds<RT, MB / 64> L;
    if (*box_fail) return;  // uniform over the grid
    if (threadIdx.x == 0) {
        L.T = T;
        L.O = O;
    }
    load_templates(L.M, T);
    match_block<RT, MB / 64>(L.M, L.T, L.O, L.work, (int64_t)blockIdx.x * MB, n, nbr_rel, nbr_id, sid, species, T,
                             code, ords, mask, cutoff, force_full, O, full_count, job_count, knn_src, knn_out);
}

// ------------------------------------------------- post-hoc cut-off (Sec. 5.1)
// Both kernels are HBM streams.  Lanes take eight atoms each (one 8-byte
// load of types, four 16-byte loads of RMSDs) when the arrays are aligned
// for it; atoms past the last full group of eight, or misaligned arrays, go
// one per lane.
__device__ inline int8_t cut_one(int8_t t, double r, double cutoff) { return r <= cutoff ? t : (int8_t)0; }

__global__ void __launch_bounds__(256) k_apply_cutoff(int64_t n, int64_t n8, const int8_t *__restrict__ best_type,
                                                      const double *__restrict__ rmsd, double cutoff,
                                                      int8_t *__restrict__ type) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n8; g += stride) {
        const uint64_t t8 = ((const uint64_t *)best_type)[g];
        const double2 *r2 = (const double2 *)rmsd + 4 * g;
        uint64_t o = 0;
#pragma unroll
        for (int h = 0; h < 4; h++) {
            const double2 r = r2[h];
            o |= (uint64_t)(uint8_t)cut_one((int8_t)(t8 >> (16 * h)), r.x, cutoff) << (16 * h);
            o |= (uint64_t)(uint8_t)cut_one((int8_t)(t8 >> (16 * h + 8)), r.y, cutoff) << (16 * h + 8);
        }
        ((uint64_t *)type)[g] = o;
    }
    for (int64_t i = 8 * n8 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
        type[i] = cut_one(best_type[i], rmsd[i], cutoff);
}

// per-type histograms: a block-private copy in LDS (when 6 * nbins fits),
// then one atomic add per non-zero bin into the global counts
constexpr int HIST_LDS_BINS = 6 * 1024;
__device__ inline void hist_add(unsigned int *h, unsigned long long *counts, bool lds, int t, double r, int nbins,
                                double rmax, double inv) {
    if (t < 0 || t > 5) return;
    int b = nbins - 1;
    if (r < rmax) b = min(nbins - 1, max(0, (int)(r * inv)));
    if (lds) atomicAdd(&h[t * nbins + b], 1u);
    else atomicAdd(&counts[t * nbins + b], 1ull);
}

__global__ void __launch_bounds__(256) k_rmsd_histogram(int64_t n, int64_t n8, const int8_t *__restrict__ best_type,
                                                        const double *__restrict__ rmsd, int nbins, double rmax,
                                                        double inv, unsigned long long *__restrict__ counts) {
    __shared__ unsigned int h[HIST_LDS_BINS];
    const bool lds = 6 * nbins <= HIST_LDS_BINS;
    if (lds)
        for (int b = threadIdx.x; b < 6 * nbins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n8; g += stride) {
        const uint64_t t8 = ((const uint64_t *)best_type)[g];
        const double2 *r2 = (const double2 *)rmsd + 4 * g;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const double2 r = r2[q];
            hist_add(h, counts, lds, (int8_t)(t8 >> (16 * q)), r.x, nbins, rmax, inv);
            hist_add(h, counts, lds, (int8_t)(t8 >> (16 * q + 8)), r.y, nbins, rmax, inv);
        }
    }
    for (int64_t i = 8 * n8 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
        hist_add(h, counts, lds, best_type[i], rmsd[i], nbins, rmax, inv);
    __syncthreads();
    if (lds)
        for (int b = threadIdx.x; b < 6 * nbins; b += blockDim.x)
            if (h[b]) atomicAdd(&counts[b], (unsigned long long)h[b]);
}

// groups of eight atoms a lane can load as one 8-byte word of types and four
// 16-byte words of RMSDs (0 if the arrays are not aligned for that)
static int64_t groups_of_eight(int64_t n, const void *t, const void *r, const void *out) {
    const bool ok = ((uintptr_t)t % 8 == 0) && ((uintptr_t)r % 16 == 0) && (!out || (uintptr_t)out % 8 == 0);
    return ok ? n / 8 : 0;
}
static unsigned stream_blocks(int64_t n) {
    // about eight resident blocks per CU of 256 lanes, each lane striding
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 256 * 8));
}

void launch_apply_cutoff(int64_t n, const int8_t *best_type, const double *rmsd, double cutoff, int8_t *type,
                         hipStream_t st) {
    const int64_t n8 = groups_of_eight(n, best_type, rmsd, type);
    hipLaunchKernelGGL(k_apply_cutoff, dim3(stream_blocks(n8 > 0 ? n8 : n)), dim3(256), 0, st, n, n8, best_type, rmsd,
                       cutoff, type);
}
void launch_rmsd_histogram(int64_t n, const int8_t *best_type, const double *rmsd, int nbins, double rmax,
                           unsigned long long *counts, hipStream_t st) {
    const int64_t n8 = groups_of_eight(n, best_type, rmsd, nullptr);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    const double inv = (double)nbins / rmax;  // the bin of r is floor(r * inv), inv rounded once on the host
    hipLaunchKernelGGL(k_rmsd_histogram, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, n, n8,
                       best_type, rmsd, nbins, rmax, inv, counts);
}

// ------------------------------------------------------- misorientation
// Sec. 7: smallest rotation angle of conj(q1) q2 q_h over the template's
// proper rotations (identity only for type NONE), as 2 atan2(|v|, |w|) of
// the best product, which stays accurate near zero.  Invalid types give NaN.
template <bool Vec>
__global__ void __launch_bounds__(256) k_misorientation(int64_t n, TablesView T, const int8_t *__restrict__ type,
                                                        const double *__restrict__ q1, const double *__restrict__ q2,
                                                        double *__restrict__ angle) {
    // every template's rotation group, staged in LDS: lanes of one type read
    // the same word (a broadcast)
    __shared__ double4 G[NT * GMAX];
    __shared__ int gbase[NT + 1];
    if (threadIdx.x == 0) {
        int b = 0;
        for (int t = 0; t < NT; t++) {
            gbase[t] = b;
            b += T.tpl[t].ngroup;
        }
        gbase[NT] = b;
    }
    __syncthreads();
    for (int t = 0; t < NT; t++)
        for (int h = threadIdx.x; h < T.tpl[t].ngroup; h += blockDim.x) {
            const double *g = T.tpl[t].gq[h];
            G[gbase[t] + h] = make_double4(g[0], g[1], g[2], g[3]);
        }
    __syncthreads();
    // Waves of mixed types would each scan the largest group among their
    // lanes (60 for ICO).  The block's pairs are regrouped by type first
    // (wave ballots give each lane its slot) and every lane takes the pair
    // in its slot: waves then mostly scan one group, and its LDS words are
    // broadcasts.  Out-of-range types form a class of their own.
    constexpr int NCLS = NT + 2;  // types 0..NT, then invalid
    __shared__ int32_t s_cnt[4][NCLS];
    __shared__ int64_t s_i[256];
    {
        const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
        int cls = -1;
        if (i0 < n) {
            const int t0 = type[i0];
            cls = (t0 < 0 || t0 > NT) ? NT + 1 : t0;
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        uint64_t bal[NCLS];
#pragma unroll
        for (int k = 0; k < NCLS; k++) bal[k] = __ballot(cls == k);
        if (lane == 0)
            for (int k = 0; k < NCLS; k++) s_cnt[wv][k] = __popcll(bal[k]);
        __syncthreads();
        int total = 0, slot = 0;
#pragma unroll
        for (int k = 0; k < NCLS; k++) {
            int before = 0, tk = 0;
            for (int w2 = 0; w2 < 4; w2++) {
                tk += s_cnt[w2][k];
                if (w2 < wv) before += s_cnt[w2][k];
            }
            if (k == cls) slot = total + before + __popcll(bal[k] & ((1ull << lane) - 1));
            total += tk;
        }
        if (cls >= 0) s_i[slot] = i0;
        __syncthreads();
        if ((int)threadIdx.x >= total) return;
    }
    const int64_t i = s_i[threadIdx.x];
    const int ty = type[i];
    double a0, a1, a2, a3, b0, b1, b2, b3;
    if (Vec) {  // 16-byte aligned quaternion arrays
        const double2 *p1 = (const double2 *)(q1 + 4 * i), *p2 = (const double2 *)(q2 + 4 * i);
        const double2 u0 = p1[0], u1 = p1[1], v0 = p2[0], v1 = p2[1];
        a0 = u0.x, a1 = -u0.y, a2 = -u1.x, a3 = -u1.y;  // conj(q1)
        b0 = v0.x, b1 = v0.y, b2 = v1.x, b3 = v1.y;
    } else {
        a0 = q1[4 * i], a1 = -q1[4 * i + 1], a2 = -q1[4 * i + 2], a3 = -q1[4 * i + 3];
        b0 = q2[4 * i], b1 = q2[4 * i + 1], b2 = q2[4 * i + 2], b3 = q2[4 * i + 3];
    }
    const double m0 = a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3, m1 = a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2;
    const double m2 = a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1, m3 = a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0;
    if (ty < 0 || ty > NT) {
        angle[i] = NAN;
        return;
    }
    // the w of m q_h is a dot product: scan the group for the largest |w|,
    // then form the vector part of that one product only
    double bw = fabs(m0);
    int best = -1;
    if (ty > 0) {
        const int h0 = gbase[ty - 1], h1 = gbase[ty];
        for (int h = h0; h < h1; h++) {
            const double4 g = G[h];
            const double c0 = fabs(m0 * g.x - m1 * g.y - m2 * g.z - m3 * g.w);
            if (c0 > bw) {
                bw = c0;
                best = h;
            }
        }
    }
    double c1 = m1, c2 = m2, c3 = m3;
    if (best >= 0) {
        const double4 g = G[best];
        c1 = m0 * g.y + m1 * g.x + m2 * g.w - m3 * g.z;
        c2 = m0 * g.z - m1 * g.w + m2 * g.x + m3 * g.y;
        c3 = m0 * g.w + m1 * g.z - m2 * g.y + m3 * g.x;
    }
    angle[i] = 2.0 * atan2(sqrt(c1 * c1 + c2 * c2 + c3 * c3), bw);
}

void launch_misorientation(int64_t n, const TablesView &T, const int8_t *type, const double *q1, const double *q2,
                           double *angle, hipStream_t st) {
    const dim3 grid((unsigned)((n + 255) / 256));
    if ((uintptr_t)q1 % 16 == 0 && (uintptr_t)q2 % 16 == 0)
        hipLaunchKernelGGL(k_misorientation<true>, grid, dim3(256), 0, st, n, T, type, q1, q2, angle);
    else
        hipLaunchKernelGGL(k_misorientation<false>, grid, dim3(256), 0, st, n, T, type, q1, q2, angle);
}

// ------------------------------------------------------------- self-check
// The strain of one match on the device, as the decision kernels compute it
// (strain_inputs, polar_p) in the working precision: K relative vectors rel
// ([K][3], template-vertex order), template t; P[9] row-major.
template <int K, typename RT>
__global__ void k_selftest_strain(const TemplateDev *__restrict__ tpl, int t, const double *__restrict__ rel,
                                  double *__restrict__ P) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const TemplateDev &D = tpl[t];
    double v[K][3];
    uint64_t tv = 0;
    for (int r = 0; r < K; r++) {
        for (int d = 0; d < 3; d++) v[r][d] = rel[3 * r + d];
        tv |= (uint64_t)r << (4 * r);
    }
    RT a0[3], At[3][3], l, Pm[3][3];
    strain_inputs<K, RT>(D, tv, v, a0, At, l);
    polar_p<RT>(At, l, Pm);
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) P[3 * x + y] = (double)Pm[x][y];
}

template <typename RT>
static void launch_selftest_strain_rt(const TablesView &T, int t, const double *rel, double *P, hipStream_t st) {
    const int k = template_k(t);
    if (k == 6) hipLaunchKernelGGL((k_selftest_strain<6, RT>), dim3(1), dim3(64), 0, st, T.tpl, t, rel, P);
    else if (k == 12) hipLaunchKernelGGL((k_selftest_strain<12, RT>), dim3(1), dim3(64), 0, st, T.tpl, t, rel, P);
    else hipLaunchKernelGGL((k_selftest_strain<14, RT>), dim3(1), dim3(64), 0, st, T.tpl, t, rel, P);
}
void launch_selftest_strain(const TablesView &T, int t, bool f32, const double *rel, double *P, hipStream_t st) {
    if (f32) launch_selftest_strain_rt<float>(T, t, rel, P, st);
    else launch_selftest_strain_rt<double>(T, t, rel, P, st);
}

// --------------------------------------------------------------- launches
// zero n int32 words (a kernel rather than a memset node, so that a captured
// stream replays it faithfully)
__global__ void k_fill_zero(int32_t *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
void launch_zero(int32_t *p, int64_t n, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, p, n);
}
void launch_bounds(const double *pos, int64_t n, double *part, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_bounds, dim3(nblocks), dim3(256), 0, st, pos, n, part);
}
void launch_bin_count(const double *pos, int64_t n, const Grid &g, int32_t *cell_of, int32_t *slot_of,
                      int32_t *count, hipStream_t st) {
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n, g, cell_of, slot_of,
                       count);
}
void launch_cell_starts(const int32_t *count, int64_t cells, int32_t *bsum, int32_t *start, hipStream_t st) {
    const int64_t items = scan_items(cells);
    hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)items), dim3(SCAN_THREADS), 0, st, count, cells, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, bsum, items);
    hipLaunchKernelGGL(k_scan_cells, dim3((unsigned)items), dim3(SCAN_THREADS), 0, st, count, cells,
                       (const int32_t *)bsum, start);
}
void launch_bin_scatter(const double *pos, int64_t n, const int32_t *cell_of, const int32_t *slot_of,
                        const int32_t *start, double *spos, int32_t *sid, hipStream_t st) {
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n, cell_of, slot_of,
                       start, spos, sid);
}
bool knn_fast_applies(const Grid &g) {
    for (int a = 0; a < 3; a++)
        if (g.periodic[a] && g.nc[a] < 5) return false;
    return true;
}
template <int NK>
static void launch_knn_nk(int64_t n, const Grid &g, const double *spos,
                          const int32_t *sid, const int32_t *start, int32_t *nbr_id, double *nbr_rel,
                          int32_t *todo, int32_t *todo_count, int32_t *box_fail, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (knn_fast_applies(g)) {
        hipLaunchKernelGGL(k_knn_fast<NK>, dim3((unsigned)xcd_pad(blocks)), dim3(256), 0, st, n, g, spos, sid,
                           start, nbr_id, nbr_rel, todo, todo_count, box_fail);
        // the atoms left over are few; 512 blocks of four waves (two per SIMD,
        // what its registers allow) stride over them
        hipLaunchKernelGGL(k_knn_exact<NK>, dim3((unsigned)std::min<int64_t>(blocks, 512)), dim3(256), 0, st, n, g,
                           spos, sid, start, nbr_id, nbr_rel, (const int32_t *)todo,
                           (const int32_t *)todo_count, box_fail);
    } else {
        hipLaunchKernelGGL(k_knn_exact<NK>, dim3((unsigned)std::min<int64_t>((n + 3) / 4, 16384)), dim3(256), 0, st, n,
                           g, spos, sid, start, nbr_id, nbr_rel, (const int32_t *)nullptr,
                           (const int32_t *)nullptr, box_fail);
    }
}
void launch_knn(int64_t n, const Grid &g, int nk, const double *spos,
                const int32_t *sid, const int32_t *start, int32_t *nbr_id, double *nbr_rel, int32_t *todo,
                int32_t *todo_count, int32_t *box_fail, hipStream_t st) {
    if (nk == VK)
        launch_knn_nk<VK>(n, g, spos, sid, start, nbr_id, nbr_rel, todo, todo_count, box_fail, st);
    else
        launch_knn_nk<KMAX>(n, g, spos, sid, start, nbr_id, nbr_rel, todo, todo_count, box_fail, st);
}
void launch_voronoi(int64_t n, const double *rel18, const int32_t *id18, uint32_t *vf, uint32_t *vlive,
                    double *nbr_rel, int32_t *nbr_id, const int32_t *box_fail, hipStream_t st) {
    const unsigned grid = (unsigned)xcd_pad((n + VB - 1) / VB);
    hipLaunchKernelGGL(k_voronoi_hull, dim3(grid), dim3(VB), 0, st, n, rel18, id18, vf, vlive, box_fail);
    hipLaunchKernelGGL(k_voronoi_order, dim3(grid), dim3(VB), 0, st, n, rel18, id18, (const uint32_t *)vf,
                       (const uint32_t *)vlive, nbr_rel, nbr_id, box_fail);
}
// Both precision forms use the FP32-storage hull kernel: every predicate is
// exact (a filter on the FP32 copies decides only when its bound proves the
// sign of the predicate on the FP64 inputs, otherwise the FP64 filter and
// the exact path run on the originals), so the hulls, codes and labellings
// are those of the FP64 kernel, with half the LDS per lane.
void launch_topo(int64_t n, const double *nbr_rel, const int32_t *nbr_id, const TablesView &T, uint32_t need,
                 int32_t *code, uint64_t *ord, const int32_t *box_fail, hipStream_t st) {
    dim3 grid((unsigned)((n + TB - 1) / TB)), block(TB);
    hipLaunchKernelGGL(k_topo, grid, block, 0, st, n, nbr_rel, nbr_id, T, need, code, ord, box_fail);
}
// ======================================== serving: one persistent kernel
// Every frame runs as nine stages of work items; the last item of a stage
// queues the next one (so stages of one frame follow each other, stages of
// different frames overlap).  A workgroup is one wave: it claims the item at
// the front of the device queue (an atomic range counter per (frame, stage)
// entry), runs it and counts it done.  Idle waves pull new frames from the
// pinned host block (one at a time, under a try-lock) and exit after a
// stretch of the device wall clock without work, or when the host sets
// stop: no wave waits on another, so every wave reaches an exit.
enum {
    PH_BOUNDS = 0,   // per-item bounds and non-finite flag
    PH_GRID = 1,     // one item: the grid from the bounds (make_grid on the device)
    PH_ZERO = 2,     // cell counters and frame counters to zero
    PH_COUNT = 3,    // cell of every atom, slot in its cell (atomic counts)
    PH_SCAN = 4,     // exclusive scan of the counts within each item, item totals
    PH_SCANTOP = 5,  // one item: exclusive scan of the item totals
    PH_SCATTER = 6,  // final cell starts (into the count array) and the sorted copy
    PH_KNN = 7,      // neighbours (fast search, exact search for what it leaves)
    PH_MATCH = 8     // hulls and codes, then the match stage, 64 atoms at a time
};

__device__ inline Grid make_grid_dev(const double (&box)[3], const double (&mn)[3], const double (&mx)[3], int64_t n,
                                     int kn) {
    // the host's make_grid (ptm_api.hip), same arithmetic
    Grid g;
    double ext[3], vol = 1.0;
    int flat = 0;
    for (int a = 0; a < 3; a++) {
        g.periodic[a] = box[a] > 0;
        ext[a] = g.periodic[a] ? box[a] : fmax(mx[a] - mn[a], 0.0);
        if (ext[a] > 0) vol *= ext[a];
        else flat++;
    }
    double h;
    if (flat == 0 && vol > 0) {
        const double rho = (double)n / vol;
        h = 0.6 * cbrt((double)kn / (4.1887902047863905 * rho));
    } else {
        h = 1.0;
        for (int a = 0; a < 3; a++) h = fmax(h, ext[a] / 16.0);
    }
    for (int iter = 0; iter < 200; iter++) {
        double cells = 1;
        for (int a = 0; a < 3; a++) {
            int nc;
            if (g.periodic[a]) nc = (int)fmin(floor(ext[a] / h), (double)(1 << 20));
            else nc = ext[a] > 0 ? (int)fmin(floor(ext[a] / h), (double)(1 << 20)) : 1;
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
        hmax = fmax(hmax, g.h[a]);
    }
    g.margin = 1e-9 * hmax;
    g.canonical = 1;
    for (int a = 0; a < 3; a++)
        if (g.periodic[a] && !(mn[a] >= 0.0 && mx[a] < box[a])) g.canonical = 0;
    return g;
}

__device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// queue entry: slot (16 bits), stage (8), generation (40)
__device__ inline unsigned long long serve_entry(int slot, int ph, unsigned long long gen) {
    return (unsigned long long)slot | ((unsigned long long)ph << 16) | (gen << 24);
}

// a stage's claim counter: the frame's generation (36 bits) over a 28-bit item index
constexpr int SERVE_IDX_BITS = 28;
constexpr unsigned long long SERVE_IDX_MASK = (1ull << SERVE_IDX_BITS) - 1;
__device__ inline unsigned long long serve_counter(unsigned long long gen) { return gen << SERVE_IDX_BITS; }

// append (slot, stage); the stage's item count and counter are set before
// (one lane)
__device__ inline void serve_push(ServeDev *dev, int slot, int ph, unsigned long long gen) {
    const unsigned long long pos = atomicAdd(&dev->tail, 1ull);
    dev->entry[pos % SERVE_FIFO] = serve_entry(slot, ph, gen);
    __threadfence();
    __hip_atomic_store(&dev->seq[pos % SERVE_FIFO], pos + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// the frame is finished: status, completion time, generation (one lane)
__device__ inline void serve_complete(ServeHost *host, int slot, unsigned long long gen, int status) {
    __threadfence_system();
    __hip_atomic_store(&host->status[slot], status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&host->t_done[slot], (long long)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&host->done[slot], gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// exclusive scan over the wave
__device__ inline long long wave_excl_scan(long long v, long long &total) {
    const int lane = threadIdx.x & 63;
    long long x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const long long y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    total = __shfl(x, 63);
    return x - v;
}

template <typename RT>
union ServeWork {
    TopoShared topo;
    MatchWork<RT, 1> mw;
};

// k-NN stage item: the fast search lane by lane, the exact one for what it
// leaves, a wave per atom (a call of its own: its registers apart)
__device__ __noinline__ void serve_knn(ServeSlot &S, int64_t r) {
    const int lane = threadIdx.x & 63;
    // the grid and the arrays in registers: the searches' stores cannot
    // alias them
    const Grid g = S.g;
    const int64_t n = S.r.n;
    const bool fast = S.fast;
    const double *spos = S.r.spos;
    const int32_t *sid = S.r.sid, *start = S.r.count;
    int32_t *nbr_id = S.r.nbr_id;
    double *nbr_rel = S.r.nbr_rel;
    int32_t *box_fail = S.r.count + S.cells + 3;
    const int64_t b = r * SERVE_ATOMS, e = min(n, b + SERVE_ATOMS);
    for (int64_t sub = b; sub < e; sub += 64) {
        const int64_t p = sub + lane;
        bool ok = true;
        if (p < e) ok = fast && knn_fast_atom<KMAX>(p, n, g, spos, sid, start, nbr_id, nbr_rel, box_fail);
        uint64_t left = __ballot(!ok);
        while (left) {
            const int l = __builtin_ctzll(left);
            left &= left - 1;
            knn_exact_atom<KMAX>(sub + l, n, g, spos, sid, start, nbr_id, nbr_rel, box_fail);
        }
    }
}

// hulls + match stage item, 64 atoms at a time (a call of its own)
// The LDS objects (templates, table view, outputs, working space) come as
// LDS-space pointers: a call's reference parameters are generic, and
// generic accesses to LDS are slower flat instructions; the generic views
// below derive from the LDS pointers, so the compiler turns their accesses
// back into LDS instructions.
// The hulls of one atom per lane, in a call of their own: its registers
// apart from the match's (LDS operands passed as LDS pointers)
__device__ __noinline__ void serve_topo(__attribute__((address_space(3))) TopoShared *Sp,
                                        __attribute__((address_space(3))) TablesView *Tp, int lane, int64_t p,
                                        int64_t n, const double *nbr_rel, const int32_t *nbr_id, uint32_t need,
                                        int32_t *code, uint64_t *ord) {
    topo_atom(*(TopoShared *)Sp, lane, p, n, nbr_rel, nbr_id, *(const TablesView *)Tp, need, code, ord);
}

template <typename RT>
__device__ __noinline__ void serve_match(__attribute__((address_space(3))) MatchShared *Mp,
                                         __attribute__((address_space(3))) TablesView *Tp,
                                         __attribute__((address_space(3))) MatchOut *Op,
                                         __attribute__((address_space(3))) ServeWork<RT> *Up, ServeSlot &S,
                                         int64_t r) {
    const MatchShared &M = *(const MatchShared *)Mp;
    const TablesView &T = *(const TablesView *)Tp;
    MatchOut &Ol = *(MatchOut *)Op;
    ServeWork<RT> &U = *(ServeWork<RT> *)Up;
    const int lane = threadIdx.x & 63;
    // the frame's parameters in registers (the stages' stores cannot alias them)
    const int64_t n = S.r.n, cells = S.cells;
    const double *nbr_rel = S.r.nbr_rel;
    const int32_t *nbr_id = S.r.nbr_id, *sid = S.r.sid;
    const int8_t *species = S.r.species;
    int32_t *code = S.r.code;
    uint64_t *ord = S.r.ord;
    int32_t *count = S.r.count, *knn_out = S.r.knn_out;
    const uint32_t mask = S.r.mask, need = S.r.need;
    const double cutoff = S.r.cutoff;
    const int64_t b = r * SERVE_ATOMS, e = min(n, b + SERVE_ATOMS);
    if (lane == 0) Ol = S.r.O;
    int32_t *full_count = count + cells + 2;
    unsigned long long *job_count = job_counter(count, cells);
    for (int64_t sub = b; sub < e; sub += 64) {
        const int64_t p = sub + lane;
        __syncthreads();  // the previous sub-block's match LDS is free; Ol is written
        if (p < e) serve_topo(&Up->topo, Tp, lane, p, n, nbr_rel, nbr_id, need, code, ord);
        // the wave's code / ord writes before other lanes read them
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
        match_block<RT, 1>(M, T, Ol, U.mw, sub, n, nbr_rel, nbr_id, sid, species, T, code, ord, mask, cutoff, 0,
                           Ol, full_count, job_count, nbr_id, knn_out);
    }
}

// Stage ph, item r of the frame in slot S (the whole wave).  Returns the
// stage's status for its last item (see serve_advance).
template <typename RT>
__device__ void serve_item(const MatchShared &M, const TablesView &Tl, MatchOut &Ol, ServeWork<RT> &U,
                           const TablesView &T, ServeSlot &S, int ph, int64_t r) {
    const int lane = threadIdx.x & 63;
    const ServeRequest &R = S.r;
    const int64_t n = R.n;
    if (ph == PH_BOUNDS) {
        const int64_t b = r * SERVE_ATOMS_LIGHT, e = min(n, b + SERVE_ATOMS_LIGHT);
        double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
        int bad = 0;
        for (int64_t i = b + lane; i < e; i += 64)
            for (int d = 0; d < 3; d++) {
                const double x = R.pos[3 * i + d];
                if (!isfinite(x)) bad = 1;
                mn[d] = fmin(mn[d], x);
                mx[d] = fmax(mx[d], x);
            }
        for (int off = 32; off > 0; off >>= 1) {
            for (int d = 0; d < 3; d++) {
                mn[d] = fmin(mn[d], __shfl_xor(mn[d], off));
                mx[d] = fmax(mx[d], __shfl_xor(mx[d], off));
            }
            bad |= __shfl_xor(bad, off);
        }
        if (lane == 0) {
            double *o = R.part + 7 * r;
            for (int d = 0; d < 3; d++) {
                o[d] = mn[d];
                o[3 + d] = mx[d];
            }
            o[6] = (double)bad;
        }
    } else if (ph == PH_GRID) {
        const int64_t nb = S.nr[PH_BOUNDS];
        double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
        int bad = 0;
        for (int64_t k = lane; k < nb; k += 64) {
            const double *o = R.part + 7 * k;
            for (int d = 0; d < 3; d++) {
                mn[d] = fmin(mn[d], o[d]);
                mx[d] = fmax(mx[d], o[3 + d]);
            }
            bad |= o[6] != 0.0;
        }
        for (int off = 32; off > 0; off >>= 1) {
            for (int d = 0; d < 3; d++) {
                mn[d] = fmin(mn[d], __shfl_xor(mn[d], off));
                mx[d] = fmax(mx[d], __shfl_xor(mx[d], off));
            }
            bad |= __shfl_xor(bad, off);
        }
        if (lane == 0) {
            const double box[3] = {R.box[0], R.box[1], R.box[2]};
            S.g = make_grid_dev(box, mn, mx, n, KMAX);
            S.cells = (int64_t)S.g.nc[0] * S.g.nc[1] * S.g.nc[2];
            bool fast = true;
            for (int a = 0; a < 3; a++)
                if (S.g.periodic[a] && S.g.nc[a] < 5) fast = false;
            S.fast = fast;
            S.bad = bad;  // non-finite coordinate: the frame stops here
        }
    } else if (ph == PH_ZERO) {
        const int64_t m = S.cells + FRAME_COUNTERS;
        const int64_t b = r * SERVE_ZERO_CELLS, e = min(m, b + SERVE_ZERO_CELLS);
        for (int64_t c = b + lane; c < e; c += 64) R.count[c] = 0;
    } else if (ph == PH_COUNT) {
        const int64_t b = r * SERVE_ATOMS_LIGHT, e = min(n, b + SERVE_ATOMS_LIGHT);
        const Grid &g = S.g;
        for (int64_t i = b + lane; i < e; i += 64) {
            const int cx = cell_coord(R.pos[3 * i + 0], g, 0);
            const int cy = cell_coord(R.pos[3 * i + 1], g, 1);
            const int cz = cell_coord(R.pos[3 * i + 2], g, 2);
            const int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
            R.cell_of[i] = c;
            R.slot_of[i] = atomicAdd(&R.count[c], 1);
        }
    } else if (ph == PH_SCAN) {
        // cells 0..cells (the last one counts zero: its start is the total)
        const int64_t m = S.cells + 1;
        const int64_t b = r * SERVE_SCAN_CELLS, e = min(m, b + SERVE_SCAN_CELLS);
        constexpr int64_t PER = SERVE_SCAN_CELLS / 64;
        const int64_t lb = b + lane * PER, le = min(e, lb + PER);
        long long sum = 0;
        for (int64_t c = lb; c < le; c++) sum += c < S.cells ? R.count[c] : 0;
        long long total;
        long long run = wave_excl_scan(sum, total);
        for (int64_t c = lb; c < le; c++) {
            R.start[c] = (int32_t)run;
            run += c < S.cells ? R.count[c] : 0;
        }
        if (lane == 0) R.bsum[r] = (int32_t)total;
    } else if (ph == PH_SCANTOP) {
        const int64_t m = S.nr[PH_SCAN];
        const int64_t per = ceil_div(m, 64);
        const int64_t lb = lane * per, le = min(m, lb + per);
        long long sum = 0;
        for (int64_t k = lb; k < le; k++) sum += R.bsum[k];
        long long total;
        long long run = wave_excl_scan(sum, total);
        for (int64_t k = lb; k < le; k++) {
            const int32_t v = R.bsum[k];
            R.bsum[k] = (int32_t)run;
            run += v;
        }
    } else if (ph == PH_SCATTER) {
        // final starts of this item's cells (the k-NN reads them from count)
        const int64_t m = S.cells + 1;
        const int64_t cb = r * SERVE_SCAN_CELLS, ce = min(m, cb + SERVE_SCAN_CELLS);
        if (cb < m) {
            const int32_t off = R.bsum[r];
            for (int64_t c = cb + lane; c < ce; c += 64) R.count[c] = R.start[c] + off;
        }
        const int64_t b = r * SERVE_ATOMS_LIGHT, e = min(n, b + SERVE_ATOMS_LIGHT);
        for (int64_t i = b + lane; i < e; i += 64) {
            const int32_t c = R.cell_of[i];
            const int64_t p = (int64_t)R.start[c] + R.bsum[c / SERVE_SCAN_CELLS] + R.slot_of[i];
            R.spos[3 * (int64_t)p] = R.pos[3 * i + 0];
            R.spos[3 * (int64_t)p + 1] = R.pos[3 * i + 1];
            R.spos[3 * (int64_t)p + 2] = R.pos[3 * i + 2];
            R.sid[p] = (int32_t)i;
        }
    } else if (ph == PH_KNN) {
        serve_knn(S, r);
    } else {  // PH_MATCH
        serve_match<RT>((__attribute__((address_space(3))) MatchShared *)&M,
                        (__attribute__((address_space(3))) TablesView *)&Tl,
                        (__attribute__((address_space(3))) MatchOut *)&Ol,
                        (__attribute__((address_space(3))) ServeWork<RT> *)&U, S, r);
    }
}

// `count` items of (slot, ph) are done: the stage's last one queues the next
// stage (or completes the frame).  Whole wave; one lane acts.  A wave counts
// its items of one stage together, when it moves to another stage or runs
// out of work: the release that makes its writes visible to the other XCDs
// (a write-back of the L2) then happens once per stage, not per item.
__device__ inline void serve_advance(ServeDev *dev, ServeHost *host, int slot, int ph, unsigned long long gen,
                                     long long count) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // these items' writes before their count
    if (lane != 0) return;
    ServeSlot &S = dev->slot[slot];
    const long long d = __hip_atomic_fetch_add(&S.done[ph], count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + count;
    if (d != S.nr[ph]) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every item's writes of the stage
    int next = ph + 1;
    if (ph == PH_GRID && S.bad) {
        serve_complete(host, slot, gen, SERVE_NONFINITE);
        return;
    }
    if (ph == PH_KNN && __hip_atomic_load(S.r.count + S.cells + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        serve_complete(host, slot, gen, SERVE_BOX);
        return;
    }
    if (ph == PH_MATCH) {
        serve_complete(host, slot, gen, SERVE_OK);
        return;
    }
    const int64_t n = S.r.n;
    long long nr = 1;
    switch (next) {
        case PH_ZERO: nr = ceil_div(S.cells + FRAME_COUNTERS, SERVE_ZERO_CELLS); break;
        case PH_COUNT: nr = ceil_div(n, SERVE_ATOMS_LIGHT); break;
        case PH_SCAN: nr = ceil_div(S.cells + 1, SERVE_SCAN_CELLS); break;
        case PH_SCANTOP: nr = 1; break;
        case PH_SCATTER: nr = max(ceil_div(S.cells + 1, SERVE_SCAN_CELLS), ceil_div(n, SERVE_ATOMS_LIGHT)); break;
        case PH_KNN: nr = ceil_div(n, SERVE_ATOMS); break;
        case PH_MATCH: nr = ceil_div(n, SERVE_ATOMS); break;
        default: nr = 1;
    }
    S.nr[next] = nr;
    S.done[next] = 0;
    __threadfence();
    __hip_atomic_store(&S.next[next], serve_counter(gen), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    serve_push(dev, slot, next, gen);
}

// An idle wave pulls the next frame the host published, if any, and queues
// its first stage.  Returns true if it did.
__device__ inline bool serve_pull(ServeDev *dev, ServeHost *host) {
    const int lane = threadIdx.x & 63;
    int slot = -1;
    if (lane == 0 && atomicCAS(&dev->poll_lock, 0, 1) == 0) {
        const unsigned long long ht = __hip_atomic_load(&host->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        const unsigned long long pulled = __hip_atomic_load(&dev->pulled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (pulled < ht) {
            slot = __hip_atomic_load(&host->ring[pulled % SERVE_SLOTS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&dev->pulled, pulled + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __hip_atomic_store(&dev->poll_lock, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    slot = __shfl(slot, 0);
    if (slot < 0) return false;
    // copy the request out of host memory, a word per lane
    ServeSlot &S = dev->slot[slot];
    constexpr int WORDS = sizeof(ServeRequest) / 8;
    static_assert(sizeof(ServeRequest) % 8 == 0, "request copied in 8-byte words");
    const unsigned long long *src = (const unsigned long long *)&host->req[slot];
    unsigned long long *dst = (unsigned long long *)&S.r;
    for (int w = lane; w < WORDS; w += 64)
        dst[w] = __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence();
    if (lane == 0) {
        const unsigned long long gen = S.r.gen;
        for (int k = 0; k < SERVE_NPH; k++) S.done[k] = 0;
        S.nr[PH_BOUNDS] = ceil_div(S.r.n, SERVE_ATOMS_LIGHT);
        S.bad = 0;
        __threadfence();
        __hip_atomic_store(&S.next[PH_BOUNDS], serve_counter(gen), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        serve_push(dev, slot, PH_BOUNDS, gen);
    }
    return true;
}

// The persistent kernel: one wave per workgroup (LDS: templates, the hull
// stage's per-lane state or the match stage's, in a union).
template <typename RT>
__global__ void __launch_bounds__(64, 2) k_serve(TablesView T, ServeDev *dev, ServeHost *host, long long idle_ticks) {
    __shared__ MatchShared M;
    __shared__ TablesView Tl;
    __shared__ MatchOut Ol;
    __shared__ ServeWork<RT> U;
    const int lane = threadIdx.x & 63;
    if (lane == 0) Tl = T;
    load_templates(M, T);
    long long idle_from = wall_clock64();
    int idle_rounds = 0;
    // the stage of this wave's items not yet counted (see serve_advance)
    int cur_slot = -1, cur_ph = 0;
    unsigned long long cur_gen = 0;
    long long pending = 0;
    for (;;) {
        int slot = -1, ph = 0;
        long long r = -1;
        unsigned long long gen = 0;
        if (lane == 0) {
            unsigned long long hd = __hip_atomic_load(&dev->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long tl = __hip_atomic_load(&dev->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (unsigned long long pos = hd; pos < tl && pos < hd + 64; pos++) {
                if (__hip_atomic_load(&dev->seq[pos % SERVE_FIFO], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                    pos + 1)
                    break;
                const unsigned long long e = dev->entry[pos % SERVE_FIFO];
                const int sl = (int)(e & 0xFFFF), p2 = (int)((e >> 16) & 0xFF);
                const unsigned long long g2 = e >> 24;
                ServeSlot &S = dev->slot[sl];
                // claim the next item.  The counter carries the frame's
                // generation: an entry left over from the slot's previous
                // frame sees another generation and leaves it alone; a claim
                // that races with the counter's reset for a new frame takes
                // an item of that frame, and runs it as such (the generation
                // comes from the counter).  Exhausted counters are not
                // incremented, so the index stays within its bits.
                const unsigned long long v = __hip_atomic_load(&S.next[p2], __ATOMIC_ACQUIRE,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                if ((v >> SERVE_IDX_BITS) == g2 && (long long)(v & SERVE_IDX_MASK) < S.nr[p2]) {
                    const unsigned long long w = __hip_atomic_fetch_add(&S.next[p2], 1ull, __ATOMIC_ACQ_REL,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
                    if ((long long)(w & SERVE_IDX_MASK) < S.nr[p2]) {
                        slot = sl;
                        ph = p2;
                        r = (long long)(w & SERVE_IDX_MASK);
                        gen = w >> SERVE_IDX_BITS;
                        break;
                    }
                }
                // exhausted (or stale): the front entry leaves the queue
                if (pos == hd && atomicCAS(&dev->head, hd, hd + 1) == hd) hd++;
            }
        }
        slot = __shfl(slot, 0);
        if (slot < 0) {
            if (pending) {
                // out of work: count what this wave did (it may finish a stage)
                serve_advance(dev, host, cur_slot, cur_ph, cur_gen, pending);
                __syncthreads();
                pending = 0;
                cur_slot = -1;
                continue;
            }
            // Idle.  Waves that find nothing back off (up to ~10 us between
            // looks at the queue), only one wave in 16 looks for new frames
            // in host memory, and the stop word (host memory too) is read
            // every 32nd idle round: idle waves keep the queue's cache lines
            // and the host link free for the working ones.
            if ((blockIdx.x & 15) == (idle_rounds & 15) && serve_pull(dev, host)) {
                idle_from = wall_clock64();
                idle_rounds = 0;
                continue;
            }
            idle_rounds++;
            if ((idle_rounds & 31) == 0 &&
                __hip_atomic_load(&host->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
                break;
            if (wall_clock64() - idle_from > idle_ticks) break;
            const int naps = idle_rounds < 6 ? (1 << idle_rounds) : 48;
            for (int z = 0; z < naps; z++) __builtin_amdgcn_s_sleep(8);
            continue;
        }
        idle_rounds = 0;
        ph = __shfl(ph, 0);
        r = __shfl(r, 0);
        gen = __shfl(gen, 0);
        if (slot != cur_slot || ph != cur_ph || gen != cur_gen) {
            // a new stage for this wave: count the previous one's items, and
            // see the new stage's inputs (an invalidation of the L2, once)
            if (pending) serve_advance(dev, host, cur_slot, cur_ph, cur_gen, pending);
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            cur_slot = slot;
            cur_ph = ph;
            cur_gen = gen;
            pending = 0;
        }
        serve_item<RT>(M, Tl, Ol, U, T, dev->slot[slot], ph, r);
        pending++;
        __syncthreads();
        idle_from = wall_clock64();
    }
    if (pending) serve_advance(dev, host, cur_slot, cur_ph, cur_gen, pending);
}

__global__ void k_wall_clock(long long *out) {
    if (threadIdx.x == 0) __hip_atomic_store(out, (long long)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_match(int64_t n, const double *nbr_rel, const int32_t *nbr_id, const int32_t *sid,
                  const int8_t *species, const TablesView &T, const int32_t *code, const uint64_t *ord,
                  uint32_t mask, double cutoff, bool force_full, const MatchOut &O, int32_t *full_count,
                  unsigned long long *job_count, const int32_t *knn_src, int32_t *knn_out, const int32_t *box_fail,
                  bool f32, hipStream_t st) {
    if (n <= 0) return;
    dim3 grid((unsigned)((n + MB - 1) / MB)), block(MB);
    if (f32)
        hipLaunchKernelGGL(k_match<float>, grid, block, 0, st, n, nbr_rel, nbr_id, sid, species, T, code, ord, mask,
                           cutoff, (int)force_full, O, full_count, job_count, knn_src, knn_out, box_fail);
    else
        hipLaunchKernelGGL(k_match<double>, grid, block, 0, st, n, nbr_rel, nbr_id, sid, species, T, code, ord,
                           mask, cutoff, (int)force_full, O, full_count, job_count, knn_src, knn_out, box_fail);
}

template <typename RT>
static int launch_serve_rt(const TablesView &T, ServeDev *dev, ServeHost *host, long long idle_ticks,
                           hipStream_t st) {
    int per_cu = 0, cus = 0, device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_serve<RT>, 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int blocks = per_cu * cus;
    hipLaunchKernelGGL(k_serve<RT>, dim3((unsigned)blocks), dim3(64), 0, st, T, dev, host, idle_ticks);
    return hipGetLastError() == hipSuccess ? blocks : 0;
}
int launch_serve(bool f32, const TablesView &T, ServeDev *dev, ServeHost *host, long long idle_ticks,
                 hipStream_t st) {
    return f32 ? launch_serve_rt<float>(T, dev, host, idle_ticks, st)
               : launch_serve_rt<double>(T, dev, host, idle_ticks, st);
}
void launch_wall_clock(long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_wall_clock, dim3(1), dim3(64), 0, st, out);
}

}  // namespace ptm
