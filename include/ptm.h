/*
 * ptm.h -- C ABI of the MI355X Polyhedral Template Matching library
 * (libptm.so).  Method: Larsen, Schmidt & Schiotz, "Robust Structural
 * Identification via Polyhedral Template Matching", arXiv:1603.05143.
 *
 * For every atom the library finds the nearest neighbours (Sec. 3, Euclidean
 * ordering), builds the convex hull of the innermost 6, 12 and 14 neighbours
 * (Sec. 4; Alg. 1 requires the central atom strictly inside), reduces the
 * hull to its orientation-preserving canonical form (Sec. 4), looks it up
 * against the SC, FCC, HCP, ICO and BCC templates (Table 1, App. A) and
 * minimises the scale-invariant RMSD of eqs. (3)-(4) over the candidate
 * correspondences (Alg. 1).  It returns type, RMSD, scale, orientation,
 * ordered neighbours, the elastic strain of eq. (6) / Sec. 8 and the alloy
 * class of Sec. 6 / Table 3.
 *
 * Conventions
 *  - Status codes only; no exception crosses this boundary.  On an error no
 *    output is written (outputs may be partially written only by
 *    PTM_E_DEVICE, after which their contents are unspecified).
 *  - Pointers are device pointers (HIP, same device as the context) unless
 *    the context was created with PTM_F_HOST_POINTERS.  The caller owns
 *    all input and output buffers; they must stay valid until the call (or
 *    ticket) completes.  The context owns its tables and scratch memory.
 *  - Real outputs are float64 in both precision forms.
 *  - One context per host thread.  Calls on one context are serialised on
 *    its stream.
 */
#ifndef PTM_H
#define PTM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptm_ctx ptm_ctx; /* opaque: device tables, scratch, stream */

typedef enum {
    PTM_OK = 0,
    PTM_E_INVALID = 1,   /* bad argument: NULL pointer, n < 0, bad box, NaN/Inf coordinate */
    PTM_E_NOMEM = 2,     /* device allocation failed or HBM budget exceeded */
    PTM_E_DEVICE = 3,    /* HIP runtime error (message in ptm_last_error) */
    PTM_E_BOX = 4,       /* periodic box too short for the neighbour shell (see ptm_classify) */
    PTM_E_TOO_LARGE = 5, /* n > PTM_MAX_ATOMS */
    PTM_E_BUSY = 6,      /* serving queue full */
    PTM_E_TIMEOUT = 7    /* ptm_wait timed out; the ticket stays valid */
} ptm_status;

#define PTM_MAX_ATOMS 2147483646LL /* atom ids are int32 */

typedef enum {
    PTM_FP64 = 0,      /* superposition, orientation and strain in FP64; the exact steps (neighbour
                          order, hull predicates, codes) are the same in both forms                */
    PTM_FP32_MIXED = 1 /* superposition etc. in FP32 where an error bound proves the decision; FP64
                          otherwise                                                                  */
} ptm_precision;

/* template_mask bits (Table 1 templates) */
enum { PTM_SC = 1u << 0, PTM_FCC = 1u << 1, PTM_HCP = 1u << 2, PTM_ICO = 1u << 3, PTM_BCC = 1u << 4,
       PTM_ALL = 0x1Fu };

/* structure type output */
enum { PTM_TYPE_NONE = 0, PTM_TYPE_SC = 1, PTM_TYPE_FCC = 2, PTM_TYPE_HCP = 3, PTM_TYPE_ICO = 4,
       PTM_TYPE_BCC = 5 };

/* alloy output (Sec. 6, Table 3; species-agnostic: "same as / other than the
 * central atom") */
enum { PTM_ALLOY_NONE = 0, PTM_ALLOY_A1 = 1, PTM_ALLOY_L10 = 2, PTM_ALLOY_L12_MAJ = 3,
       PTM_ALLOY_L12_MIN = 4, PTM_ALLOY_FCC_OTHER = 5, PTM_ALLOY_A2 = 6, PTM_ALLOY_B2 = 7,
       PTM_ALLOY_BCC_OTHER = 8 };

/* context flags */
enum { PTM_F_HOST_POINTERS = 1u << 0, /* inputs/outputs are host pointers (staged through HBM) */
       PTM_F_PROFILE = 1u << 1,       /* record HIP events between pipeline stages */
       /* Topological neighbour ordering (Sec. 3) instead of the Euclidean one:
        * the 18 nearest neighbours (Sec. 9) are ordered by the area of the
        * interface between the Voronoi cell of the centre (taken with respect
        * to these 18) and theirs, larger first, then by 1/d; areas are compared
        * on a grid of 2^-20 of the cell surface, so equal areas tie and fall to
        * the Euclidean rank.  The first 6 / 12 / 14 of this order form the
        * hulls.  Atoms with fewer than 18 neighbours in the frame, or whose
        * cell is unbounded, keep the Euclidean order.  The knn output stays
        * Euclidean.  Costs 504 more bytes of scratch per atom. */
       PTM_F_TOPOLOGICAL = 1u << 2,
       /* decide every atom that has a candidate by the full rule (every
        * candidate superposed in FP64, ties by template and representative,
        * Alg. 1) instead of the working-precision common rule: results are
        * unchanged, only slower.  For tests of the full rule's path. */
       PTM_F_FULL_RULE = 1u << 3,
       /* serving (ptm_submit / ptm_wait) through one persistent kernel: the
        * frame is handed over in pinned host memory and every stage of it
        * (bounds, grid, binning and its scan, k-NN, hulls, match) runs as
        * work items of that kernel, frames overlapping stage by stage; no
        * launch or host round trip per frame.  The kernel exits after
        * 20 ms without work and is relaunched by the next ptm_submit or
        * ptm_wait.  Euclidean ordering only (with PTM_F_TOPOLOGICAL:
        * PTM_E_INVALID at ptm_create).  A non-finite coordinate is reported
        * by ptm_wait (PTM_E_INVALID), not by ptm_submit.  ptm_submit waits
        * on the host for the context stream's prior work. */
       PTM_F_PERSISTENT = 1u << 4 };

/* pipeline stages reported by ptm_stage_times */
enum { PTM_STAGE_BOUNDS = 0, PTM_STAGE_BIN = 1, PTM_STAGE_KNN = 2,
       PTM_STAGE_TOPO = 3 /* hulls of 6, 12, 14 neighbours, codes, lookup */,
       PTM_STAGE_MATCH = 4 /* superposition of every candidate, decision, orientation, strain, alloy,
                              write-back */,
       PTM_NSTAGES = 5 };

typedef struct {
    int device;                /* HIP device ordinal */
    ptm_precision precision;   /* PTM_FP64 or PTM_FP32_MIXED */
    void *hip_stream;          /* hipStream_t to run on; NULL = the context's own (non-blocking) stream.
                                  Device inputs written by work on another stream must be complete (or
                                  that stream waited on) before a call: the library orders its work on
                                  this stream only.  ptm_submit frames wait for this stream's prior
                                  work before they start. */
    uint64_t hbm_budget_bytes; /* cap on scratch + in-flight frames; 0 = no cap */
    uint32_t flags;            /* PTM_F_* */
} ptm_config;

/* Per-atom outputs, n entries each (arrays with a second dimension are
 * row-major [n][m]).  Every pointer except type may be NULL to skip it
 * (type too when n == 0).  Device outputs (contexts without
 * PTM_F_HOST_POINTERS): quat and quat_fz 16-byte aligned, neighbours
 * 8-byte aligned (records are written as 16- and 8-byte pairs; any HIP or
 * PyTorch allocation is), else PTM_E_INVALID. */
typedef struct {
    int8_t *type;        /* PTM_TYPE_*: best template if its RMSD <= rmsd_cutoff, else NONE      */
    int8_t *alloy;       /* PTM_ALLOY_*; NONE when species == NULL or type not FCC/BCC            */
    double *rmsd;        /* minimum eq.(3) RMSD over enabled templates; +inf if no candidate        */
    double *scale;       /* optimal s of eq.(3) (1/length); 0 if no candidate                      */
    double *quat;        /* [n][4] (w,x,y,z) of the rotation template -> sample, w >= 0; (1,0,0,0)
                            if no candidate                                                          */
    int32_t *neighbours; /* [n][14] atom ids in template-vertex order; -1 past k or if no candidate */
    double *strain;      /* [n][9] symmetric P of the left polar decomposition A = P U of eq.(6)   */
    int32_t *knn;        /* [n][14] atom ids in Euclidean order (Sec. 3); -1 past the last neighbour */
    /* derived from the best match (0, or (1,0,0,0), if there is no candidate) */
    double *vm_strain;       /* von Mises shear strain of P, sqrt(3/2 sum P_ij^2 - 1/2 (tr P)^2) (Sec. 8)  */
    double *strain_residual; /* residual of the least-squares fit of eq.(6): sum of squares over the N
                                normalised points (Falk-Langer D^2_min, Sec. 8)                            */
    double *nn_distance;     /* nearest-neighbour distance the fit implies: the distance of template
                                vertex 0 from the centre in eq.(4) units divided by s (the hydrostatic
                                part recovered from the scale, Sec. 8)                                  */
    double *quat_fz;         /* [n][4] the orientation in the fundamental zone (Sec. 7): of the
                                equivalent q x conj(q_h), h in the template's proper rotation group,
                                the one of largest w (the first in group order on ties), w >= 0       */
    int8_t *best_type;       /* the template of the minimum-RMSD match whatever rmsd_cutoff (NONE only
                                without a candidate): with rmsd, the input of ptm_apply_cutoff and
                                ptm_rmsd_histogram, so that the cut-off can be chosen after the
                                analysis (Sec. 5.1)                                                      */
} ptm_outputs;

/* Frame statistics returned by ptm_wait. */
typedef struct {
    double submit_time_us;   /* host clock at ptm_submit */
    double start_time_us;    /* host clock when the frame's work was enqueued on the device */
    double complete_time_us; /* host-clock time of the frame's completion on the device */
    int64_t n_atoms;
    uint64_t scratch_bytes;  /* pooled device scratch the frame held (counted against the budget) */
} ptm_frame_stats;

/* Create a context on cfg->device: builds the template tables (all
 * triangulations, canonical codes, rotation groups; Sec. 4, App. A) and
 * uploads them.  *out receives the context, or NULL on error.
 * Errors: PTM_E_INVALID (NULL arguments, bad precision), PTM_E_DEVICE (no
 * such device / HIP failure), PTM_E_NOMEM. */
ptm_status ptm_create(const ptm_config *cfg, ptm_ctx **out);

/* Classify n_atoms atoms of one frame (Alg. 1 for every atom).
 *   positions  [n][3] float64, any values; periodic axes are wrapped.
 *   species    [n] int8 or NULL (alloy output then NONE).
 *   box        host pointer to 3 doubles: > 0 periodic length of an
 *              orthorhombic box along that axis, 0 open.  Negative, NaN or
 *              Inf -> PTM_E_INVALID.
 *   template_mask  PTM_* bits of the templates to consider (0 allowed).
 *   rmsd_cutoff    keep the type iff RMSD <= cutoff (+inf = no cut-off,
 *                  Sec. 5.1); must not be NaN.
 * Stream-ordered on the context's stream; synchronises before returning.
 * Periodic boxes (Sec. 5 samples): neighbours are minimum images, which are
 * the periodic crystal's neighbours only when every atom's 14th neighbour
 * (18th with PTM_F_TOPOLOGICAL) lies strictly closer than half of each
 * periodic box length -- every other image of an atom is at least half a
 * length away.  Otherwise (tested as 4 d^2 < L*L in FP64, d^2 the squared
 * minimum-image distance; also when a frame with a periodic axis gives some
 * atom fewer than 14 / 18 neighbours) the call returns PTM_E_BOX and writes
 * no output: replicate the cell first.
 * Errors: PTM_E_INVALID, PTM_E_TOO_LARGE, PTM_E_NOMEM, PTM_E_DEVICE,
 * PTM_E_BOX.  n_atoms == 0 returns PTM_OK without touching the device. */
ptm_status ptm_classify(ptm_ctx *ctx, const double *positions, const int8_t *species,
                        const double *box, int64_t n_atoms, uint32_t template_mask,
                        double rmsd_cutoff, const ptm_outputs *out);

/* Largest frame of ptm_classify_noalloc. */
#define PTM_NOALLOC_MAX_ATOMS 65536

/* ptm_classify that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, outputs and errors as
 * ptm_classify on a device-pointer context; the pipeline's scratch is a
 * static 104 MiB array that each device the library runs on holds until the
 * process ends (room for n_atoms <= PTM_NOALLOC_MAX_ATOMS with either
 * neighbour ordering).  n_atoms above that -> PTM_E_TOO_LARGE, a
 * PTM_F_HOST_POINTERS context -> PTM_E_INVALID, both before any device work.
 * Every call on one device shares that array and leaves its contents behind:
 * calls that overlap on one device (from several contexts or threads) race.
 * Synchronises before returning, like ptm_classify. */
ptm_status ptm_classify_noalloc(ptm_ctx *ctx, const double *positions, const int8_t *species,
                                const double *box, int64_t n_atoms, uint32_t template_mask,
                                double rmsd_cutoff, const ptm_outputs *out);

/* Serving: enqueue one frame without waiting (continuous batching: frames
 * are admitted while the HBM budget allows, their work overlaps on the
 * device).  Arguments as ptm_classify; buffers must stay valid until
 * ptm_wait returns PTM_OK for the ticket.  Errors: as ptm_classify, plus
 * PTM_E_BUSY when the budget cannot admit the frame now (retry after a
 * ptm_wait). */
ptm_status ptm_submit(ptm_ctx *ctx, const double *positions, const int8_t *species,
                      const double *box, int64_t n_atoms, uint32_t template_mask,
                      double rmsd_cutoff, const ptm_outputs *out, uint64_t *ticket);

/* Wait for a ticket (timeout_us < 0: forever; 0: poll).  PTM_E_TIMEOUT if
 * not yet complete (the ticket stays valid); PTM_E_INVALID for an unknown
 * ticket; PTM_E_BOX when the frame's periodic box is too short (as for
 * ptm_classify: no output is written, the ticket is consumed).  stats may be
 * NULL. */
ptm_status ptm_wait(ptm_ctx *ctx, uint64_t ticket, int64_t timeout_us, ptm_frame_stats *stats);

/* Destroy a context (waits for in-flight tickets).  NULL is a no-op. */
void ptm_destroy(ptm_ctx *ctx);

/* Static description of a status code. */
const char *ptm_status_string(ptm_status s);

/* Last error message of a context (empty string if none; never NULL). */
const char *ptm_last_error(const ptm_ctx *ctx);

/* Device time in milliseconds of each pipeline stage of the most recent
 * ptm_classify on a context created with PTM_F_PROFILE, measured with HIP
 * events on the stream the kernels run on: ms[PTM_STAGE_*] for
 * min(n, PTM_NSTAGES) entries (0 for a stage that did not run).
 * PTM_E_INVALID if the context was not created with PTM_F_PROFILE. */
ptm_status ptm_stage_times(const ptm_ctx *ctx, double *ms, int n);

/* Work counts of the most recent ptm_classify on a PTM_F_PROFILE context:
 * info[PTM_INFO_*] for min(n, PTM_NINFO) entries.  Same errors as
 * ptm_stage_times. */
enum { PTM_INFO_CELLS = 0,      /* cells of the binning grid */
       PTM_INFO_KNN_EXACT = 1,  /* atoms whose neighbours the exact (whole-wave) search found */
       PTM_INFO_PAIRS = 2,      /* (atom, candidate correspondence) pairs superposed */
       PTM_INFO_DECIDE_FULL = 3, /* atoms decided by the full rule (near tie, FP32 margin) */
       PTM_NINFO = 4 };
ptm_status ptm_frame_info(const ptm_ctx *ctx, int64_t *info, int n);

/* Misorientation angles (Sec. 7): for i < n, angle[i] = the smallest
 * rotation angle (radians, in [0, pi]) of conj(q1_i) x q2_i x q_h over the
 * proper rotation group of template type[i] (PTM_TYPE_*; NONE: no symmetry,
 * the plain angle between the two orientations).  q1, q2: [n][4] unit
 * quaternions (w,x,y,z) as written to ptm_outputs.quat; type: [n] int8;
 * angle: [n] double.  Device pointers (host pointers on a PTM_F_HOST_POINTERS
 * context), caller-owned; runs on the context's stream and synchronises.
 * A type outside 0..5 gives NaN (device pointers) or PTM_E_INVALID before
 * any work (host pointers); PTM_E_INVALID also for NULL arrays with n > 0
 * or n < 0. */
ptm_status ptm_misorientation(ptm_ctx *ctx, const int8_t *type, const double *q1, const double *q2, int64_t n,
                              double *angle);

/* Post-hoc cut-off (Sec. 5.1: RMSD_max can be chosen after the analysis):
 * type[i] = best_type[i] if rmsd[i] <= rmsd_cutoff, else PTM_TYPE_NONE, for
 * i < n.  Arrays as written by ptm_classify (device pointers, or host ones
 * on a PTM_F_HOST_POINTERS context), caller-owned; the context's stream,
 * synchronised.  PTM_E_INVALID for NULL arrays with n > 0 or n < 0. */
ptm_status ptm_apply_cutoff(ptm_ctx *ctx, const int8_t *best_type, const double *rmsd, int64_t n,
                            double rmsd_cutoff, int8_t *type);

/* RMSD histograms per structure type (Sec. 5.1, Fig. 4: the way to pick
 * RMSD_max): counts[t * nbins + b] (host array of 6 * nbins int64,
 * overwritten) = number of atoms with best_type t and rmsd in bin b of
 * nbins equal bins over [0, rmax); an RMSD >= rmax (or +inf) counts in the
 * last bin.  best_type, rmsd as for ptm_apply_cutoff.  PTM_E_INVALID for
 * NULL arrays with n > 0, n < 0, nbins outside 1..65536 or rmax <= 0. */
ptm_status ptm_rmsd_histogram(ptm_ctx *ctx, const int8_t *best_type, const double *rmsd, int64_t n, int nbins,
                              double rmax, int64_t *counts);

/* Template facts of the library's own tables, for checks without a device:
 * info[0]=k, info[1]=rotation group order, info[2]=triangulations,
 * info[3]=distinct table keys (orientation-preserving start-edge codes of
 * the triangulations), info[4]=candidate correspondences kept after the
 * reduction by the template's rotation group (App. A).  Returns PTM_E_INVALID for t outside 0..4. */
ptm_status ptm_template_info(int t, int64_t info[5]);

#ifdef __cplusplus
}
#endif
#endif /* PTM_H */
