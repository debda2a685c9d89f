/*
 * ptm_selftest.h -- self-check entry points of libptm.so.
 *
 * They run the library's own device arithmetic compiled for the host, so the
 * exact orientation predicate with Simulation of Simplicity (used for the
 * hull of Sec. 4 of arXiv:1603.05143) and the library's canonical code can
 * be checked on a machine without a GPU.  They are not part of the
 * classification path.  All pointers are host pointers.
 */
#ifndef PTM_SELFTEST_H
#define PTM_SELFTEST_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Sign (+1/-1) of det[b-a; c-a; d-a] for the rows a,b,c,d of p12[4][3],
 * exact, with Simulation of Simplicity by the four distinct ranks (the
 * lowest rank is perturbed most).  Returns 0 only if ranks are not distinct. */
int ptm_selftest_orient(const double *p12, const int32_t *ranks4);

/* Exact sign (-1/0/+1) of det[a; b; c] for the rows of p9[3][3]. */
int ptm_selftest_det3(const double *p9);

/* Key set of a triangulated sphere with k <= 14 vertices given as ntri
 * outward counter-clockwise triangles (int32 [ntri][3]): the start-edge
 * codes (k words each) of its start edges from vertices of minimum
 * degree, u ascending, then counter-clockwise around u from its
 * lowest-numbered neighbour (the first is the one the topology kernel looks
 * up).  Writes up to max_codes codes to codes[max_codes][k] and their
 * number to *n_codes.  Isomorphic graphs have equal key sets and the first
 * code of a graph lies in the key set of exactly the graphs isomorphic to
 * it.  Returns 0, or -1 if the triangles are not a closed oriented
 * triangulation. */
int ptm_selftest_codes(int k, const int32_t *tris, int ntri, uint64_t *codes, int max_codes, int32_t *n_codes);

/* Eq. (3) superposition for a fixed correspondence with the library's QCP
 * solver: obs and tpl are [N][3] (N <= 15, not centred / not normalised).
 * Writes rmsd, scale and the quaternion (w,x,y,z) rotating the template
 * onto the observation.  Returns 0, or -1 for N out of range. */
int ptm_selftest_superpose(int N, const double *obs, const double *tpl, double *rmsd, double *scale, double *q);

/* Decision (+1/-1, or 0 if undecided) of the FP32-storage orientation filter
 * of the FP32-mixed form on the FP32 roundings of p12[4][3]; a decided
 * sign must equal the exact sign of det[b-a; c-a; d-a] on the FP64 inputs. */
int ptm_selftest_orient_f32filter(const double *p12);

/* Same for det[a; b; c] (p9[3][3]). */
int ptm_selftest_det3_f32filter(const double *p9);

/* ptm_selftest_superpose evaluated in FP32 the way the FP32-mixed form
 * evaluates a candidate (centring in FP64, covariance, QCP and residual in
 * FP32).  excess (nullable) receives the bound d2 the FP32-mixed decision
 * keeps with the candidate: the amount by which the FP32 eigen-solve's
 * rotation and scale can raise RMSD^2 above its minimum, from the
 * conditioning of the top eigenpair of Horn's matrix (+inf when FP32
 * cannot resolve it: nearly equal top eigenvalues, or an eigenpair whose
 * Rayleigh quotient has not converged). */
int ptm_selftest_superpose_f32(int N, const double *obs, const double *tpl, double *rmsd, double *scale, double *q,
                               double *excess);

/* Strain of one match (eq. (6) least-squares fit with the pseudoinverse of
 * the normalised template, then P of the left polar decomposition A = P U
 * with U right-handed; Sec. 8) by the library's strain arithmetic: template
 * t (0..4), obs[k+1][3] the observed points in template-vertex order with
 * the centre first, precision PTM_FP64 (0) or PTM_FP32_MIXED (1, the FP32
 * arithmetic of that form).  Host evaluation; P[9] row-major.  Returns 0,
 * or -1 for t or precision out of range. */
int ptm_selftest_strain(int t, int precision, const double *obs, double *P);

/* The same on the device of a context, by the code the decision kernels
 * run, in the context's precision.  Host pointers; synchronous on the
 * context's stream.  Returns 0 (PTM_OK) or a ptm_status code. */
struct ptm_ctx;
int ptm_selftest_strain_device(struct ptm_ctx *ctx, int t, const double *obs, double *P);

#ifdef __cplusplus
}
#endif
#endif
