// ptm_device.hpp -- device arithmetic of the HIP path (also compiled for
// the host so the self-check entry points can exercise it without a GPU).
//
//  * orientation predicates with an FP64 (or FP32) error-bounded filter and
//    an exact fallback on floating-point expansions (error-free sums and
//    products, Dekker/Knuth; expansion growth after Shewchuk 1997), plus
//    Simulation of Simplicity (Edelsbrunner & Muecke 1990) for exact zeros
//    -- the hull of Sec. 4 is thereby a function of the input alone;
//  * the QCP solve of the superposition of eqs. (2)-(4) (Theobald 2005; Liu
//    et al. 2010): characteristic polynomial of Horn's 4x4 matrix, Newton
//    from an upper bound, eigenvector from the adjugate;
//  * cyclic Jacobi for 3x3 symmetric matrices, and the strain of eq. (6) and
//    Sec. 8 (pseudoinverse fit, symmetric factor of the left polar
//    decomposition with a right-handed rotation).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ptm_tables.hpp"

namespace ptm {

#define PTM_HD __host__ __device__ inline

// ------------------------------------------------------------------ exact
struct Expansion {
    int n;
    double c[112];
};

PTM_HD void exact_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bv = s - a;
    double av = s - bv;
    e = (a - av) + (b - bv);
}

PTM_HD void exact_prod(double a, double b, double &p, double &e) {
    p = a * b;
    e = fma(a, b, -p);
}

// x += b exactly; zero components dropped
PTM_HD void exp_grow(Expansion &x, double b) {
    double q = b;
    int m = 0;
    for (int i = 0; i < x.n; i++) {
        double s, h;
        exact_sum(q, x.c[i], s, h);
        q = s;
        if (h != 0.0) x.c[m++] = h;
    }
    if (q != 0.0) x.c[m++] = q;
    x.n = m;
}

PTM_HD int exp_sign(const Expansion &x) {
    for (int i = x.n - 1; i >= 0; i--)
        if (x.c[i] != 0.0) return x.c[i] > 0.0 ? 1 : -1;
    return 0;
}

// x += sgn * a*b*c exactly
PTM_HD void exp_add_prod3(Expansion &x, double a, double b, double c, double sgn) {
    double p, e;
    exact_prod(a, b, p, e);
    double p1, e1, p2, e2;
    exact_prod(p, c, p1, e1);
    exact_prod(e, c, p2, e2);
    exp_grow(x, sgn * p1);
    exp_grow(x, sgn * e1);
    exp_grow(x, sgn * p2);
    exp_grow(x, sgn * e2);
}

PTM_HD void exp_add_prod2(Expansion &x, double a, double b, double sgn) {
    double p, e;
    exact_prod(a, b, p, e);
    exp_grow(x, sgn * p);
    exp_grow(x, sgn * e);
}

// x += sgn * det[p; q; r] (rows, raw coordinates) exactly
PTM_HD void exp_add_det3(Expansion &x, const double *p, const double *q, const double *r, double sgn) {
    exp_add_prod3(x, p[0], q[1], r[2], sgn);
    exp_add_prod3(x, p[0], q[2], r[1], -sgn);
    exp_add_prod3(x, p[1], q[0], r[2], -sgn);
    exp_add_prod3(x, p[1], q[2], r[0], sgn);
    exp_add_prod3(x, p[2], q[0], r[1], sgn);
    exp_add_prod3(x, p[2], q[1], r[0], -sgn);
}

// Sign of det of the 4x4 matrix with rows (p_i, 1): Laplace expansion along
// the constant column, each 3x3 minor evaluated exactly.
#ifdef __HIP_DEVICE_COMPILE__
__attribute__((noinline))
#endif
__host__ __device__ inline int lambda4_sign_exact(const double *a, const double *b, const double *c, const double *d) {
    Expansion x;
    x.n = 0;
    exp_add_det3(x, b, c, d, -1.0);
    exp_add_det3(x, a, c, d, 1.0);
    exp_add_det3(x, a, b, d, -1.0);
    exp_add_det3(x, a, b, c, 1.0);
    return exp_sign(x);
}

// exact sign of det[[p_i, p_j, 1], [q_i, q_j, 1], [r_i, r_j, 1]] on coordinates (i, j)
#ifdef __HIP_DEVICE_COMPILE__
__attribute__((noinline))
#endif
__host__ __device__ inline int orient2_sign_exact(const double *p, const double *q, const double *r, int i, int j) {
    Expansion x;
    x.n = 0;
    exp_add_prod2(x, p[i], q[j], 1.0);
    exp_add_prod2(x, p[j], q[i], -1.0);
    exp_add_prod2(x, p[i], r[j], -1.0);
    exp_add_prod2(x, p[j], r[i], 1.0);
    exp_add_prod2(x, q[i], r[j], 1.0);
    exp_add_prod2(x, q[j], r[i], -1.0);
    return exp_sign(x);
}

PTM_HD int sgn_diff(double a, double b) { return a > b ? 1 : (a < b ? -1 : 0); }

// Simulation of Simplicity for the 4x4 orientation determinant.  Rows sorted
// by increasing rank r0 < r1 < r2 < r3; rank r's coordinate j is perturbed by
// eps^(2^(3r+2-j)) (j = 0,1,2 for x,y,z), so the lowest rank moves most and z
// before y before x.  The perturbed determinant is a polynomial in eps whose
// coefficients are signed minors; in order of decreasing size the
// non-vanishing candidates are listed below as (sign, minor).  Returns the
// sign of det L_sorted(eps).
#ifdef __HIP_DEVICE_COMPILE__
__attribute__((noinline))
#endif
__host__ __device__ inline int sos_lambda4_sorted(const double *p0, const double *p1, const double *p2,
                                           const double *p3) {
    int s;
    // eps(r0,z): +det[x y 1] of rows 1,2,3
    if ((s = orient2_sign_exact(p1, p2, p3, 0, 1))) return s;
    // eps(r0,y): -det[x z 1] of rows 1,2,3
    if ((s = orient2_sign_exact(p1, p2, p3, 0, 2))) return -s;
    // eps(r0,x): +det[y z 1] of rows 1,2,3
    if ((s = orient2_sign_exact(p1, p2, p3, 1, 2))) return s;
    // eps(r1,z): -det[x y 1] of rows 0,2,3
    if ((s = orient2_sign_exact(p0, p2, p3, 0, 1))) return -s;
    // eps(r0,y) eps(r1,z): +(x2 - x3)
    if ((s = sgn_diff(p2[0], p3[0]))) return s;
    // eps(r0,x) eps(r1,z): -(y2 - y3)
    if ((s = sgn_diff(p2[1], p3[1]))) return -s;
    // eps(r1,y): +det[x z 1] of rows 0,2,3
    if ((s = orient2_sign_exact(p0, p2, p3, 0, 2))) return s;
    // eps(r0,z) eps(r1,y): -(x2 - x3)
    if ((s = sgn_diff(p2[0], p3[0]))) return -s;
    // eps(r0,x) eps(r1,y): +(z2 - z3)
    if ((s = sgn_diff(p2[2], p3[2]))) return s;
    // eps(r1,x): -det[y z 1] of rows 0,2,3
    if ((s = orient2_sign_exact(p0, p2, p3, 1, 2))) return -s;
    // eps(r0,z) eps(r1,x): +(y2 - y3)
    if ((s = sgn_diff(p2[1], p3[1]))) return s;
    // eps(r0,y) eps(r1,x): -(z2 - z3)
    if ((s = sgn_diff(p2[2], p3[2]))) return -s;
    // eps(r2,z): +det[x y 1] of rows 0,1,3
    if ((s = orient2_sign_exact(p0, p1, p3, 0, 1))) return s;
    // eps(r0,y) eps(r2,z): -(x1 - x3)
    if ((s = sgn_diff(p1[0], p3[0]))) return -s;
    // eps(r0,x) eps(r2,z): +(y1 - y3)
    if ((s = sgn_diff(p1[1], p3[1]))) return s;
    // eps(r1,y) eps(r2,z): +(x0 - x3)
    if ((s = sgn_diff(p0[0], p3[0]))) return s;
    // eps(r0,x) eps(r1,y) eps(r2,z): +1
    return 1;
}

// orientation of (a,b,c,d) := det[b-a; c-a; d-a] (> 0: d on the side the
// normal (b-a)x(c-a) points to), exactly, with SoS by the ranks ra..rd
#ifdef __HIP_DEVICE_COMPILE__
__attribute__((noinline))
#endif
__host__ __device__ inline int orient_exact_sos(const double *a, const double *b, const double *c, const double *d, int ra,
                            int rb, int rc, int rd) {
    int s = lambda4_sign_exact(a, b, c, d);
    if (s) return -s;
    const double *p[4] = {a, b, c, d};
    int r[4] = {ra, rb, rc, rd};
    int parity = 1;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3 - i; j++)
            if (r[j] > r[j + 1]) {
                int tr = r[j]; r[j] = r[j + 1]; r[j + 1] = tr;
                const double *tp = p[j]; p[j] = p[j + 1]; p[j + 1] = tp;
                parity = -parity;
            }
    return -parity * sos_lambda4_sorted(p[0], p[1], p[2], p[3]);
}

// Semi-static filter for det[b-a; c-a; d-a] in FP64 with exact inputs.
// Returns the sign, or 0 when the error bound does not decide it.  The
// evaluation uses differences against d (det[a-d; b-d; c-d] = -orient) and
// the bound 10 u x permanent (u = 2^-53) covers the 3 input differences, 2 products,
// 1 subtraction, 1 product and 2 additions of each term.
PTM_HD int orient_filter64(const double *a, const double *b, const double *c, const double *d) {
    double adx = a[0] - d[0], ady = a[1] - d[1], adz = a[2] - d[2];
    double bdx = b[0] - d[0], bdy = b[1] - d[1], bdz = b[2] - d[2];
    double cdx = c[0] - d[0], cdy = c[1] - d[1], cdz = c[2] - d[2];
    double m1 = bdx * cdy, m2 = cdx * bdy;
    double m3 = cdx * ady, m4 = adx * cdy;
    double m5 = adx * bdy, m6 = bdx * ady;
    double det = adz * (m1 - m2) + bdz * (m3 - m4) + cdz * (m5 - m6);
    double perm = (fabs(m1) + fabs(m2)) * fabs(adz) + (fabs(m3) + fabs(m4)) * fabs(bdz) +
                  (fabs(m5) + fabs(m6)) * fabs(cdz);
    double bound = 1.1102230246251565e-15 * perm;  // 10 unit roundoffs of perm
    if (det > bound) return -1;
    if (det < -bound) return 1;
    return 0;
}

// det[a; b; c] (raw coordinates) filter; 0 if undecided
PTM_HD int det3_filter64(const double *a, const double *b, const double *c) {
    double m1 = b[1] * c[2], m2 = b[2] * c[1];
    double m3 = b[2] * c[0], m4 = b[0] * c[2];
    double m5 = b[0] * c[1], m6 = b[1] * c[0];
    double det = a[0] * (m1 - m2) + a[1] * (m3 - m4) + a[2] * (m5 - m6);
    double perm = fabs(a[0]) * (fabs(m1) + fabs(m2)) + fabs(a[1]) * (fabs(m3) + fabs(m4)) +
                  fabs(a[2]) * (fabs(m5) + fabs(m6));
    double bound = 8.8817841970012523e-16 * perm;  // 8 unit roundoffs
    if (det > bound) return 1;
    if (det < -bound) return -1;
    return 0;
}

// Static error bounds.  For a point set whose coordinates are at most m in
// magnitude every entry of the difference matrix of an orientation test is
// at most 2m, and a perturbation of at most e per entry moves each of the six
// products of the 3x3 determinant by at most 3 (2m)^2 e (first order), so the
// determinant by at most 18 (2m)^2 e; for det[a; b; c] on the raw points the
// same argument gives 18 m^2 e.  The bounds below are fixed per atom (m = the
// largest coordinate of its neighbour vectors), so a test costs the
// determinant alone.  Tiny sets (bound below 1e-290) are never decided.
//
// FP32 storage and FP32 arithmetic: each coordinate x32 is the FP32
// rounding of the exact FP64 input (|x32 - x| <= 2^-24 |x|; m is taken from
// the x32 with a factor 1 + 2^-22).  Orientation: a difference computed in
// FP32 is off the exact one by at most 2^-24 (|a| + |d|) + 2^-24 |a32 - d32|
// <= 2^-22 m, which moves the determinant by at most 18 (2m)^2 2^-22 m =
// 288 2^-24 m^3; the FP32 evaluation (three roundings inside each of the six
// triple products, two in the sums) adds at most 5 2^-24 times the
// permanent, <= 6 (2m)^3 = 48 m^3: 528 2^-24 m^3 = 3.15e-5 m^3 -> 3.3e-5 m^3.
// det[a; b; c]: 18 m^3 2^-24 for the inputs, 5 2^-24 6 m^3 for the
// evaluation: 48 2^-24 m^3 = 2.9e-6 m^3 -> 3.0e-6 m^3.  Outside 1e-9 < M <
// 1e12 (FP32 underflow or overflow of the products) the filter never
// decides.  A decided sign is the exact sign of the predicate on the FP64
// inputs.
PTM_HD double f32_orient_bound(double m) {
    double M = m * (1.0 + 0x1p-22);
    return (M > 1e-9 && M < 1e12) ? 3.3e-5 * M * M * M : INFINITY;
}
PTM_HD double f32_det3_bound(double m) {
    double M = m * (1.0 + 0x1p-22);
    return (M > 1e-9 && M < 1e12) ? 3.0e-6 * M * M * M : INFINITY;
}
// FP64 inputs: the rounding of the differences (e = 2^-53 2m) and 10 unit
// roundoffs of the evaluation on a permanent of at most 6 (2m)^3 give
// (144 + 480) 2^-53 m^3 = 6.9e-14 m^3 -> 7e-14 m^3; det3: 8 unit roundoffs
// of at most 6 m^3 -> 5.4e-15 m^3.
PTM_HD double f64_orient_bound(double m) { return fmax(7e-14 * m * m * m, 1e-290); }
PTM_HD double f64_det3_bound(double m) { return fmax(5.4e-15 * m * m * m, 1e-290); }

// det[a-d; b-d; c-d] = -det[b-a; c-a; d-a] from FP32 points in FP32
// arithmetic: the value the FP32 orientation filter compares with its bound
PTM_HD float orient_det_f32in(const float *a, const float *b, const float *c, const float *d) {
    // fused multiply-adds round once where a product and a sum round twice,
    // so the error bound of the unfused evaluation covers them
#pragma clang fp contract(fast)
    const float adx = a[0] - d[0], ady = a[1] - d[1], adz = a[2] - d[2];
    const float bdx = b[0] - d[0], bdy = b[1] - d[1], bdz = b[2] - d[2];
    const float cdx = c[0] - d[0], cdy = c[1] - d[1], cdz = c[2] - d[2];
    return adz * (bdx * cdy - cdx * bdy) + bdz * (cdx * ady - adx * cdy) + cdz * (adx * bdy - bdx * ady);
}

// det[b-a; c-a; d-a] sign from FP32 points in FP32 arithmetic; 0 when |det| <=
// bound (f32_orient_bound).
PTM_HD int orient_filter_f32in(const float *a, const float *b, const float *c, const float *d, double bound) {
    const float det = orient_det_f32in(a, b, c, d);
    const float bf = (float)bound;
    if (det > bf) return -1;
    if (det < -bf) return 1;
    return 0;
}

// det[a; b; c] from FP32 points in FP32 arithmetic: the value the FP32
// determinant filter compares with its bound
PTM_HD float det3_f32in(const float *a, const float *b, const float *c) {
    // fused multiply-adds round once where a product and a sum round twice,
    // so the error bound of the unfused evaluation covers them
#pragma clang fp contract(fast)
    return a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
}

// det[a; b; c] sign from FP32 points in FP32 arithmetic; 0 when |det| <=
// bound (f32_det3_bound)
PTM_HD int det3_filter_f32in(const float *a, const float *b, const float *c, double bound) {
    const float det = det3_f32in(a, b, c);
    const float bf = (float)bound;
    if (det > bf) return 1;
    if (det < -bf) return -1;
    return 0;
}

// FP64 filters with a static bound (same evaluation as orient_filter64 /
// det3_filter64, without the per-test permanent)
PTM_HD int orient_filter64b(const double *a, const double *b, const double *c, const double *d, double bound) {
    // fused multiply-adds round once where a product and a sum round twice,
    // so the error bound of the unfused evaluation covers them
#pragma clang fp contract(fast)
    double adx = a[0] - d[0], ady = a[1] - d[1], adz = a[2] - d[2];
    double bdx = b[0] - d[0], bdy = b[1] - d[1], bdz = b[2] - d[2];
    double cdx = c[0] - d[0], cdy = c[1] - d[1], cdz = c[2] - d[2];
    double det = adz * (bdx * cdy - cdx * bdy) + bdz * (cdx * ady - adx * cdy) + cdz * (adx * bdy - bdx * ady);
    if (det > bound) return -1;
    if (det < -bound) return 1;
    return 0;
}

PTM_HD int det3_filter64b(const double *a, const double *b, const double *c, double bound) {
    // fused multiply-adds round once where a product and a sum round twice,
    // so the error bound of the unfused evaluation covers them
#pragma clang fp contract(fast)
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                 a[2] * (b[0] * c[1] - b[1] * c[0]);
    if (det > bound) return 1;
    if (det < -bound) return -1;
    return 0;
}

#ifdef __HIP_DEVICE_COMPILE__
__attribute__((noinline))
#endif
__host__ __device__ inline int det3_sign_exact(const double *a, const double *b, const double *c) {
    Expansion x;
    x.n = 0;
    exp_add_det3(x, a, b, c, 1.0);
    return exp_sign(x);
}

PTM_HD int orient_sos64(const double *a, const double *b, const double *c, const double *d, int ra, int rb,
                        int rc, int rd) {
    int s = orient_filter64(a, b, c, d);
    if (s) return s;
    return orient_exact_sos(a, b, c, d, ra, rb, rc, rd);
}

PTM_HD int det3_sign64(const double *a, const double *b, const double *c) {
    int s = det3_filter64(a, b, c);
    if (s) return s;
    return det3_sign_exact(a, b, c);
}

// the same with a static filter bound (f64_orient_bound / f64_det3_bound)
PTM_HD int orient_sos64b(const double *a, const double *b, const double *c, const double *d, int ra, int rb,
                         int rc, int rd, double bound) {
    int s = orient_filter64b(a, b, c, d, bound);
    if (s) return s;
    return orient_exact_sos(a, b, c, d, ra, rb, rc, rd);
}

PTM_HD int det3_sign64b(const double *a, const double *b, const double *c, double bound) {
    int s = det3_filter64b(a, b, c, bound);
    if (s) return s;
    return det3_sign_exact(a, b, c);
}

// ------------------------------------------------------------------- QCP
template <typename T>
struct RealTraits;
template <>
struct RealTraits<double> {
    static constexpr double newton_tol = 1e-15;
    static constexpr double jacobi_off = 1e-36;
    static constexpr double polar_step = 1e-8;
};
template <>
struct RealTraits<float> {
    static constexpr float newton_tol = 2e-7f;
    static constexpr float jacobi_off = 1e-14f;
    static constexpr float polar_step = 2e-4f;
};

// Largest eigenvalue and eigenvector of Horn's matrix for S_xy = sum b_x a_y
// (template b, observation a); q (w,x,y,z) rotates b onto a.  Ga, Gb are the
// inner products of the two sets (upper bound sqrt(Ga Gb) on lambda).
// cond (optional) receives a conditioning measure of the computed top
// eigenpair, 0 when it cannot be trusted: sqrt(best) / lambda^3, best the
// largest squared column norm of adj(K - lambda I) -- for an exact top
// eigenpair that column is |prod_j (lambda - lambda_j)| times a component
// of the eigenvector (at least 1/2 in the largest), so cond bounds the
// product of the gaps to the other three eigenvalues; each gap is at most
// 4 lambda (K is traceless), hence the smallest gap is at least
// cond * lambda / 16.  That reading holds only for a converged eigenpair:
// Newton approaches the largest root from above (lambda >= lambda_1) and
// the Rayleigh quotient rho = q^T K q is at most lambda_1, so
// lambda - rho >= 0 bounds both the eigenvalue error and the eigenvector's
// suboptimality; cond is 0 unless lambda - rho <= 64 u lambda (u the unit
// roundoff of T), and 0 if lambda <= 0.
template <typename T>
__host__ __device__ inline T qcp_solve(const T S[3][3], T Ga, T Gb, T q[4], T *cond = nullptr) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    const T Sxx = S[0][0], Sxy = S[0][1], Sxz = S[0][2];
    const T Syx = S[1][0], Syy = S[1][1], Syz = S[1][2];
    const T Szx = S[2][0], Szy = S[2][1], Szz = S[2][2];
    T K[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
                 {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
                 {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
                 {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
    // characteristic polynomial lambda^4 + c2 lambda^2 + c1 lambda + c0
    T ss = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) ss += S[i][j] * S[i][j];
    T c2 = T(-2) * ss;
    T detS = Sxx * (Syy * Szz - Syz * Szy) - Sxy * (Syx * Szz - Syz * Szx) + Sxz * (Syx * Szy - Syy * Szx);
    T c1 = T(-8) * detS;
    // c0 = det K by complementary 2x2 minors of rows (0,1) and (2,3)
    T s01 = K[0][0] * K[1][1] - K[0][1] * K[1][0], s02 = K[0][0] * K[1][2] - K[0][2] * K[1][0];
    T s03 = K[0][0] * K[1][3] - K[0][3] * K[1][0], s12 = K[0][1] * K[1][2] - K[0][2] * K[1][1];
    T s13 = K[0][1] * K[1][3] - K[0][3] * K[1][1], s23 = K[0][2] * K[1][3] - K[0][3] * K[1][2];
    T t01 = K[2][0] * K[3][1] - K[2][1] * K[3][0], t02 = K[2][0] * K[3][2] - K[2][2] * K[3][0];
    T t03 = K[2][0] * K[3][3] - K[2][3] * K[3][0], t12 = K[2][1] * K[3][2] - K[2][2] * K[3][1];
    T t13 = K[2][1] * K[3][3] - K[2][3] * K[3][1], t23 = K[2][2] * K[3][3] - K[2][3] * K[3][2];
    T c0 = s01 * t23 - s02 * t13 + s03 * t12 + s12 * t03 - s13 * t02 + s23 * t01;
    T lam = sqrt(Ga * Gb);
    for (int it = 0; it < 60; it++) {
        T l2 = lam * lam;
        T f = (l2 + c2) * l2 + c1 * lam + c0;
        T fp = T(4) * l2 * lam + T(2) * c2 * lam + c1;
        if (fp == T(0)) break;
        T step = f / fp;
        lam -= step;
        if (fabs(step) <= RealTraits<T>::newton_tol * fabs(lam) + T(1e-30)) break;
    }
    // eigenvector: the adjugate column of (K - lam I) with the largest norm
    T A[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) A[i][j] = K[i][j] - (i == j ? lam : T(0));
    T best = -1;
    q[0] = 1; q[1] = q[2] = q[3] = 0;
    for (int col = 0; col < 4; col++) {
        // cofactors C_{col,i} = (-1)^{col+i} det(A without row col, col i)
        T v[4];
        for (int i = 0; i < 4; i++) {
            int r[3], c[3], nr = 0, nc = 0;
            for (int t = 0; t < 4; t++) {
                if (t != col) r[nr++] = t;
                if (t != i) c[nc++] = t;
            }
            T m = A[r[0]][c[0]] * (A[r[1]][c[1]] * A[r[2]][c[2]] - A[r[1]][c[2]] * A[r[2]][c[1]]) -
                  A[r[0]][c[1]] * (A[r[1]][c[0]] * A[r[2]][c[2]] - A[r[1]][c[2]] * A[r[2]][c[0]]) +
                  A[r[0]][c[2]] * (A[r[1]][c[0]] * A[r[2]][c[1]] - A[r[1]][c[1]] * A[r[2]][c[0]]);
            v[i] = ((col + i) & 1) ? -m : m;
        }
        T n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
        if (n2 > best) {
            best = n2;
            T inv = n2 > T(0) ? T(1) / sqrt(n2) : T(0);
            for (int i = 0; i < 4; i++) q[i] = v[i] * inv;
        }
    }
    if (!(best > T(0))) { q[0] = 1; q[1] = q[2] = q[3] = 0; }
    if (cond) {
        T c = (lam > T(0) && best > T(0)) ? sqrt(best) / (lam * lam * lam) : T(0);
        T rho = 0;
        for (int i = 0; i < 4; i++) {
            T kq = K[i][0] * q[0] + K[i][1] * q[1] + K[i][2] * q[2] + K[i][3] * q[3];
            rho += q[i] * kq;
        }
        const T unit = sizeof(T) == 4 ? T(0x1p-24) : T(0x1p-53);
        if (!(lam - rho <= T(64) * unit * lam)) c = T(0);
        *cond = c;
    }
    return lam;
}

// Bound d2 on how far the FP32 residual sum exceeds its minimum, per point
// (on RMSD^2), from the eigen-solve.  With s = lambda / Ga the residual at
// (s, q) exceeds the minimum by ((lambda - lambda_1)^2 + 2 lambda
// (lambda_1 - rho)) / Ga (rho = q^T K q), which is second order in the
// eigenvector's error when the eigenpair is converged and well separated:
// the eigenvector's error is about c u lambda / gap per direction, so the
// excess per point is at most 35 c^2 u^2 / cond (the gaps are at least
// cond lambda / 16, lambda^2 / (Ga N) is at most Gb / N, about 1); with
// c = 10 that is 3500 u^2 / cond.  Other eigenpairs (cond below 1/8, or a
// Rayleigh quotient that leaves lambda by more than rounding) get no finite
// bound: FP32 arithmetic cannot resolve nearly equal top eigenvalues, and
// their atoms are decided in FP64.
__host__ __device__ inline float f32_excess_bound(float lam, float cond, float Ga) {
    const float unit = 0x1p-24f;
    if (!(Ga > 0.f) || !(lam > 0.f) || !(cond >= 0.125f)) return INFINITY;
    return 3500.f * unit * unit / cond;
}

template <typename T>
__host__ __device__ inline void quat_rot(const T q[4], T R[3][3]) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    T w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

// cyclic Jacobi for a symmetric 3x3 matrix; returns eigenvalues in d and
// eigenvectors in the columns of V
template <typename T>
__host__ __device__ inline void jacobi3(T A[3][3], T d[3], T V[3][3]) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) V[i][j] = (i == j) ? T(1) : T(0);
    for (int sweep = 0; sweep < 12; sweep++) {
        T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        T dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= RealTraits<T>::jacobi_off * dg) break;
        for (int p = 0; p < 2; p++)
            for (int r = p + 1; r < 3; r++) {
                T apr = A[p][r];
                if (apr == T(0)) continue;
                T h = A[r][r] - A[p][p];
                T th = T(0.5) * h / apr;
                T t = T(1) / (fabs(th) + sqrt(th * th + T(1)));
                if (th < T(0)) t = -t;
                T c = T(1) / sqrt(t * t + T(1)), s = t * c;
                for (int m = 0; m < 3; m++) {
                    T amp = A[m][p], amr = A[m][r];
                    A[m][p] = c * amp - s * amr;
                    A[m][r] = s * amp + c * amr;
                }
                for (int m = 0; m < 3; m++) {
                    T apm = A[p][m], arm = A[r][m];
                    A[p][m] = c * apm - s * arm;
                    A[r][m] = s * apm + c * arm;
                }
                for (int m = 0; m < 3; m++) {
                    T vmp = V[m][p], vmr = V[m][r];
                    V[m][p] = c * vmp - s * vmr;
                    V[m][r] = s * vmp + c * vmr;
                }
            }
    }
    d[0] = A[0][0]; d[1] = A[1][1]; d[2] = A[2][2];
}

// ---------------------------------------------------------------- strain
// eq.(6) inputs of a match, gathered point by point: with the barycentre cb
// of the K + 1 points (FP64; the centre is the origin), the centred points
// are a_0 = -cb (the centre) and a_r = v_r - cb, the difference taken in
// FP64 and then rounded to RT; A^T l = sum_i V+_{:,i} a_i^T (V+ the
// pseudoinverse of the normalised template, column tv(r) + 1 for rank r)
// and l = mean |a_i| (eq. 4, W' = a / l).  strain_begin takes the centre,
// strain_add one neighbour, and the caller divides l by K + 1 at the end
// (TPL: a template table entry with the pseudoinverse vpinv).
template <typename RT, typename TPL>
__host__ __device__ inline void strain_begin(const TPL &D, const double (&cb)[3], RT (&a0)[3],
                                             RT (&At)[3][3], RT &l) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    for (int d = 0; d < 3; d++) a0[d] = (RT)(-cb[d]);
    l = sqrt(a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2]);
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) At[x][y] = (RT)D.vpinv[x][0] * a0[y];
}

template <typename RT, typename TPL>
__host__ __device__ inline void strain_add(const TPL &D, int col, const RT (&ar)[3], RT (&At)[3][3],
                                           RT &l) {
#pragma clang fp contract(fast)
    l += sqrt(ar[0] * ar[0] + ar[1] * ar[1] + ar[2] * ar[2]);
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) At[x][y] += (RT)D.vpinv[x][col] * ar[y];
}

// The same for K neighbour vectors v held in an array (rank order; tv:
// nibble r = template vertex of rank r): the self-check entry points use
// it, with the arithmetic of the match kernel.
template <int K, typename RT>
__host__ __device__ inline void strain_inputs(const TemplateDev &D, uint64_t tv, const double (&v)[K][3],
                                              RT (&a0)[3], RT (&At)[3][3], RT &l) {
    double cb[3] = {0, 0, 0};
    for (int rr = 0; rr < K; rr++)
        for (int d = 0; d < 3; d++) cb[d] += v[rr][d];
    for (int d = 0; d < 3; d++) cb[d] /= (K + 1);
    strain_begin<RT>(D, cb, a0, At, l);
    for (int rr = 0; rr < K; rr++) {
        RT ar[3];
        for (int d = 0; d < 3; d++) ar[d] = (RT)(v[rr][d] - cb[d]);
        strain_add<RT>(D, (int)((tv >> (4 * rr)) & 0xF) + 1, ar, At, l);
    }
    l /= RT(K + 1);
}

// Sec. 8: the symmetric factor P of the left polar decomposition A = P U,
// U orthogonal and right-handed, from At = A^T l.  For det A > 0, U is the
// limit of Newton's iteration X <- (X + X^-T) / 2 from X = A (quadratic
// convergence: a step of size e leaves an error of about e^2 / 2, so the
// iteration stops after a step below polar_step, with X then exact to the
// working precision) and P = A U^T, symmetrised.  Otherwise, or if the iteration has not settled
// after 12 steps: A A^T = X S^2 X^T (cyclic Jacobi) and P = X diag(s) X^T,
// where the smallest singular value takes the sign of det A: then det P has
// the sign of det A and U = P^-1 A is a proper rotation (for det A > 0,
// P = (A A^T)^(1/2) in both branches).
template <typename RT>
__host__ __device__ inline void polar_p(const RT (&At)[3][3], RT l, RT (&P)[3][3]) {
    // products and sums may fuse into FMAs here (one rounding instead of two; no
    // result depends on a particular rounding)
#pragma clang fp contract(fast)
    RT A[3][3];
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) A[x][y] = At[y][x] / l;
    const RT detA = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                    A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                    A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (detA > RT(0)) {
        RT X[3][3];
        for (int x = 0; x < 3; x++)
            for (int y = 0; y < 3; y++) X[x][y] = A[x][y];
        bool settled = false;
        for (int it = 0; it < 12 && !settled; it++) {
            // X^-T = cofactor matrix / det X
            const RT C[3][3] = {{X[1][1] * X[2][2] - X[1][2] * X[2][1], X[1][2] * X[2][0] - X[1][0] * X[2][2],
                                 X[1][0] * X[2][1] - X[1][1] * X[2][0]},
                                {X[0][2] * X[2][1] - X[0][1] * X[2][2], X[0][0] * X[2][2] - X[0][2] * X[2][0],
                                 X[0][1] * X[2][0] - X[0][0] * X[2][1]},
                                {X[0][1] * X[1][2] - X[0][2] * X[1][1], X[0][2] * X[1][0] - X[0][0] * X[1][2],
                                 X[0][0] * X[1][1] - X[0][1] * X[1][0]}};
            const RT inv = RT(1) / (X[0][0] * C[0][0] + X[0][1] * C[0][1] + X[0][2] * C[0][2]);
            RT step = 0;
            for (int x = 0; x < 3; x++)
                for (int y = 0; y < 3; y++) {
                    const RT xn = RT(0.5) * (X[x][y] + C[x][y] * inv);
                    step = fmax(step, fabs(xn - X[x][y]));
                    X[x][y] = xn;
                }
            settled = step <= RealTraits<RT>::polar_step;
        }
        if (settled) {
            RT Q[3][3];
            for (int x = 0; x < 3; x++)
                for (int y = 0; y < 3; y++) {
                    RT s = 0;
                    for (int m = 0; m < 3; m++) s += A[x][m] * X[y][m];
                    Q[x][y] = s;
                }
            for (int x = 0; x < 3; x++)
                for (int y = 0; y < 3; y++) P[x][y] = RT(0.5) * (Q[x][y] + Q[y][x]);
            return;
        }
    }
    RT AA[3][3];
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) {
            RT s = 0;
            for (int m = 0; m < 3; m++) s += At[m][x] * At[m][y];
            AA[x][y] = s / (l * l);
        }
    RT ev[3], V[3][3];
    jacobi3<RT>(AA, ev, V);
    int sm = ev[1] < ev[0] ? 1 : 0;
    if (ev[2] < ev[sm]) sm = 2;
    for (int m = 0; m < 3; m++) ev[m] = sqrt(fmax(ev[m], RT(0)));
    const RT det = At[0][0] * (At[1][1] * At[2][2] - At[1][2] * At[2][1]) -
                   At[0][1] * (At[1][0] * At[2][2] - At[1][2] * At[2][0]) +
                   At[0][2] * (At[1][0] * At[2][1] - At[1][1] * At[2][0]);
    if (det < RT(0)) ev[sm] = -ev[sm];
    for (int x = 0; x < 3; x++)
        for (int y = 0; y < 3; y++) {
            RT s = 0;
            for (int m = 0; m < 3; m++) s += V[x][m] * ev[m] * V[y][m];
            P[x][y] = s;
        }
}

}  // namespace ptm
