// Exact potential of one linearly magnetised tetrahedron at one target
// (Sec. 2.1), shared by the near-field, direct-sum and surrogate kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace tfmm {

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

// ---------------------------------------------------------------------------
// P2P / direct sum: exact potential of linearly magnetised tets (Sec. 2.1).
//
// For a tet with outward face normals n_k (face k opposite corner k), target
// x, d_i = v_i - x, the potential is (integration by parts into the faces)
//   4 pi u_T(x) = sum_k alpha_k(x) I0_k(x) + sum_e gamma_e g_e(x)
// with the face single-layer integral of a constant density
//   I0_k = sum_{e in k} t0_{k,e} f_e - h_k Omega_k,
// the edge terms  f_e = ln((R_b + l_b)/(R_a + l_a)),
//                 g_e = R0_e^2 f_e + l_b R_b - l_a R_a  (edge e = (a, b)),
// h_k = n_k . d (signed height), Omega_k the signed solid angle of face k,
// t0_{k,e} the in-plane distance of x's projection to edge e, and the field
// coefficients (G = dM/dr, M_0 the value at corner 0)
//   alpha_k = M(x).n_k + h_k (n_k.G n_k - div M / 2),  M(x) = M_0 - G d_0,
//   gamma_e = 1/2 sum_{faces k of e} (G^T n_k) . u_{k,e},
// u_{k,e} the outward in-plane normal of edge e in face k.
//
// Corner order after orientation (positive volume) fixes the faces, counter-
// clockwise about the outward normal:
//   F0 = (1,2,3), F1 = (0,3,2), F2 = (0,1,3), F3 = (0,2,1)
// and edges e0..e5 = (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).
// ---------------------------------------------------------------------------
constexpr int kEa[6] = {0, 0, 0, 1, 1, 2};
constexpr int kEb[6] = {1, 2, 3, 2, 3, 3};
// face k: its three edges and the orientation sign of each
constexpr int kFe[4][3] = {{3, 5, 4}, {2, 5, 1}, {0, 4, 2}, {1, 3, 0}};
constexpr double kFs[4][3] = {{1, 1, -1}, {1, -1, -1}, {1, 1, -1}, {1, -1, -1}};
// face k: counter-clockwise corners
constexpr int kFv[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

struct TetGeom {
    double v[4][3];
    double n[4][3];
    double il[6];  // 1 / edge length
};
struct TetField {
    double a[4];     // M_0 . n_k
    double b[4][3];  // G^T n_k
    double c[4];     // n_k . G n_k - div M / 2
    double g[6];     // gamma_e
};

// Geometry of a tet with corners G.v: unit outward normals, inverse edge
// lengths, and (returned) the gradients gl of the barycentric coordinates and
// the unit edge vectors eh.
__device__ inline void tet_geometry(TetGeom &G, double gl[4][3], double eh[6][3])
{
    double N[4][3];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int a = kFv[f][0], b = kFv[f][1], c = kFv[f][2];
        double u[3], w[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            u[k] = G.v[b][k] - G.v[a][k];
            w[k] = G.v[c][k] - G.v[a][k];
        }
        N[f][0] = u[1] * w[2] - u[2] * w[1];
        N[f][1] = u[2] * w[0] - u[0] * w[2];
        N[f][2] = u[0] * w[1] - u[1] * w[0];
        const double inv = 1.0 / sqrt(N[f][0] * N[f][0] + N[f][1] * N[f][1] + N[f][2] * N[f][2]);
#pragma unroll
        for (int k = 0; k < 3; ++k) G.n[f][k] = N[f][k] * inv;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = G.v[kEb[e]][k] - G.v[kEa[e]][k];
        const double il = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        G.il[e] = il;
#pragma unroll
        for (int k = 0; k < 3; ++k) eh[e][k] = d[k] * il;
    }
    // gradients of the barycentric coordinates
    double e1[3], e2[3], e3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e1[k] = G.v[1][k] - G.v[0][k];
        e2[k] = G.v[2][k] - G.v[0][k];
        e3[k] = G.v[3][k] - G.v[0][k];
    }
    gl[1][0] = e2[1] * e3[2] - e2[2] * e3[1];
    gl[1][1] = e2[2] * e3[0] - e2[0] * e3[2];
    gl[1][2] = e2[0] * e3[1] - e2[1] * e3[0];
    gl[2][0] = e3[1] * e1[2] - e3[2] * e1[1];
    gl[2][1] = e3[2] * e1[0] - e3[0] * e1[2];
    gl[2][2] = e3[0] * e1[1] - e3[1] * e1[0];
    gl[3][0] = e1[1] * e2[2] - e1[2] * e2[1];
    gl[3][1] = e1[2] * e2[0] - e1[0] * e2[2];
    gl[3][2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double idet = 1.0 / (e1[0] * gl[1][0] + e1[1] * gl[1][1] + e1[2] * gl[1][2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        gl[1][k] *= idet;
        gl[2][k] *= idet;
        gl[3][k] *= idet;
        gl[0][k] = -(gl[1][k] + gl[2][k] + gl[3][k]);
    }
}

// Field coefficients (a, b, c, g) of the affine magnetisation with nodal
// values m[corner][axis] on a tet of geometry G, gl, eh.
__device__ inline void tet_field(const TetGeom &G, const double gl[4][3], const double eh[6][3], const double m[4][3],
                                 TetField &F1)
{
    {
        // div M = sum_i M_i . grad lambda_i
        double divM = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) divM += m[c][0] * gl[c][0] + m[c][1] * gl[c][1] + m[c][2] * gl[c][2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // G^T n = sum_i (M_i . n) grad lambda_i
            double b[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double mn = m[c][0] * G.n[k][0] + m[c][1] * G.n[k][1] + m[c][2] * G.n[k][2];
                b[0] += mn * gl[c][0];
                b[1] += mn * gl[c][1];
                b[2] += mn * gl[c][2];
            }
            F1.a[k] = m[0][0] * G.n[k][0] + m[0][1] * G.n[k][1] + m[0][2] * G.n[k][2];
            F1.b[k][0] = b[0];
            F1.b[k][1] = b[1];
            F1.b[k][2] = b[2];
            F1.c[k] = (b[0] * G.n[k][0] + b[1] * G.n[k][1] + b[2] * G.n[k][2]) - 0.5 * divM;
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) F1.g[e] = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int e = kFe[k][j];
                const double s = kFs[k][j];
                // u_{k,e} = (s e_hat) x n_k
                const double ux = s * (eh[e][1] * G.n[k][2] - eh[e][2] * G.n[k][1]);
                const double uy = s * (eh[e][2] * G.n[k][0] - eh[e][0] * G.n[k][2]);
                const double uz = s * (eh[e][0] * G.n[k][1] - eh[e][1] * G.n[k][0]);
                F1.g[e] += 0.5 * (F1.b[k][0] * ux + F1.b[k][1] * uy + F1.b[k][2] * uz);
            }
    }
}

// Geometry of tet t (corners from tet_xyz [12][T]) and the coefficients of
// one field (nodal values Mf [n_nodes][3]); the geometry is written to
// *Gout when Gout is not null.
__device__ inline void tet_prepare(const double *__restrict__ tet_xyz, const int32_t *__restrict__ tet_node, int64_t T,
                                   int64_t t, const double *__restrict__ Mf, TetGeom *Gout, TetField &F1)
{
    TetGeom G;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) G.v[c][k] = tet_xyz[(int64_t)(3 * c + k) * T + t];
    double gl[4][3], eh[6][3];
    tet_geometry(G, gl, eh);
    if (Gout) *Gout = G;
    double m[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t nd = tet_node[(int64_t)c * T + t];
#pragma unroll
        for (int k = 0; k < 3; ++k) m[c][k] = Mf[3 * nd + k];
    }
    tet_field(G, gl, eh, m, F1);
}

// The distance band of the near-field surrogate: 2 <= |x - c| / diam < 6
// (c the centroid, diam the longest edge).  band_geom and in_band are the only
// place the band is decided, with explicit fused operations, so that every
// kernel that splits pairs by it rounds identically.
constexpr double kBandLo = 2.0, kBandHi = 6.0;
__device__ __forceinline__ void band_geom(const double v[4][3], double c[3], double &id2)
{
    double l2 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) {
            const double dx = v[b][0] - v[a][0], dy = v[b][1] - v[a][1], dz = v[b][2] - v[a][2];
            l2 = fmax(l2, fma(dx, dx, fma(dy, dy, dz * dz)));
        }
    id2 = 1.0 / l2;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = 0.25 * ((v[0][k] + v[1][k]) + (v[2][k] + v[3][k]));
}
__device__ __forceinline__ bool in_band(const double x[3], const double c[3], double id2)
{
    const double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz)) * id2;
    return r2 >= kBandLo * kBandLo && r2 < kBandHi * kBandHi;
}

// n / d for finite nonzero d of moderate range: the hardware reciprocal
// estimate, two Newton-Raphson steps r <- r + r (1 - d r), then the quotient
// with one residual correction q <- q + r (n - d q).
__device__ __forceinline__ double div_nr(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    const double q = n * r;
    return fma(r, fma(-d, q, n), q);
}

// 1/sqrt(a) for positive finite normal a: the hardware estimate and two
// Newton-Raphson steps r <- r + r (1 - a r^2) / 2, then one more on the
// residual (the estimate's ~2^-23 relative error squares per step).
__device__ __forceinline__ double rsqrt_nr(double a)
{
    double r = __builtin_amdgcn_rsq(a);
    double h = a * r;
    double e = fma(-h, r, 1.0);
    r = fma(0.5 * r, e, r);
    h = a * r;
    e = fma(-h, r, 1.0);
    r = fma(0.5 * r, e, r);
    h = a * r;
    e = fma(-h, r, 1.0);
    return fma(0.5 * r, e, r);
}

// ln(num / den) for positive finite num, den, with one division: writing
// num = a 2^i, den = b 2^j (a, b in [1/2, 1)), the ratio a/b is brought into
// [1/sqrt2, sqrt2) by a factor 2 on a or b (the differences below are then
// exact), and ln(a/b) = 2 atanh(s), s = (a - b)/(a + b), |s| <= 0.1716, is
// summed by its odd series sum s^(2k+1)/(2k+1) to k = 9 (the tail is below
// s^21/21 / (1 - s^2) < 4.1e-18, 2.4e-17 relative to 2 atanh(s));
// the power of two enters as (i - j) ln 2 with ln 2 split into a 32-bit-exact
// head and a tail (Cody & Waite).
__device__ __forceinline__ double log_ratio(double num, double den)
{
    int ei, ej;
    double a = frexp(num, &ei), b = frexp(den, &ej);
    const double kSqrt2 = 1.4142135623730951;
    const bool lo = a * kSqrt2 < b;            // a/b < 1/sqrt2
    const bool hi = !lo && a > b * kSqrt2;     // a/b > sqrt2
    a = ldexp(a, lo ? 1 : 0);  // exact doubling, no select of doubles
    b = ldexp(b, hi ? 1 : 0);
    const int e = ei - ej + (hi ? 1 : 0) - (lo ? 1 : 0);
    const double sv = div_nr(a - b, a + b);
    const double z = sv * sv;
    double q = 1.0 / 19.0;
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    const double t = 2.0 * sv * z * q;  // 2 atanh(s) - 2 s
    const double kLn2Hi = 6.93147180369123816490e-01, kLn2Lo = 1.90821492927058770002e-10;
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, t) + 2.0 * sv);
}

// The edge integral ln((R_b + l_b)/(R_a + l_a)) in a cancellation-free form.
// With P = R_b + |l_b| and Q = R_a + |l_a| (sums of non-negative terms): it is
// ln(P/Q) for l_a >= 0, -ln(P/Q) = ln((R_a - l_a)/(R_b - l_b)) for l_b <= 0,
// and ln(PQ/R0^2) = ln((R_b + l_b)(R_a - l_a)/R0^2) in between (where
// R_a^2 - l_a^2 = R_b^2 - l_b^2 = R0^2).  log_ratio is exactly odd under the
// exchange of its arguments, so the sign flip gives the same value as the
// swapped ratio.  0 when a corner coincides with the target or the ratio
// degenerates (its factors t0 and R0^2 vanish there).  Branch free: every
// candidate is formed and one is selected.  With kMask the logarithm of a
// degenerate ratio is taken of 1/1; without it the logarithm of the
// degenerate arguments (possibly not finite) is computed and discarded by the
// final select, which copies bits and never propagates it: four selects
// fewer, which the shared-entity loop gains from, while the per-tet kernel
// (measured at 16 fields) is faster with the mask.
template <bool kMask = true>
__device__ __forceinline__ double edge_log(double Ra, double Rb, double la, double lb, double r0sq)
{
    const bool fwd = la >= 0.0, mid = !fwd && lb > 0.0;
    const double p = Rb + fabs(lb), q = Ra + fabs(la);
    const double num = mid ? p * q : p;
    const double den = mid ? r0sq : q;
    const bool ok = (Ra > 0.0) && (Rb > 0.0) && (den > 0.0) && (num > 0.0);
    const double f = kMask ? log_ratio(ok ? num : 1.0, ok ? den : 1.0) : log_ratio(num, den);
    const double fs = (fwd || mid) ? f : -f;
    return ok ? fs : 0.0;
}

// atan2(y, x) in (-pi, pi], 0 for y = x = 0, with one division: with
// a = min(|x|, |y|), b = max(|x|, |y|), atan(a/b) in [0, pi/4] is reduced to
// t in [0, tan(pi/8)] by t = a/b or, above tan(pi/8), pi/4 - atan(t),
// t = (b - a)/(b + a); atan(t) = t + t^3 Q(t^2) with Q the degree-10
// polynomial interpolating (atan(sqrt z)/sqrt z - 1)/z at the Chebyshev
// points of [0, tan(pi/8)^2] (relative error of atan(t) below 5e-18); the
// octant and quadrant follow by pi/2 - r and pi - r, the sign from y.
__device__ __forceinline__ double atan2_nr(double y, double x)
{
    const double ay = fabs(y), ax = fabs(x);
    const double b = fmax(ay, ax), a = fmin(ay, ax);
    const double kTanPi8 = 0.41421356237309503;
    const bool big = a > kTanPi8 * b;
    const double num = big ? b - a : a;
    const double den = big ? b + a : (b > 0.0 ? b : 1.0);
    const double t = div_nr(num, den);
    const double z = t * t;
    double q = -1.91768871190622589893e-2;
    q = fma(q, z, 3.923165829558719130283e-2);
    q = fma(q, z, -5.085449737940259861323e-2);
    q = fma(q, z, 5.858148912802209881646e-2);
    q = fma(q, z, -6.664511447381948000098e-2);
    q = fma(q, z, 7.692183190826086563693e-2);
    q = fma(q, z, -9.090904578123901890479e-2);
    q = fma(q, z, 1.111111101525636172749e-1);
    q = fma(q, z, -1.428571428466654292249e-1);
    q = fma(q, z, 1.999999999999552067782e-1);
    q = fma(q, z, -3.333333333333333015966e-1);
    const double at = fma(t * z, q, t);
    const double kPi = 3.141592653589793116, kPi2 = 1.5707963267948965580, kPi4 = 0.78539816339744827900;
    double r = big ? kPi4 - at : at;
    r = ay > ax ? kPi2 - r : r;
    r = x < 0.0 ? kPi - r : r;
    return copysign(r, y);
}

// Geometric integrals of one pair (target x, tet G): the face integrals I0_k,
// the edge terms g_e, the signed heights h_k and d_0 = v_0 - x; the potential
// of a field is then the contraction pair_contract with its coefficients.
struct PairGeo {
    double I0[4], ge[6], h[4], d0[3];
};

// The edges are taken one at a time (the edges (a, b) listed first in the
// faces give the faces' triple products for the solid angles).
__device__ __forceinline__ void pair_geometry(const double x[3], const TetGeom &G, PairGeo &P)
{
    double d[4][3], R2[4], R[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int k = 0; k < 3; ++k) d[c][k] = G.v[c][k] - x[k];
        R2[c] = d[c][0] * d[c][0] + d[c][1] * d[c][1] + d[c][2] * d[c][2];
        R[c] = sqrt(R2[c]);
    }
    double D[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) D[a][b] = D[b][a] = d[a][0] * d[b][0] + d[a][1] * d[b][1] + d[a][2] * d[b][2];
    double det[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = kFv[k][0];
        P.h[k] = G.n[k][0] * d[a][0] + G.n[k][1] * d[a][1] + G.n[k][2] * d[a][2];
        P.I0[k] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int a = kEa[e], b = kEb[e];
        const double il = G.il[e];
        double cx[3];
        cx[0] = d[a][1] * d[b][2] - d[a][2] * d[b][1];
        cx[1] = d[a][2] * d[b][0] - d[a][0] * d[b][2];
        cx[2] = d[a][0] * d[b][1] - d[a][1] * d[b][0];
        const double r0sq = (cx[0] * cx[0] + cx[1] * cx[1] + cx[2] * cx[2]) * (il * il);
        const double la = (D[a][b] - R2[a]) * il;  // (v_a - x) . e_hat
        const double lb = (R2[b] - D[a][b]) * il;  // (v_b - x) . e_hat
        // f = ln((R_b + l_b)/(R_a + l_a)) in a form free of cancellation
        const double fe = edge_log(R[a], R[b], la, lb, r0sq);
        const double fl = fe * il;
        P.ge[e] = r0sq * fe + lb * R[b] - la * R[a];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (kFe[k][j] != e) continue;
                // t0 |e| = s n_k . (d_a x d_b)
                P.I0[k] += kFs[k][j] * (G.n[k][0] * cx[0] + G.n[k][1] * cx[1] + G.n[k][2] * cx[2]) * fl;
                if (j == 0) {  // det[d_a, d_b, d_c] = d_c . (d_a x d_b)
                    const int c = kFv[k][2];
                    det[k] = kFs[k][0] * (d[c][0] * cx[0] + d[c][1] * cx[1] + d[c][2] * cx[2]);
                }
            }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = kFv[k][0], b = kFv[k][1], c = kFv[k][2];
        const double den = R[a] * R[b] * R[c] + D[a][b] * R[c] + D[a][c] * R[b] + D[b][c] * R[a];
        P.I0[k] -= P.h[k] * (2.0 * atan2_nr(det[k], den));  // - h_k Omega_k
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) P.d0[k] = d[0][k];
}

// 4 pi u_T(x) of one field from the pair's geometric integrals.
__device__ __forceinline__ double pair_contract(const PairGeo &P, const TetField &F1)
{
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // alpha_k = M(x).n_k + h_k (n_k.G n_k - div M / 2)
        const double alpha =
            F1.a[k] - (P.d0[0] * F1.b[k][0] + P.d0[1] * F1.b[k][1] + P.d0[2] * F1.b[k][2]) + F1.c[k] * P.h[k];
        v = fma(alpha, P.I0[k], v);
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) v = fma(F1.g[e], P.ge[e], v);
    return v;
}

// One pair (target x, tet G with FCH fields): adds 4 pi u_T(x) of every field
// to acc.
template <int FCH>
__device__ __forceinline__ void pair_accumulate(const double x[3], const TetGeom &G, const TetField *fld,
                                                double (&acc)[FCH])
{
    PairGeo P;
    pair_geometry(x, G, P);
#pragma unroll
    for (int f = 0; f < FCH; ++f) acc[f] += pair_contract(P, fld[f]);
}

}  // namespace tfmm
