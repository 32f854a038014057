// HIP kernels of the tetrahedral FMM for CDNA4 (gfx950), FP64.
//
//   p2m   multipole coefficients of a leaf (eq. expCoeffs) from the tets'
//         geometric moments (exact quadrature, once per plan) and affine M
//   m2m   binomial shift of child multipoles to the parent centre
//   m2l   multipole -> local translation of the Cartesian Taylor expansion on
//         FP64 matrix cores, target cells in tiles sharing translation keys
//   l2l   binomial shift of a local expansion to the child centres
//   l2p   evaluation of the local expansion at the targets (adds into u)
//   p2p   exact near-field tet-to-target potential (Sec. 2.1), source-major:
//         one workgroup per block of <= 64 tets of a source leaf, the tets'
//         geometry and field coefficients staged in LDS, every lane a target,
//         atomically accumulated into u
//
// Multi-indices |n| <= p are stored in graded order: degree ascending, within
// a degree n_x descending, then n_y descending.  idx(n) = d(d+1)(d+2)/6 +
// r(r+1)/2 + n_z with d = |n| and r = n_y + n_z.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/tetfmm.h"
#include "device.h"
#include "pair.h"

namespace tfmm {

// ---------------------------------------------------------------------------
// constant tables
// ---------------------------------------------------------------------------
constexpr int kPmax = TFMM_PMAX;
constexpr int kNcoefMax = (kPmax + 1) * (kPmax + 2) * (kPmax + 3) / 6;

struct MiTable {
    int8_t v[kNcoefMax][4];  // nx, ny, nz, |n|
};
constexpr MiTable make_mi()
{
    MiTable t{};
    int k = 0;
    for (int d = 0; d <= kPmax; ++d)
        for (int nx = d; nx >= 0; --nx)
            for (int ny = d - nx; ny >= 0; --ny) {
                t.v[k][0] = (int8_t)nx;
                t.v[k][1] = (int8_t)ny;
                t.v[k][2] = (int8_t)(d - nx - ny);
                t.v[k][3] = (int8_t)d;
                ++k;
            }
    return t;
}
struct BinomTable {
    double c[2 * kPmax + 1][2 * kPmax + 1];
    double invfact[2 * kPmax + 1];
};
constexpr BinomTable make_binom()
{
    BinomTable t{};
    for (int n = 0; n <= 2 * kPmax; ++n)
        for (int r = 0; r <= 2 * kPmax; ++r) t.c[n][r] = 0.0;
    for (int n = 0; n <= 2 * kPmax; ++n) {
        t.c[n][0] = 1.0;
        for (int r = 1; r <= n; ++r) t.c[n][r] = t.c[n - 1][r - 1] + (r <= n - 1 ? t.c[n - 1][r] : 0.0);
    }
    double f = 1.0;
    for (int n = 0; n <= 2 * kPmax; ++n) {
        if (n > 0) f *= n;
        t.invfact[n] = 1.0 / f;
    }
    return t;
}
__constant__ MiTable c_mi = make_mi();
// compile-time view of the same table (loops unrolled over a template order)
constexpr MiTable kMi = make_mi();
__host__ __device__ constexpr int mi_x(int m) { return kMi.v[m][0]; }
__host__ __device__ constexpr int mi_y(int m) { return kMi.v[m][1]; }
__host__ __device__ constexpr int mi_z(int m) { return kMi.v[m][2]; }
__constant__ BinomTable c_bin = make_binom();

__device__ __forceinline__ int mi_index(int nx, int ny, int nz)
{
    int d = nx + ny + nz, r = ny + nz;
    return d * (d + 1) * (d + 2) / 6 + r * (r + 1) / 2 + nz;
}
__host__ __device__ constexpr int ncoef_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }


// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  A grid of 8 * ceil(n/8) workgroups in x is remapped so that XCD x
// runs items [x * per, (x + 1) * per): neighbouring items (Morton order) share
// an L2.  Returns -1 for the padding workgroups.
constexpr int kXcds = 8;
__host__ __device__ constexpr unsigned xcd_grid(int n) { return (unsigned)(kXcds * ((n + kXcds - 1) / kXcds)); }
__device__ __forceinline__ int xcd_item(int n)
{
    const int w = blockIdx.x, per = (n + kXcds - 1) / kXcds;
    const int item = (w % kXcds) * per + w / kXcds;
    return item < n ? item : -1;
}

// cell int fields
enum { CI_TBEG = 0, CI_TEND, CI_XBEG, CI_XEND, CI_CBEG, CI_NCHILD, CI_PARENT, CI_LEVEL, CI_N };

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------
__global__ void k_fill(double *__restrict__ a, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

// ---------------------------------------------------------------------------
// P2M (eq. expCoeffs).  M is affine on a tet, M_k(y) = M_k(c) + sum_d G_kd
// (y_d - c_d) with G = dM/dy, so with the geometric moments of the tet about
// its leaf centre c,  S_m = int_T (y - c)^m dy  (|m| <= p),
//   Q_n = sum_k n_k int_T M_k(y) (y - c)^{n - e_k} dy
//       = sum_k n_k [ M_k(c) S_{n-e_k} + sum_d G_kd S_{n-e_k+e_d} ].
// S depends on the mesh only: k_tet_moments computes it once per plan with
// an exact collapsed Gauss-Jacobi rule (degree p); k_p2m streams it.
// ---------------------------------------------------------------------------
constexpr int kMomThreads = 256;
constexpr int kMomChunk = 256;

// One workgroup per leaf holding tets: S of each of its tets, [T][ncoef].
__global__ __launch_bounds__(kMomThreads) void k_tet_moments(const int32_t *__restrict__ cells,
                                                             const int32_t *__restrict__ cell_i,
                                                             const double *__restrict__ cell_c, int64_t C,
                                                             const double *__restrict__ tet_xyz, int64_t T,
                                                             const double *__restrict__ quad, int nq, int p,
                                                             int points, double *__restrict__ mom)
{
    __shared__ double s_pw[kMomChunk][3][kPmax + 1];  // powers 0..p of (y - c)
    __shared__ double s_w[kMomChunk];
    const int cell = cells[blockIdx.x];
    const int tbeg = cell_i[CI_N * cell + CI_TBEG], tend = cell_i[CI_N * cell + CI_TEND];
    const double cc[3] = {cell_c[cell], cell_c[C + cell], cell_c[2 * C + cell]};
    const int ncoef = ncoef_of(p);
    const int tid = threadIdx.x;
    if (points) {  // point sources: S_m = (y - c)^m at the point
        for (int i = tid; i < (tend - tbeg) * ncoef; i += kMomThreads) {
            const int t = tbeg + i / ncoef, m = i % ncoef;
            double r = 1.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double y = tet_xyz[(int64_t)k * T + t] - cc[k];
                for (int j = 0; j < c_mi.v[m][k]; ++j) r *= y;
            }
            mom[(int64_t)t * ncoef + m] = r;
        }
        return;
    }
    for (int t = tbeg; t < tend; ++t) {
        double v[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k) v[c][k] = tet_xyz[(int64_t)(3 * c + k) * T + t];
        double e[3][3];
#pragma unroll
        for (int c = 1; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k) e[c - 1][k] = v[c][k] - v[0][k];
        const double vol6 = fabs(e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                                 e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                                 e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]));
        double acc[2] = {0.0, 0.0};
        for (int base = 0; base < nq; base += kMomChunk) {
            __syncthreads();
            const int q = base + tid;
            if (q < nq) {
                const double l1 = quad[4 * q], l2 = quad[4 * q + 1], l3 = quad[4 * q + 2];
                const double l0 = 1.0 - (l1 + l2 + l3);
                s_w[tid] = quad[4 * q + 3] * vol6;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double y = ((l0 * (v[0][k] - cc[k]) + l1 * (v[1][k] - cc[k])) + l2 * (v[2][k] - cc[k])) +
                                     l3 * (v[3][k] - cc[k]);
                    double pw = 1.0;
                    for (int j = 0; j <= p; ++j) {
                        s_pw[tid][k][j] = pw;
                        pw *= y;
                    }
                }
            }
            __syncthreads();
            const int n = min(kMomChunk, nq - base);
            for (int r = 0; r < 2; ++r) {
                const int m = tid + r * kMomThreads;
                if (m >= ncoef) break;
                const int a = c_mi.v[m][0], b = c_mi.v[m][1], c = c_mi.v[m][2];
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += s_w[i] * (s_pw[i][0][a] * s_pw[i][1][b] * s_pw[i][2][c]);
                acc[r] += s;
            }
        }
        for (int r = 0; r < 2; ++r) {
            const int m = tid + r * kMomThreads;
            if (m < ncoef) mom[(int64_t)t * ncoef + m] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------------
// P2M.  One workgroup per leaf holding tets (XCD-contiguous), FC fields per
// workgroup (blockIdx.y = field chunk).  With the per-tet moments
// S_m = int_T (y - c)^m (exact, once per plan) and, per field, the affine
// magnetisation M(y) = M(c) + G (y - c) of the tet,
//   Q_n = sum_T sum_k n_k [M_k(c) S_{n-e_k} + sum_d G_kd S_{n-e_k+e_d}].
// Tets are staged kP2MStage at a time: their moments and the 12 field values
// of every (tet, field) pair (one thread each) go to LDS, then every thread
// accumulates its coefficients n over the staged tets for all FC fields.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int field_chunk(int F) { return F >= 16 ? 16 : (F >= 4 ? 4 : 1); }
constexpr int kP2MThreads = 256;
constexpr int kP2MStage = 16;

// M(c) [3] and G [3][3] of tet t for one field (nodal values Mf).
__device__ inline void tet_affine_field(const double *__restrict__ tet_xyz, const int32_t *__restrict__ tet_node,
                                        int64_t T, int64_t t, const double *__restrict__ Mf, const double c[3],
                                        double *__restrict__ out)
{
    double v[4][3], mm[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int nd = tet_node[(int64_t)q * T + t];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + t];
            mm[q][k] = Mf[3 * (int64_t)nd + k];
        }
    }
    double e1[3], e2[3], e3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e1[k] = v[1][k] - v[0][k];
        e2[k] = v[2][k] - v[0][k];
        e3[k] = v[3][k] - v[0][k];
    }
    // gradients of the barycentric coordinates
    double g[4][3];
    g[1][0] = e2[1] * e3[2] - e2[2] * e3[1];
    g[1][1] = e2[2] * e3[0] - e2[0] * e3[2];
    g[1][2] = e2[0] * e3[1] - e2[1] * e3[0];
    g[2][0] = e3[1] * e1[2] - e3[2] * e1[1];
    g[2][1] = e3[2] * e1[0] - e3[0] * e1[2];
    g[2][2] = e3[0] * e1[1] - e3[1] * e1[0];
    g[3][0] = e1[1] * e2[2] - e1[2] * e2[1];
    g[3][1] = e1[2] * e2[0] - e1[0] * e2[2];
    g[3][2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double idet = 1.0 / (e1[0] * g[1][0] + e1[1] * g[1][1] + e1[2] * g[1][2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g[1][k] *= idet;
        g[2][k] *= idet;
        g[3][k] *= idet;
        g[0][k] = -(g[1][k] + g[2][k] + g[3][k]);
    }
    const double dc[3] = {c[0] - v[0][0], c[1] - v[0][1], c[2] - v[0][2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double G[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) G[b] = mm[0][a] * g[0][b] + mm[1][a] * g[1][b] + mm[2][a] * g[2][b] + mm[3][a] * g[3][b];
        out[a] = mm[0][a] + (G[0] * dc[0] + G[1] * dc[1] + G[2] * dc[2]);  // M_a(c)
        out[3 + 3 * a] = G[0];
        out[4 + 3 * a] = G[1];
        out[5 + 3 * a] = G[2];
    }
}

// Dynamic LDS: S [kP2MStage][ncoef], W [kP2MStage][FC][12] doubles.
template <int FC>
__global__ __launch_bounds__(kP2MThreads) void k_p2m(const int32_t *__restrict__ cells, const int32_t *__restrict__ cell_i,
                                                     const double *__restrict__ cell_c, int64_t C,
                                                     const double *__restrict__ tet_xyz, const int32_t *__restrict__ tet_node,
                                                     int64_t T, const double *__restrict__ mom,
                                                     const double *__restrict__ M, int64_t n_nodes, int F, int p,
                                                     int ncells, int points, LevelOrders lo, double *__restrict__ Q)
{
    extern __shared__ double s_dyn[];
    const int ncoef = ncoef_of(p);
    double *s_S = s_dyn;                        // [kP2MStage][ncoef]
    double *s_W = s_dyn + kP2MStage * ncoef;    // [kP2MStage][FC][12]
    const int item = xcd_item(ncells);
    if (item < 0) return;
    const int cell = cells[item];
    const int f0 = blockIdx.y * FC;
    const int tbeg = cell_i[CI_N * cell + CI_TBEG], tend = cell_i[CI_N * cell + CI_TEND];
    const int tid = threadIdx.x;
    const double cc[3] = {cell_c[cell], cell_c[C + cell], cell_c[2 * C + cell]};
    double acc[2][FC];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < FC; ++j) acc[r][j] = 0.0;
    for (int sb = tbeg; sb < tend; sb += kP2MStage) {
        const int nt = min(kP2MStage, tend - sb);
        __syncthreads();
        for (int i = tid; i < nt * ncoef; i += blockDim.x) s_S[i] = mom[(int64_t)sb * ncoef + i];
        for (int i = tid; i < nt * FC; i += blockDim.x) {
            const int t = i / FC, j = i - t * FC;
            if (f0 + j < F && points) {  // a dipole: M(c) = its moment, no gradient
                const double *m = M + ((int64_t)(f0 + j) * n_nodes + tet_node[sb + t]) * 3;
                double *w = s_W + (t * FC + j) * 12;
                for (int q = 0; q < 12; ++q) w[q] = q < 3 ? m[q] : 0.0;
            } else if (f0 + j < F)
                tet_affine_field(tet_xyz, tet_node, T, sb + t, M + (int64_t)(f0 + j) * n_nodes * 3, cc,
                                 s_W + (t * FC + j) * 12);
            else
                for (int q = 0; q < 12; ++q) s_W[(t * FC + j) * 12 + q] = 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int n = tid + r * kP2MThreads;
            if (n >= ncoef) continue;
            const int nv[3] = {c_mi.v[n][0], c_mi.v[n][1], c_mi.v[n][2]};
            // indices of S_{n-e_k} and S_{n-e_k+e_d}
            int si[3][4];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int b[3] = {nv[0], nv[1], nv[2]};
                b[k] = b[k] > 0 ? b[k] - 1 : 0;
                si[k][0] = mi_index(b[0], b[1], b[2]);
                si[k][1] = mi_index(b[0] + 1, b[1], b[2]);
                si[k][2] = mi_index(b[0], b[1] + 1, b[2]);
                si[k][3] = mi_index(b[0], b[1], b[2] + 1);
            }
            for (int t = 0; t < nt; ++t) {
                const double *S = s_S + t * ncoef;
                double sv[3][4];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int q = 0; q < 4; ++q) sv[k][q] = nv[k] ? nv[k] * S[si[k][q]] : 0.0;
#pragma unroll
                for (int j = 0; j < FC; ++j) {
                    const double *w = s_W + (t * FC + j) * 12;
                    double sacc = acc[r][j];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        sacc += w[k] * sv[k][0] + w[3 + 3 * k] * sv[k][1] + w[4 + 3 * k] * sv[k][2] +
                                w[5 + 3 * k] * sv[k][3];
                    acc[r][j] = sacc;
                }
            }
        }
    }
    // kept to the order of the leaf's level (the rest stays zero)
    const int nkeep = ncoef_of(lo.q[cell_i[CI_N * cell + CI_LEVEL]]);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int n = tid + r * kP2MThreads;
        if (n >= ncoef) continue;
#pragma unroll
        for (int j = 0; j < FC; ++j)
            if (f0 + j < F) Q[((int64_t)(f0 + j) * C + cell) * ncoef + n] = n < nkeep ? acc[r][j] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// M2M and L2L as three one-dimensional binomial shifts.  The shift by t of a
// multipole (k <= n) or local (k >= m, |k| <= p) expansion factorises over the
// axes, C(n, k) t^(n-k) = prod_i C(n_i, k_i) t_i^(n_i - k_i), so it is applied
// axis by axis (at most p + 1 terms per coefficient and axis).  A workgroup
// holds kShiftItems items (children) of 32 lanes each, one field
// (blockIdx.y); LDS holds two buffers of kShiftItems x ncoef doubles.
// ---------------------------------------------------------------------------
constexpr int kShiftItems = 8;
constexpr int kShiftThreads = 32 * kShiftItems;

template <bool Up>
__device__ __forceinline__ void shift_pass(const double *__restrict__ in, double *__restrict__ out, int ncoef, int p,
                                           int ax, double t, int lane)
{
    for (int n = lane; n < ncoef; n += 32) {
        int v[3] = {c_mi.v[n][0], c_mi.v[n][1], c_mi.v[n][2]};
        const int a = v[ax], rest = c_mi.v[n][3] - a;
        double acc = 0.0, pw = 1.0;
        if (Up) {  // out_n = sum_{k <= a} C(a, k) t^(a-k) in_(.., k, ..)
            for (int k = a; k >= 0; --k) {
                v[ax] = k;
                acc += c_bin.c[a][k] * pw * in[mi_index(v[0], v[1], v[2])];
                pw *= t;
            }
        } else {  // out_m = sum_{a <= k <= p - rest} C(k, a) t^(k-a) in_(.., k, ..)
            for (int k = a; k <= p - rest; ++k) {
                v[ax] = k;
                acc += c_bin.c[k][a] * pw * in[mi_index(v[0], v[1], v[2])];
                pw *= t;
            }
        }
        out[n] = acc;
    }
}

// M2M: one workgroup per parent of a level; child g of the parent is item g.
//   Q_n(P) = sum_children sum_{k <= n} C(n,k) (c_C - c_P)^{n-k} Q_k(C)
__global__ __launch_bounds__(kShiftThreads) void k_m2m(const int32_t *__restrict__ cells, const int32_t *__restrict__ cell_i,
                                                       const double *__restrict__ cell_c, int64_t C, int p, int pout,
                                                       double *__restrict__ Q)
{
    extern __shared__ double s_dyn[];
    const int ncoef = ncoef_of(p), nkeep = ncoef_of(pout);
    double *s_a = s_dyn, *s_b = s_dyn + kShiftItems * ncoef;
    const int cell = cells[blockIdx.x];
    const int f = blockIdx.y;
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    const int cbeg = cell_i[CI_N * cell + CI_CBEG], nch = cell_i[CI_N * cell + CI_NCHILD];
    const int ch = cbeg + g;
    const bool act = g < nch && cell_i[CI_N * ch + CI_TEND] > cell_i[CI_N * ch + CI_TBEG];
    double t[3] = {0.0, 0.0, 0.0};
    if (act) {
        for (int n = lane; n < ncoef; n += 32) s_a[g * ncoef + n] = Q[((int64_t)f * C + ch) * ncoef + n];
#pragma unroll
        for (int k = 0; k < 3; ++k) t[k] = cell_c[k * C + ch] - cell_c[k * C + cell];
    }
    __syncthreads();
    if (act) shift_pass<true>(s_a + g * ncoef, s_b + g * ncoef, ncoef, p, 0, t[0], lane);
    __syncthreads();
    if (act) shift_pass<true>(s_b + g * ncoef, s_a + g * ncoef, ncoef, p, 1, t[1], lane);
    __syncthreads();
    if (act) shift_pass<true>(s_a + g * ncoef, s_b + g * ncoef, ncoef, p, 2, t[2], lane);
    __syncthreads();
    for (int n = threadIdx.x; n < ncoef; n += blockDim.x) {
        double q = 0.0;
        for (int c = 0; c < nch && c < kShiftItems; ++c)
            if (cell_i[CI_N * (cbeg + c) + CI_TEND] > cell_i[CI_N * (cbeg + c) + CI_TBEG]) q += s_b[c * ncoef + n];
        Q[((int64_t)f * C + cell) * ncoef + n] = n < nkeep ? q : 0.0;  // kept to the parent level's order
    }
}

// L2L: items are kShiftItems consecutive child cells of a level (each with
// its own parent).
//   l_m(C) += sum_{k >= m, |k| <= p} C(k,m) (c_C - c_P)^{k-m} l_k(P)
__global__ __launch_bounds__(kShiftThreads) void k_l2l(const int32_t *__restrict__ cells, int ncells,
                                                       const int32_t *__restrict__ cell_i,
                                                       const double *__restrict__ cell_c, int64_t C, int p, int pout,
                                                       double *__restrict__ L)
{
    extern __shared__ double s_dyn[];
    const int ncoef = ncoef_of(p), nkeep = ncoef_of(pout);
    double *s_a = s_dyn, *s_b = s_dyn + kShiftItems * ncoef;
    const int f = blockIdx.y;
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    const int it = blockIdx.x * kShiftItems + g;
    const bool act = it < ncells;
    int cell = 0;
    double t[3] = {0.0, 0.0, 0.0};
    if (act) {
        cell = cells[it];
        const int par = cell_i[CI_N * cell + CI_PARENT];
        for (int n = lane; n < ncoef; n += 32) s_a[g * ncoef + n] = L[((int64_t)f * C + par) * ncoef + n];
#pragma unroll
        for (int k = 0; k < 3; ++k) t[k] = cell_c[k * C + cell] - cell_c[k * C + par];
    }
    __syncthreads();
    if (act) shift_pass<false>(s_a + g * ncoef, s_b + g * ncoef, ncoef, p, 0, t[0], lane);
    __syncthreads();
    if (act) shift_pass<false>(s_b + g * ncoef, s_a + g * ncoef, ncoef, p, 1, t[1], lane);
    __syncthreads();
    if (act) {
        shift_pass<false>(s_a + g * ncoef, s_b + g * ncoef, ncoef, p, 2, t[2], lane);
        // the lanes that wrote out[n] add it (no barrier needed)
        for (int n = lane; n < nkeep; n += 32) L[((int64_t)f * C + cell) * ncoef + n] += s_b[g * ncoef + n];
    }
}

constexpr int kM2LWaves = 4;


// The two matrix-core shapes used by M2L: 16x16x4 with FP64 or FP32 operands.
// A (16 x 4): lane l holds row l%16, column l/16; B (4 x 16): lane l holds
// row l/16, column l%16.  The 16x16 result: lane l, register r holds
// column l%16 and row (l/16) + 4r (FP64) or 4(l/16) + r (FP32).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using v4 = double __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    using v4 = float __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ---------------------------------------------------------------------------
// Harmonic reduction of the translation.  D_k = d^k (1/|R|) is harmonic, so
// D_{k + 2e_z} = -D_{k + 2e_x} - D_{k + 2e_y}: every term of the contraction
// sum_n D_{n+m} Qt_n with n_z >= 2 folds, degree by degree, onto the n_z <= 1
// terms (Qr = reduced multipoles), and every output with m_z >= 2 follows from
// the m_z <= 1 outputs of the same degree.  Both keep |n| and |m|, so the
// truncation |n| + |m| <= p is unchanged and the result is the same
// contraction up to rounding, with (p+1)^2 instead of ncoef(p) indices per
// side (81 vs 165 at p = 8).
//
// Reduced indices (z <= 1), degree d block at d^2:
//   ridx(x, y, 0) = d^2 + y,   ridx(x, y, 1) = d^2 + d + 1 + y.
// Derivative table per key, entries with k_z <= 2 only, degree d block at
//   sd(d) = 0 (d = 0), 1 + 3 d (d - 1) / 2:  didx = sd(d) + {0, d + 1, 2d + 1}[k_z] + k_y.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int nr_of(int p) { return (p + 1) * (p + 1); }
__host__ __device__ constexpr int nd_of(int p) { return 1 + 3 * p * (p + 1) / 2; }
__host__ __device__ constexpr int rdeg(int j)
{
    int d = 0;
    while ((d + 1) * (d + 1) <= j) ++d;
    return d;
}
__host__ __device__ constexpr int ridx(int x, int y, int z)
{
    const int d = x + y + z;
    return d * d + z * (d + 1) + y;
}
__host__ __device__ constexpr int didx_of(int x, int y, int z)
{
    const int d = x + y + z;
    return (d == 0 ? 0 : 1 + 3 * d * (d - 1) / 2) + (z == 0 ? 0 : (z == 1 ? d + 1 : 2 * d + 1)) + y;
}
constexpr int kNrMax = (kPmax + 1) * (kPmax + 1);
constexpr int kNdMax = 1 + 3 * kPmax * (kPmax + 1) / 2;
struct RedTable {
    int8_t r[kNrMax][4];  // reduced index -> x, y, z, d
    int8_t d[kNdMax][4];  // table index -> x, y, z, d
};
constexpr RedTable make_red()
{
    RedTable t{};
    for (int d = 0; d <= kPmax; ++d)
        for (int z = 0; z <= 2; ++z)
            for (int y = 0; y + z <= d; ++y) {
                const int x = d - y - z;
                if (z <= 1) {
                    const int j = ridx(x, y, z);
                    t.r[j][0] = (int8_t)x, t.r[j][1] = (int8_t)y, t.r[j][2] = (int8_t)z, t.r[j][3] = (int8_t)d;
                }
                const int k = didx_of(x, y, z);
                t.d[k][0] = (int8_t)x, t.d[k][1] = (int8_t)y, t.d[k][2] = (int8_t)z, t.d[k][3] = (int8_t)d;
            }
    return t;
}
__constant__ RedTable c_red = make_red();

// MFMA tiling of the reduced contraction: rows m = reduced indices of degree
// <= p - 1 (degree p rows only meet n = 0, and Q_0 = 0), in tiles of 16;
// columns n = 1 .. nr(p) - 1 in steps of 4; row tile rt only needs columns
// of degree <= p - |m_min(rt)|.
__host__ __device__ constexpr int m2l_nrows(int P) { return P * P; }
__host__ __device__ constexpr int m2l_nrt(int P) { return (m2l_nrows(P) + 15) / 16; }
__host__ __device__ constexpr int m2l_ks(int P, int rt)
{
    const int d = rdeg(16 * rt);
    if (d >= P) return 0;
    return (nr_of(P - d) - 1 + 3) / 4;
}
__host__ __device__ constexpr int m2l_kstr(int P)
{
    int k = 4 * m2l_ks(P, 0) + 1;  // columns 0 .. 4 KS
    while (k % 16 != 1) ++k;       // odd row stride: spreads the 16 columns over the banks
    return k;
}
// Column steps of wave W: ks = W, W + kM2LWaves, ... of every row tile.
__host__ __device__ constexpr int m2l_wave_steps(int P, int W)
{
    int s = 0;
    for (int rt = 0; rt < m2l_nrt(P); ++rt) {
        const int KS = m2l_ks(P, rt);
        if (KS > W) s += (KS - W + kM2LWaves - 1) / kM2LWaves;
    }
    return s;
}
template <int P, int W>
using M2LIdx = int[m2l_wave_steps(P, W) > 0 ? m2l_wave_steps(P, W) : 1];

// Derivative tables: one thread per key, 2^(dl (|k| + 1)) D_k(rho) for
// |k| <= p, k_z <= 2, with D_k by
//   |k| r^2 D_k = -(2|k| - 1) sum_i k_i rho_i D_{k-e_i} - (|k| - 1) sum_i k_i (k_i - 1) D_{k-2e_i}
// (every term on the right has k_z no larger than k's).
__global__ void k_m2l_table(const int32_t *__restrict__ keys, int nkeys, int p, double *__restrict__ D)
{
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= nkeys) return;
    const int nd = nd_of(p);
    const int dl = keys[4 * key];
    const double unit = dl >= 0 ? 0.5 : ldexp(0.5, dl);  // rho = k * unit
    const double Rx = keys[4 * key + 1] * unit, Ry = keys[4 * key + 2] * unit, Rz = keys[4 * key + 3] * unit;
    const double r2 = (Rx * Rx + Ry * Ry) + Rz * Rz;
    double *row = D + (int64_t)key * nd;
    row[0] = 1.0 / sqrt(r2);
    for (int k = 1; k < nd; ++k) {
        const int kx = c_red.d[k][0], ky = c_red.d[k][1], kz = c_red.d[k][2], d = c_red.d[k][3];
        double s1 = 0.0, s2 = 0.0;
        if (kx > 0) s1 += kx * Rx * row[didx_of(kx - 1, ky, kz)];
        if (ky > 0) s1 += ky * Ry * row[didx_of(kx, ky - 1, kz)];
        if (kz > 0) s1 += kz * Rz * row[didx_of(kx, ky, kz - 1)];
        if (kx > 1) s2 += kx * (kx - 1) * row[didx_of(kx - 2, ky, kz)];
        if (ky > 1) s2 += ky * (ky - 1) * row[didx_of(kx, ky - 2, kz)];
        if (kz > 1) s2 += kz * (kz - 1) * row[didx_of(kx, ky, kz - 2)];
        row[k] = -((2.0 * d - 1.0) * s1 + (d - 1.0) * s2) / (d * r2);
    }
    // level-difference factor 2^(dl (|k| + 1)) (exact)
    for (int k = 0; k < nd; ++k) row[k] = ldexp(row[k], dl * (c_red.d[k][3] + 1));
}

__global__ void k_to_float(const double *__restrict__ a, int64_t n, float *__restrict__ b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (float)a[i];
}

// Reduced scaled multipoles of the cells holding tets; one thread per
// (cell, reduced index n = (a, b, c), c <= 1):
//   Qr_n = (-1)^|n| s_B^-|n| sum_{j >= 0} (-1)^j sum_{i <= j} C(j, i) Q_n'/n'!,
//   n' = (a - 2i, b - 2(j - i), c + 2j).
template <typename T>
__global__ void k_qreduce(const double *__restrict__ Q, const int32_t *__restrict__ cell_i, int64_t C, double side,
                          int p, int qpad, T *__restrict__ Qr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    const int ncoef = ncoef_of(p);
    if (i >= C * qpad) return;
    const int64_t c = i / qpad;
    const int n = (int)(i % qpad);
    double v = 0.0;
    if (n < nr_of(p) && cell_i[CI_N * c + CI_TEND] > cell_i[CI_N * c + CI_TBEG]) {
        const int a = c_red.r[n][0], b = c_red.r[n][1], cz = c_red.r[n][2], d = c_red.r[n][3];
        const double *q = Q + ((int64_t)f * C + c) * ncoef;
        for (int j = 0; cz + 2 * j <= d; ++j) {
            double sj = 0.0;
            for (int k = 0; k <= j; ++k) {
                const int x = a - 2 * k, y = b - 2 * (j - k), z = cz + 2 * j;
                if (x < 0 || y < 0) continue;
                sj += c_bin.c[j][k] * q[mi_index(x, y, z)] * c_bin.invfact[x] * c_bin.invfact[y] * c_bin.invfact[z];
            }
            v += (j & 1) ? -sj : sj;
        }
        const double is = 1.0 / ldexp(side, -cell_i[CI_N * c + CI_LEVEL]);
        double sp = 1.0;
        for (int j = 0; j < d; ++j) sp *= is;
        v *= ((d & 1) ? -sp : sp);
    }
    Qr[((int64_t)f * C + c) * qpad + n] = (T)v;
}

// Steps of wave W in issue order: column step ks = W, W + 4, ... (outer),
// row tiles rt with ks < KS(rt) (inner), so consecutive MFMAs of a wave feed
// different accumulators; row tile 0 (the longest) rotates over 2 of its own.
// m2l_wave_index gives this lane's D-table index of the A-operand element of
// every step (the zero slot ND outside |n| + |m| <= P).
template <int P, int W>
__device__ __forceinline__ void m2l_wave_index(int lane, M2LIdx<P, W> &didx)
{
    constexpr int NR = nr_of(P), NROW = m2l_nrows(P), ND = nd_of(P), NRT = m2l_nrt(P), KS0 = m2l_ks(P, 0);
    int s = 0;
#pragma unroll
    for (int ks = W; ks < KS0; ks += kM2LWaves) {
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
            if (ks < m2l_ks(P, rt)) {
                const int m = 16 * rt + (lane & 15), n = 1 + 4 * ks + (lane >> 4);
                int di = ND;  // the zero slot of the staged D row
                if (m < NROW && n < NR && c_red.r[m][3] + c_red.r[n][3] <= P)
                    di = didx_of(c_red.r[m][0] + c_red.r[n][0], c_red.r[m][1] + c_red.r[n][1],
                                 c_red.r[m][2] + c_red.r[n][2]);
                didx[s++] = di;
            }
        }
    }
}

template <typename T, int P, int W>
__device__ __forceinline__ void m2l_wave_mfma(typename Mfma<T>::v4 (&acc)[m2l_nrt(P)], typename Mfma<T>::v4 (&acc0)[2],
                                              const T *s_D, const T *s_Q, const M2LIdx<P, W> &didx, int lane)
{
    constexpr int NRT = m2l_nrt(P), KSTR = m2l_kstr(P), KS0 = m2l_ks(P, 0);
    const T *qcol = s_Q + (lane & 15) * KSTR + 1 + (lane >> 4);
    int s = 0, r0 = 0;
#pragma unroll
    for (int ks = W; ks < KS0; ks += kM2LWaves) {
        const T b = qcol[4 * ks];
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
            if (ks < m2l_ks(P, rt)) {
                const T a = s_D[didx[s++]];
                if (rt == 0) {
                    acc0[r0 & 1] = Mfma<T>::mma(a, b, acc0[r0 & 1]);
                    ++r0;
                } else {
                    acc[rt] = Mfma<T>::mma(a, b, acc[rt]);
                }
            }
        }
    }
}

// Geometry of a tile: TPT target cells x FPT fields = 16 MFMA columns,
// column c = t * FPT + g (target slot t, field f0 + g).
struct M2LCols {
    int tpt, fpt, f0, F;
    int dstr;  // row stride of the derivative tables (the plan's order; P may be lower)
};

// One workgroup of kM2LWaves wavefronts per target tile (see k_m2l_mfma).
// Two LDS buffers: while the MFMAs of key e read buffer e&1, the operands of
// key e+1 are loaded into registers and stored to the other buffer; one
// barrier per key.  Thread tid stages column tid/16, coefficients
// n = tid%16 + 16 j.
constexpr int kM2LSeg = 128;  // M2L entries whose metadata is staged in LDS at once
constexpr int kM2LAhead = 2;  // lookahead entries staged with a segment (matrix-core form)

template <typename T, int P, int W>
__device__ __forceinline__ void m2l_tile(const int32_t *__restrict__ tile_rng, const int32_t *__restrict__ ent_key,
                                         const int32_t *__restrict__ ent_src, const int32_t *__restrict__ keys,
                                         const T *__restrict__ Dtab, const T *__restrict__ Qr, int qpad, int64_t C,
                                         M2LCols cols, int tile, T *s_D, T *s_Q, int32_t *s_src, int32_t *s_kk,
                                         typename Mfma<T>::v4 (&acc)[m2l_nrt(P)])
{
    using v4 = typename Mfma<T>::v4;
    constexpr int NR = nr_of(P), ND = nd_of(P), KSTR = m2l_kstr(P), DSTR = ND + 1;
    constexpr int NT = 64 * kM2LWaves;
    static_assert(NT == 256, "16 columns x 16 threads");
    constexpr int QREG = (NR + 15) / 16, DREG = (ND + NT - 1) / NT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int tcol = tid >> 4, tn = tid & 15;
    const int tslot = tcol / cols.fpt, field = cols.f0 + tcol % cols.fpt;
    M2LIdx<P, W> didx;
    m2l_wave_index<P, W>(lane, didx);
    v4 acc0[2] = {v4{0, 0, 0, 0}, v4{0, 0, 0, 0}};
    const int e0 = tile_rng[2 * tile], e1 = tile_rng[2 * tile + 1];
    int qdeg[QREG];
#pragma unroll
    for (int j = 0; j < QREG; ++j) qdeg[j] = rdeg(tn + 16 * j);
    // Entry metadata (key id, its level difference, the source cell of every
    // tile slot) is staged in LDS a segment of kM2LSeg entries (plus
    // kM2LAhead lookahead entries) at a time, so the loop issues no global
    // load whose address depends on another global load.  The table row and
    // multipoles of an entry are loaded two entries ahead, into one of two
    // register sets: those of entry e + 2 are in flight while the MFMAs of
    // entry e run and entry e + 1 is stored to LDS, so a load has two entries
    // of matrix work to arrive in.  Loads go to clamped, in-bounds addresses
    // unconditionally and are masked when stored (exec-masked loads make the
    // compiler wait for every outstanding load where the branches join).
    const bool active = field < cols.F;
    const T *qf = Qr + (int64_t)(active ? field : 0) * C * qpad;
    int seg = e0;
    auto stage_seg = [&]() {
        const int ne = min(e1 - seg, kM2LSeg + kM2LAhead);
        for (int i = tid; i < ne * cols.tpt; i += NT) s_src[i] = ent_src[(int64_t)seg * cols.tpt + i];
        for (int i = tid; i < ne; i += NT) {
            const int key = ent_key[seg + i];
            s_kk[2 * i] = key;
            s_kk[2 * i + 1] = keys[4 * key];
        }
    };
    struct Ops {
        T q[QREG], d[DREG];
        int dl;
        bool ok;
    };
    auto fetch = [&](Ops &o, int e) {
        const int r = e - seg;
        const int key = s_kk[2 * r];
        o.dl = s_kk[2 * r + 1];
        const int src = s_src[r * cols.tpt + tslot];
#pragma unroll
        for (int j = 0; j < DREG; ++j) {
            const int k = tid + NT * j;
            o.d[j] = Dtab[(int64_t)key * cols.dstr + (k < ND ? k : ND - 1)];
        }
        o.ok = active && src >= 0;
        const T *q = qf + (int64_t)(o.ok ? src : 0) * qpad;
#pragma unroll
        for (int j = 0; j < QREG; ++j) {
            const int n = tn + 16 * j;
            o.q[j] = q[n < NR ? n : NR - 1];
        }
    };
    auto store = [&](const Ops &o, int buf) {
        T *D = s_D + buf * DSTR;
        T *Qb = s_Q + buf * 16 * KSTR + tcol * KSTR;
#pragma unroll
        for (int j = 0; j < DREG; ++j) {
            const int k = tid + NT * j;
            if (k < ND) D[k] = o.d[j];
        }
#pragma unroll
        for (int j = 0; j < QREG; ++j) {
            const int n = tn + 16 * j;
            if (n < NR) Qb[n] = o.ok ? ldexp(o.q[j], -o.dl * qdeg[j]) : (T)0;  // 2^(-dl |n|), exact
        }
    };
    if (e0 >= e1) return;
    stage_seg();
    __syncthreads();
    Ops oa, ob;
    fetch(oa, e0);
    store(oa, 0);
    if (e0 + 1 < e1) fetch(oa, e0 + 1);
    __syncthreads();
    // Entry e is in LDS buffer (e - e0) & 1, `cur` holds the loads of entry
    // e + 1 and `nxt` takes those of entry e + 2.
    auto step = [&](Ops &cur, Ops &nxt, int e) {
        const int buf = (e - e0) & 1;
        if (e + 2 < e1) fetch(nxt, e + 2);
        m2l_wave_mfma<T, P, W>(acc, acc0, s_D + buf * DSTR, s_Q + buf * 16 * KSTR, didx, lane);
        if (e + 1 < e1) store(cur, buf ^ 1);
        __syncthreads();
        if (e + 3 < e1 && e + 3 - seg == kM2LSeg + kM2LAhead) {  // the next fetch leaves the segment
            seg = e + 3;
            stage_seg();
            __syncthreads();
        }
    };
    for (int e = e0; e < e1; e += 2) {
        step(oa, ob, e);
        if (e + 1 < e1) step(ob, oa, e + 1);
    }
    acc[0] += acc0[0] + acc0[1];
}

// ---------------------------------------------------------------------------
// M2L on matrix cores.
//
// With cell sides s and the scaled multipoles
//   Qt_n(B) = (-1)^|n| Q_n(B) / (n! s_B^|n|),
// and rho = (c_A - c_B) / s_B, dl = level(B) - level(A), the translation is
//   l_m(A) = 1 / (4 pi m! s_A^(|m|+1)) * Lt_m(A),
//   Lt_m(A) = sum_B 2^(dl (|m|+1)) sum_{|n|>=1, |n|+|m|<=p} D_{n+m}(rho) Qt_n(B),
// D_k = d^k (1/|rho|) depending only on the key (dl, rho): one table row per
// distinct key serves every level, and all magnitudes are O(1) (the FP32 form
// needs no other scaling).  The level factor splits exactly as
// 2^(dl (|n|+|m|+1)) * 2^(-dl |n|): the first is in the key's table, the
// second is applied to the multipoles as they are staged.  The contraction runs on the harmonic reduction
// (reduced multipoles Qr, outputs Lr with m_z <= 1); the epilogue expands Lr
// to all m by
//   Lt_(x, y, c + 2j) = (-1)^j sum_{i <= j} C(j, i) Lr_(x + 2i, y + 2(j - i), c).
// A tile (16 MFMA columns: TPT target cells of one level x FPT fields) runs
// through the keys its cells use; per key the source multipoles form the B
// operand (columns without that key are zero), the Hankel matrix
// H[m][n] = D_{n+m} the A operand, and the 16x16x4 MFMA accumulates Lr for
// all columns in registers.  Four wavefronts split the column steps; their
// partial sums meet in LDS.
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__(64 * kM2LWaves, 2) void k_m2l_mfma(
    const int32_t *__restrict__ tile_tgt, const int32_t *__restrict__ tile_rng, const int32_t *__restrict__ ent_key,
    const int32_t *__restrict__ ent_src, const int32_t *__restrict__ keys, const T *__restrict__ Dtab,
    const T *__restrict__ Qr, int qpad, const int32_t *__restrict__ cell_i, double side, int64_t C, int tpt, int fpt,
    int F, int ntiles, int dstr, int lstr, double *__restrict__ L)
{
    using v4 = typename Mfma<T>::v4;
    constexpr int NC = ncoef_of(P), NROW = m2l_nrows(P), ND = nd_of(P), NRT = m2l_nrt(P), KSTR = m2l_kstr(P);
    static_assert(KSTR >= NROW, "the staging buffer doubles as the reduction buffer");
    static_assert(kM2LWaves == 4, "wave specialisation below");
    static_assert(2 * sizeof(T) >= sizeof(double), "reduction buffer fits in the staging buffers");
    __shared__ T s_D[2 * (ND + 1)];
    __shared__ __align__(16) T s_Q[2 * 16 * KSTR];
    __shared__ int32_t s_src[(kM2LSeg + kM2LAhead) * 16], s_kk[2 * (kM2LSeg + kM2LAhead)];
    const int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const M2LCols cols{tpt, fpt, (int)blockIdx.y * fpt, F, dstr};
    for (int i = tid; i < 2 * 16 * KSTR; i += blockDim.x) s_Q[i] = (T)0;  // column padding stays zero
    for (int i = tid; i < 2 * (ND + 1); i += blockDim.x) s_D[i] = (T)0;   // zero slot ND of each buffer
    __syncthreads();
    v4 acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) acc[rt] = v4{0, 0, 0, 0};
    switch (wave) {
    case 0: m2l_tile<T, P, 0>(tile_rng, ent_key, ent_src, keys, Dtab, Qr, qpad, C, cols, tile, s_D, s_Q, s_src, s_kk, acc); break;
    case 1: m2l_tile<T, P, 1>(tile_rng, ent_key, ent_src, keys, Dtab, Qr, qpad, C, cols, tile, s_D, s_Q, s_src, s_kk, acc); break;
    case 2: m2l_tile<T, P, 2>(tile_rng, ent_key, ent_src, keys, Dtab, Qr, qpad, C, cols, tile, s_D, s_Q, s_src, s_kk, acc); break;
    default: m2l_tile<T, P, 3>(tile_rng, ent_key, ent_src, keys, Dtab, Qr, qpad, C, cols, tile, s_D, s_Q, s_src, s_kk, acc); break;
    }
    // sum the waves' partial accumulators in LDS (FP64): red[c][m], c = column
    __syncthreads();
    double *red = reinterpret_cast<double *>(s_Q);
    for (int i = tid; i < 16 * KSTR; i += blockDim.x) red[i] = 0.0;
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * rt + Mfma<T>::row(lane, r);
            if (m < NROW) atomicAdd(&red[(lane & 15) * KSTR + m], (double)acc[rt][r]);
        }
    __syncthreads();
    // expand to all m, then l_m(A) = Lt_m / (4 pi m! s_A^(|m|+1))
    for (int i = tid; i < 16 * NC; i += blockDim.x) {
        const int c = i / NC, m = i - c * NC;
        const int field = cols.f0 + c % fpt;
        const int A = tile_tgt[tile * tpt + c / fpt];
        if (A < 0 || field >= F) continue;
        const int mx = c_mi.v[m][0], my = c_mi.v[m][1], mz = c_mi.v[m][2], dm = c_mi.v[m][3];
        double lt = 0.0;
        if (dm < P) {
            const int j = mz >> 1, cz = mz & 1;
            for (int k = 0; k <= j; ++k) lt += c_bin.c[j][k] * red[c * KSTR + ridx(mx + 2 * k, my + 2 * (j - k), cz)];
            if (j & 1) lt = -lt;
        }
        const double is = 1.0 / ldexp(side, -cell_i[CI_N * A + CI_LEVEL]);
        double sp = is;
        for (int k = 0; k < dm; ++k) sp *= is;
        atomicAdd(&L[((int64_t)field * C + A) * lstr + m],
                  lt * kInv4Pi * sp * c_bin.invfact[mx] * c_bin.invfact[my] * c_bin.invfact[mz]);
    }
}

// ---------------------------------------------------------------------------
// M2L packed by key (FP64, fewer than 16 fields).
//
// The contraction is that of k_m2l_mfma (scaled, harmonically reduced
// multipoles; Hankel operand H[m][n] = D_{n+m} of the key; outputs Lr with
// m_z <= 1), but the 16 matrix-core columns of a step are 16 / fpt
// translations of one key x fpt fields, taken from a block of up to
// nb = slots / fpt target cells: every column carries a translation except
// in the last group of each key.  The reduced locals of the block's
// (cell, field) slots are summed in LDS (FP64) and added to Lr once per
// work item; k_lr_expand then expands Lr to all m and adds it to L.
//
// Each wavefront takes a contiguous run of the item's groups (consecutive
// groups mostly share the key).  The key's derivative row is staged in the
// wavefront's own LDS row when the key changes; the multipoles of the next
// group are loaded into registers while the matrix cores work on the
// current one (two register sets, loop unrolled by two).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int m2l_all_steps(int P)
{
    int s = 0;
    for (int rt = 0; rt < m2l_nrt(P); ++rt) s += m2l_ks(P, rt);
    return s;
}
// LDS accumulator slots (target cell x field) of one packed block
__host__ __device__ constexpr int m2lp_slots(int P) { return P <= 8 ? 128 : 64; }
constexpr int kM2LPWaves = 4;

template <typename T, int P>
__global__ __launch_bounds__(64 * kM2LPWaves, P <= 8 ? 2 : 1) void k_m2l_pack(
    const int32_t *__restrict__ item, int nitems, const int32_t *__restrict__ blk_cells, int nb, int tpg,
    const int32_t *__restrict__ grp_key, const int32_t *__restrict__ grp_src, const uint8_t *__restrict__ grp_slot,
    const int32_t *__restrict__ keys, const T *__restrict__ Dtab, int dstr, const T *__restrict__ Qr, int qpad,
    int64_t C, int fpt, int F, double *__restrict__ Lr, int lrs)
{
    using v4 = typename Mfma<T>::v4;
    constexpr int NR = nr_of(P), ND = nd_of(P), NROW = m2l_nrows(P), NRT = m2l_nrt(P), KS0 = m2l_ks(P, 0);
    constexpr int NS = m2l_all_steps(P), NSLOT = m2lp_slots(P), DSTR = ND + 1;
    // odd row stride of the accumulators: the 16 columns of an output
    // register (the same row of 16 slots) fall in 16 different bank pairs
    // when their slots differ mod 16, as the packer arranges
    constexpr int LSTR = NROW | 1;
    __shared__ double s_L[NSLOT * LSTR];
    __shared__ T s_D[kM2LPWaves][2][DSTR];
    const int it = blockIdx.x;
    if (it >= nitems) return;
    // the wavefront index made visibly uniform: the group bounds, keys and
    // the key-change branch then live in scalar registers, and reading a key
    // does not wait for the vector loads of the prefetched multipoles
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 15, pair = col / fpt, fsub = col % fpt, field = (int)blockIdx.y * fpt + fsub;
    const bool fok = field < F;
    for (int i = tid; i < NSLOT * LSTR; i += blockDim.x) s_L[i] = 0.0;
    if (lane < 2) s_D[w][lane][ND] = (T)0;  // the zero slot of each row
    // this lane's table index of the A operand of every step (ks-major,
    // row tiles inner; the zero slot outside |n| + |m| <= P)
    int didx[NS];
    {
        int s = 0;
#pragma unroll
        for (int ks = 0; ks < KS0; ++ks) {
            const int n = 1 + 4 * ks + (lane >> 4);
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
                if (ks < m2l_ks(P, rt)) {
                    const int m = 16 * rt + (lane & 15);
                    int di = ND;
                    if (m < NROW && n < NR && c_red.r[m][3] + c_red.r[n][3] <= P)
                        di = didx_of(c_red.r[m][0] + c_red.r[n][0], c_red.r[m][1] + c_red.r[n][1],
                                     c_red.r[m][2] + c_red.r[n][2]);
                    didx[s++] = di;
                }
        }
    }
    __syncthreads();
    const int blk = item[3 * it], g0 = item[3 * it + 1], g1 = item[3 * it + 2];
    const int wg0 = g0 + (int)((int64_t)(g1 - g0) * w / kM2LPWaves);
    const int wg1 = g0 + (int)((int64_t)(g1 - g0) * (w + 1) / kM2LPWaves);
    const T *qf = Qr + (int64_t)(fok ? field : 0) * C * qpad;
    constexpr int DREG = (ND + 63) / 64;
    struct Ops {
        T b[KS0], d[DREG];
        int slot, key, dl;
        bool ok, newkey;
    };
    // loads of group g (the derivative row too when its key differs from
    // the previous group's): clamped addresses, masked when used
    auto fetch = [&](Ops &o, int g) {
        const int src = grp_src[(int64_t)g * tpg + pair];
        o.slot = grp_slot[(int64_t)g * tpg + pair];
        o.ok = fok && src >= 0;
        const T *q = qf + (int64_t)(o.ok ? src : 0) * qpad;
#pragma unroll
        for (int ks = 0; ks < KS0; ++ks) {
            const int n = 1 + 4 * ks + (lane >> 4);
            o.b[ks] = q[n < NR ? n : NR - 1];
        }
        o.key = grp_key[g];
        o.newkey = g == wg0 || grp_key[g - 1] != o.key;  // uniform over the wavefront
        if (o.newkey) {
            o.dl = keys[4 * o.key];
#pragma unroll
            for (int j = 0; j < DREG; ++j) {
                const int k = lane + 64 * j;
                o.d[j] = Dtab[(int64_t)o.key * dstr + (k < ND ? k : ND - 1)];
            }
        }
    };
    int buf = 0, dl = 0;
    auto run = [&](const Ops &o, int g) {
        if (o.newkey) {
            buf ^= 1;
            T *D = s_D[w][buf];
#pragma unroll
            for (int j = 0; j < DREG; ++j) {
                const int k = lane + 64 * j;
                if (k < ND) D[k] = o.d[j];
            }
            dl = o.dl;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const T *D = s_D[w][buf];
        // B operand: the multipoles times 2^(-dl |n|) (exact).  Columns of
        // empty slots and rows n >= NR hold finite values that meet zero A
        // entries or are never added out, so they need no masking.
        T b[KS0];
        if (dl == 0) {  // uniform over the wavefront
#pragma unroll
            for (int ks = 0; ks < KS0; ++ks) b[ks] = o.b[ks];
        } else {
#pragma unroll
            for (int ks = 0; ks < KS0; ++ks) {
                const int n = 1 + 4 * ks + (lane >> 4);
                const int deg = (int)sqrtf((float)n);  // exact: the degree block of n starts at deg^2
                b[ks] = (T)ldexp(o.b[ks], -dl * deg);
            }
        }
        v4 acc[NRT], acc0[2] = {v4{0, 0, 0, 0}, v4{0, 0, 0, 0}};
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) acc[rt] = v4{0, 0, 0, 0};
        int s = 0, r0 = 0;
#pragma unroll
        for (int ks = 0; ks < KS0; ++ks)
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
                if (ks < m2l_ks(P, rt)) {
                    const T a = D[didx[s++]];
                    if (rt == 0) {
                        acc0[r0 & 1] = Mfma<T>::mma(a, b[ks], acc0[r0 & 1]);
                        ++r0;
                    } else {
                        acc[rt] = Mfma<T>::mma(a, b[ks], acc[rt]);
                    }
                }
        acc[0] = acc0[0] + acc0[1];
        if (o.ok) {
            double *Ls = s_L + (o.slot * fpt + fsub) * LSTR;
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * rt + Mfma<T>::row(lane, r);
                    if (m < NROW) atomicAdd(&Ls[m], (double)acc[rt][r]);
                }
        }
    };
    if (wg0 < wg1) {
        Ops oa, ob;
        fetch(oa, wg0);
        for (int g = wg0; g < wg1; g += 2) {
            if (g + 1 < wg1) fetch(ob, g + 1);
            run(oa, g);
            if (g + 1 < wg1) {
                if (g + 2 < wg1) fetch(oa, g + 2);
                run(ob, g + 1);
            }
        }
    }
    __syncthreads();
    // add the block's reduced locals to Lr
    for (int i = tid; i < NSLOT * NROW; i += blockDim.x) {
        const int c = i / NROW, m = i - c * NROW;
        const double v = s_L[c * LSTR + m];
        if (v == 0.0) continue;
        const int fld = (int)blockIdx.y * fpt + c % fpt, cell = c / fpt < nb ? blk_cells[(int64_t)blk * nb + c / fpt] : -1;
        if (cell >= 0 && fld < F) atomicAdd(&Lr[((int64_t)fld * C + cell) * lrs + m], v);
    }
}

// L_m(A) += Lt_m(A) / (4 pi m! s_A^(|m|+1)), Lt expanded from the reduced
// locals Lr (see k_m2l_mfma), for |m| < the order of A's level; one thread
// per (cell, m), fields in blockIdx.y.
__global__ void k_lr_expand(const double *__restrict__ Lr, int lrs, const int32_t *__restrict__ cell_i, double side,
                            int64_t C, int ncoef, LevelOrders lo, double *__restrict__ L)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C * ncoef) return;
    const int64_t A = i / ncoef;
    const int m = (int)(i - A * ncoef), f = blockIdx.y;
    const int lev = cell_i[CI_N * A + CI_LEVEL];
    const int mx = c_mi.v[m][0], my = c_mi.v[m][1], mz = c_mi.v[m][2], dm = c_mi.v[m][3];
    if (dm >= lo.q[lev]) return;
    const double *red = Lr + ((int64_t)f * C + A) * lrs;
    const int j = mz >> 1, cz = mz & 1;
    double lt = 0.0;
    for (int k = 0; k <= j; ++k) lt += c_bin.c[j][k] * red[ridx(mx + 2 * k, my + 2 * (j - k), cz)];
    if (lt == 0.0) return;
    if (j & 1) lt = -lt;
    const double is = 1.0 / ldexp(side, -lev);
    double sp = is;
    for (int k = 0; k < dm; ++k) sp *= is;
    L[((int64_t)f * C + A) * ncoef + m] += lt * kInv4Pi * sp * c_bin.invfact[mx] * c_bin.invfact[my] * c_bin.invfact[mz];
}

// ---------------------------------------------------------------------------
// M2L with split BF16 operands on matrix cores (v_mfma_f32_16x16x32_bf16).
//
// The FP32 operands of the FP32 form (derivative rows and reduced multipoles,
// all O(1) by the level scaling) are split as they are staged into LDS,
// x = x0 + x1 + x2 with x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1)
// (each difference exact in FP32), and the product is formed from the part
// products of total order < NP: NP = 2 takes a0 b0 + a0 b1 + a1 b0 (BF16x3),
// NP = 3 adds a1 b1 + a0 b2 + a2 b0 (BF16x6), accumulated in FP32.
// Operand layout: A (16 x 32): lane l holds row l%16, columns 8(l/16) + i;
// B (32 x 16): lane l holds rows 8(l/16) + i, column l%16; result as the
// FP32 16x16x4 form (row 4(l/16) + r, column l%16).
// Column steps are 32 wide (n = 1 + 32 ks + ...); the (row tile, step) pairs
// are dealt to two wavefronts in turn.
// ---------------------------------------------------------------------------
constexpr int kM2LBWaves = 2;
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));

__host__ __device__ constexpr int m2lb_ks(int P, int rt)
{
    const int d = rdeg(16 * rt);
    if (d >= P) return 0;
    return (nr_of(P - d) - 1 + 31) / 32;
}
__host__ __device__ constexpr int m2lb_kstr(int P) { return 32 * m2lb_ks(P, 0) + 8; }  // bf16 per staged column
// number of (rt, ks) steps of wave W: steps in order ks-major, dealt in turn
__host__ __device__ constexpr int m2lb_wave_steps(int P, int W)
{
    int s = 0, c = 0;
    for (int ks = 0; ks < m2lb_ks(P, 0); ++ks)
        for (int rt = 0; rt < m2l_nrt(P); ++rt)
            if (ks < m2lb_ks(P, rt)) {
                if (s % kM2LBWaves == W) ++c;
                ++s;
            }
    return c;
}
// row tile and column step of the j-th step of wave W
__host__ __device__ constexpr int m2lb_step(int P, int W, int j, bool want_rt)
{
    int s = 0, c = 0;
    for (int ks = 0; ks < m2lb_ks(P, 0); ++ks)
        for (int rt = 0; rt < m2l_nrt(P); ++rt)
            if (ks < m2lb_ks(P, rt)) {
                if (s % kM2LBWaves == W) {
                    if (c == j) return want_rt ? rt : ks;
                    ++c;
                }
                ++s;
            }
    return 0;
}

__device__ __forceinline__ void bf16_split3(float x, __bf16 &x0, __bf16 &x1, __bf16 &x2)
{
    x0 = (__bf16)x;
    const float r1 = x - (float)x0;
    x1 = (__bf16)r1;
    x2 = (__bf16)(r1 - (float)x1);
}

template <int P, int NP, int W>
__device__ __forceinline__ void m2lb_tile(const int32_t *__restrict__ tile_rng, const int32_t *__restrict__ ent_key,
                                          const int32_t *__restrict__ ent_src, const int32_t *__restrict__ keys,
                                          const float *__restrict__ Dtab, const float *__restrict__ Qr, int qpad,
                                          int64_t C, M2LCols cols, int tile, __bf16 *s_D, __bf16 *s_Q,
                                          int32_t *s_src, int32_t *s_kk, Mfma<float>::v4 (&acc)[m2l_nrt(P)])
{
    constexpr int NR = nr_of(P), NROW = m2l_nrows(P), ND = nd_of(P), KSTR = m2lb_kstr(P), DSTR = ND + 1;
    constexpr int NT = 64 * kM2LBWaves, NS = m2lb_wave_steps(P, W);
    static_assert(NT % 16 == 0, "16 columns");
    constexpr int TPC = NT / 16;  // staging threads per column
    constexpr int QREG = (NR + TPC - 1) / TPC, DREG = (ND + NT - 1) / NT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int tcol = tid / TPC, tn = tid % TPC;
    const int tslot = tcol / cols.fpt, field = cols.f0 + tcol % cols.fpt;
    // A-operand table indices of this lane, per step (the zero slot ND outside |n| + |m| <= P)
    int didx[NS > 0 ? NS : 1][8];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int rt = m2lb_step(P, W, j, true), ks = m2lb_step(P, W, j, false);
        const int m = 16 * rt + (lane & 15);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int n = 1 + 32 * ks + 8 * (lane >> 4) + i;
            int di = ND;
            if (m < NROW && n < NR && c_red.r[m][3] + c_red.r[n][3] <= P)
                di = didx_of(c_red.r[m][0] + c_red.r[n][0], c_red.r[m][1] + c_red.r[n][1], c_red.r[m][2] + c_red.r[n][2]);
            didx[j][i] = di;
        }
    }
    const int e0 = tile_rng[2 * tile], e1 = tile_rng[2 * tile + 1];
    float pq[QREG], pd[DREG];
    int pdl = 0, qdeg[QREG];
#pragma unroll
    for (int j = 0; j < QREG; ++j) qdeg[j] = rdeg(tn + TPC * j);
    // entry metadata staged in LDS by segments, loads as in m2l_tile
    const bool active = field < cols.F;
    const float *qf = Qr + (int64_t)(active ? field : 0) * C * qpad;
    int seg = e0;
    auto stage_seg = [&]() {
        const int ne = min(e1 - seg, kM2LSeg + 1);
        for (int i = tid; i < ne * cols.tpt; i += NT) s_src[i] = ent_src[(int64_t)seg * cols.tpt + i];
        for (int i = tid; i < ne; i += NT) {
            const int key = ent_key[seg + i];
            s_kk[2 * i] = key;
            s_kk[2 * i + 1] = keys[4 * key];
        }
    };
    bool qok = false;
    auto fetch = [&](int e) {
        const int r = e - seg;
        const int key = s_kk[2 * r];
        pdl = s_kk[2 * r + 1];
        const int src = s_src[r * cols.tpt + tslot];
#pragma unroll
        for (int j = 0; j < DREG; ++j) {
            const int k = tid + NT * j;
            pd[j] = Dtab[(int64_t)key * cols.dstr + (k < ND ? k : ND - 1)];
        }
        qok = active && src >= 0;
        const float *q = qf + (int64_t)(qok ? src : 0) * qpad;
#pragma unroll
        for (int j = 0; j < QREG; ++j) {
            const int n = tn + TPC * j;
            pq[j] = q[n < NR ? n : NR - 1];
        }
    };
    auto store = [&](int buf) {
        __bf16 *D = s_D + buf * 3 * DSTR;
#pragma unroll
        for (int j = 0; j < DREG; ++j) {
            const int k = tid + NT * j;
            if (k < ND) bf16_split3(pd[j], D[k], D[DSTR + k], D[2 * DSTR + k]);
        }
        __bf16 *Qb = s_Q + buf * 3 * 16 * KSTR + tcol * KSTR;
#pragma unroll
        for (int j = 0; j < QREG; ++j) {
            const int n = tn + TPC * j;
            if (n >= 1 && n < NR)  // column n is stored at n - 1
                bf16_split3(qok ? ldexpf(pq[j], -pdl * qdeg[j]) : 0.0f, Qb[n - 1], Qb[16 * KSTR + n - 1],
                            Qb[32 * KSTR + n - 1]);
        }
    };
    if (e0 >= e1) return;
    stage_seg();
    __syncthreads();
    fetch(e0);
    store(0);
    __syncthreads();
    for (int e = e0; e < e1; ++e) {
        const int buf = (e - e0) & 1;
        if (e + 1 < e1) fetch(e + 1);
        const __bf16 *D = s_D + buf * 3 * DSTR;
        const __bf16 *Qb = s_Q + buf * 3 * 16 * KSTR + (lane & 15) * KSTR + 8 * (lane >> 4);
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int rt = m2lb_step(P, W, j, true), ks = m2lb_step(P, W, j, false);
            bf16x8 a[NP], b[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                b[q] = *reinterpret_cast<const bf16x8 *>(Qb + q * 16 * KSTR + 32 * ks);
#pragma unroll
                for (int i = 0; i < 8; ++i) a[q][i] = D[q * DSTR + didx[j][i]];
            }
            // smallest terms first
            if constexpr (NP == 3) {
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc[rt], 0, 0, 0);
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc[rt], 0, 0, 0);
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc[rt], 0, 0, 0);
            }
            acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc[rt], 0, 0, 0);
            acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc[rt], 0, 0, 0);
            acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc[rt], 0, 0, 0);
        }
        if (e + 1 < e1) store(buf ^ 1);
        __syncthreads();
        if (e + 1 - seg == kM2LSeg && e + 1 < e1) {
            seg = e + 1;
            stage_seg();
            __syncthreads();
        }
    }
}

template <int P, int NP>
__global__ __launch_bounds__(64 * kM2LBWaves, 2) void k_m2l_bf16(
    const int32_t *__restrict__ tile_tgt, const int32_t *__restrict__ tile_rng, const int32_t *__restrict__ ent_key,
    const int32_t *__restrict__ ent_src, const int32_t *__restrict__ keys, const float *__restrict__ Dtab,
    const float *__restrict__ Qr, int qpad, const int32_t *__restrict__ cell_i, double side, int64_t C, int tpt, int fpt,
    int F, int ntiles, int dstr, int lstr, double *__restrict__ L)
{
    using v4 = Mfma<float>::v4;
    constexpr int NC = ncoef_of(P), NROW = m2l_nrows(P), ND = nd_of(P), NRT = m2l_nrt(P), KSTR = m2lb_kstr(P);
    constexpr int RSTR = NROW + 1;  // reduction buffer row stride (doubles)
    static_assert(kM2LBWaves == 2, "wave specialisation below");
    static_assert(16 * RSTR * sizeof(double) <= 2 * 3 * 16 * KSTR * sizeof(__bf16), "reduction buffer fits");
    __shared__ __bf16 s_D[2 * 3 * (ND + 1)];
    __shared__ __align__(16) __bf16 s_Q[2 * 3 * 16 * KSTR];
    __shared__ int32_t s_src[(kM2LSeg + 1) * 16], s_kk[2 * (kM2LSeg + 1)];
    const int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const M2LCols cols{tpt, fpt, (int)blockIdx.y * fpt, F, dstr};
    for (int i = tid; i < 2 * 3 * 16 * KSTR; i += blockDim.x) s_Q[i] = (__bf16)0.0f;  // padding stays zero
    for (int i = tid; i < 2 * 3 * (ND + 1); i += blockDim.x) s_D[i] = (__bf16)0.0f;   // zero slots
    __syncthreads();
    v4 acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) acc[rt] = v4{0, 0, 0, 0};
    if (wave == 0)
        m2lb_tile<P, NP, 0>(tile_rng, ent_key, ent_src, keys, Dtab, Qr, qpad, C, cols, tile, s_D, s_Q, s_src, s_kk,
                            acc);
    else
        m2lb_tile<P, NP, 1>(tile_rng, ent_key, ent_src, keys, Dtab, Qr, qpad, C, cols, tile, s_D, s_Q, s_src, s_kk,
                            acc);
    __syncthreads();
    double *red = reinterpret_cast<double *>(s_Q);
    for (int i = tid; i < 16 * RSTR; i += blockDim.x) red[i] = 0.0;
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * rt + Mfma<float>::row(lane, r);
            if (m < NROW) atomicAdd(&red[(lane & 15) * RSTR + m], (double)acc[rt][r]);
        }
    __syncthreads();
    for (int i = tid; i < 16 * NC; i += blockDim.x) {
        const int c = i / NC, m = i - c * NC;
        const int field = cols.f0 + c % fpt;
        const int A = tile_tgt[tile * tpt + c / fpt];
        if (A < 0 || field >= F) continue;
        const int mx = c_mi.v[m][0], my = c_mi.v[m][1], mz = c_mi.v[m][2], dm = c_mi.v[m][3];
        double lt = 0.0;
        if (dm < P) {
            const int j = mz >> 1, cz = mz & 1;
            for (int k = 0; k <= j; ++k) lt += c_bin.c[j][k] * red[c * RSTR + ridx(mx + 2 * k, my + 2 * (j - k), cz)];
            if (j & 1) lt = -lt;
        }
        const double is = 1.0 / ldexp(side, -cell_i[CI_N * A + CI_LEVEL]);
        double sp = is;
        for (int k = 0; k < dm; ++k) sp *= is;
        atomicAdd(&L[((int64_t)field * C + A) * lstr + m],
                  lt * kInv4Pi * sp * c_bin.invfact[mx] * c_bin.invfact[my] * c_bin.invfact[mz]);
    }
}

// ---------------------------------------------------------------------------
// L2P.  One thread per target (octree order) and field (blockIdx.y); adds
// into u[f][perm[i]].
//   u(x) = sum_m l_m (x - c)^m
// The order is a template parameter, so the loop over m unrolls and every
// monomial is a product of three powers held in registers.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_l2p(const double *__restrict__ tgt_xyz, const int32_t *__restrict__ tgt_perm,
                                             const int32_t *__restrict__ tgt_leaf, int64_t N,
                                             const double *__restrict__ cell_c, int64_t C,
                                             const double *__restrict__ L, double *__restrict__ u)
{
    constexpr int NC = ncoef_of(P);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (i >= N) return;
    const int leaf = tgt_leaf[i];
    const double y[3] = {tgt_xyz[i] - cell_c[leaf], tgt_xyz[N + i] - cell_c[C + leaf],
                         tgt_xyz[2 * N + i] - cell_c[2 * C + leaf]};
    double pw[3][P + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pw[k][0] = 1.0;
#pragma unroll
        for (int j = 1; j <= P; ++j) pw[k][j] = pw[k][j - 1] * y[k];
    }
    const double *Ll = L + ((int64_t)f * C + leaf) * NC;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < NC; ++m) s = fma(Ll[m], pw[0][mi_x(m)] * pw[1][mi_y(m)] * pw[2][mi_z(m)], s);
    atomicAdd(&u[(int64_t)f * N + tgt_perm[i]], s);  // the near field is added concurrently
}

// One workgroup per P2P block (<= 64 tets of a source leaf and the targets of
// its near target leaves): one wavefront for one or two fields, four for more
// (they share the staged field coefficients).  Tets are staged in LDS BT at a
// time, thread l preparing field l % FCH of tet l / FCH (geometry 240 B + 208
// B per field per tet; 8 tets for 32 fields); every thread then takes targets
// ib + l, ib + l + NT, ... over the staged tets and adds its potentials
// atomically.  With band_skip the pairs of the surrogate's distance band
// (in_band) are left out: they are evaluated from the band pair list.
// WIDE: four wavefronts also for one or two fields (a plan's tuning choice).
__host__ __device__ constexpr int p2p_threads(int FCH, bool wide) { return FCH <= 2 && !wide ? 64 : 256; }
__host__ __device__ constexpr int p2p_stage(int FCH, bool wide)
{
    return FCH <= 2 ? (wide ? 64 / FCH : 16) : (FCH >= 32 ? 8 : (FCH >= 16 ? 16 : (FCH >= 8 ? 32 : 64)));
}

template <int FCH, bool WIDE>
__global__ __launch_bounds__(p2p_threads(FCH, WIDE), 2) void k_p2p(const int32_t *__restrict__ blk, int nblk, int band_skip, int64_t T,
                                                     const double *__restrict__ tet_xyz, const int32_t *__restrict__ tet_node,
                                                     const int32_t *__restrict__ idx, const double *__restrict__ tgt_xyz,
                                                     const int32_t *__restrict__ tgt_perm, int64_t N,
                                                     const double *__restrict__ M, int64_t n_nodes, int f0,
                                                     double *__restrict__ u)
{
    constexpr int BT = p2p_stage(FCH, WIDE), NT = p2p_threads(FCH, WIDE);
    static_assert(BT * FCH <= NT, "one thread per staged tet and field");
    __shared__ TetGeom s_g[BT];
    __shared__ TetField s_f[BT][FCH];
    __shared__ double s_bc[BT][4];  // band test: centroid, 1 / diam^2
    const int b = xcd_item(nblk);
    if (b < 0) return;
    const int tb = blk[4 * b], te = blk[4 * b + 1], ib = blk[4 * b + 2], ie = blk[4 * b + 3];
    const int lane = threadIdx.x;
    for (int sb = tb; sb < te; sb += BT) {
        const int nt = min(BT, te - sb);
        __syncthreads();
        {
            const int t = lane / FCH, f = lane % FCH;
            if (t < nt) {
                tet_prepare(tet_xyz, tet_node, T, sb + t, M + (int64_t)(f0 + f) * n_nodes * 3, f == 0 ? &s_g[t] : nullptr,
                            s_f[t][f]);
                if (band_skip && f == 0) {
                    double v[4][3];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int k = 0; k < 3; ++k) v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + sb + t];
                    band_geom(v, s_bc[t], s_bc[t][3]);
                }
            }
        }
        __syncthreads();
        for (int i = ib + lane; i < ie; i += NT) {
            const int s = idx[i];
            const double x[3] = {tgt_xyz[s], tgt_xyz[N + s], tgt_xyz[2 * N + s]};
            double acc[FCH];
#pragma unroll
            for (int f = 0; f < FCH; ++f) acc[f] = 0.0;
#pragma unroll 1
            for (int t = 0; t < nt; ++t) {
                if (band_skip && in_band(x, s_bc[t], s_bc[t][3])) continue;
                pair_accumulate<FCH>(x, s_g[t], s_f[t], acc);
            }
            const int64_t o = tgt_perm[s];
#pragma unroll
            for (int f = 0; f < FCH; ++f) atomicAdd(&u[(int64_t)(f0 + f) * N + o], acc[f] * kInv4Pi);
        }
    }
}

// ---------------------------------------------------------------------------
// Direct sum: every target against every tet.  Far from a tet the closed form
// of pair_accumulate adds terms much larger than their sum and loses about
// (d/diam)^4 eps (d = |x - centroid|, diam = the longest edge).  From 3
// diameters on the pair is instead integrated by a collapsed Gauss-Jacobi
// rule of the integrand of eq. approx1,
//   4 pi u_T(x) = 6|V| sum_q w_q M(y_q) . (x - y_q) / |x - y_q|^3
//               = 6|V| sum_i M_i . K_i,
//   K_i = sum_q w_q lambda_i(q) (x - y_q) / |x - y_q|^3,
// K independent of the field, with the rules of degree 13, 11, 9 and 7 for
// the bands [3, 6), [6, 12), [12, 24) and [24, inf) diameters (rule error
// below ~1e-14 of |M| V / (4 pi d^2)).  One workgroup of 256 threads per DT consecutive tets
// staged in LDS; every thread takes targets lane, lane + 256, ... and adds
// its sums over the staged tets atomically.
// ---------------------------------------------------------------------------
struct FarTet {
    double c[3];     // centroid
    double id2;      // 1 / diam^2
    double e[3][3];  // v_1 - v_0, v_2 - v_0, v_3 - v_0
    double vol6;     // 6 |V|
};
__host__ __device__ constexpr int direct_stage(int FCH) { return FCH >= 32 ? 4 : (FCH >= 16 ? 8 : 16); }

template <int FCH>
__global__ __launch_bounds__(256, 2) void k_direct(int nblk, int64_t T, const double *__restrict__ tet_xyz,
                                                const int32_t *__restrict__ tet_node,
                                                const double *__restrict__ tgt_xyz,
                                                const int32_t *__restrict__ tgt_perm, int64_t N,
                                                const double *__restrict__ M, int64_t n_nodes, int f0,
                                                const double *__restrict__ rule, double *__restrict__ u)
{
    constexpr int DT = direct_stage(FCH);
    static_assert(DT * FCH <= 256, "one thread per staged tet and field");
    __shared__ TetGeom s_g[DT];
    __shared__ TetField s_f[DT][FCH];
    __shared__ FarTet s_t[DT];
    __shared__ double s_m[DT][FCH][12];
    const int b = xcd_item(nblk);
    if (b < 0) return;
    const int64_t tb = (int64_t)b * DT;
    const int nt = (int)min<int64_t>(DT, T - tb);
    const int lane = threadIdx.x;
    {
        const int t = lane / FCH, f = lane % FCH;
        if (t < nt) {
            const int64_t tt = tb + t;
            const double *Mf = M + (int64_t)(f0 + f) * n_nodes * 3;
            tet_prepare(tet_xyz, tet_node, T, tt, Mf, f == 0 ? &s_g[t] : nullptr, s_f[t][f]);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t nd = tet_node[(int64_t)c * T + tt];
#pragma unroll
                for (int k = 0; k < 3; ++k) s_m[t][f][3 * c + k] = Mf[3 * nd + k];
            }
            if (f == 0) {
                double v[4][3];
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int k = 0; k < 3; ++k) v[c][k] = tet_xyz[(int64_t)(3 * c + k) * T + tt];
                FarTet &F = s_t[t];
                double l2 = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int q = a + 1; q < 4; ++q) {
                        const double dx = v[q][0] - v[a][0], dy = v[q][1] - v[a][1], dz = v[q][2] - v[a][2];
                        l2 = fmax(l2, dx * dx + dy * dy + dz * dz);
                    }
                F.id2 = 1.0 / l2;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    F.c[k] = 0.25 * ((v[0][k] + v[1][k]) + (v[2][k] + v[3][k]));
                    F.e[0][k] = v[1][k] - v[0][k];
                    F.e[1][k] = v[2][k] - v[0][k];
                    F.e[2][k] = v[3][k] - v[0][k];
                }
                const double det = F.e[0][0] * (F.e[1][1] * F.e[2][2] - F.e[1][2] * F.e[2][1]) -
                                   F.e[0][1] * (F.e[1][0] * F.e[2][2] - F.e[1][2] * F.e[2][0]) +
                                   F.e[0][2] * (F.e[1][0] * F.e[2][1] - F.e[1][1] * F.e[2][0]);
                F.vol6 = fabs(det);
            }
        }
    }
    __syncthreads();
    const double r2b[kFarBands] = {kFarRatio[0] * kFarRatio[0], kFarRatio[1] * kFarRatio[1],
                                   kFarRatio[2] * kFarRatio[2], kFarRatio[3] * kFarRatio[3]};
    for (int64_t i = lane; i < N; i += 256) {
        const double x[3] = {tgt_xyz[i], tgt_xyz[N + i], tgt_xyz[2 * N + i]};
        double acc[FCH];
#pragma unroll
        for (int f = 0; f < FCH; ++f) acc[f] = 0.0;
#pragma unroll 1
        for (int t = 0; t < nt; ++t) {
            const FarTet &F = s_t[t];
            const double dc0 = x[0] - F.c[0], dc1 = x[1] - F.c[1], dc2 = x[2] - F.c[2];
            const double rat2 = (dc0 * dc0 + dc1 * dc1 + dc2 * dc2) * F.id2;
            if (rat2 < r2b[0]) {
                pair_accumulate<FCH>(x, s_g[t], s_f[t], acc);
                continue;
            }
            const int band = rat2 < r2b[1] ? 0 : (rat2 < r2b[2] ? 1 : (rat2 < r2b[3] ? 2 : 3));
            const int q0 = band == 0 ? kFarOff[0] : (band == 1 ? kFarOff[1] : (band == 2 ? kFarOff[2] : kFarOff[3]));
            const int q1 = band == 0 ? kFarOff[1] : (band == 1 ? kFarOff[2] : (band == 2 ? kFarOff[3] : kFarOff[4]));
            const double xv[3] = {x[0] - s_g[t].v[0][0], x[1] - s_g[t].v[0][1], x[2] - s_g[t].v[0][2]};
            double S[3] = {0.0, 0.0, 0.0}, K[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll 2
            for (int q = q0; q < q1; ++q) {
                const double l1 = rule[4 * q], l2 = rule[4 * q + 1], l3 = rule[4 * q + 2], w = rule[4 * q + 3];
                double d[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) d[k] = xv[k] - (l1 * F.e[0][k] + l2 * F.e[1][k] + l3 * F.e[2][k]);
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                const double ri = rsqrt_nr(r2);
                const double wr = w * ri * ri * ri;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double kk = wr * d[k];
                    S[k] += kk;
                    K[0][k] = fma(l1, kk, K[0][k]);
                    K[1][k] = fma(l2, kk, K[1][k]);
                    K[2][k] = fma(l3, kk, K[2][k]);
                }
            }
            // K_0 = S - K_1 - K_2 - K_3 (lambda_0 = 1 - lambda_1 - lambda_2 - lambda_3)
#pragma unroll
            for (int f = 0; f < FCH; ++f) {
                const double *m = s_m[t][f];
                double v = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    v += m[k] * (S[k] - K[0][k] - K[1][k] - K[2][k]) + m[3 + k] * K[0][k] + m[6 + k] * K[1][k] +
                         m[9 + k] * K[2][k];
                acc[f] = fma(F.vol6, v, acc[f]);
            }
        }
        const int64_t o = tgt_perm[i];
#pragma unroll
        for (int f = 0; f < FCH; ++f) atomicAdd(&u[(int64_t)(f0 + f) * N + o], acc[f] * kInv4Pi);
    }
}

// ---------------------------------------------------------------------------
// Point dipoles (the second source kind): u(x) = 1/(4 pi) sum_i m_i . (x - y_i)
// / |x - y_i|^3 over the sources of the near leaves (or all, direct sum); a
// target at a source's own position takes nothing from it.  Blocks as in
// k_p2p; the positions and the FCH moments of kPtStage sources are staged in
// LDS, every thread takes targets ib + l, ib + l + 256, ...
// ---------------------------------------------------------------------------
constexpr int kPtStage = 128, kPtThreads = 256;
constexpr int kP2PTets = 64;  // sources per block of the dipole direct sum

template <int FCH>
__global__ __launch_bounds__(kPtThreads) void k_p2p_points(const int32_t *__restrict__ blk, int nblk, int direct_src,
                                                           int64_t T, const double *__restrict__ src_xyz,
                                                           const int32_t *__restrict__ src_node,
                                                           const int32_t *__restrict__ idx,
                                                           const double *__restrict__ tgt_xyz,
                                                           const int32_t *__restrict__ tgt_perm, int64_t N,
                                                           const double *__restrict__ M, int64_t n_nodes, int f0,
                                                           double *__restrict__ u)
{
    __shared__ double s_y[kPtStage][3];
    __shared__ double s_m[kPtStage][FCH][3];
    const int b = xcd_item(nblk);
    if (b < 0) return;
    int tb, te, ib, ie;
    if (direct_src) {
        tb = b * kP2PTets;
        te = min<int64_t>(T, tb + kP2PTets);
        ib = 0;
        ie = (int)N;
    } else {
        tb = blk[4 * b];
        te = blk[4 * b + 1];
        ib = blk[4 * b + 2];
        ie = blk[4 * b + 3];
    }
    const int lane = threadIdx.x;
    for (int sb = tb; sb < te; sb += kPtStage) {
        const int ns = min(kPtStage, te - sb);
        __syncthreads();
        for (int i = lane; i < ns; i += kPtThreads) {
#pragma unroll
            for (int k = 0; k < 3; ++k) s_y[i][k] = src_xyz[(int64_t)k * T + sb + i];
            const int64_t nd = src_node[sb + i];
#pragma unroll
            for (int f = 0; f < FCH; ++f)
#pragma unroll
                for (int k = 0; k < 3; ++k) s_m[i][f][k] = M[((int64_t)(f0 + f) * n_nodes + nd) * 3 + k];
        }
        __syncthreads();
        for (int i = ib + lane; i < ie; i += kPtThreads) {
            const int s = direct_src ? i : idx[i];
            const double x[3] = {tgt_xyz[s], tgt_xyz[N + s], tgt_xyz[2 * N + s]};
            double acc[FCH];
#pragma unroll
            for (int f = 0; f < FCH; ++f) acc[f] = 0.0;
            for (int j = 0; j < ns; ++j) {
                const double d0 = x[0] - s_y[j][0], d1 = x[1] - s_y[j][1], d2 = x[2] - s_y[j][2];
                const double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
                const double w = r2 > 0.0 ? 1.0 / (r2 * sqrt(r2)) : 0.0;
#pragma unroll
                for (int f = 0; f < FCH; ++f)
                    acc[f] = fma(w, (s_m[j][f][0] * d0 + s_m[j][f][1] * d1) + s_m[j][f][2] * d2, acc[f]);
            }
            const int64_t o = tgt_perm[s];
#pragma unroll
            for (int f = 0; f < FCH; ++f) atomicAdd(&u[(int64_t)(f0 + f) * N + o], acc[f] * kInv4Pi);
        }
    }
}

// ---------------------------------------------------------------------------
// Single-field near field over the shared mesh entities of a source chunk.
//
// Summed over the tets T of a chunk, the pair formula regroups by entity:
//   4 pi u(x) = sum_edges [ f_e il_e B_e(y) + Gamma_e g_e ] - sum_faces A_F(y) h_F Omega_F
// with y = x - c (c the chunk's node centroid), f_e the edge log (the line
// integral of 1/R, independent of the edge direction), g_e = R0^2 f +
// l_b R_b - l_a R_a (also direction independent), h_F Omega_F the face's
// height times solid angle in any fixed orientation (the product does not
// change with it), and the field weights
//   A_F(y)   = sum_{T, k: face k of T is F} alpha_{T,k}(y)                     (affine)
//   B_e(y)   = sum_{T, k, e in face k} s_{k,e} alpha_{T,k}(y) n_k.(d_a x d_b)  (quadratic)
//   Gamma_e  = sum_{T: e in T} gamma_{T,e}
// (alpha affine in y, d = v - x).  k_topo_coef forms them once per evaluation;
// k_p2p_topo then evaluates one square root per node, one log per edge and
// one solid angle per face of the chunk for every target.
// ---------------------------------------------------------------------------
// One wavefront takes kTopoChunksPerWave chunks, 16 lanes (one per tet) each.
constexpr int kTopoChunksPerWave = 4;
static_assert(kTopoTets <= 64 / kTopoChunksPerWave, "one lane per tet of a chunk");

__global__ __launch_bounds__(64) void k_topo_coef(const int32_t *__restrict__ ch_i, const double *__restrict__ ch_c,
                                                  int nch, const int32_t *__restrict__ inc,
                                                  const double *__restrict__ tet_xyz,
                                                  const int32_t *__restrict__ tet_node, int64_t T,
                                                  const double *__restrict__ M, double *__restrict__ A,
                                                  double *__restrict__ Bc)
{
    constexpr int LPC = 64 / kTopoChunksPerWave;  // lanes per chunk
    __shared__ double s_Aw[kTopoChunksPerWave][kTopoFaces][4];
    __shared__ double s_Bw[kTopoChunksPerWave][kTopoEdges][11];
    const int sub = (int)threadIdx.x / LPC, tl = (int)threadIdx.x % LPC;
    const int ch = (int)blockIdx.x * kTopoChunksPerWave + sub;
    const bool live = ch < nch;
    const int chl = live ? ch : nch - 1;  // clamped: reads stay in bounds, nothing is written
    const int tb = ch_i[8 * chl], nt = live ? ch_i[8 * chl + 1] : 0, eoff = ch_i[8 * chl + 4],
              ne = ch_i[8 * chl + 5], foff = ch_i[8 * chl + 6], nf = ch_i[8 * chl + 7];
    const double c[3] = {ch_c[3 * chl], ch_c[3 * chl + 1], ch_c[3 * chl + 2]};
    double (*s_A)[4] = s_Aw[sub];
    double (*s_B)[11] = s_Bw[sub];
    for (int i = threadIdx.x; i < kTopoChunksPerWave * kTopoFaces * 4; i += blockDim.x) (&s_Aw[0][0][0])[i] = 0.0;
    for (int i = threadIdx.x; i < kTopoChunksPerWave * kTopoEdges * 11; i += blockDim.x) (&s_Bw[0][0][0])[i] = 0.0;
    __syncthreads();
    if (tl < nt) {
        const int64_t t = tb + tl;
        TetGeom G;
        TetField Fd;
        tet_prepare(tet_xyz, tet_node, T, t, M, &G, Fd);
        double w[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k) w[q][k] = G.v[q][k] - c[k];
        const int32_t *ti = inc + 10 * t;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double *n = G.n[k];
            const int a = kFv[k][0];
            // alpha_k(y) = a0 + a1 . y
            const double a1[3] = {Fd.b[k][0] - Fd.c[k] * n[0], Fd.b[k][1] - Fd.c[k] * n[1], Fd.b[k][2] - Fd.c[k] * n[2]};
            const double a0 = Fd.a[k] - (w[0][0] * Fd.b[k][0] + w[0][1] * Fd.b[k][1] + w[0][2] * Fd.b[k][2]) +
                              Fd.c[k] * (n[0] * w[a][0] + n[1] * w[a][1] + n[2] * w[a][2]);
            double *Af = s_A[ti[6 + k]];
            atomicAdd(&Af[0], a0);
            atomicAdd(&Af[1], a1[0]);
            atomicAdd(&Af[2], a1[1]);
            atomicAdd(&Af[3], a1[2]);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int e = kFe[k][j];
                const double sg = kFs[k][j];
                const int ea = kEa[e], eb = kEb[e];
                // n . ((w_a - y) x (w_b - y)) = t0 + t1 . y
                const double cx[3] = {w[ea][1] * w[eb][2] - w[ea][2] * w[eb][1], w[ea][2] * w[eb][0] - w[ea][0] * w[eb][2],
                                      w[ea][0] * w[eb][1] - w[ea][1] * w[eb][0]};
                const double t0 = n[0] * cx[0] + n[1] * cx[1] + n[2] * cx[2];
                const double u[3] = {w[ea][0] - w[eb][0], w[ea][1] - w[eb][1], w[ea][2] - w[eb][2]};
                const double t1[3] = {u[1] * n[2] - u[2] * n[1], u[2] * n[0] - u[0] * n[2], u[0] * n[1] - u[1] * n[0]};
                double *Be = s_B[ti[e]];
                atomicAdd(&Be[0], sg * a0 * t0);
                atomicAdd(&Be[1], sg * (a0 * t1[0] + t0 * a1[0]));
                atomicAdd(&Be[2], sg * (a0 * t1[1] + t0 * a1[1]));
                atomicAdd(&Be[3], sg * (a0 * t1[2] + t0 * a1[2]));
                atomicAdd(&Be[4], sg * a1[0] * t1[0]);
                atomicAdd(&Be[5], sg * (a1[0] * t1[1] + a1[1] * t1[0]));
                atomicAdd(&Be[6], sg * (a1[0] * t1[2] + a1[2] * t1[0]));
                atomicAdd(&Be[7], sg * a1[1] * t1[1]);
                atomicAdd(&Be[8], sg * (a1[1] * t1[2] + a1[2] * t1[1]));
                atomicAdd(&Be[9], sg * a1[2] * t1[2]);
            }
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) atomicAdd(&s_B[ti[e]][10], Fd.g[e]);
    }
    __syncthreads();
    if (!live) return;
    for (int i = tl; i < nf * 4; i += LPC) A[(int64_t)foff * 4 + i] = (&s_A[0][0])[i];
    for (int i = tl; i < ne * 11; i += LPC) Bc[(int64_t)eoff * 11 + i] = (&s_B[0][0])[i];
}

// NT = 64: one wavefront per workgroup; NT = 256: four wavefronts share the
// staged chunk (less LDS per wavefront).  The 256-thread form asks for 4
// workgroups per CU but its 41 KB of LDS admits 3 (3 waves per SIMD); the
// register allocation under that request gives the tightest entity loops
// (asking for 3 lets it take 144 VGPRs, and the edge and face loops grow by
// 7 and 9 instructions).
template <int NT>
__global__ __launch_bounds__(NT, NT == 64 ? 2 : 4) void k_p2p_topo(const int32_t *__restrict__ blk, int nblk,
                                                    const int32_t *__restrict__ ch_i, const double *__restrict__ ch_c,
                                                    const double *__restrict__ nw, const int32_t *__restrict__ eab,
                                                    const double *__restrict__ eil, const int32_t *__restrict__ fpqr,
                                                    const double *__restrict__ fn, const double *__restrict__ fa2,
                                                    const double *__restrict__ A,
                                                    const double *__restrict__ Bc, const int32_t *__restrict__ idx,
                                                    const double *__restrict__ tgt_xyz,
                                                    const int32_t *__restrict__ tgt_perm, int64_t N,
                                                    double *__restrict__ u)
{
    __shared__ double s_w[kTopoNodes][4];  // rows of 4: node offsets are shifts, not multiplies
    __shared__ double s_R[kTopoNodes][NT];
    __shared__ int s_ea[kTopoEdges], s_eb[kTopoEdges];
    __shared__ double s_il[kTopoEdges], s_B[kTopoEdges][11];
    __shared__ int s_fp[kTopoFaces], s_fq[kTopoFaces], s_fr[kTopoFaces];
    __shared__ double s_fn[kTopoFaces][3], s_fa[kTopoFaces], s_A[kTopoFaces][4];
    const int b = xcd_item(nblk);
    if (b < 0) return;
    const int cb = blk[4 * b], ce = blk[4 * b + 1], ib = blk[4 * b + 2], ie = blk[4 * b + 3];
    const int lane = threadIdx.x;
    for (int ch = cb; ch < ce; ++ch) {
        const int noff = ch_i[8 * ch + 2], nn = ch_i[8 * ch + 3], eoff = ch_i[8 * ch + 4], ne = ch_i[8 * ch + 5],
                  foff = ch_i[8 * ch + 6], nf = ch_i[8 * ch + 7];
        const double c[3] = {ch_c[3 * ch], ch_c[3 * ch + 1], ch_c[3 * ch + 2]};
        __syncthreads();
        for (int i = lane; i < nn * 3; i += NT) s_w[i / 3][i % 3] = nw[(int64_t)noff * 3 + i];
        for (int i = lane; i < ne; i += NT) {
            s_ea[i] = eab[2 * ((int64_t)eoff + i)];
            s_eb[i] = eab[2 * ((int64_t)eoff + i) + 1];
            s_il[i] = eil[eoff + i];
        }
        for (int i = lane; i < ne * 11; i += NT) (&s_B[0][0])[i] = Bc[(int64_t)eoff * 11 + i];
        for (int i = lane; i < nf; i += NT) {
            s_fp[i] = fpqr[3 * ((int64_t)foff + i)];
            s_fq[i] = fpqr[3 * ((int64_t)foff + i) + 1];
            s_fr[i] = fpqr[3 * ((int64_t)foff + i) + 2];
        }
        for (int i = lane; i < nf * 3; i += NT) (&s_fn[0][0])[i] = fn[(int64_t)foff * 3 + i];
        for (int i = lane; i < nf; i += NT) s_fa[i] = fa2[foff + i];
        for (int i = lane; i < nf * 4; i += NT) (&s_A[0][0])[i] = A[(int64_t)foff * 4 + i];
        __syncthreads();
        for (int i = ib + lane; i < ie; i += NT) {
            const int s = idx[i];
            const double y[3] = {tgt_xyz[s] - c[0], tgt_xyz[N + s] - c[1], tgt_xyz[2 * N + s] - c[2]};
            const double m[10] = {1.0,         y[0],        y[1],        y[2],        y[0] * y[0],
                                  y[0] * y[1], y[0] * y[2], y[1] * y[1], y[1] * y[2], y[2] * y[2]};
#pragma unroll 1
            for (int j = 0; j < nn; ++j) {
                const double d0 = s_w[j][0] - y[0], d1 = s_w[j][1] - y[1], d2 = s_w[j][2] - y[2];
                s_R[j][lane] = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
            }
            double acc = 0.0;
#pragma unroll 1
            for (int e = 0; e < ne; ++e) {
                const int a = s_ea[e], bb = s_eb[e];
                const double il = s_il[e];
                const double da[3] = {s_w[a][0] - y[0], s_w[a][1] - y[1], s_w[a][2] - y[2]};
                const double db[3] = {s_w[bb][0] - y[0], s_w[bb][1] - y[1], s_w[bb][2] - y[2]};
                const double Ra = s_R[a][lane], Rb = s_R[bb][lane];
                const double Dab = da[0] * db[0] + da[1] * db[1] + da[2] * db[2];
                const double la = fma(-Ra, Ra, Dab) * il;  // (v_a - x) . e_hat
                const double lb = fma(Rb, Rb, -Dab) * il;  // (v_b - x) . e_hat
                const double cx0 = da[1] * db[2] - da[2] * db[1], cx1 = da[2] * db[0] - da[0] * db[2],
                             cx2 = da[0] * db[1] - da[1] * db[0];
                const double r0sq = (cx0 * cx0 + cx1 * cx1 + cx2 * cx2) * (il * il);
                const double f = edge_log<false>(Ra, Rb, la, lb, r0sq);
                const double g = r0sq * f + lb * Rb - la * Ra;
                const double *Be = s_B[e];
                double bq = Be[0];
#pragma unroll
                for (int q = 1; q < 10; ++q) bq = fma(Be[q], m[q], bq);
                acc = fma(f * il, bq, fma(Be[10], g, acc));
            }
#pragma unroll 1
            for (int fi = 0; fi < nf; ++fi) {
                const int pp = s_fp[fi], qq = s_fq[fi], rr = s_fr[fi];
                const double dp[3] = {s_w[pp][0] - y[0], s_w[pp][1] - y[1], s_w[pp][2] - y[2]};
                const double dq[3] = {s_w[qq][0] - y[0], s_w[qq][1] - y[1], s_w[qq][2] - y[2]};
                const double dr[3] = {s_w[rr][0] - y[0], s_w[rr][1] - y[1], s_w[rr][2] - y[2]};
                const double Rp = s_R[pp][lane], Rq = s_R[qq][lane], Rr = s_R[rr][lane];
                const double Dpq = dp[0] * dq[0] + dp[1] * dq[1] + dp[2] * dq[2];
                const double Dpr = dp[0] * dr[0] + dp[1] * dr[1] + dp[2] * dr[2];
                const double Dqr = dq[0] * dr[0] + dq[1] * dr[1] + dq[2] * dr[2];
                const double den = Rp * Rq * Rr + Dpq * Rr + Dpr * Rq + Dqr * Rp;
                const double h = s_fn[fi][0] * dp[0] + s_fn[fi][1] * dp[1] + s_fn[fi][2] * dp[2];
                // [d_p, d_q, d_r] = d_p . ((q - p) x (r - p)) = h |(q - p) x (r - p)|
                const double det = h * s_fa[fi];
                const double af = s_A[fi][0] + (s_A[fi][1] * y[0] + s_A[fi][2] * y[1] + s_A[fi][3] * y[2]);
                acc = fma(-af * h, 2.0 * atan2_nr(det, den), acc);
            }
            atomicAdd(&u[tgt_perm[s]], acc * kInv4Pi);
        }
    }
}

// ---------------------------------------------------------------------------
// Stored near-field operator (Sec. 2.1: the direct part is linear in the
// nodal magnetisation, so its node-to-node coefficients can be kept for a
// fixed mesh).  u_T(x) = sum_{corners c, axes j} C_{T,c,j}(x) M_{node(T,c), j}
// where C_{T,c,j}(x) is the potential of the field that is the unit vector e_j
// at corner c and zero at the other corners.  k_near_assemble evaluates the
// pair formula for these 12 unit fields (staged in LDS like the fields of
// k_p2p) for every near (target, tet) pair and adds the coefficients into the
// target's row of its leaf block [nt][3][ncols]; the column of a node is found
// by binary search in the leaf's sorted column list.
// ---------------------------------------------------------------------------
constexpr int kNearAsmTets = 16, kNearAsmThreads = 256;

__global__ __launch_bounds__(kNearAsmThreads) void k_near_assemble(
    const int32_t *__restrict__ blk, int nblk, int64_t T, const double *__restrict__ tet_xyz,
    const int32_t *__restrict__ tet_node, const int32_t *__restrict__ idx, const double *__restrict__ tgt_xyz,
    int64_t N, const int32_t *__restrict__ tgt_leaf, const int32_t *__restrict__ cell_i,
    const int64_t *__restrict__ near_off, const int32_t *__restrict__ near_nc, const int32_t *__restrict__ near_cols,
    double *__restrict__ val)
{
    __shared__ TetGeom s_g[kNearAsmTets];
    __shared__ TetField s_f[kNearAsmTets][12];
    __shared__ int32_t s_n[kNearAsmTets][4];
    const int b = xcd_item(nblk);
    if (b < 0) return;
    const int tb = blk[4 * b], te = blk[4 * b + 1], ib = blk[4 * b + 2], ie = blk[4 * b + 3];
    const int lane = threadIdx.x;
    for (int sb = tb; sb < te; sb += kNearAsmTets) {
        const int nt = min(kNearAsmTets, te - sb);
        __syncthreads();
        {
            const int t = lane / 12, f = lane % 12;
            if (t < nt) {
                TetGeom G;
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int k = 0; k < 3; ++k) G.v[c][k] = tet_xyz[(int64_t)(3 * c + k) * T + sb + t];
                double gl[4][3], eh[6][3];
                tet_geometry(G, gl, eh);
                double m[4][3];
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int k = 0; k < 3; ++k) m[c][k] = (3 * c + k == f) ? 1.0 : 0.0;
                tet_field(G, gl, eh, m, s_f[t][f]);
                if (f == 0) {
                    s_g[t] = G;
#pragma unroll
                    for (int c = 0; c < 4; ++c) s_n[t][c] = tet_node[(int64_t)c * T + sb + t];
                }
            }
        }
        __syncthreads();
        for (int i = ib + lane; i < ie; i += kNearAsmThreads) {
            const int s = idx[i];
            const double x[3] = {tgt_xyz[s], tgt_xyz[N + s], tgt_xyz[2 * N + s]};
            const int32_t a = tgt_leaf[s];
            const int64_t voff = near_off[2 * a + 1];
            if (voff < 0) continue;
            const int nc = near_nc[a];
            const int32_t *cl = near_cols + near_off[2 * a];
            double *row = val + voff + (int64_t)(s - cell_i[8 * a + 2]) * 3 * nc;
#pragma unroll 1
            for (int t = 0; t < nt; ++t) {
                PairGeo P;
                pair_geometry(x, s_g[t], P);
#pragma unroll 1
                for (int c = 0; c < 4; ++c) {
                    const int32_t node = s_n[t][c];
                    int lo = 0, hi = nc;  // first column >= node
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (cl[mid] < node) lo = mid + 1; else hi = mid;
                    }
                    if (lo >= nc || cl[lo] != node) continue;
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        atomicAdd(&row[(int64_t)j * nc + lo], pair_contract(P, s_f[t][3 * c + j]) * kInv4Pi);
                }
            }
        }
    }
}

// Applies the stored operator.  Work item = up to kNearRows consecutive target
// rows of one leaf (they share the leaf's column list): one wavefront per
// item, lanes striding the columns; per column the node's M is gathered once
// for FC fields and applied to every row of the item (three coalesced
// coefficient streams per row).  Row sums are reduced across the wavefront
// and added into u (L2P adds concurrently).
constexpr int kNearRows = 4, kNearItemsPerBlock = 4;

template <int FC>
__global__ __launch_bounds__(64 * kNearItemsPerBlock) void k_near_apply(
    int nitems, const int32_t *__restrict__ items, const int32_t *__restrict__ cell_i,
    const int64_t *__restrict__ near_off, const int32_t *__restrict__ near_nc, const int32_t *__restrict__ near_cols,
    const double *__restrict__ val, const int32_t *__restrict__ tgt_perm, int64_t N, const double *__restrict__ M,
    int64_t n_nodes, int F, double *__restrict__ u)
{
    const int blk = xcd_item((nitems + kNearItemsPerBlock - 1) / kNearItemsPerBlock);
    if (blk < 0) return;
    const int lane = threadIdx.x & 63;
    // one item per wavefront, its index made visibly uniform (the item's
    // bounds, column list and rows are then read on the scalar path)
    const int it = blk * kNearItemsPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (it >= nitems) return;
    const int32_t a = items[2 * it], r0 = items[2 * it + 1];
    const int xb = cell_i[8 * a + 2];
    const int nr = min(kNearRows, cell_i[8 * a + 3] - xb - r0);
    const int64_t voff = near_off[2 * a + 1];
    const int nc = near_nc[a];
    const int32_t *cl = near_cols + near_off[2 * a];
    const double *row = val + voff + (int64_t)r0 * 3 * nc;
    const int f0 = blockIdx.y * FC;
    double acc[kNearRows][FC];
#pragma unroll
    for (int r = 0; r < kNearRows; ++r)
#pragma unroll
        for (int f = 0; f < FC; ++f) acc[r][f] = 0.0;
    for (int c = lane; c < nc; c += 64) {
        const int64_t n = cl[c];
        double w[kNearRows][3];
#pragma unroll
        for (int r = 0; r < kNearRows; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) w[r][k] = r < nr ? row[((int64_t)r * 3 + k) * nc + c] : 0.0;
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            if (f0 + f < F) {
                const double *m = M + ((int64_t)(f0 + f) * n_nodes + n) * 3;
                const double m0 = m[0], m1 = m[1], m2 = m[2];
#pragma unroll
                for (int r = 0; r < kNearRows; ++r)
                    acc[r][f] = fma(w[r][0], m0, fma(w[r][1], m1, fma(w[r][2], m2, acc[r][f])));
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kNearRows; ++r)
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            double v = acc[r][f];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && r < nr && f0 + f < F) atomicAdd(&u[(int64_t)(f0 + f) * N + tgt_perm[xb + r0 + r]], v);
        }
}

// ---------------------------------------------------------------------------
// Demagnetising field and energy from nodal potentials (P1 interpolation):
// per tet H_T = -grad u = -sum_i u_i grad lambda_i, and
//   E / mu0 = 1/2 sum_T int_T M . grad u = 1/2 sum_T V_T (mean_i M_i) . grad u_T
// (M affine on the tet).  One thread per tet (octree order); the block sums
// are added in a fixed order by k_sum_blocks.
// ---------------------------------------------------------------------------
constexpr int kEnergyThreads = 256;

// grad u of the P1 interpolant on tet t (octree order) of the nodal values u,
// with its corner node ids, 6|V| and the mean nodal M (when M is not null).
__device__ inline void p1_gradient(const double *__restrict__ tet_xyz, const int32_t *__restrict__ tet_node, int64_t T,
                                   int64_t t, const double *__restrict__ u, const double *__restrict__ M,
                                   double gu[3], int64_t nd[4], double &vol6, double mbar[3])
{
    double v[4][3], uc[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) mbar[k] = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        nd[c] = tet_node[(int64_t)c * T + t];
        uc[c] = u[nd[c]];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[c][k] = tet_xyz[(int64_t)(3 * c + k) * T + t];
            if (M) mbar[k] += 0.25 * M[3 * nd[c] + k];
        }
    }
    double e1[3], e2[3], e3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e1[k] = v[1][k] - v[0][k];
        e2[k] = v[2][k] - v[0][k];
        e3[k] = v[3][k] - v[0][k];
    }
    // grad u = (u1-u0) g1 + (u2-u0) g2 + (u3-u0) g3, g_i = rows of the inverse Jacobian
    double g1[3], g2[3], g3[3];
    g1[0] = e2[1] * e3[2] - e2[2] * e3[1];
    g1[1] = e2[2] * e3[0] - e2[0] * e3[2];
    g1[2] = e2[0] * e3[1] - e2[1] * e3[0];
    g2[0] = e3[1] * e1[2] - e3[2] * e1[1];
    g2[1] = e3[2] * e1[0] - e3[0] * e1[2];
    g2[2] = e3[0] * e1[1] - e3[1] * e1[0];
    g3[0] = e1[1] * e2[2] - e1[2] * e2[1];
    g3[1] = e1[2] * e2[0] - e1[0] * e2[2];
    g3[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double det = e1[0] * g1[0] + e1[1] * g1[1] + e1[2] * g1[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) gu[k] = ((uc[1] - uc[0]) * g1[k] + (uc[2] - uc[0]) * g2[k] + (uc[3] - uc[0]) * g3[k]) / det;
    vol6 = fabs(det);
}

__global__ __launch_bounds__(kEnergyThreads) void k_demag(const double *__restrict__ tet_xyz,
                                                          const int32_t *__restrict__ tet_node,
                                                          const int32_t *__restrict__ tet_perm, int64_t T,
                                                          const double *__restrict__ M, const double *__restrict__ u,
                                                          double *__restrict__ H, double *__restrict__ part)
{
    __shared__ double s_e[kEnergyThreads];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (t < T) {
        double gu[3], vol6, mbar[3];
        int64_t nd[4];
        p1_gradient(tet_xyz, tet_node, T, t, u, M, gu, nd, vol6, mbar);
        e = 0.5 * (vol6 / 6.0) * (mbar[0] * gu[0] + mbar[1] * gu[1] + mbar[2] * gu[2]);
        if (H) {
            const int64_t o = tet_perm[t];
#pragma unroll
            for (int k = 0; k < 3; ++k) H[3 * o + k] = -gu[k];
        }
    }
    s_e[threadIdx.x] = e;
    __syncthreads();
    for (int w = kEnergyThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_e[threadIdx.x] += s_e[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_e[0];
}

// Mass-lumped nodal field (the lumped L2 projection of the P1 field onto the
// nodes): H_j = sum_{T ni j} (V_T / 4) H_T / w_j, w_j = sum_{T ni j} V_T / 4.
// k_demag_scatter adds (V_T / 4) H_T of every tet to its corners (and, when w
// is not null, V_T / 4 to the weights); k_lump_divide divides by w.
__global__ __launch_bounds__(kEnergyThreads) void k_demag_scatter(const double *__restrict__ tet_xyz,
                                                                  const int32_t *__restrict__ tet_node, int64_t T,
                                                                  const double *__restrict__ u, double *__restrict__ Hn,
                                                                  double *__restrict__ w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double gu[3], vol6, mbar[3];
    int64_t nd[4];
    p1_gradient(tet_xyz, tet_node, T, t, u, nullptr, gu, nd, vol6, mbar);
    const double q = vol6 / 24.0;  // V_T / 4
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int k = 0; k < 3; ++k) atomicAdd(&Hn[3 * nd[c] + k], -q * gu[k]);
        if (w) atomicAdd(&w[nd[c]], q);
    }
}

__global__ void k_lump_divide(double *__restrict__ Hn, const double *__restrict__ w, int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double wj = w[j];
    const double r = wj > 0.0 ? 1.0 / wj : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) Hn[3 * j + k] *= r;
}

__global__ __launch_bounds__(kEnergyThreads) void k_sum_blocks(const double *__restrict__ part, int n,
                                                               double *__restrict__ out)
{
    __shared__ double s_e[kEnergyThreads];
    double e = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) e += part[i];
    s_e[threadIdx.x] = e;
    __syncthreads();
    for (int w = kEnergyThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_e[threadIdx.x] += s_e[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s_e[0];
}

// ---------------------------------------------------------------------------
// The near field's own elementary functions, one call per element (for
// checking them against an independent implementation).
// ---------------------------------------------------------------------------
__global__ void k_elementary(int fn, const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                             double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = a[i], y = b[i];
    double r;
    switch (fn) {
    case 0: r = log_ratio(x, y); break;
    case 1: r = atan2_nr(x, y); break;
    case 2: r = div_nr(x, y); break;
    default: r = rsqrt_nr(x); break;
    }
    out[i] = r;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
std::vector<int32_t> xcd_dispatch_items(int n)
{
    std::vector<int32_t> out;
    out.reserve(n > 0 ? n : 0);
    const int per = (n + kXcds - 1) / kXcds;
    for (int w = 0; w < kXcds * per; ++w) {
        const int item = (w % kXcds) * per + w / kXcds;
        if (item < n) out.push_back(item);
    }
    return out;
}

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw DeviceError{std::string(what) + ": " + hipGetErrorString(e)};
}

namespace {

// Calls fn with std::integral_constant<int, field_chunk(F)>.
// Calls fn with std::integral_constant<int, p> for 1 <= p <= kPmax.
template <class Fn>
void with_order(int p, Fn &&fn)
{
    switch (p) {
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    case 3: fn(std::integral_constant<int, 3>{}); break;
    case 4: fn(std::integral_constant<int, 4>{}); break;
    case 5: fn(std::integral_constant<int, 5>{}); break;
    case 6: fn(std::integral_constant<int, 6>{}); break;
    case 7: fn(std::integral_constant<int, 7>{}); break;
    case 8: fn(std::integral_constant<int, 8>{}); break;
    case 9: fn(std::integral_constant<int, 9>{}); break;
    default: fn(std::integral_constant<int, 10>{}); break;
    }
}

template <class Fn>
void launch_fc(int F, Fn &&fn)
{
    switch (field_chunk(F)) {
    case 16: fn(std::integral_constant<int, 16>{}); break;
    case 4: fn(std::integral_constant<int, 4>{}); break;
    default: fn(std::integral_constant<int, 1>{}); break;
    }
}

hipEvent_t pool_event(DevicePlan &dp)
{
    if (dp.events_used == dp.event_pool.size()) {
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "hipEventCreate");
        dp.event_pool.push_back(e);
    }
    return dp.event_pool[dp.events_used++];
}

// Records an event pair around one phase on the evaluation stream; nothing is
// synchronised here.
struct KTimer {
    DevicePlan &dp;
    int slot;
    hipStream_t st;
    hipEvent_t a = nullptr;
    KTimer(DevicePlan &d, int s, hipStream_t stream) : dp(d), slot(s), st(stream)
    {
        if (!dp.timing) return;
        if (dp.spans.size() >= 4096) collect_timing(dp);
        a = pool_event(dp);
        hip_check(hipEventRecord(a, st), "hipEventRecord");
    }
    ~KTimer() noexcept(false)
    {
        if (!dp.timing) return;
        hipEvent_t b = pool_event(dp);
        hip_check(hipEventRecord(b, st), "hipEventRecord");
        dp.spans.push_back({slot, a, b});
    }
};

// Ragged batches evaluated as one merged plan: mesh i's nodal M (device
// [n_i][3]) times scale[i] into rows off[i] .. off[i+1] of the merged M, and
// the merged u back into each mesh's u (device [n_i]).
__device__ __forceinline__ int batch_mesh(const int64_t *__restrict__ off, int n, int64_t j)
{
    int lo = 0, hi = n;  // last i with off[i] <= j
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}
__global__ void k_batch_gather(const double *const *__restrict__ M, const int64_t *__restrict__ off,
                               const double *__restrict__ scale, int n, double *__restrict__ out)
{
    const int64_t N = off[n];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        const int i = batch_mesh(off, n, j);
        const double *m = M[i] + 3 * (j - off[i]);
        const double s = scale[i];
        out[3 * j] = s * m[0];
        out[3 * j + 1] = s * m[1];
        out[3 * j + 2] = s * m[2];
    }
}
__global__ void k_batch_scatter(const double *__restrict__ u, const int64_t *__restrict__ off, int n,
                                double *const *__restrict__ U)
{
    const int64_t N = off[n];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        const int i = batch_mesh(off, n, j);
        U[i][j - off[i]] = u[j];
    }
}
void fill(double *a, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    k_fill<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(a, n, v);
    hip_check(hipGetLastError(), "k_fill launch");
}

template <int FCH, bool WIDE>
void launch_p2p_w(DevicePlan &dp, bool band_skip, int f0, const double *M, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const unsigned nblk = (unsigned)dp.n_p2p_blk;
    if (nblk == 0) return;
    k_p2p<FCH, WIDE><<<dim3(xcd_grid((int)nblk)), dim3(p2p_threads(FCH, WIDE)), 0, st>>>(
        dp.p2p_blk, (int)nblk, band_skip ? 1 : 0, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx, dp.tgt_xyz,
        dp.tgt_perm, hp.n_targets, M, hp.n_nodes, f0, u);
    hip_check(hipGetLastError(), "k_p2p launch");
}

template <int FCH>
void launch_p2p(DevicePlan &dp, bool band_skip, int f0, const double *M, double *u, hipStream_t st)
{
    if constexpr (FCH <= 2) {
        if (dp.p2p_wide) {
            launch_p2p_w<FCH, true>(dp, band_skip, f0, M, u, st);
            return;
        }
    }
    launch_p2p_w<FCH, false>(dp, band_skip, f0, M, u, st);
}

void run_p2p_points(DevicePlan &dp, bool direct, const double *M, int32_t F, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const unsigned nblk = direct ? (unsigned)((hp.n_tets + kP2PTets - 1) / kP2PTets) : (unsigned)dp.n_p2p_blk;
    if (nblk == 0) return;
    for (int f = 0; f < F;) {
        const int left = F - f;
#define TFMM_P2P_POINTS(FCV)                                                                                       \
    k_p2p_points<FCV><<<dim3(xcd_grid((int)nblk)), dim3(kPtThreads), 0, st>>>(                                      \
        dp.p2p_blk, (int)nblk, direct ? 1 : 0, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx, dp.tgt_xyz,            \
        dp.tgt_perm, hp.n_targets, M, hp.n_nodes, f, u)
        if (left >= 8) {
            TFMM_P2P_POINTS(8);
            f += 8;
        } else if (left >= 4) {
            TFMM_P2P_POINTS(4);
            f += 4;
        } else if (left >= 2) {
            TFMM_P2P_POINTS(2);
            f += 2;
        } else {
            TFMM_P2P_POINTS(1);
            f += 1;
        }
#undef TFMM_P2P_POINTS
        hip_check(hipGetLastError(), "k_p2p_points launch");
    }
}

// Near field by the pair integrals: point dipoles (or, direct, the dipole
// sum); one field of tets over the shared mesh entities; otherwise the
// per-tet kernel, without the band's pairs when band_skip.
void run_p2p(DevicePlan &dp, bool direct, const double *M, int32_t F, double *u, hipStream_t st, bool band_skip = false)
{
    if (dp.hp.points) {
        run_p2p_points(dp, direct, M, F, u, st);
        return;
    }
    if (direct) throw DeviceError{"the tet direct sum runs in k_direct"};
    if (!band_skip && F == 1 && dp.p2p_topo && dp.n_topo_ch > 0) {
        const HostPlan &hp = dp.hp;
        k_topo_coef<<<dim3((unsigned)((dp.n_topo_ch + kTopoChunksPerWave - 1) / kTopoChunksPerWave)), dim3(64), 0, st>>>(dp.topo_ch_i, dp.topo_ch_c, dp.n_topo_ch, dp.topo_inc,
                                                             dp.tet_xyz, dp.tet_node, hp.n_tets, M, dp.topo_A,
                                                             dp.topo_B);
        hip_check(hipGetLastError(), "k_topo_coef launch");
        const int nblk = dp.n_p2p_blk;
        if (dp.p2p_wide)
            k_p2p_topo<256><<<dim3(xcd_grid(nblk)), dim3(256), 0, st>>>(
                dp.topo_blk, nblk, dp.topo_ch_i, dp.topo_ch_c, dp.topo_w, dp.topo_ab, dp.topo_il, dp.topo_pqr,
                dp.topo_n, dp.topo_a2, dp.topo_A, dp.topo_B, dp.p2p_idx, dp.tgt_xyz, dp.tgt_perm, hp.n_targets, u);
        else
            k_p2p_topo<64><<<dim3(xcd_grid(nblk)), dim3(64), 0, st>>>(
                dp.topo_blk, nblk, dp.topo_ch_i, dp.topo_ch_c, dp.topo_w, dp.topo_ab, dp.topo_il, dp.topo_pqr,
                dp.topo_n, dp.topo_a2, dp.topo_A, dp.topo_B, dp.p2p_idx, dp.tgt_xyz, dp.tgt_perm, hp.n_targets, u);
        hip_check(hipGetLastError(), "k_p2p_topo launch");
        return;
    }
    int f = 0;
    while (f < F) {
        const int left = F - f;
        if (left >= 32) {
            launch_p2p<32>(dp, band_skip, f, M, u, st);
            f += 32;
        } else if (left >= 16) {
            launch_p2p<16>(dp, band_skip, f, M, u, st);
            f += 16;
        } else if (left >= 8) {
            launch_p2p<8>(dp, band_skip, f, M, u, st);
            f += 8;
        } else if (left >= 4) {
            launch_p2p<4>(dp, band_skip, f, M, u, st);
            f += 4;
        } else if (left >= 2) {
            launch_p2p<2>(dp, band_skip, f, M, u, st);
            f += 2;
        } else {
            launch_p2p<1>(dp, band_skip, f, M, u, st);
            f += 1;
        }
    }
}

// Near field from the stored operator (F fields, FC per pass).
void run_near_stored(DevicePlan &dp, const double *M, int32_t F, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const int64_t N = hp.n_targets;
    if (N == 0 || dp.near_nvals == 0) return;
    const int ni = dp.near_nitems;
    if (ni == 0) return;
    const int nblk = (ni + kNearItemsPerBlock - 1) / kNearItemsPerBlock;
    const int fc = F >= 8 ? 8 : (F >= 4 ? 4 : (F >= 2 ? 2 : 1));
    const dim3 grid(xcd_grid(nblk), (unsigned)((F + fc - 1) / fc));
    const dim3 thr(64 * kNearItemsPerBlock);
#define TFMM_NEAR_APPLY(FCV)                                                                                       \
    k_near_apply<FCV><<<grid, thr, 0, st>>>(ni, dp.near_items, dp.cell_i, dp.near_off, dp.near_nc, dp.near_cols,    \
                                            dp.near_val, dp.tgt_perm, N, M, hp.n_nodes, F, u)
    switch (fc) {
    case 8: TFMM_NEAR_APPLY(8); break;
    case 4: TFMM_NEAR_APPLY(4); break;
    case 2: TFMM_NEAR_APPLY(2); break;
    default: TFMM_NEAR_APPLY(1); break;
    }
#undef TFMM_NEAR_APPLY
    hip_check(hipGetLastError(), "k_near_apply launch");
}

// Near field of an evaluation: the stored operator when the plan holds one;
// with the surrogate switched on, the exact integrals outside the band and
// the band's pairs by the network (or a control); else the pair integrals.
void run_near(DevicePlan &dp, const double *M, int32_t F, double *u, hipStream_t st)
{
    if (dp.near_stored) {
        run_near_stored(dp, M, F, u, st);
    } else if (dp.sur_mode != TFMM_SUR_OFF && !dp.hp.points) {
        run_p2p(dp, false, M, F, u, st, true);
        run_band_pairs(dp, dp.sur_mode, M, F, u, st);
    } else {
        run_p2p(dp, false, M, F, u, st);
    }
}

template <typename T, int P>
void launch_m2l_p(DevicePlan &dp, const DevicePlan::Tiles &tl, const T *D, const T *Qt, int fpt, int32_t F,
                  hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const unsigned groups = (unsigned)((F + fpt - 1) / fpt);
    k_m2l_mfma<T, P><<<dim3(tl.ntiles, groups), dim3(64 * kM2LWaves), 0, st>>>(
        tl.tile_tgt, tl.tile_rng, tl.ent_key, tl.ent_src, dp.m2l_keys, D, Qt, dp.qpad, dp.cell_i, hp.side,
        (int64_t)hp.cells.size(), tl.tpt, fpt, F, tl.ntiles, m2l_table_width(hp.p), dp.ncoef, dp.L);
    hip_check(hipGetLastError(), "k_m2l_mfma launch");
}

template <int P, int NP>
void launch_m2lb_p(DevicePlan &dp, const DevicePlan::Tiles &tl, const float *D, const float *Qt, int fpt, int32_t F,
                   hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const unsigned groups = (unsigned)((F + fpt - 1) / fpt);
    k_m2l_bf16<P, NP><<<dim3(tl.ntiles, groups), dim3(64 * kM2LBWaves), 0, st>>>(
        tl.tile_tgt, tl.tile_rng, tl.ent_key, tl.ent_src, dp.m2l_keys, D, Qt, dp.qpad, dp.cell_i, hp.side,
        (int64_t)hp.cells.size(), tl.tpt, fpt, F, tl.ntiles, m2l_table_width(hp.p), dp.ncoef, dp.L);
    hip_check(hipGetLastError(), "k_m2l_bf16 launch");
}

// (p: the order of the translation, the plan's or a level's)
template <int NP>
void launch_m2lb_t(DevicePlan &dp, const DevicePlan::Tiles &tl, const float *D, const float *Qt, int fpt, int32_t F,
                   hipStream_t st, int p)
{
    switch (p) {
    case 1: launch_m2lb_p<1, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 2: launch_m2lb_p<2, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 3: launch_m2lb_p<3, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 4: launch_m2lb_p<4, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 5: launch_m2lb_p<5, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 6: launch_m2lb_p<6, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 7: launch_m2lb_p<7, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 8: launch_m2lb_p<8, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 9: launch_m2lb_p<9, NP>(dp, tl, D, Qt, fpt, F, st); break;
    case 10: launch_m2lb_p<10, NP>(dp, tl, D, Qt, fpt, F, st); break;
    default: throw DeviceError{"unsupported expansion order"};
    }
}

template <typename T>
void launch_m2l_t(DevicePlan &dp, const DevicePlan::Tiles &tl, const T *D, const T *Qt, int fpt, int32_t F,
                  hipStream_t st, int p)
{
    switch (p) {
    case 1: launch_m2l_p<T, 1>(dp, tl, D, Qt, fpt, F, st); break;
    case 2: launch_m2l_p<T, 2>(dp, tl, D, Qt, fpt, F, st); break;
    case 3: launch_m2l_p<T, 3>(dp, tl, D, Qt, fpt, F, st); break;
    case 4: launch_m2l_p<T, 4>(dp, tl, D, Qt, fpt, F, st); break;
    case 5: launch_m2l_p<T, 5>(dp, tl, D, Qt, fpt, F, st); break;
    case 6: launch_m2l_p<T, 6>(dp, tl, D, Qt, fpt, F, st); break;
    case 7: launch_m2l_p<T, 7>(dp, tl, D, Qt, fpt, F, st); break;
    case 8: launch_m2l_p<T, 8>(dp, tl, D, Qt, fpt, F, st); break;
    case 9: launch_m2l_p<T, 9>(dp, tl, D, Qt, fpt, F, st); break;
    case 10: launch_m2l_p<T, 10>(dp, tl, D, Qt, fpt, F, st); break;
    default: throw DeviceError{"unsupported expansion order"};
    }
}

template <typename T, int P>
void launch_m2l_pack_p(DevicePlan &dp, const DevicePlan::Packs &k, const T *D, const T *Qt, int fpt, int32_t F,
                       hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    if (k.nitems == 0) return;
    if (k.nb * fpt != m2lp_slots(P) || k.tpg * fpt != 16 || k.p != P)
        throw DeviceError{"M2L packs do not match the translation order"};
    const unsigned groups = (unsigned)((F + fpt - 1) / fpt);
    k_m2l_pack<T, P><<<dim3((unsigned)k.nitems, groups), dim3(64 * kM2LPWaves), 0, st>>>(
        k.item, k.nitems, k.blk_cells, k.nb, k.tpg, k.grp_key, k.grp_src, k.grp_slot, dp.m2l_keys, D,
        m2l_table_width(hp.p), Qt, dp.qpad, (int64_t)hp.cells.size(), fpt, F, dp.Lr, m2l_nrows(hp.p));
    hip_check(hipGetLastError(), "k_m2l_pack launch");
}

template <typename T>
void launch_m2l_pack_t(DevicePlan &dp, const DevicePlan::Packs &k, const T *D, const T *Qt, int fpt, int32_t F,
                       hipStream_t st, int p)
{
    switch (p) {
    case 1: launch_m2l_pack_p<T, 1>(dp, k, D, Qt, fpt, F, st); break;
    case 2: launch_m2l_pack_p<T, 2>(dp, k, D, Qt, fpt, F, st); break;
    case 3: launch_m2l_pack_p<T, 3>(dp, k, D, Qt, fpt, F, st); break;
    case 4: launch_m2l_pack_p<T, 4>(dp, k, D, Qt, fpt, F, st); break;
    case 5: launch_m2l_pack_p<T, 5>(dp, k, D, Qt, fpt, F, st); break;
    case 6: launch_m2l_pack_p<T, 6>(dp, k, D, Qt, fpt, F, st); break;
    case 7: launch_m2l_pack_p<T, 7>(dp, k, D, Qt, fpt, F, st); break;
    case 8: launch_m2l_pack_p<T, 8>(dp, k, D, Qt, fpt, F, st); break;
    case 9: launch_m2l_pack_p<T, 9>(dp, k, D, Qt, fpt, F, st); break;
    case 10: launch_m2l_pack_p<T, 10>(dp, k, D, Qt, fpt, F, st); break;
    default: throw DeviceError{"unsupported expansion order"};
    }
}

// Scaled multipoles, then the translations, in the plan's M2L precision.
// Field tile width of M2L for F fields: FPT fields x 16/FPT target cells.
int m2l_fpt(int32_t F)
{
    int fpt = 1;
    while (fpt * 2 <= std::min<int32_t>(F, 16)) fpt *= 2;
    return fpt;
}

// Whether M2L runs in the packed form: FP64 translations of fewer than 16
// fields (the tiles of 16 or more fields carry one target cell x 16 fields,
// every column used; the FP32 and split-BF16 tiles are faster than their
// packed forms, whose few matrix-core cycles per group leave the LDS
// accumulation as the bound).
bool m2l_packed(const DevicePlan &dp, int32_t F)
{
    return dp.m2l_pack && m2l_fpt(F) < 16 && dp.m2l_precision == TFMM_M2L_FP64;
}
int m2l_pack_slot(int fpt)
{
    int s = 0;
    while ((1 << s) < fpt) ++s;
    return s;
}

// The translations of one tile list at order p in the plan's M2L precision.
void launch_m2l_tiles(DevicePlan &dp, const DevicePlan::Tiles &tl, int fpt, int32_t F, hipStream_t st, int p)
{
    if (tl.ntiles == 0) return;
    if (dp.m2l_precision == TFMM_M2L_BF16X3)
        launch_m2lb_t<2>(dp, tl, dp.m2l_Df, dp.Qtf, fpt, F, st, p);
    else if (dp.m2l_precision == TFMM_M2L_BF16X6)
        launch_m2lb_t<3>(dp, tl, dp.m2l_Df, dp.Qtf, fpt, F, st, p);
    else if (dp.m2l_precision == TFMM_M2L_FP32)
        launch_m2l_t<float>(dp, tl, dp.m2l_Df, dp.Qtf, fpt, F, st, p);
    else
        launch_m2l_t<double>(dp, tl, dp.m2l_D, dp.Qt, fpt, F, st, p);
}

void run_m2l(DevicePlan &dp, int32_t F, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const int64_t C = (int64_t)hp.cells.size();
    const int fpt = m2l_fpt(F);
    if (hp.m2l_src.empty()) return;
    const int64_t nq = C * dp.qpad;
    const dim3 qgrid((unsigned)((nq + 255) / 256), F);
    if (dp.m2l_precision != TFMM_M2L_FP64) {  // FP32 operands (FP32, BF16x3, BF16x6)
        if (!dp.m2l_Df || dp.qtf_cap < F) throw DeviceError{"M2L buffers not prepared"};
        k_qreduce<float><<<qgrid, dim3(256), 0, st>>>(dp.Q, dp.cell_i, C, hp.side, hp.p, dp.qpad, dp.Qtf);
    } else {
        if (dp.qt_cap < F) throw DeviceError{"M2L buffers not prepared"};
        k_qreduce<double><<<qgrid, dim3(256), 0, st>>>(dp.Q, dp.cell_i, C, hp.side, hp.p, dp.qpad, dp.Qt);
    }
    hip_check(hipGetLastError(), "k_qreduce launch");
    if (m2l_packed(dp, F)) {
        if (dp.lr_cap < F) throw DeviceError{"M2L buffers not prepared"};
        const int lrs = m2l_nrows(hp.p);
        fill(dp.Lr, (int64_t)F * C * lrs, 0.0, st);
        auto go = [&](const DevicePlan::Packs &k, int p) {
            launch_m2l_pack_t<double>(dp, k, dp.m2l_D, dp.Qt, fpt, F, st, p);
        };
        if (!dp.level_orders) {
            go(dp.m2l_packs[m2l_pack_slot(fpt)], hp.p);
        } else {
            for (size_t lv = 0; lv < dp.lvl_packs.size(); ++lv) go(dp.lvl_packs[lv], dp.lo.q[lv]);
        }
        const int64_t n = C * dp.ncoef;
        k_lr_expand<<<dim3((unsigned)((n + 255) / 256), (unsigned)F), dim3(256), 0, st>>>(
            dp.Lr, lrs, dp.cell_i, hp.side, C, dp.ncoef, dp.lo, dp.L);
        hip_check(hipGetLastError(), "k_lr_expand launch");
        return;
    }
    if (!dp.level_orders) {
        launch_m2l_tiles(dp, ensure_m2l_tiles(dp, 16 / fpt), fpt, F, st, hp.p);
        return;
    }
    // per-level orders: one launch per target level at that level's order
    // (the source multipoles already hold no terms above their own level's)
    const std::vector<DevicePlan::Tiles> &lt = ensure_m2l_level_tiles(dp, 16 / fpt);
    for (size_t lv = 0; lv < lt.size(); ++lv) launch_m2l_tiles(dp, lt[lv], fpt, F, st, dp.lo.q[lv]);
}

}  // namespace

void batch_gather(const double *const *M, const int64_t *off, const double *scale, int n, int64_t N, double *out,
                  hipStream_t st)
{
    if (N <= 0) return;
    k_batch_gather<<<dim3((unsigned)std::min<int64_t>((N + 255) / 256, 65536)), dim3(256), 0, st>>>(M, off, scale, n,
                                                                                                   out);
    hip_check(hipGetLastError(), "k_batch_gather launch");
}
void batch_scatter(const double *u, const int64_t *off, int n, int64_t N, double *const *U, hipStream_t st)
{
    if (N <= 0) return;
    k_batch_scatter<<<dim3((unsigned)std::min<int64_t>((N + 255) / 256, 65536)), dim3(256), 0, st>>>(u, off, n, U);
    hip_check(hipGetLastError(), "k_batch_scatter launch");
}


void store_near(DevicePlan &dp, hipStream_t st)
{
    if (dp.near_stored) return;
    const HostPlan &hp = dp.hp;
    NearOpLayout lay;
    build_near_operator_layout(hp, lay);
    const size_t C = hp.cells.size();
    const size_t b_off = sizeof(int64_t) * 2 * std::max<size_t>(C, 1), b_nc = sizeof(int32_t) * std::max<size_t>(C, 1),
                 b_cols = sizeof(int32_t) * std::max<size_t>(lay.cols.size(), 1),
                 b_val = sizeof(double) * (size_t)std::max<int64_t>(lay.nvals, 1);
    // apply work items: (leaf, first row) per kNearRows rows of a leaf block
    std::vector<int32_t> items;
    for (size_t a = 0; a < C; ++a) {
        if (lay.leaf_off[2 * a + 1] < 0) continue;
        const Cell &K = hp.cells[a];
        for (int32_t r = 0; r < K.xend - K.xbeg; r += kNearRows) {
            items.push_back((int32_t)a);
            items.push_back(r);
        }
    }
    const size_t b_items = sizeof(int32_t) * std::max<size_t>(items.size(), 1);
    void *p[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    const size_t sz[5] = {b_off, b_nc, b_cols, b_val, b_items};
    for (int i = 0; i < 5; ++i) {
        const hipError_t e = hipMalloc(&p[i], sz[i]);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; ++j) (void)hipFree(p[j]);
            if (e == hipErrorOutOfMemory)
                throw PlanError{TFMM_ENOMEM, "stored near-field operator: device memory exhausted (" +
                                                 std::to_string(b_val >> 20) + " MiB of coefficients)"};
            hip_check(e, "hipMalloc near operator");
        }
    }
    dp.near_off = (int64_t *)p[0];
    dp.near_nc = (int32_t *)p[1];
    dp.near_cols = (int32_t *)p[2];
    dp.near_val = (double *)p[3];
    dp.near_items = (int32_t *)p[4];
    dp.near_nitems = (int32_t)(items.size() / 2);
    dp.near_nvals = lay.nvals;
    dp.near_ncols = (int64_t)lay.cols.size();
    dp.near_nnz = lay.nnz;
    dp.near_bytes = (int64_t)(b_off + b_nc + b_cols + b_val + b_items);
    dp.device_bytes += dp.near_bytes;
    try {
        if (!items.empty())
            hip_check(hipMemcpy(dp.near_items, items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice),
                      "hipMemcpy near items");
        hip_check(hipMemcpy(dp.near_off, lay.leaf_off.data(), sizeof(int64_t) * lay.leaf_off.size(), hipMemcpyHostToDevice),
                  "hipMemcpy near offsets");
        hip_check(hipMemcpy(dp.near_nc, lay.leaf_nc.data(), sizeof(int32_t) * lay.leaf_nc.size(), hipMemcpyHostToDevice),
                  "hipMemcpy near counts");
        if (!lay.cols.empty())
            hip_check(hipMemcpy(dp.near_cols, lay.cols.data(), sizeof(int32_t) * lay.cols.size(), hipMemcpyHostToDevice),
                      "hipMemcpy near columns");
        fill(dp.near_val, lay.nvals, 0.0, st);
        if (dp.n_p2p_blk > 0) {
            k_near_assemble<<<dim3(xcd_grid(dp.n_p2p_blk)), dim3(kNearAsmThreads), 0, st>>>(
                dp.p2p_blk, dp.n_p2p_blk, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx, dp.tgt_xyz, hp.n_targets,
                dp.tgt_leaf, dp.cell_i, dp.near_off, dp.near_nc, dp.near_cols, dp.near_val);
            hip_check(hipGetLastError(), "k_near_assemble launch");
        }
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize (near operator)");
    } catch (...) {
        drop_near(dp);  // a failed assembly leaves no operator behind
        throw;
    }
    dp.near_stored = true;
    ++dp.schedule_gen;
}

void drop_near(DevicePlan &dp)
{
    if (!dp.near_off) return;
    (void)hipDeviceSynchronize();  // also called on a failure path: freeing must not throw
    void *p[5] = {dp.near_off, dp.near_nc, dp.near_cols, dp.near_val, dp.near_items};
    for (void *q : p)
        if (q) (void)hipFree(q);
    dp.near_items = nullptr;
    dp.near_nitems = 0;
    dp.near_off = nullptr;
    dp.near_nc = nullptr;
    dp.near_cols = nullptr;
    dp.near_val = nullptr;
    dp.device_bytes -= dp.near_bytes;
    dp.near_bytes = dp.near_nvals = dp.near_ncols = dp.near_nnz = 0;
    dp.near_stored = false;
    ++dp.schedule_gen;
}

void build_tet_moments(DevicePlan &dp)
{
    if (dp.n_p2m_cells == 0) return;
    k_tet_moments<<<dim3(dp.n_p2m_cells), dim3(kMomThreads)>>>(dp.p2m_cells, dp.cell_i, dp.cell_c,
                                                               (int64_t)dp.hp.cells.size(), dp.tet_xyz, dp.hp.n_tets,
                                                               dp.quad, dp.nq, dp.hp.p, dp.hp.points ? 1 : 0,
                                                               dp.tet_mom);
    hip_check(hipGetLastError(), "k_tet_moments launch");
    hip_check(hipDeviceSynchronize(), "k_tet_moments");
}

void build_m2l_table(DevicePlan &dp)
{
    if (dp.n_m2l_keys == 0) return;
    k_m2l_table<<<dim3((dp.n_m2l_keys + 63) / 64), dim3(64)>>>(dp.m2l_keys, dp.n_m2l_keys, dp.hp.p, dp.m2l_D);
    hip_check(hipGetLastError(), "k_m2l_table launch");
    hip_check(hipDeviceSynchronize(), "k_m2l_table");
}

static void free_tiles(DevicePlan &dp, DevicePlan::Tiles &t)
{
    for (int32_t *q : {t.tile_tgt, t.tile_rng, t.ent_key, t.ent_src})
        if (q) (void)hipFree(q);
    dp.device_bytes -= t.bytes;
    t = DevicePlan::Tiles{};
}

static void upload_tiles(DevicePlan &dp, const M2LTiles &h, int tpt, DevicePlan::Tiles &t)
{
    auto up = [&](const std::vector<int32_t> &v, int32_t *&d) {
        const size_t b = sizeof(int32_t) * std::max<size_t>(v.size(), 1);
        hip_check(hipMalloc(&d, b), "hipMalloc M2L tiles");
        t.bytes += (int64_t)b;
        dp.device_bytes += (int64_t)b;
        if (!v.empty())
            hip_check(hipMemcpy(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice), "hipMemcpy M2L tiles");
    };
    up(h.tile_tgt, t.tile_tgt);
    up(h.tile_rng, t.tile_rng);
    up(h.ent_key, t.ent_key);
    up(h.ent_src, t.ent_src);
    t.ntiles = (int32_t)(h.tile_rng.size() / 2);
    t.nent = (int64_t)h.ent_key.size();
    t.tpt = tpt;
    t.max_ent = dp.m2l_max_ent;
}

DevicePlan::Tiles &ensure_m2l_tiles(DevicePlan &dp, int tpt)
{
    int slot = 0;
    while ((16 >> slot) != tpt && slot < 4) ++slot;
    if ((16 >> slot) != tpt) throw DeviceError{"bad M2L tile width"};
    DevicePlan::Tiles &t = dp.m2l_tiles[slot];
    if (t.tpt == tpt && t.max_ent == dp.m2l_max_ent) return t;
    // a captured graph may hold the old tile pointers
    ++dp.schedule_gen;
    free_tiles(dp, t);
    M2LTiles h;
    build_m2l_tiles(dp.hp, tpt, dp.m2l_max_ent, h);
    upload_tiles(dp, h, tpt, t);
    return t;
}

void drop_m2l_level_tiles(DevicePlan &dp)
{
    if (!dp.lvl_tiles.empty()) ++dp.schedule_gen;  // a captured graph may hold them
    for (auto &t : dp.lvl_tiles) free_tiles(dp, t);
    dp.lvl_tiles.clear();
}

const std::vector<DevicePlan::Tiles> &ensure_m2l_level_tiles(DevicePlan &dp, int tpt)
{
    if (!dp.lvl_tiles.empty() && dp.lvl_tiles[0].tpt == tpt && dp.lvl_tiles[0].max_ent == dp.m2l_max_ent)
        return dp.lvl_tiles;
    drop_m2l_level_tiles(dp);
    ++dp.schedule_gen;
    dp.lvl_tiles.resize((size_t)dp.hp.depth + 1);
    for (int lv = 0; lv <= dp.hp.depth; ++lv) {
        M2LTiles h;
        build_m2l_tiles(dp.hp, tpt, dp.m2l_max_ent, h, lv);
        upload_tiles(dp, h, tpt, dp.lvl_tiles[lv]);
    }
    return dp.lvl_tiles;
}

static void free_packs(DevicePlan &dp, DevicePlan::Packs &k)
{
    void *q[] = {k.blk_cells, k.item, k.grp_key, k.grp_src, k.grp_slot};
    for (void *x : q)
        if (x) (void)hipFree(x);
    dp.device_bytes -= k.bytes;
    k = DevicePlan::Packs{};
}

void free_m2l_packs(DevicePlan &dp)
{
    bool any = !dp.lvl_packs.empty();
    for (auto &k : dp.m2l_packs) {
        any = any || k.nb != 0;
        free_packs(dp, k);
    }
    for (auto &k : dp.lvl_packs) free_packs(dp, k);
    dp.lvl_packs.clear();
    if (any) ++dp.schedule_gen;  // a captured graph may hold them
}

// Packs of fpt fields for translations of order p (all levels, or one).
static void build_packs(DevicePlan &dp, int fpt, int p, int only_level, DevicePlan::Packs &k)
{
    M2LPacks h;
    build_m2l_packs(dp.hp, m2lp_slots(p) / fpt, 16 / fpt, dp.m2l_max_grp, h, only_level);
    auto up = [&](const auto &v, auto *&d) {
        using E = typename std::decay_t<decltype(v)>::value_type;
        const size_t b = sizeof(E) * std::max<size_t>(v.size(), 1);
        hip_check(hipMalloc(&d, b), "hipMalloc M2L packs");
        k.bytes += (int64_t)b;
        dp.device_bytes += (int64_t)b;
        if (!v.empty())
            hip_check(hipMemcpy(d, v.data(), sizeof(E) * v.size(), hipMemcpyHostToDevice), "hipMemcpy M2L packs");
    };
    up(h.blk_cells, k.blk_cells);
    up(h.item, k.item);
    up(h.grp_key, k.grp_key);
    up(h.grp_src, k.grp_src);
    up(h.grp_slot, k.grp_slot);
    k.nb = h.nb;
    k.tpg = h.tpg;
    k.max_grp = dp.m2l_max_grp;
    k.p = p;
    k.nitems = (int32_t)(h.item.size() / 3);
    k.ngrp = (int64_t)h.grp_key.size();
    k.npairs = 0;
    for (int32_t s : h.grp_src) k.npairs += s >= 0;
}

static void ensure_m2l_packs(DevicePlan &dp, int32_t F)
{
    if (!m2l_packed(dp, F)) return;
    const HostPlan &hp = dp.hp;
    const int fpt = m2l_fpt(F);
    if (!dp.level_orders) {
        DevicePlan::Packs &k = dp.m2l_packs[m2l_pack_slot(fpt)];
        if (k.nb == 0 || k.max_grp != dp.m2l_max_grp || k.p != hp.p) {
            ++dp.schedule_gen;
            free_packs(dp, k);
            build_packs(dp, fpt, hp.p, -1, k);
        }
    } else {
        bool ok = dp.lvl_packs.size() == (size_t)hp.depth + 1;
        for (size_t lv = 0; ok && lv < dp.lvl_packs.size(); ++lv) {
            const DevicePlan::Packs &k = dp.lvl_packs[lv];
            ok = k.tpg * fpt == 16 && k.max_grp == dp.m2l_max_grp && k.p == dp.lo.q[lv];
        }
        if (!ok) {
            ++dp.schedule_gen;
            for (auto &k : dp.lvl_packs) free_packs(dp, k);
            dp.lvl_packs.assign((size_t)hp.depth + 1, DevicePlan::Packs{});
            for (int lv = 0; lv <= hp.depth; ++lv) build_packs(dp, fpt, dp.lo.q[lv], lv, dp.lvl_packs[lv]);
        }
    }
    if (dp.lr_cap < F) {
        ++dp.schedule_gen;
        if (dp.Lr) (void)hipFree(dp.Lr);
        dp.Lr = nullptr;
        dp.lr_cap = 0;
        hip_check(hipMalloc(&dp.Lr, sizeof(double) * (size_t)F * hp.cells.size() * m2l_nrows(hp.p)), "hipMalloc Lr");
        dp.lr_cap = F;
    }
}

void collect_timing(DevicePlan &dp)
{
    for (const auto &sp : dp.spans) {
        hip_check(hipEventSynchronize(sp.b), "hipEventSynchronize");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, sp.a, sp.b), "hipEventElapsedTime");
        dp.kt_ms[sp.slot] += ms;
        dp.kt_n[sp.slot] += 1;
    }
    dp.spans.clear();
    dp.events_used = 0;
}

void reset_timing(DevicePlan &dp)
{
    dp.spans.clear();
    dp.events_used = 0;
    for (int i = 0; i < KT_COUNT; ++i) {
        dp.kt_ms[i] = 0.0;
        dp.kt_n[i] = 0;
    }
}

void ensure_expansions(DevicePlan &dp, int32_t F)
{
    if (F <= dp.Fcap) return;
    ++dp.schedule_gen;  // a captured graph may hold the old Q and L
    if (dp.Q) (void)hipFree(dp.Q);
    if (dp.L) (void)hipFree(dp.L);
    dp.Q = dp.L = nullptr;
    dp.Fcap = 0;
    const size_t bytes = sizeof(double) * (size_t)F * dp.hp.cells.size() * dp.ncoef;
    hip_check(hipMalloc(&dp.Q, bytes), "hipMalloc Q");
    hip_check(hipMalloc(&dp.L, bytes), "hipMalloc L");
    dp.Fcap = F;
}

void prepare_evaluate(DevicePlan &dp, int32_t F)
{
    const int64_t C = (int64_t)dp.hp.cells.size();
    if (dp.sur_mode != TFMM_SUR_OFF && !dp.hp.points && !dp.near_stored) {
        if (dp.sur_mode == TFMM_SUR_MLP && !dp.sur_wb)
            throw PlanError{TFMM_EINVAL, "the surrogate is switched on but no network is attached"};
        build_band_list(dp, nullptr);
    }
    if (!dp.side) {
        hip_check(hipStreamCreateWithFlags(&dp.side, hipStreamNonBlocking), "hipStreamCreate");
        hip_check(hipEventCreateWithFlags(&dp.ev_fork, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventCreateWithFlags(&dp.ev_join, hipEventDisableTiming), "hipEventCreate");
    }
    ensure_expansions(dp, F);
    if (m2l_packed(dp, F)) {
        ensure_m2l_packs(dp, F);
    } else {
        ensure_m2l_tiles(dp, 16 / m2l_fpt(F));
        if (dp.level_orders) ensure_m2l_level_tiles(dp, 16 / m2l_fpt(F));
    }
    if (dp.m2l_precision != TFMM_M2L_FP64) {
        if (!dp.m2l_Df) {
            ++dp.schedule_gen;
            const int64_t n = (int64_t)dp.n_m2l_keys * nd_of(dp.hp.p);
            hip_check(hipMalloc(&dp.m2l_Df, sizeof(float) * std::max<int64_t>(n, 1)), "hipMalloc M2L table f32");
            k_to_float<<<dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536))), dim3(256)>>>(
                dp.m2l_D, n, dp.m2l_Df);
            hip_check(hipGetLastError(), "k_to_float launch");
            hip_check(hipDeviceSynchronize(), "k_to_float");
        }
        if (dp.qtf_cap < F) {
            ++dp.schedule_gen;
            if (dp.Qtf) (void)hipFree(dp.Qtf);
            dp.Qtf = nullptr;
            dp.qtf_cap = 0;
            hip_check(hipMalloc(&dp.Qtf, sizeof(float) * (size_t)F * C * dp.qpad), "hipMalloc Qt f32");
            dp.qtf_cap = F;
        }
    } else if (dp.qt_cap < F) {
        ++dp.schedule_gen;
        if (dp.Qt) (void)hipFree(dp.Qt);
        dp.Qt = nullptr;
        dp.qt_cap = 0;
        hip_check(hipMalloc(&dp.Qt, sizeof(double) * (size_t)F * C * dp.qpad), "hipMalloc Qt");
        dp.qt_cap = F;
    }
}

// Times one configuration: the median of three evaluations (after one warm
// evaluation) with events on st.
static float time_config(DevicePlan &dp, const double *M, double *u, hipStream_t st)
{
    prepare_evaluate(dp, 1);
    run_evaluate(dp, M, 1, u, st);
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "hipEventCreate");
    hip_check(hipEventCreate(&b), "hipEventCreate");
    float ms[3];
    for (float &m : ms) {
        hip_check(hipEventRecord(a, st), "hipEventRecord");
        run_evaluate(dp, M, 1, u, st);
        hip_check(hipEventRecord(b, st), "hipEventRecord");
        hip_check(hipEventSynchronize(b), "hipEventSynchronize");
        hip_check(hipEventElapsedTime(&m, a, b), "hipEventElapsedTime");
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(ms, ms + 3);
    return ms[1];
}

void autotune(DevicePlan &dp, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    double *M = nullptr, *u = nullptr;
    hip_check(hipMalloc(&M, sizeof(double) * 3 * std::max<int64_t>(hp.n_nodes, 1)), "hipMalloc tuning M");
    if (hipMalloc(&u, sizeof(double) * std::max<int64_t>(hp.n_targets, 1)) != hipSuccess) {
        (void)hipFree(M);
        throw DeviceError{"hipMalloc tuning u failed"};
    }
    const bool timing = dp.timing;
    dp.timing = false;
    try {
        fill(M, 3 * hp.n_nodes, 1.0, st);
        // M2L form and work item size, then the P2P workgroup shape; every
        // candidate computes the same contraction, only the schedule differs
        int best_ent = dp.m2l_max_ent, best_grp = dp.m2l_max_grp;
        bool best_pack = false;
        float best = -1.f;
        dp.m2l_pack = false;
        for (int ent : {128, 256, 512, 1024}) {
            dp.m2l_max_ent = ent;
            const float t = time_config(dp, M, u, st);
            if (best < 0.f || t < best) best = t, best_ent = ent;
        }
        dp.m2l_max_ent = best_ent;
        dp.m2l_pack = true;
        if (m2l_packed(dp, 1)) {
            for (int grp : {256, 512}) {
                dp.m2l_max_grp = grp;
                const float t = time_config(dp, M, u, st);
                if (t < best) best = t, best_grp = grp, best_pack = true;
            }
        }
        dp.m2l_pack = best_pack;
        dp.m2l_max_grp = best_grp;
        // the work lists of the form not taken are rebuilt if it is set later
        if (best_pack)
            free_tiles(dp, dp.m2l_tiles[0]);
        else
            free_m2l_packs(dp);
        bool best_wide = false;
        for (bool wide : {false, true}) {
            dp.p2p_wide = wide;
            const float t = time_config(dp, M, u, st);
            if (!wide || t < best) best = t, best_wide = wide;
        }
        dp.p2p_wide = best_wide;
        ++dp.schedule_gen;
        prepare_evaluate(dp, 1);
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    } catch (...) {
        dp.timing = timing;
        (void)hipFree(M);
        (void)hipFree(u);
        throw;
    }
    dp.timing = timing;
    (void)hipFree(M);
    (void)hipFree(u);
}

void run_evaluate(DevicePlan &dp, const double *M, int32_t F, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const int64_t C = (int64_t)hp.cells.size();
    const int p = hp.p;
    prepare_evaluate(dp, F);
    dp.last_F = F;
    // u = 0, then the near field (P2P, needs only M) runs on the plan's side
    // stream while the expansions are formed; both add into u atomically.
    // Under stream capture (batch graphs) the near field stays on st, after
    // the far field.
    fill(u, (int64_t)F * hp.n_targets, 0.0, st);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(st, &cap), "hipStreamIsCapturing");
    // with per-phase timing on, the phases run one after another (isolated times)
    const bool fork = cap == hipStreamCaptureStatusNone && !dp.timing;
    auto fork_p2p = [&]() {
        hip_check(hipEventRecord(dp.ev_fork, st), "hipEventRecord");
        hip_check(hipStreamWaitEvent(dp.side, dp.ev_fork, 0), "hipStreamWaitEvent");
        {
            KTimer kt(dp, KT_P2P, dp.side);
            run_near(dp, M, F, u, dp.side);
        }
        hip_check(hipEventRecord(dp.ev_join, dp.side), "hipEventRecord");
    };
    if (fork) fork_p2p();
    fill(dp.Q, (int64_t)F * C * dp.ncoef, 0.0, st);
    fill(dp.L, (int64_t)F * C * dp.ncoef, 0.0, st);
    const size_t shift_lds = sizeof(double) * 2 * kShiftItems * (size_t)dp.ncoef;
    {
        KTimer kt(dp, KT_P2M, st);
        if (dp.n_p2m_cells > 0) launch_fc(F, [&](auto fc) {
            constexpr int FC = decltype(fc)::value;
            const size_t lds = sizeof(double) * (size_t)kP2MStage * (dp.ncoef + 12 * FC);
            k_p2m<FC><<<dim3(xcd_grid(dp.n_p2m_cells), (F + FC - 1) / FC), dim3(kP2MThreads), lds, st>>>(
                dp.p2m_cells, dp.cell_i, dp.cell_c, C, dp.tet_xyz, dp.tet_node, hp.n_tets, dp.tet_mom, M, hp.n_nodes, F,
                p, dp.n_p2m_cells, hp.points ? 1 : 0, dp.lo, dp.Q);
            hip_check(hipGetLastError(), "k_p2m launch");
        });
    }
    {
        KTimer kt(dp, KT_M2M, st);
        for (int Lv = hp.depth - 1; Lv >= 0; --Lv) {
            int b = dp.m2m_level_ptr[Lv], e = dp.m2m_level_ptr[Lv + 1];
            if (e > b) {
                k_m2m<<<dim3(e - b, F), dim3(kShiftThreads), shift_lds, st>>>(dp.m2m_cells + b, dp.cell_i, dp.cell_c,
                                                                                  C, p, dp.lo.q[Lv], dp.Q);
                hip_check(hipGetLastError(), "k_m2m launch");
            }
        }
    }
    {
        KTimer kt(dp, KT_M2L, st);
        run_m2l(dp, F, st);
    }
    {
        KTimer kt(dp, KT_L2L, st);
        for (int Lv = 1; Lv <= hp.depth; ++Lv) {
            int b = dp.l2l_level_ptr[Lv], e = dp.l2l_level_ptr[Lv + 1];
            if (e > b) {
                k_l2l<<<dim3((e - b + kShiftItems - 1) / kShiftItems, F), dim3(kShiftThreads), shift_lds, st>>>(
                    dp.l2l_cells + b, e - b, dp.cell_i, dp.cell_c, C, p, dp.lo.q[Lv], dp.L);
                hip_check(hipGetLastError(), "k_l2l launch");
            }
        }
    }
    {
        KTimer kt(dp, KT_L2P, st);
        const unsigned nb = (unsigned)((hp.n_targets + 255) / 256);
        with_order(p, [&](auto pc) {
            constexpr int PP = decltype(pc)::value;
            k_l2p<PP><<<dim3(nb, F), dim3(256), 0, st>>>(dp.tgt_xyz, dp.tgt_perm, dp.tgt_leaf, hp.n_targets, dp.cell_c,
                                                         C, dp.L, u);
        });
        hip_check(hipGetLastError(), "k_l2p launch");
    }
    if (fork) {
        hip_check(hipStreamWaitEvent(st, dp.ev_join, 0), "hipStreamWaitEvent");
    } else {
        KTimer kt(dp, KT_P2P, st);
        run_near(dp, M, F, u, st);
    }
}

double run_demag(DevicePlan &dp, const double *M, const double *u, double *H, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    if (!hp.targets_are_nodes) throw DeviceError{"the plan's targets are not its nodes"};
    const int64_t T = hp.n_tets;
    const int nb = (int)((T + kEnergyThreads - 1) / kEnergyThreads);
    double *part = nullptr;
    hip_check(hipMalloc(&part, sizeof(double) * (size_t)(nb + 1)), "hipMalloc energy");
    double E = 0.0;
    hipError_t err = hipSuccess;
    if (T > 0) {
        k_demag<<<nb, kEnergyThreads, 0, st>>>(dp.tet_xyz, dp.tet_node, dp.tet_perm, T, M, u, H, part);
        k_sum_blocks<<<1, kEnergyThreads, 0, st>>>(part, nb, part + nb);
        err = hipGetLastError();
        if (err == hipSuccess) err = hipMemcpyAsync(&E, part + nb, sizeof(double), hipMemcpyDeviceToHost, st);
        if (err == hipSuccess) err = hipStreamSynchronize(st);
    }
    (void)hipFree(part);
    hip_check(err, "demag energy");
    return E;
}

void run_elementary(int fn, const double *a, const double *b, int64_t n, double *out)
{
    double *d = nullptr;
    hip_check(hipMalloc(&d, sizeof(double) * 3 * (size_t)n), "hipMalloc elementary");
    hipError_t e = hipMemcpy(d, a, sizeof(double) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + n, b, sizeof(double) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_elementary<<<(unsigned)((n + 255) / 256), 256>>>(fn, d, d + n, n, d + 2 * n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, d + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    hip_check(e, "elementary functions");
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point: one file-scope device array of
// kNoAllocScratchDoubles doubles; every device the library runs on holds its
// own copy until the process ends.  In host code the array's name is only a
// stand-in (not a device address), so host code reaches it through the
// address hipGetSymbolAddress returns on each device, taken once per device
// with that device current and kept.  Every call on a device shares that
// device's array (it keeps the last call's contents): calls that overlap on
// one device race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

static double *scratch_address(int device)
{
    static std::mutex mu;
    static std::vector<double *> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) throw DeviceError{"no device"};
    if ((int)addr.size() <= device) addr.resize((size_t)device + 1, nullptr);
    if (!addr[device]) {
        int cur = -1;
        hip_check(hipGetDevice(&cur), "hipGetDevice");
        if (cur != device) throw DeviceError{"scratch address requested for a device that is not current"};
        void *p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        addr[device] = static_cast<double *>(p);
    }
    return addr[device];
}

void run_demag_noalloc(DevicePlan &dp, const double *M, const double *u, double *H, double *energy_dev,
                       hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    if (!hp.targets_are_nodes) throw DeviceError{"the plan's targets are not its nodes"};
    const int64_t T = hp.n_tets;
    const int64_t nb = (T + kEnergyThreads - 1) / kEnergyThreads;
    if (nb + 1 > kNoAllocScratchDoubles)
        throw PlanError{TFMM_EINVAL, "tfmm_demag_energy_noalloc: " + std::to_string(T) + " tets exceed the limit of " +
                                         std::to_string((int64_t)TFMM_NOALLOC_MAX_TETS)};
    double *part = scratch_address(dp.device);
    // every slot read below is written first in this call (block partials,
    // then their sum): nothing has to start at zero
    if (T > 0) {
        k_demag<<<(unsigned)nb, kEnergyThreads, 0, st>>>(dp.tet_xyz, dp.tet_node, dp.tet_perm, T, M, u, H, part);
        k_sum_blocks<<<1, kEnergyThreads, 0, st>>>(part, (int)nb, energy_dev);
    } else {
        k_sum_blocks<<<1, kEnergyThreads, 0, st>>>(part, 0, energy_dev);
    }
    hip_check(hipGetLastError(), "demag energy (no allocation) launch");
}

void run_demag_nodes(DevicePlan &dp, const double *u, double *Hn, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    if (!hp.targets_are_nodes) throw DeviceError{"the plan's targets are not its nodes"};
    const int64_t T = hp.n_tets, N = hp.n_nodes;
    const unsigned nb = (unsigned)((T + kEnergyThreads - 1) / kEnergyThreads);
    fill(Hn, 3 * N, 0.0, st);
    if (!dp.node_lump) {  // lumped volumes, once per plan
        hip_check(hipMalloc(&dp.node_lump, sizeof(double) * (size_t)std::max<int64_t>(N, 1)), "hipMalloc lumped volumes");
        dp.device_bytes += (int64_t)(sizeof(double) * (size_t)std::max<int64_t>(N, 1));
        fill(dp.node_lump, N, 0.0, st);
        if (T > 0)
            k_demag_scatter<<<nb, kEnergyThreads, 0, st>>>(dp.tet_xyz, dp.tet_node, T, u, Hn, dp.node_lump);
    } else if (T > 0) {
        k_demag_scatter<<<nb, kEnergyThreads, 0, st>>>(dp.tet_xyz, dp.tet_node, T, u, Hn, nullptr);
    }
    if (N > 0) k_lump_divide<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(Hn, dp.node_lump, N);
    hip_check(hipGetLastError(), "lumped field launch");
}

void run_direct(DevicePlan &dp, const double *M, int32_t F, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    fill(u, (int64_t)F * hp.n_targets, 0.0, st);
    if (hp.points) {
        run_p2p(dp, true, M, F, u, st);
        return;
    }
    if (hp.n_tets == 0 || hp.n_targets == 0) return;
    for (int f = 0; f < F;) {
        const int left = F - f;
        const int fch = left >= 32 ? 32 : (left >= 16 ? 16 : (left >= 8 ? 8 : (left >= 4 ? 4 : (left >= 2 ? 2 : 1))));
        auto go = [&](auto fc) {
            constexpr int FC = decltype(fc)::value;
            const int nblk = (int)((hp.n_tets + direct_stage(FC) - 1) / direct_stage(FC));
            k_direct<FC><<<dim3(xcd_grid(nblk)), dim3(256), 0, st>>>(nblk, hp.n_tets, dp.tet_xyz, dp.tet_node,
                                                                     dp.tgt_xyz, dp.tgt_perm, hp.n_targets, M,
                                                                     hp.n_nodes, f, dp.far_rule, u);
        };
        switch (fch) {
        case 32: go(std::integral_constant<int, 32>{}); break;
        case 16: go(std::integral_constant<int, 16>{}); break;
        case 8: go(std::integral_constant<int, 8>{}); break;
        case 4: go(std::integral_constant<int, 4>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        default: go(std::integral_constant<int, 1>{}); break;
        }
        hip_check(hipGetLastError(), "k_direct launch");
        f += fch;
    }
}

// ---------------------------------------------------------------------------
// quadrature: Gauss-Jacobi nodes on [0, 1] for the weight (1 - t)^alpha by
// bracketing the sign changes of the Jacobi polynomial and bisection, weights
// from the classical closed form; collapsed onto the simplex.
// ---------------------------------------------------------------------------
namespace {

void jacobi_eval(int n, double a, double x, double &P, double &dP)
{
    // P_n^{(a,0)}(x) by the three-term recurrence, derivative by the standard identity
    double p0 = 1.0, p1 = 0.5 * (a + 2.0) * x + 0.5 * a;
    if (n == 0) {
        P = 1.0;
        dP = 0.0;
        return;
    }
    const double b = 0.0;
    for (int k = 2; k <= n; ++k) {
        const double c = 2.0 * k + a + b;
        const double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
        const double a2 = (c - 1.0) * (a * a - b * b);
        const double a3 = (c - 2.0) * (c - 1.0) * c;
        const double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
        const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    const double c = 2.0 * n + a + b;
    dP = (n * (a - b - c * x) * p1 + 2.0 * (n + a) * (n + b) * p0) / (c * (1.0 - x * x));
}

void gauss_jacobi01(int n, double a, std::vector<double> &t, std::vector<double> &w)
{
    t.clear();
    w.clear();
    const int grid = 20000;
    double xl = -1.0 + 1e-14, Pl, dPl;
    jacobi_eval(n, a, xl, Pl, dPl);
    for (int i = 1; i <= grid && (int)t.size() < n; ++i) {
        double xr = -1.0 + 2.0 * i / grid - (i == grid ? 1e-14 : 0.0), Pr, dPr;
        jacobi_eval(n, a, xr, Pr, dPr);
        if ((Pl < 0.0) != (Pr < 0.0)) {
            double lo = xl, hi = xr, flo = Pl;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), fm, dm;
                jacobi_eval(n, a, mid, fm, dm);
                if ((fm < 0.0) == (flo < 0.0)) {
                    lo = mid;
                    flo = fm;
                } else {
                    hi = mid;
                }
            }
            double x = 0.5 * (lo + hi), P, dP;
            jacobi_eval(n, a, x, P, dP);
            // classical weight for weight (1-x)^a on [-1,1], b = 0
            const double lw = std::lgamma(n + a + 1.0) + std::lgamma(n + 1.0) - std::lgamma(n + a + 1.0) -
                              std::lgamma(n + 1.0) + (a + 1.0) * std::log(2.0);
            const double wx = std::exp(lw) / ((1.0 - x * x) * dP * dP);
            t.push_back(0.5 * (x + 1.0));
            w.push_back(wx * std::pow(2.0, -a - 1.0));
        }
        xl = xr;
        Pl = Pr;
    }
}

}  // namespace

std::vector<double> simplex_rule(int deg, int *npts)
{
    const int q = (deg + 2) / 2;  // 2q - 1 >= deg
    std::vector<double> ta, wa, tb, wb, tc, wc;
    gauss_jacobi01(q, 2.0, ta, wa);
    gauss_jacobi01(q, 1.0, tb, wb);
    gauss_jacobi01(q, 0.0, tc, wc);
    std::vector<double> out;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                const double a = ta[i], b = tb[j], c = tc[k];
                out.push_back(a);
                out.push_back((1.0 - a) * b);
                out.push_back((1.0 - a) * (1.0 - b) * c);
                out.push_back(wa[i] * wb[j] * wc[k]);
            }
    *npts = q * q * q;
    return out;
}

}  // namespace tfmm
