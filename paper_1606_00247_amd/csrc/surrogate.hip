// Learned surrogate of the near-field pair integral at intermediate distance.
//
// For a tet T (corners v_i, diameter = longest edge, centroid c, volume V) and
// a target x with 2 <= rho = |x - c| / diam < 6 the potential is linear in the
// nodal magnetisation and homogeneous of degree one in length:
//   u_T(x) = diam * sum_{i,a} C_ia M_ia,
// C a function of the corners seen from the target.  The tet's own multipole
// expansion about c truncated at |n| <= 2 (the dipole and quadrupole terms of
// the Taylor expansion of Sec. 2.2) gives most of it in closed form,
//   4 pi diam Cq_ia = (V / R^3) [R_a / 4 + (3 R_a (R . w_i) / R^2 - w_ia) / 20],
// R = x - c, w_i = v_i - c; a multilayer perceptron predicts the rest: it maps
// the tet's corners seen from the target, as 16 scale-free O(1) numbers (the
// unit direction R / |R|, w_i / diam and 1 / rho), to
// y = kYScale (C - Cq) rho^4 / Vh (Vh = V / diam^3; the residual falls like
// rho^-4, so y is O(1) over the band), and the 12 coefficients are contracted
// with the 4 nodal M exactly.  Layers 16 -> H -> H -> H -> 12 with ReLU.
// Training pairs are drawn from the plan's own band pairs (the pairs the
// evaluation hands to the network); their targets come from the exact pair
// integral (unit nodal fields).  Training runs in FP32 (Adam); inference uses BF16
// weights and activations on matrix cores with FP32 accumulation, the
// quadrupole part and the contraction in FP64.
//
// In an evaluation with the surrogate on, the near-field pairs of the band
// are taken out of the exact near-field kernel and evaluated from a list of
// band pairs (built once per plan, ordered by target within each P2P block)
// by the network, or by one of two controls: the quadrupole part alone (the
// network's base) or a 27-point Gauss-Jacobi rule (degree 5) of the integrand.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/tetfmm.h"
#include "device.h"
#include "pair.h"

namespace tfmm {

namespace {

constexpr int kIn = 16, kOut = 12;
constexpr double kYScale = 2048.0;  // y = kYScale (C - Cq) rho^4 / Vh

// splitmix64 (Steele, Lea and Flood 2014): the counter-based generator of the
// training samples.
__host__ __device__ inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__device__ inline double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

// Parameter layout (FP32): W1 [12][H], b1 [H], W2 [H][H], b2, W3 [H][H], b3,
// W4 [H][12], b4 [12]; W[k][n] maps input k to output n.
struct Layout {
    int H;
    size_t w[4], b[4], n;
    __host__ __device__ explicit Layout(int h) : H(h)
    {
        const int K[4] = {kIn, h, h, h}, N[4] = {h, h, h, kOut};
        size_t o = 0;
        for (int l = 0; l < 4; ++l) {
            w[l] = o;
            o += (size_t)K[l] * N[l];
            b[l] = o;
            o += N[l];
        }
        n = o;
    }
    __host__ __device__ int K(int l) const { return l == 0 ? kIn : H; }
    __host__ __device__ int N(int l) const { return l == 3 ? kOut : H; }
};

// diameter (longest edge), centroid and Vh = V / diam^3 of corners v
__device__ inline void tet_scales(const double v[4][3], double c[3], double &diam, double &vh)
{
    double l2 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) {
            const double dx = v[b][0] - v[a][0], dy = v[b][1] - v[a][1], dz = v[b][2] - v[a][2];
            l2 = fmax(l2, dx * dx + dy * dy + dz * dz);
        }
    diam = sqrt(l2);
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = 0.25 * ((v[0][k] + v[1][k]) + (v[2][k] + v[3][k]));
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const double e3[3] = {v[3][0] - v[0][0], v[3][1] - v[0][1], v[3][2] - v[0][2]};
    const double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                       e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    vh = fabs(det) / 6.0 / (l2 * diam);
}

// 4 pi diam Cq_j of the 12 unit fields j = 3 i + a (component a at corner i):
// the tet's multipole expansion about its centroid c truncated at |n| <= 2,
//   q_{3i+a} = (V / R^3) [R_a / 4 + (3 R_a (R . w_i) / R^2 - w_ia) / 20],
// R = x - c, w_i = v_i - c (the moments int_T lambda_i = V/4 and
// int_T lambda_i (y - c) = V w_i / 20 of the barycentric field lambda_i e_a).
__device__ inline void quad_coeffs(const double x[3], const double v[4][3], const double c[3], double q[12])
{
    const double R[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double ir = rsqrt_nr(r2);
    const double ir2 = ir * ir;
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const double e3[3] = {v[3][0] - v[0][0], v[3][1] - v[0][1], v[3][2] - v[0][2]};
    const double V = fabs(e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                          e1[2] * (e2[0] * e3[1] - e2[1] * e3[0])) / 6.0;
    const double f = V * ir * ir2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double w[3] = {v[i][0] - c[0], v[i][1] - c[1], v[i][2] - c[2]};
        const double rw = 3.0 * (R[0] * w[0] + R[1] * w[1] + R[2] * w[2]) * ir2;
#pragma unroll
        for (int a = 0; a < 3; ++a) q[3 * i + a] = f * (0.25 * R[a] + 0.05 * (R[a] * rw - w[a]));
    }
}

// The network's 16 inputs for target x and a tet (corners v, centroid c,
// longest edge diam), all O(1) and scale free: the unit direction
// R / |R| (R = x - c), the corners about the centroid in units of the
// diameter (v_i - c) / diam, and 1 / rho = diam / |R|.
__device__ inline void sur_features(const double x[3], const double v[4][3], const double c[3], double diam,
                                    double f[kIn])
{
    const double R[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    const double ir = rsqrt_nr(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    const double id = 1.0 / diam;
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = R[k] * ir;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) f[3 + 3 * i + k] = (v[i][k] - c[k]) * id;
    f[15] = diam * ir;
}

// One training sample per thread: inputs X [n][16], targets Y [n][12].  The
// pair is drawn from the plan's list of band pairs (the near-field pairs the
// evaluation hands to the network) when given, else a tet of the plan with a
// target at a uniform direction and rho uniform in [2, 6).
__global__ void k_sur_gen(const double *__restrict__ tet_xyz, int64_t T, const int32_t *__restrict__ pairs,
                          int64_t npairs, const double *__restrict__ tgt_xyz, int64_t N, uint64_t seed, int n,
                          float *__restrict__ X, float *__restrict__ Y)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t h0 = splitmix64(seed ^ splitmix64((uint64_t)s));
    const uint64_t h1 = splitmix64(h0), h2 = splitmix64(h1), h3 = splitmix64(h2);
    int64_t t;
    double x[3];
    TetGeom G;
    double c[3], diam, vh;
    if (pairs && npairs > 0) {
        const int64_t k = (int64_t)(h0 % (uint64_t)npairs);
        const int64_t tg = pairs[2 * k];
        t = pairs[2 * k + 1];
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = tgt_xyz[d * N + tg];
    } else {
        t = (int64_t)(h0 % (uint64_t)T);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) G.v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + t];
    tet_scales(G.v, c, diam, vh);
    if (!(pairs && npairs > 0)) {
        const double zc = 2.0 * u01(h1) - 1.0, ph = 6.283185307179586 * u01(h2);
        const double sr = sqrt(fmax(0.0, 1.0 - zc * zc));
        const double rho = kBandLo + (kBandHi - kBandLo) * u01(h3);
        x[0] = c[0] + rho * diam * sr * cos(ph);
        x[1] = c[1] + rho * diam * sr * sin(ph);
        x[2] = c[2] + rho * diam * zc;
    }
    const double dist = sqrt((x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) + (x[2] - c[2]) * (x[2] - c[2]));
    const double rho = dist / diam;
    double gl[4][3], eh[6][3];
    tet_geometry(G, gl, eh);
    TetField fld[kOut];
#pragma unroll 1
    for (int j = 0; j < kOut; ++j) {  // unit field: component j % 3 at corner j / 3
        double m[4][3] = {};
        m[j / 3][j % 3] = 1.0;
        tet_field(G, gl, eh, m, fld[j]);
    }
    double acc[kOut];
#pragma unroll
    for (int j = 0; j < kOut; ++j) acc[j] = 0.0;
    pair_accumulate<kOut>(x, G, fld, acc);
    double q[kOut];
    quad_coeffs(x, G.v, c, q);
    const double rho2 = rho * rho;
    const double scale = kYScale * kInv4Pi / diam * rho2 * rho2 / vh;
    double f[kIn];
    sur_features(x, G.v, c, diam, f);
#pragma unroll
    for (int j = 0; j < kIn; ++j) X[(int64_t)s * kIn + j] = (float)f[j];
#pragma unroll
    for (int j = 0; j < kOut; ++j) Y[(int64_t)s * kOut + j] = (float)((acc[j] - q[j]) * scale);
}

// Z [B][N] = A [B][K] W [K][N] + b; out = relu(Z) (relu) or Z.
constexpr int kTile = 16;
__global__ void k_lin_fwd(const float *__restrict__ A, const float *__restrict__ W, const float *__restrict__ bias,
                          int B, int K, int N, bool relu, float *__restrict__ out)
{
    __shared__ float sa[kTile][kTile + 1], sw[kTile][kTile + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int row = blockIdx.y * kTile + ty, col = blockIdx.x * kTile + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += kTile) {
        sa[ty][tx] = (row < B && k0 + tx < K) ? A[(int64_t)row * K + k0 + tx] : 0.f;
        sw[ty][tx] = (k0 + ty < K && col < N) ? W[(int64_t)(k0 + ty) * N + col] : 0.f;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTile; ++k) acc += sa[ty][k] * sw[k][tx];
        __syncthreads();
    }
    if (row < B && col < N) {
        const float z = acc + bias[col];
        out[(int64_t)row * N + col] = relu ? fmaxf(z, 0.f) : z;
    }
}

// dA [B][K] = (dZ [B][N] W^T) * (A > 0)  (A: the layer input, a ReLU output)
__global__ void k_lin_bwd_data(const float *__restrict__ dZ, const float *__restrict__ W, const float *__restrict__ A,
                               int B, int K, int N, float *__restrict__ dA)
{
    __shared__ float sd[kTile][kTile + 1], sw[kTile][kTile + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int row = blockIdx.y * kTile + ty, col = blockIdx.x * kTile + tx;  // col indexes K
    float acc = 0.f;
    for (int n0 = 0; n0 < N; n0 += kTile) {
        sd[ty][tx] = (row < B && n0 + tx < N) ? dZ[(int64_t)row * N + n0 + tx] : 0.f;
        // sw[n][k] = W[k][n]
        sw[ty][tx] = (n0 + ty < N && blockIdx.x * kTile + tx < K) ? W[(int64_t)(blockIdx.x * kTile + tx) * N + n0 + ty]
                                                                   : 0.f;
        __syncthreads();
#pragma unroll
        for (int n = 0; n < kTile; ++n) acc += sd[ty][n] * sw[n][tx];
        __syncthreads();
    }
    if (row < B && col < K) dA[(int64_t)row * K + col] = A[(int64_t)row * K + col] > 0.f ? acc : 0.f;
}

// dW [K][N] = A^T dZ, db [N] = sum_b dZ  (over the batch)
__global__ void k_lin_bwd_w(const float *__restrict__ A, const float *__restrict__ dZ, int B, int K, int N,
                            float *__restrict__ dW, float *__restrict__ db)
{
    __shared__ float sa[kTile][kTile + 1], sd[kTile][kTile + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int k = blockIdx.y * kTile + ty, n = blockIdx.x * kTile + tx;
    float acc = 0.f, accb = 0.f;
    for (int b0 = 0; b0 < B; b0 += kTile) {
        // sa[b][k], sd[b][n]
        sa[ty][tx] = (b0 + ty < B && blockIdx.y * kTile + tx < K) ? A[(int64_t)(b0 + ty) * K + blockIdx.y * kTile + tx]
                                                                   : 0.f;
        sd[ty][tx] = (b0 + ty < B && n < N) ? dZ[(int64_t)(b0 + ty) * N + n] : 0.f;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < kTile; ++b) {
            acc += sa[b][ty] * sd[b][tx];
            accb += sd[b][tx];
        }
        __syncthreads();
    }
    if (k < K && n < N) dW[(int64_t)k * N + n] = acc;
    if (blockIdx.y == 0 && ty == 0 && n < N) db[n] = accb;
}

// dY = 2 (Y - T) / (B * 12); loss += sum (Y - T)^2 / (B * 12)
__global__ void k_sur_loss(const float *__restrict__ Yp, const float *__restrict__ Yt, int n, float *__restrict__ dY,
                           double *__restrict__ loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (i < n) {
        const float e = Yp[i] - Yt[i];
        dY[i] = 2.f * e / (float)n;
        e2 = e * e;
    }
    for (int o = 32; o > 0; o >>= 1) e2 += __shfl_down(e2, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, (double)e2 / (double)n);
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_f32_to_bf16_t(const float *__restrict__ W, int K, int N, int KP, int NP, int dup,
                                __bf16 *__restrict__ out)
{
    // out [NP][KP] = W^T, zero padded; with dup the K rows are repeated once
    // (columns K .. 2K - 1 take the weights of the low parts of the inputs)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP * KP) return;
    const int n = i / KP, k0 = i % KP;
    const int k = (dup && k0 >= K && k0 < 2 * K) ? k0 - K : k0;
    out[i] = (__bf16)((n < N && k < K) ? W[(int64_t)k * N + n] : 0.f);
}

// Device buffers of one training or gradient pass.
struct Work {
    int H = 0, B = 0;
    float *X = nullptr, *Yt = nullptr, *A[3] = {}, *Yp = nullptr, *dY = nullptr, *dA[3] = {};
    float *grad = nullptr;
    double *loss = nullptr;
    void alloc(int h, int b, size_t nparam)
    {
        H = h;
        B = b;
        auto f = [&](float *&p, size_t n) { hip_check(hipMalloc(&p, sizeof(float) * n), "hipMalloc surrogate"); };
        f(X, (size_t)B * kIn);
        f(Yt, (size_t)B * kOut);
        f(Yp, (size_t)B * kOut);
        f(dY, (size_t)B * kOut);
        for (int l = 0; l < 3; ++l) {
            f(A[l], (size_t)B * H);
            f(dA[l], (size_t)B * H);
        }
        f(grad, nparam);
        hip_check(hipMalloc(&loss, sizeof(double)), "hipMalloc surrogate");
    }
    ~Work()
    {
        for (float *p : {X, Yt, Yp, dY, A[0], A[1], A[2], dA[0], dA[1], dA[2], grad})
            if (p) (void)hipFree(p);
        if (loss) (void)hipFree(loss);
    }
};

// Forward and backward of the loss on the batch in w.X / w.Yt; gradients to
// w.grad, the loss added to *w.loss.
void forward_backward(const Layout &L, const float *P, Work &w, hipStream_t st)
{
    const dim3 blk(kTile, kTile);
    auto grid = [&](int cols, int rows) { return dim3((cols + kTile - 1) / kTile, (rows + kTile - 1) / kTile); };
    const float *in = w.X;
    for (int l = 0; l < 3; ++l) {
        k_lin_fwd<<<grid(L.N(l), w.B), blk, 0, st>>>(in, P + L.w[l], P + L.b[l], w.B, L.K(l), L.N(l), true, w.A[l]);
        in = w.A[l];
    }
    k_lin_fwd<<<grid(kOut, w.B), blk, 0, st>>>(in, P + L.w[3], P + L.b[3], w.B, L.H, kOut, false, w.Yp);
    const int n = w.B * kOut;
    k_sur_loss<<<(n + 255) / 256, 256, 0, st>>>(w.Yp, w.Yt, n, w.dY, w.loss);
    const float *dz = w.dY;
    for (int l = 3; l >= 0; --l) {
        const float *a = l == 0 ? w.X : w.A[l - 1];
        k_lin_bwd_w<<<grid(L.N(l), L.K(l)), blk, 0, st>>>(a, dz, w.B, L.K(l), L.N(l), w.grad + L.w[l], w.grad + L.b[l]);
        if (l > 0) {
            k_lin_bwd_data<<<grid(L.K(l), w.B), blk, 0, st>>>(dz, P + L.w[l], w.A[l - 1], w.B, L.K(l), L.N(l),
                                                               w.dA[l - 1]);
            dz = w.dA[l - 1];
        }
    }
    hip_check(hipGetLastError(), "surrogate training launch");
}

// ---------------------------------------------------------------------------
// Band pairs: the (target, tet) pairs of the near field with
// 2 <= |x - c| / diam < 6 (in_band), listed once per plan per P2P block (the
// block's tets x its target list), target-major, so that the pairs of a
// wavefront come in runs of one target.  k_band_count counts them per block;
// k_band_fill writes them at the block's offset as (sorted target index, tet).
// ---------------------------------------------------------------------------
constexpr int kBandThreads = 256;
constexpr int kBandMaxTets = 64;  // tets per P2P block

struct BandTetG {
    double c[3];
    double id2;
};

__device__ inline int stage_band_tets(const int32_t *__restrict__ blk, int b, int64_t T,
                                      const double *__restrict__ tet_xyz, BandTetG *s_b, int &ib, int &ie, int &tb)
{
    tb = blk[4 * b];
    const int te = blk[4 * b + 1];
    ib = blk[4 * b + 2];
    ie = blk[4 * b + 3];
    const int nt = min(te - tb, kBandMaxTets);
    if ((int)threadIdx.x < nt) {
        double v[4][3];
        const int64_t t = tb + threadIdx.x;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k) v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + t];
        band_geom(v, s_b[threadIdx.x].c, s_b[threadIdx.x].id2);
    }
    return nt;
}

__global__ __launch_bounds__(kBandThreads) void k_band_count(const int32_t *__restrict__ blk, int nblk, int64_t T,
                                                            const double *__restrict__ tet_xyz,
                                                            const int32_t *__restrict__ idx,
                                                            const double *__restrict__ tgt_xyz, int64_t N,
                                                            int64_t *__restrict__ cnt)
{
    __shared__ BandTetG s_b[kBandMaxTets];
    __shared__ int64_t s_n[kBandThreads / 64];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    int ib, ie, tb;
    const int nt = stage_band_tets(blk, b, T, tet_xyz, s_b, ib, ie, tb);
    __syncthreads();
    int64_t n = 0;
    for (int i = ib + threadIdx.x; i < ie; i += kBandThreads) {
        const int s = idx[i];
        const double x[3] = {tgt_xyz[s], tgt_xyz[N + s], tgt_xyz[2 * N + s]};
        for (int t = 0; t < nt; ++t) n += in_band(x, s_b[t].c, s_b[t].id2) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) n += __shfl_down(n, o);
    if ((threadIdx.x & 63) == 0) s_n[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int w = 0; w < kBandThreads / 64; ++w) tot += s_n[w];
        cnt[b] = tot;
    }
}

__global__ __launch_bounds__(kBandThreads) void k_band_fill(const int32_t *__restrict__ blk, int nblk, int64_t T,
                                                           const double *__restrict__ tet_xyz,
                                                           const int32_t *__restrict__ idx,
                                                           const double *__restrict__ tgt_xyz, int64_t N,
                                                           const int64_t *__restrict__ off,
                                                           int32_t *__restrict__ pairs)
{
    __shared__ BandTetG s_b[kBandMaxTets];
    __shared__ int s_scan[kBandThreads];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    int ib, ie, tb;
    const int nt = stage_band_tets(blk, b, T, tet_xyz, s_b, ib, ie, tb);
    __syncthreads();
    int64_t base = off[b];
    for (int i0 = ib; i0 < ie; i0 += kBandThreads) {
        const int i = i0 + threadIdx.x;
        int s = 0, n = 0;
        double x[3] = {0.0, 0.0, 0.0};
        if (i < ie) {
            s = idx[i];
            x[0] = tgt_xyz[s];
            x[1] = tgt_xyz[N + s];
            x[2] = tgt_xyz[2 * N + s];
            for (int t = 0; t < nt; ++t) n += in_band(x, s_b[t].c, s_b[t].id2) ? 1 : 0;
        }
        // inclusive scan of n over the block (Hillis-Steele)
        s_scan[threadIdx.x] = n;
        __syncthreads();
        for (int o = 1; o < kBandThreads; o <<= 1) {
            const int add = (int)threadIdx.x >= o ? s_scan[threadIdx.x - o] : 0;
            __syncthreads();
            s_scan[threadIdx.x] += add;
            __syncthreads();
        }
        const int incl = s_scan[threadIdx.x], total = s_scan[kBandThreads - 1];
        if (i < ie && n > 0) {
            int64_t k = base + incl - n;
            for (int t = 0; t < nt; ++t)
                if (in_band(x, s_b[t].c, s_b[t].id2)) {
                    pairs[2 * k] = s;
                    pairs[2 * k + 1] = tb + t;
                    ++k;
                }
        }
        base += total;
        __syncthreads();
    }
}

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x4 = float __attribute__((ext_vector_type(4)));

// One dense layer of the network for the 64 rows (pairs) of a wavefront:
// out [64][NP] = act(in [64][KP] W + b), W as [NP][KP] BF16 (transposed,
// zero padded) in global memory, activations BF16 in LDS.
template <int KP, int NP, bool LAST>
__device__ __forceinline__ void mlp_layer(const __bf16 *in, const __bf16 *__restrict__ Wt, const float *__restrict__ b,
                                          int N, __bf16 *out, float *outf, int lane)
{
#pragma unroll 1
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll 1
        for (int nb = 0; nb < NP / 16; ++nb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KP / 32; ++kb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(in + (16 * rb + (lane & 15)) * KP + 32 * kb + 8 * (lane >> 4));
                const bf16x8 w = *reinterpret_cast<const bf16x8 *>(Wt + (16 * nb + (lane & 15)) * KP + 32 * kb + 8 * (lane >> 4));
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w, acc, 0, 0, 0);
            }
            const int col = 16 * nb + (lane & 15);
            const float bias = col < N ? b[col] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + 4 * (lane >> 4) + r;
                const float z = acc[r] + bias;
                if (LAST)
                    outf[row * NP + col] = z;
                else
                    out[row * NP + col] = (__bf16)fmaxf(z, 0.f);
            }
        }
}

// ---------------------------------------------------------------------------
// Band pairs of an evaluation: one wavefront per 64 listed pairs.  Every pair
// gets the 12 coefficients q_j = 4 pi u_T(x) of the unit nodal fields j by
//   kBandExact  the exact pair integral (pair_geometry / pair_contract),
//   kBandMLP    the quadrupole part plus the network's residual,
//   kBandGauss  the 27-point collapsed Gauss-Jacobi rule (degree 5),
//   kBandQuad   the quadrupole part alone,
// contracted with each field's nodal M in FP64; the lanes of one target are
// summed by a segmented scan across the wavefront and the last lane of each
// run adds the sum into u.  The network's first layer takes every input as
// two BF16 parts, hi = bf16(s), lo = bf16(s - hi), against the same weights
// (24 of the 32 columns of the padded matrix-core step), so the inputs enter
// with ~16 significant bits.
// ---------------------------------------------------------------------------
enum { kBandExact = 0, kBandMLP = 1, kBandGauss = 2, kBandQuad = 3 };

template <int MODE, int H>
__global__ __launch_bounds__(64, 3) void k_band_eval(const int32_t *__restrict__ pairs, int64_t npairs, int64_t T,
                                                 const double *__restrict__ tet_xyz,
                                                 const int32_t *__restrict__ tet_node,
                                                 const double *__restrict__ tgt_xyz,
                                                 const int32_t *__restrict__ tgt_perm, int64_t N,
                                                 const double *__restrict__ M, int64_t n_nodes, int F,
                                                 const __bf16 *__restrict__ Wt, const float *__restrict__ P,
                                                 const double *__restrict__ rule, int nrule, double *__restrict__ u)
{
    constexpr bool NET = MODE == kBandMLP;
    constexpr int KP0 = 32, NPL = 16;  // padded input and output widths
    __shared__ __align__(16) __bf16 s_a[NET ? 64 * H : 8];
    __shared__ __align__(16) __bf16 s_b[NET ? 64 * H : 8];
    __shared__ float s_y[NET ? 64 * NPL : 1];
    const int lane = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = p < npairs;
    const int64_t pp = valid ? p : npairs - 1;
    const int s = pairs[2 * pp];
    const int64_t t = pairs[2 * pp + 1];
    const double x[3] = {tgt_xyz[s], tgt_xyz[N + s], tgt_xyz[2 * N + s]};
    double v[4][3];
    int64_t nd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        nd[q] = tet_node[(int64_t)q * T + t];
#pragma unroll
        for (int k = 0; k < 3; ++k) v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + t];
    }
    double coef[kOut];
    if constexpr (MODE == kBandExact) {
        TetGeom G;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k) G.v[q][k] = v[q][k];
        double gl[4][3], eh[6][3];
        tet_geometry(G, gl, eh);
        PairGeo PG;
        pair_geometry(x, G, PG);
#pragma unroll 1
        for (int j = 0; j < kOut; ++j) {
            double m[4][3] = {};
            m[j / 3][j % 3] = 1.0;
            TetField F1;
            tet_field(G, gl, eh, m, F1);
            coef[j] = pair_contract(PG, F1);
        }
    } else if constexpr (MODE == kBandGauss) {
        const double e[3][3] = {{v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]},
                                {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]},
                                {v[3][0] - v[0][0], v[3][1] - v[0][1], v[3][2] - v[0][2]}};
        const double vol6 = fabs(e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                                 e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                                 e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]));
        const double xv[3] = {x[0] - v[0][0], x[1] - v[0][1], x[2] - v[0][2]};
        double S[3] = {0.0, 0.0, 0.0}, K[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (int q = 0; q < nrule; ++q) {
            const double l1 = rule[4 * q], l2 = rule[4 * q + 1], l3 = rule[4 * q + 2], w = rule[4 * q + 3];
            double d[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) d[k] = xv[k] - (l1 * e[0][k] + l2 * e[1][k] + l3 * e[2][k]);
            const double ri = rsqrt_nr(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
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
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            coef[k] = vol6 * (S[k] - K[0][k] - K[1][k] - K[2][k]);
            coef[3 + k] = vol6 * K[0][k];
            coef[6 + k] = vol6 * K[1][k];
            coef[9 + k] = vol6 * K[2][k];
        }
    } else {
        double c[3], diam, vh;
        tet_scales(v, c, diam, vh);
        quad_coeffs(x, v, c, coef);
        if constexpr (NET) {
            const Layout L(H);
            const double dist =
                sqrt((x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) + (x[2] - c[2]) * (x[2] - c[2]));
            const double rho = dist / diam;
            __bf16 *row = s_a + lane * KP0;
            double fin[kIn];
            sur_features(x, v, c, diam, fin);
            static_assert(2 * kIn <= KP0, "hi and lo parts of every input fit one matrix-core step");
#pragma unroll
            for (int j = 0; j < kIn; ++j) {
                const float sj = (float)fin[j];
                const __bf16 hi = (__bf16)sj;
                row[j] = hi;
                row[kIn + j] = (__bf16)(sj - (float)hi);
            }
#pragma unroll
            for (int j = 2 * kIn; j < KP0; ++j) row[j] = (__bf16)0.f;
            __syncthreads();
            mlp_layer<KP0, H, false>(s_a, Wt, P + L.b[0], H, s_b, nullptr, lane);
            __syncthreads();
            mlp_layer<H, H, false>(s_b, Wt + H * KP0, P + L.b[1], H, s_a, nullptr, lane);
            __syncthreads();
            mlp_layer<H, H, false>(s_a, Wt + H * KP0 + H * H, P + L.b[2], H, s_b, nullptr, lane);
            __syncthreads();
            mlp_layer<H, NPL, true>(s_b, Wt + H * KP0 + 2 * H * H, P + L.b[3], kOut, nullptr, s_y, lane);
            __syncthreads();
            const double rho2 = rho * rho;
            const double g = 4.0 * 3.141592653589793 * diam * vh / (kYScale * rho2 * rho2);
#pragma unroll
            for (int j = 0; j < kOut; ++j) coef[j] = fma(g, (double)s_y[lane * NPL + j], coef[j]);
        }
    }
    // contraction with every field, one sum per run of equal targets
    const int key = valid ? s : -1 - lane;
    const int knext = __shfl_down(key, 1);
    const bool tail = valid && (lane == 63 || knext != key);
    const int64_t o = tgt_perm[s];
#pragma unroll 1
    for (int f = 0; f < F; ++f) {
        const double *Mf = M + (int64_t)f * n_nodes * 3;
        double val = 0.0;
        if (valid) {
#pragma unroll
            for (int j = 0; j < kOut; ++j) val = fma(coef[j], Mf[3 * nd[j / 3] + j % 3], val);
            val *= kInv4Pi;
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double vo = __shfl_up(val, d);
            const int ko = __shfl_up(key, d);
            if (lane >= d && ko == key) val += vo;
        }
        if (tail) atomicAdd(&u[(int64_t)f * N + o], val);
    }
}

}  // namespace

int surrogate_param_count(int H) { return (H == 32 || H == 64 || H == 128) ? (int)Layout(H).n : -1; }

void surrogate_set(DevicePlan &dp, int H, const std::vector<float> &params)
{
    const Layout L(H);
    if (params.size() != L.n) throw DeviceError{"surrogate parameter count does not match the width"};
    if (H != 32 && H != 64 && H != 128) throw DeviceError{"surrogate width must be 32, 64 or 128"};
    if (dp.sur_w) (void)hipFree(dp.sur_w);
    if (dp.sur_wb) (void)hipFree(dp.sur_wb);
    dp.sur_w = nullptr;
    dp.sur_wb = nullptr;
    hip_check(hipMalloc(&dp.sur_w, sizeof(float) * L.n), "hipMalloc surrogate");
    hip_check(hipMemcpy(dp.sur_w, params.data(), sizeof(float) * L.n, hipMemcpyHostToDevice), "hipMemcpy surrogate");
    // BF16 weights, transposed and padded: [H][32], [H][H], [H][H], [16][H]
    const size_t nb = (size_t)H * 32 + 2 * (size_t)H * H + 16 * (size_t)H;
    hip_check(hipMalloc(&dp.sur_wb, sizeof(__bf16) * nb), "hipMalloc surrogate");
    __bf16 *o = reinterpret_cast<__bf16 *>(dp.sur_wb);
    const int KP[4] = {32, H, H, H}, NP[4] = {H, H, H, 16};
    for (int l = 0; l < 4; ++l) {
        const int n = NP[l] * KP[l];
        k_f32_to_bf16_t<<<(n + 255) / 256, 256>>>(dp.sur_w + L.w[l], L.K(l), L.N(l), KP[l], NP[l], l == 0 ? 1 : 0, o);
        o += n;
    }
    hip_check(hipGetLastError(), "surrogate upload launch");
    hip_check(hipDeviceSynchronize(), "surrogate upload");
    dp.sur_hidden = H;
    ++dp.schedule_gen;  // a captured graph may hold the old weights
}

void surrogate_grad(int H, const float *params, const float *X, const float *Y, int B, float *grad, double *loss)
{
    const Layout L(H);
    Work w;
    w.alloc(H, B, L.n);
    float *P = nullptr;
    hip_check(hipMalloc(&P, sizeof(float) * L.n), "hipMalloc surrogate");
    try {
        hip_check(hipMemcpy(P, params, sizeof(float) * L.n, hipMemcpyHostToDevice), "hipMemcpy");
        hip_check(hipMemcpy(w.X, X, sizeof(float) * B * kIn, hipMemcpyHostToDevice), "hipMemcpy");
        hip_check(hipMemcpy(w.Yt, Y, sizeof(float) * B * kOut, hipMemcpyHostToDevice), "hipMemcpy");
        hip_check(hipMemset(w.loss, 0, sizeof(double)), "hipMemset");
        forward_backward(L, P, w, nullptr);
        hip_check(hipMemcpy(grad, w.grad, sizeof(float) * L.n, hipMemcpyDeviceToHost), "hipMemcpy");
        hip_check(hipMemcpy(loss, w.loss, sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
    } catch (...) {
        (void)hipFree(P);
        throw;
    }
    (void)hipFree(P);
}

void surrogate_samples(DevicePlan &dp, uint64_t seed, int n, float *X, float *Y)
{
    build_band_list(dp, nullptr);
    float *dX = nullptr, *dY = nullptr;
    hip_check(hipMalloc(&dX, sizeof(float) * n * kIn), "hipMalloc");
    if (hipMalloc(&dY, sizeof(float) * n * kOut) != hipSuccess) {
        (void)hipFree(dX);
        throw DeviceError{"hipMalloc failed"};
    }
    k_sur_gen<<<(n + 63) / 64, 64>>>(dp.tet_xyz, dp.hp.n_tets, dp.band_pairs, dp.n_band_pairs, dp.tgt_xyz,
                                     dp.hp.n_targets, seed, n, dX, dY);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(X, dX, sizeof(float) * n * kIn, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Y, dY, sizeof(float) * n * kOut, hipMemcpyDeviceToHost);
    (void)hipFree(dX);
    (void)hipFree(dY);
    hip_check(e, "surrogate samples");
}

double surrogate_train(DevicePlan &dp, int H, int steps, int B, float lr, uint64_t seed, std::vector<float> &params)
{
    const Layout L(H);
    build_band_list(dp, nullptr);  // training pairs: the plan's own band pairs
    // He initialisation, biases zero
    params.assign(L.n, 0.f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < 4; ++l) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (float)L.K(l)));
        for (size_t i = 0; i < (size_t)L.K(l) * L.N(l); ++i) params[L.w[l] + i] = nd(rng);
    }
    Work w;
    w.alloc(H, B, L.n);
    float *P = nullptr, *m = nullptr, *v = nullptr;
    auto cleanup = [&]() {
        for (float *q : {P, m, v})
            if (q) (void)hipFree(q);
    };
    double last = 0.0;
    const int tail = std::max(1, steps / 20);
    try {
        hip_check(hipMalloc(&P, sizeof(float) * L.n), "hipMalloc");
        hip_check(hipMalloc(&m, sizeof(float) * L.n), "hipMalloc");
        hip_check(hipMalloc(&v, sizeof(float) * L.n), "hipMalloc");
        hip_check(hipMemcpy(P, params.data(), sizeof(float) * L.n, hipMemcpyHostToDevice), "hipMemcpy");
        hip_check(hipMemset(m, 0, sizeof(float) * L.n), "hipMemset");
        hip_check(hipMemset(v, 0, sizeof(float) * L.n), "hipMemset");
        hip_check(hipMemset(w.loss, 0, sizeof(double)), "hipMemset");
        for (int it = 0; it < steps; ++it) {
            if (it == steps - tail) {
                hip_check(hipMemset(w.loss, 0, sizeof(double)), "hipMemset");
            }
            k_sur_gen<<<(B + 63) / 64, 64>>>(dp.tet_xyz, dp.hp.n_tets, dp.band_pairs, dp.n_band_pairs, dp.tgt_xyz,
                                             dp.hp.n_targets, splitmix64(seed + 1 + (uint64_t)it), B, w.X, w.Yt);
            forward_backward(L, P, w, nullptr);
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.f - std::pow(b1, (float)(it + 1)), c2 = 1.f - std::pow(b2, (float)(it + 1));
            const float lrt = lr * (0.05f + 0.95f * 0.5f * (1.f + std::cos(3.14159265f * (float)it / (float)steps)));
            k_adam<<<(unsigned)((L.n + 255) / 256), 256>>>(P, w.grad, m, v, (int64_t)L.n, lrt, b1, b2, c1, c2);
            hip_check(hipGetLastError(), "surrogate training launch");
        }
        hip_check(hipMemcpy(&last, w.loss, sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
        hip_check(hipMemcpy(params.data(), P, sizeof(float) * L.n, hipMemcpyDeviceToHost), "hipMemcpy");
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    surrogate_set(dp, H, params);
    return last / (double)tail;
}

namespace {
__global__ void k_zero(double *__restrict__ a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}
}  // namespace

void build_band_list(DevicePlan &dp, hipStream_t st)
{
    if (dp.band_built) return;
    const HostPlan &hp = dp.hp;
    const int nblk = dp.n_p2p_blk;
    std::vector<int64_t> cnt((size_t)std::max(nblk, 1), 0), off((size_t)std::max(nblk, 1) + 1, 0);
    int64_t *dcnt = nullptr;
    hip_check(hipMalloc(&dcnt, sizeof(int64_t) * (cnt.size() + 1)), "hipMalloc band counts");
    try {
        if (nblk > 0) {
            k_band_count<<<nblk, kBandThreads, 0, st>>>(dp.p2p_blk, nblk, hp.n_tets, dp.tet_xyz, dp.p2p_idx, dp.tgt_xyz,
                                                        hp.n_targets, dcnt);
            hip_check(hipGetLastError(), "k_band_count launch");
            hip_check(hipMemcpyAsync(cnt.data(), dcnt, sizeof(int64_t) * nblk, hipMemcpyDeviceToHost, st),
                      "hipMemcpy band counts");
            hip_check(hipStreamSynchronize(st), "band counts");
        }
        for (int b = 0; b < nblk; ++b) off[b + 1] = off[b] + cnt[b];
        const int64_t n = off[nblk > 0 ? nblk : 0];
        int32_t *pairs = nullptr;
        const hipError_t e = hipMalloc(&pairs, sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(n, 1));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw PlanError{TFMM_ENOMEM, "band pair list: device memory exhausted (" + std::to_string(n) + " pairs)"};
        }
        dp.band_pairs = pairs;
        dp.n_band_pairs = n;
        dp.device_bytes += (int64_t)(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(n, 1));
        if (nblk > 0 && n > 0) {
            hip_check(hipMemcpyAsync(dcnt, off.data(), sizeof(int64_t) * nblk, hipMemcpyHostToDevice, st),
                      "hipMemcpy band offsets");
            k_band_fill<<<nblk, kBandThreads, 0, st>>>(dp.p2p_blk, nblk, hp.n_tets, dp.tet_xyz, dp.p2p_idx, dp.tgt_xyz,
                                                       hp.n_targets, dcnt, dp.band_pairs);
            hip_check(hipGetLastError(), "k_band_fill launch");
        }
        int nr = 0;
        std::vector<double> rule = simplex_rule(5, &nr);  // the Gauss control: 27 points, degree 5
        hip_check(hipMalloc(&dp.band_rule, sizeof(double) * rule.size()), "hipMalloc band rule");
        hip_check(hipMemcpyAsync(dp.band_rule, rule.data(), sizeof(double) * rule.size(), hipMemcpyHostToDevice, st),
                  "hipMemcpy band rule");
        dp.n_band_rule = nr;
        hip_check(hipStreamSynchronize(st), "band list");
    } catch (...) {
        (void)hipFree(dcnt);
        throw;
    }
    (void)hipFree(dcnt);
    dp.band_built = true;
    ++dp.schedule_gen;
}

void run_band_pairs(DevicePlan &dp, int mode, const double *M, int32_t F, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    if (!dp.band_built) throw DeviceError{"band pair list not built"};
    const int64_t n = dp.n_band_pairs;
    if (n == 0) return;
    const unsigned grid = (unsigned)((n + 63) / 64);
    const __bf16 *Wt = reinterpret_cast<const __bf16 *>(dp.sur_wb);
#define TFMM_BAND(MODE, H)                                                                                          \
    k_band_eval<MODE, H><<<grid, 64, 0, st>>>(dp.band_pairs, n, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.tgt_xyz,     \
                                             dp.tgt_perm, hp.n_targets, M, hp.n_nodes, F, Wt, dp.sur_w, dp.band_rule, \
                                             dp.n_band_rule, u)
    switch (mode) {
    case kBandMLP:
        if (!dp.sur_wb) throw DeviceError{"no surrogate attached"};
        if (dp.sur_hidden == 32)
            TFMM_BAND(kBandMLP, 32);
        else if (dp.sur_hidden == 64)
            TFMM_BAND(kBandMLP, 64);
        else
            TFMM_BAND(kBandMLP, 128);
        break;
    case kBandGauss: TFMM_BAND(kBandGauss, 32); break;
    case kBandQuad: TFMM_BAND(kBandQuad, 32); break;
    default: TFMM_BAND(kBandExact, 32); break;
    }
#undef TFMM_BAND
    hip_check(hipGetLastError(), "k_band_eval launch");
}

void run_band(DevicePlan &dp, bool use_sur, const double *M, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    if (use_sur && !dp.sur_wb) throw DeviceError{"no surrogate attached"};
    build_band_list(dp, st);
    k_zero<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>((hp.n_targets + 255) / 256, 65536)), 256, 0, st>>>(
        u, hp.n_targets);
    run_band_pairs(dp, use_sur ? kBandMLP : kBandExact, M, 1, u, st);
}

}  // namespace tfmm
