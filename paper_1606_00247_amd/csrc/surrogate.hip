// Learned surrogate of the near-field pair integral at intermediate distance.
//
// For a tet T (corners v_i, diameter = longest edge, centroid c, volume V) and
// a target x with 2 <= rho = |x - c| / diam < 6 the potential is linear in the
// nodal magnetisation and homogeneous of degree one in length:
//   u_T(x) = diam * sum_{i,a} C_ia M_ia,
// C a function of the corners seen from the target.  A multilayer perceptron
// maps the 12 inputs s_i = (v_i - x) / |x - c| (scale free, O(1)) to
// y = 16 pi C rho^2 / Vh (Vh = V / diam^3; the dipole term of y is the unit
// vector from c to x, so y is O(1)); the 12 outputs are contracted with the
// 4 nodal M exactly.  Layers 12 -> H -> H -> H -> 12
// with ReLU.  Training pairs are drawn from the plan's tets with uniform
// directions and rho uniform in [2, 6); their targets come from the exact
// pair integral (unit nodal fields).  Training runs in FP32 (Adam);
// inference uses BF16 weights and activations on matrix cores with FP32
// accumulation.
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

constexpr double kBandLo = 2.0, kBandHi = 6.0;
constexpr int kIn = 12, kOut = 12;
constexpr double kYScale = 16.0 * 3.141592653589793;  // y = kYScale C rho^2 / Vh

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

// One training sample per thread: inputs X [n][12], targets Y [n][12].
__global__ void k_sur_gen(const double *__restrict__ tet_xyz, int64_t T, uint64_t seed, int n, float *__restrict__ X,
                          float *__restrict__ Y)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t h0 = splitmix64(seed ^ splitmix64((uint64_t)s));
    const uint64_t h1 = splitmix64(h0), h2 = splitmix64(h1), h3 = splitmix64(h2);
    const int64_t t = (int64_t)(h0 % (uint64_t)T);
    TetGeom G;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) G.v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + t];
    double c[3], diam, vh;
    tet_scales(G.v, c, diam, vh);
    const double zc = 2.0 * u01(h1) - 1.0, ph = 6.283185307179586 * u01(h2);
    const double sr = sqrt(fmax(0.0, 1.0 - zc * zc));
    const double rho = kBandLo + (kBandHi - kBandLo) * u01(h3);
    const double x[3] = {c[0] + rho * diam * sr * cos(ph), c[1] + rho * diam * sr * sin(ph), c[2] + rho * diam * zc};
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
    const double scale = kYScale * kInv4Pi / diam * rho * rho / vh;
    const double dist = rho * diam;
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
        X[(int64_t)s * kIn + j] = (float)((G.v[j / 3][j % 3] - x[j % 3]) / dist);
        Y[(int64_t)s * kOut + j] = (float)(acc[j] * scale);
    }
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

__global__ void k_f32_to_bf16_t(const float *__restrict__ W, int K, int N, int KP, int NP, __bf16 *__restrict__ out)
{
    // out [NP][KP] = W^T, zero padded
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP * KP) return;
    const int n = i / KP, k = i % KP;
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
// Band potential over the near-field pairs of a plan (one field): pairs with
// 2 <= rho < 6 only, by the exact integral (SUR = false) or by the network
// (SUR = true).  One wavefront per P2P block; tets staged 16 at a time.
// ---------------------------------------------------------------------------
constexpr int kBandStage = 16;

__global__ void k_zero(double *__restrict__ a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x4 = float __attribute__((ext_vector_type(4)));

struct BandTet {
    double v[4][3];
    double m[4][3];
    double c[3];
    double diam, vh;
};

// One dense layer of the network for the 64 rows (pairs) of a wavefront:
// out [64][NP] = act(in [64][KP] W + b), W as [NP][KP] BF16 (transposed,
// zero padded) in global memory, activations BF16 in LDS.
template <int KP, int NP, bool LAST>
__device__ __forceinline__ void mlp_layer(const __bf16 *in, const __bf16 *__restrict__ Wt, const float *__restrict__ b,
                                          int N, __bf16 *out, float *outf, int lane)
{
#pragma unroll 1
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
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

template <bool SUR, int H>
__global__ __launch_bounds__(64) void k_band(const int32_t *__restrict__ blk, int nblk, int64_t T,
                                            const double *__restrict__ tet_xyz, const int32_t *__restrict__ tet_node,
                                            const int32_t *__restrict__ idx, const double *__restrict__ tgt_xyz,
                                            const int32_t *__restrict__ tgt_perm, int64_t N,
                                            const double *__restrict__ M, const __bf16 *__restrict__ Wt,
                                            const float *__restrict__ P, double *__restrict__ u)
{
    constexpr int KP0 = 32, NPL = 16;  // padded input and output widths
    __shared__ BandTet s_t[kBandStage];
    __shared__ TetGeom s_g[SUR ? 1 : kBandStage];
    __shared__ TetField s_f[SUR ? 1 : kBandStage];
    __shared__ __align__(16) __bf16 s_a[SUR ? 64 * H : 8];
    __shared__ __align__(16) __bf16 s_b[SUR ? 64 * H : 8];
    __shared__ float s_y[SUR ? 64 * NPL : 1];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int tb = blk[4 * b], te = blk[4 * b + 1], ib = blk[4 * b + 2], ie = blk[4 * b + 3];
    const int lane = threadIdx.x;
    const Layout L(H);
    for (int sb = tb; sb < te; sb += kBandStage) {
        const int nt = min(kBandStage, te - sb);
        __syncthreads();
        if (lane < nt) {
            const int64_t t = sb + lane;
            BandTet &B = s_t[lane];
            for (int q = 0; q < 4; ++q) {
                const int64_t nd = tet_node[(int64_t)q * T + t];
                for (int k = 0; k < 3; ++k) {
                    B.v[q][k] = tet_xyz[(int64_t)(3 * q + k) * T + t];
                    B.m[q][k] = M[3 * nd + k];
                }
            }
            tet_scales(B.v, B.c, B.diam, B.vh);
            if constexpr (!SUR) tet_prepare(tet_xyz, tet_node, T, t, M, &s_g[lane], s_f[lane]);
        }
        __syncthreads();
        // every lane of the wavefront takes part in every round (matrix cores)
        for (int i0 = ib; i0 < ie; i0 += 64) {
            const int i = i0 + lane;
            const bool valid = i < ie;
            const int s = valid ? idx[i] : idx[ib];
            const double x[3] = {tgt_xyz[s], tgt_xyz[N + s], tgt_xyz[2 * N + s]};
            double acc = 0.0;
            for (int t = 0; t < nt; ++t) {
                const BandTet &B = s_t[t];
                const double dx = x[0] - B.c[0], dy = x[1] - B.c[1], dz = x[2] - B.c[2];
                const double rho = sqrt(dx * dx + dy * dy + dz * dz) / B.diam;
                const bool band = valid && rho >= kBandLo && rho < kBandHi;
                if constexpr (!SUR) {
                    if (band) {
                        double a1[1] = {0.0};
                        pair_accumulate<1>(x, s_g[t], &s_f[t], a1);
                        acc += a1[0] * kInv4Pi;
                    }
                } else {
                    __bf16 *row = s_a + lane * KP0;
                    const double dist = rho * B.diam;
#pragma unroll
                    for (int j = 0; j < KP0; ++j)
                        row[j] = (__bf16)(j < kIn ? (float)((B.v[j / 3][j % 3] - x[j % 3]) / dist) : 0.f);
                    __syncthreads();
                    mlp_layer<KP0, H, false>(s_a, Wt, P + L.b[0], H, s_b, nullptr, lane);
                    __syncthreads();
                    mlp_layer<H, H, false>(s_b, Wt + H * KP0, P + L.b[1], H, s_a, nullptr, lane);
                    __syncthreads();
                    mlp_layer<H, H, false>(s_a, Wt + H * KP0 + H * H, P + L.b[2], H, s_b, nullptr, lane);
                    __syncthreads();
                    mlp_layer<H, NPL, true>(s_b, Wt + H * KP0 + 2 * H * H, P + L.b[3], kOut, nullptr, s_y, lane);
                    __syncthreads();
                    if (band) {
                        double v = 0.0;
#pragma unroll
                        for (int j = 0; j < kOut; ++j) v += (double)s_y[lane * NPL + j] * B.m[j / 3][j % 3];
                        acc += v * B.diam * B.vh / (kYScale * rho * rho);
                    }
                    __syncthreads();
                }
            }
            if (valid && acc != 0.0) atomicAdd(&u[tgt_perm[s]], acc);
        }
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
        k_f32_to_bf16_t<<<(n + 255) / 256, 256>>>(dp.sur_w + L.w[l], L.K(l), L.N(l), KP[l], NP[l], o);
        o += n;
    }
    hip_check(hipGetLastError(), "surrogate upload launch");
    hip_check(hipDeviceSynchronize(), "surrogate upload");
    dp.sur_hidden = H;
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
    float *dX = nullptr, *dY = nullptr;
    hip_check(hipMalloc(&dX, sizeof(float) * n * kIn), "hipMalloc");
    if (hipMalloc(&dY, sizeof(float) * n * kOut) != hipSuccess) {
        (void)hipFree(dX);
        throw DeviceError{"hipMalloc failed"};
    }
    k_sur_gen<<<(n + 63) / 64, 64>>>(dp.tet_xyz, dp.hp.n_tets, seed, n, dX, dY);
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
            k_sur_gen<<<(B + 63) / 64, 64>>>(dp.tet_xyz, dp.hp.n_tets, splitmix64(seed + 1 + (uint64_t)it), B, w.X, w.Yt);
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

void run_band(DevicePlan &dp, bool use_sur, const double *M, double *u, hipStream_t st)
{
    const HostPlan &hp = dp.hp;
    const unsigned n = (unsigned)dp.n_p2p_blk;
    k_zero<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>((hp.n_targets + 255) / 256, 65536)), 256, 0, st>>>(
        u, hp.n_targets);
    if (n == 0) return;
    if (!use_sur) {
        k_band<false, 32><<<n, 64, 0, st>>>(dp.p2p_blk, (int)n, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx,
                                            dp.tgt_xyz, dp.tgt_perm, hp.n_targets, M, nullptr, nullptr, u);
    } else {
        if (!dp.sur_wb) throw DeviceError{"no surrogate loaded"};
        const __bf16 *Wt = reinterpret_cast<const __bf16 *>(dp.sur_wb);
        switch (dp.sur_hidden) {
        case 32:
            k_band<true, 32><<<n, 64, 0, st>>>(dp.p2p_blk, (int)n, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx,
                                               dp.tgt_xyz, dp.tgt_perm, hp.n_targets, M, Wt, dp.sur_w, u);
            break;
        case 64:
            k_band<true, 64><<<n, 64, 0, st>>>(dp.p2p_blk, (int)n, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx,
                                               dp.tgt_xyz, dp.tgt_perm, hp.n_targets, M, Wt, dp.sur_w, u);
            break;
        default:
            k_band<true, 128><<<n, 64, 0, st>>>(dp.p2p_blk, (int)n, hp.n_tets, dp.tet_xyz, dp.tet_node, dp.p2p_idx,
                                                dp.tgt_xyz, dp.tgt_perm, hp.n_targets, M, Wt, dp.sur_w, u);
            break;
        }
    }
    hip_check(hipGetLastError(), "k_band launch");
}

}  // namespace tfmm
