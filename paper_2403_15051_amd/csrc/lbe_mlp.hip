// Network of the learned warm start (not part of the paper's method): a multilayer perceptron
// 6 -> 256 -> 256 -> 256 -> 256 -> 5 with SiLU hidden activations and a linear output, trained by
// mean-squared error with Adam.  Every matrix product is one tiled kernel on the matrix cores:
// BF16 operands with FP32 accumulation (v_mfma_f32_16x16x32_bf16), or FP32 operands
// (v_mfma_f32_16x16x4_f32) for checks; activations, gradients, master weights and Adam moments
// are FP32.  Parameters are packed layer by layer as W [fan_out][fan_in] (row-major), b [fan_out].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbe_internal.h"

namespace {

constexpr int kNL = 5;
constexpr int kFanIn[kNL] = {6, 256, 256, 256, 256};
constexpr int kFanOut[kNL] = {256, 256, 256, 256, 5};
constexpr int kIn = 6, kOut = 5, kHid = 256;

constexpr int64_t weight_off(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; k++) o += (int64_t)kFanIn[k] * kFanOut[k] + kFanOut[k];
    return o;
}
constexpr int64_t bias_off(int l) { return weight_off(l) + (int64_t)kFanIn[l] * kFanOut[l]; }
constexpr int64_t kParams = weight_off(kNL);
static_assert(kParams == 200453, "parameter count");

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

enum Epi { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_DSILU = 3 };

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 4;

__device__ inline float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

// C[M][N] (row stride ldc) = epilogue(sum_k A(m, k) B(k, n)), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn].  Tile 64 x 64 per workgroup of four waves, each wave 32 x 32 as
// 2 x 2 MFMA tiles of 16 x 16; K staged in LDS 32 at a time (zero-filled past M, N, K).
// Epilogues: store; + bias then SiLU (pre-activation to Zout); + bias; times SiLU'(Zin).
// With gridDim.z > 1 (plain store only) workgroup z sums the z-th of gridDim.z K ranges into
// C + z M ldc, to be summed by k_splitk_sum.
template <bool BF16, int EPI>
__global__ void __launch_bounds__(256)
    k_gemm(int M, int N, int K, const float* __restrict__ A, long sam, long sak, const float* __restrict__ B,
           long sbk, long sbn, float* __restrict__ C, int ldc, const float* __restrict__ bias,
           float* __restrict__ Zout, const float* __restrict__ Zin)
{
    __shared__ float As[BM][LDK];  // [m][k]
    __shared__ float Bs[BN][LDK];  // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const bool a_kfast = sak == 1, b_kfast = sbk == 1;
    const int kper = ((K + gridDim.z - 1) / gridDim.z + BK - 1) / BK * BK;
    const int kbeg = blockIdx.z * kper, kend = min(K, kbeg + kper);
    if (gridDim.z > 1) C += (long)blockIdx.z * M * ldc;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        for (int e = tid; e < BM * BK; e += 256) {
            // walk the staged tile along whichever index is contiguous in memory
            int r, kk;
            if (a_kfast) { r = e / BK; kk = e % BK; } else { kk = e / BM; r = e % BM; }
            const int m = m0 + r, k = k0 + kk;
            As[r][kk] = (m < M && k < kend) ? A[(long)m * sam + (long)k * sak] : 0.f;
            if (b_kfast) { r = e / BK; kk = e % BK; } else { kk = e / BN; r = e % BN; }
            const int n = n0 + r, k2 = k0 + kk;
            Bs[r][kk] = (n < N && k2 < kend) ? B[(long)k2 * sbk + (long)n * sbn] : 0.f;
        }
        __syncthreads();
        if constexpr (BF16) {
            const int kq = 8 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < 2; i++) {
                v8bf a;
                const int ra = wm + 16 * i + (lane & 15);
#pragma unroll
                for (int q = 0; q < 8; q++) a[q] = (__bf16)As[ra][kq + q];
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    v8bf b;
                    const int cb = wn + 16 * j + (lane & 15);
#pragma unroll
                    for (int q = 0; q < 8; q++) b[q] = (__bf16)Bs[cb][kq + q];
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int kk = k4 + (lane >> 4);
#pragma unroll
                for (int i = 0; i < 2; i++) {
                    const float a = As[wm + 16 * i + (lane & 15)][kk];
#pragma unroll
                    for (int j = 0; j < 2; j++) {
                        const float b = Bs[wn + 16 * j + (lane & 15)][kk];
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= M || n >= N) continue;
                const long o = (long)m * ldc + n;
                float v = acc[i][j][r];
                if constexpr (EPI == EPI_BIAS_SILU) {
                    const float z = v + bias[n];
                    Zout[o] = z;
                    v = z * sigmoidf(z);
                } else if constexpr (EPI == EPI_BIAS) {
                    v += bias[n];
                } else if constexpr (EPI == EPI_DSILU) {
                    const float z = Zin[o];
                    const float s = sigmoidf(z);
                    v *= s * (1.0f + z * (1.0f - s));
                }
                C[o] = v;
            }
}

// C[m][n] = sum over z < nz of P[z][m][n] (fixed order), P of row stride N.
__global__ void __launch_bounds__(256) k_splitk_sum(int M, int N, int nz, const float* __restrict__ P,
                                                    float* __restrict__ C, int ldc)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= M * N) return;
    float s = 0.f;
    for (int z = 0; z < nz; z++) s += P[(long)z * M * N + e];
    C[(long)(e / N) * ldc + e % N] = s;
}

// out[n] = sum over rows of D[m][n] (fixed order: four interleaved row groups, then their sum).
__global__ void __launch_bounds__(256) k_colsum(int M, int N, const float* __restrict__ D, int ld,
                                                float* __restrict__ out)
{
    __shared__ double part[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    double s = 0;
    if (n < N)
        for (int m = g; m < M; m += 4) s += D[(long)m * ld + n];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N) out[n] = (float)(((part[0][c] + part[1][c]) + part[2][c]) + part[3][c]);
}

// Mean-squared error over R x kOut and its derivative; loss[0] = this batch's mean, loss[1] += its
// sum (one workgroup, fixed-order tree).
__global__ void __launch_bounds__(256) k_loss(int R, const float* __restrict__ Y, const float* __restrict__ T,
                                              float* __restrict__ dY, double* __restrict__ loss)
{
    __shared__ double red[256];
    const int n = R * kOut;
    const float sc = 2.0f / (float)n;
    double s = 0;
    for (int e = threadIdx.x; e < n; e += 256) {
        const float d = Y[e] - T[e];
        dY[e] = sc * d;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = red[0] / n;
        loss[1] += red[0];
    }
}

__global__ void __launch_bounds__(256) k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1 - b1) * gi;
    const float vi = b2 * v[i] + (1 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

struct Norm5 {
    float mean[kOut], inv[kOut];
};

// Minibatch rows j = (a (off + i) + b) mod N of the data set (an affine permutation per epoch),
// targets standardised.
__global__ void __launch_bounds__(256) k_gather(int64_t N, uint64_t a, uint64_t b, int64_t off, int rows,
                                                const float* __restrict__ X, const float* __restrict__ T, Norm5 nm,
                                                float* __restrict__ Xb, float* __restrict__ Tb)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    const uint64_t j = (uint64_t)((((unsigned __int128)a * (uint64_t)(off + i)) + b) % (uint64_t)N);
#pragma unroll
    for (int c = 0; c < kIn; c++) Xb[(long)i * kIn + c] = X[j * kIn + c];
#pragma unroll
    for (int c = 0; c < kOut; c++) Tb[(long)i * kOut + c] = (T[j * kOut + c] - nm.mean[c]) * nm.inv[c];
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxSplit = 8;

uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

struct lbe_mlp {
    int gemm = LBE_GEMM_BF16;
    int max_rows = 0;
    hipStream_t stream = nullptr;
    float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
    float *Z[4] = {}, *H[4] = {};
    float *Y = nullptr, *dY = nullptr, *dA = nullptr, *dB = nullptr, *Xb = nullptr, *Tb = nullptr;
    float* split = nullptr;  // partial sums of split-K products [kMaxSplit][256][256]
    double* loss = nullptr;
    double out_mean[kOut] = {0, 0, 0, 0, 0};
    double out_scale[kOut] = {1, 1, 1, 1, 1};
    int64_t t = 0;  // Adam steps taken
    std::string err;
};

namespace {

size_t mlp_bytes(int rows)
{
    const size_t F = sizeof(float), R = (size_t)rows;
    return 4 * a256(kParams * F) + 8 * a256(R * kHid * F) + 2 * a256(R * kOut * F) + 2 * a256(R * kHid * F) +
           a256(R * kIn * F) + a256(R * kOut * F) + a256(2 * sizeof(double)) +
           a256((size_t)kMaxSplit * kHid * kHid * F);
}

lbe_status merr(lbe_mlp* m, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LBE_OK;
    if (m) m->err = std::string(what) + ": " + hipGetErrorString(e);
    return LBE_EDEVICE;
}

template <bool BF16, int EPI>
hipError_t gemm_t(hipStream_t s, int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk,
                  long sbn, float* C, int ldc, const float* bias, float* Zout, const float* Zin, int nz = 1)
{
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, nz);
    hipLaunchKernelGGL((k_gemm<BF16, EPI>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias,
                       Zout, Zin);
    return hipGetLastError();
}

hipError_t gemm(const lbe_mlp* m, hipStream_t s, int epi, int M, int N, int K, const float* A, long sam, long sak,
                const float* B, long sbk, long sbn, float* C, int ldc, const float* bias = nullptr,
                float* Zout = nullptr, const float* Zin = nullptr)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const bool bf = m->gemm == LBE_GEMM_BF16;
    // long-K products with few output tiles (the weight gradients) are split over K
    const int tiles = ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
    int nz = 1;
    if (epi == EPI_STORE && tiles < 64 && (size_t)M * N <= (size_t)kHid * kHid)
        nz = std::max(1, std::min(kMaxSplit, K / 256));
    if (nz > 1) {
        hipError_t e = bf ? gemm_t<true, EPI_STORE>(s, M, N, K, A, sam, sak, B, sbk, sbn, m->split, N, nullptr,
                                                     nullptr, nullptr, nz)
                          : gemm_t<false, EPI_STORE>(s, M, N, K, A, sam, sak, B, sbk, sbn, m->split, N, nullptr,
                                                      nullptr, nullptr, nz);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_splitk_sum, dim3((M * N + 255) / 256), dim3(256), 0, s, M, N, nz, m->split, C, ldc);
        return hipGetLastError();
    }
#define LBE_GEMM_CASE(E)                                                                                   \
    case E:                                                                                                \
        return bf ? gemm_t<true, E>(s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Zout, Zin)         \
                  : gemm_t<false, E>(s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Zout, Zin);
    switch (epi) {
        LBE_GEMM_CASE(EPI_STORE)
        LBE_GEMM_CASE(EPI_BIAS_SILU)
        LBE_GEMM_CASE(EPI_BIAS)
        LBE_GEMM_CASE(EPI_DSILU)
    }
#undef LBE_GEMM_CASE
    return hipErrorInvalidValue;
}

// Forward pass of `rows` <= max_rows input rows X [rows][6]; outputs (standardised targets) in m->Y.
hipError_t forward(lbe_mlp* m, const float* X, int rows, hipStream_t s)
{
    const float* P = m->params;
    hipError_t e = gemm(m, s, EPI_BIAS_SILU, rows, kHid, kIn, X, kIn, 1, P + weight_off(0), 1, kIn, m->H[0], kHid,
                        P + bias_off(0), m->Z[0]);
    for (int l = 1; l < 4 && e == hipSuccess; l++)
        e = gemm(m, s, EPI_BIAS_SILU, rows, kHid, kHid, m->H[l - 1], kHid, 1, P + weight_off(l), 1, kHid, m->H[l],
                 kHid, P + bias_off(l), m->Z[l]);
    if (e == hipSuccess)
        e = gemm(m, s, EPI_BIAS, rows, kOut, kHid, m->H[3], kHid, 1, P + weight_off(4), 1, kHid, m->Y, kOut,
                 P + bias_off(4));
    return e;
}

// Backward pass after forward() and k_loss (dY in m->dY): gradients of every layer in m->grads.
hipError_t backward(lbe_mlp* m, const float* X, int rows, hipStream_t s)
{
    const float* P = m->params;
    float* G = m->grads;
    auto colsum = [&](const float* D, int N, float* out) {
        hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64), dim3(256), 0, s, rows, N, D, N, out);
        return hipGetLastError();
    };
    // output layer: dW4 = dY^T H3, db4, dZ3 = (dY W4) * silu'(Z3)
    hipError_t e = gemm(m, s, EPI_STORE, kOut, kHid, rows, m->dY, 1, kOut, m->H[3], kHid, 1, G + weight_off(4), kHid);
    if (e == hipSuccess) e = colsum(m->dY, kOut, G + bias_off(4));
    float* dz = m->dA;
    float* other = m->dB;
    if (e == hipSuccess)
        e = gemm(m, s, EPI_DSILU, rows, kHid, kOut, m->dY, kOut, 1, P + weight_off(4), kHid, 1, dz, kHid, nullptr,
                 nullptr, m->Z[3]);
    for (int l = 3; l >= 1 && e == hipSuccess; l--) {
        e = gemm(m, s, EPI_STORE, kHid, kHid, rows, dz, 1, kHid, m->H[l - 1], kHid, 1, G + weight_off(l), kHid);
        if (e == hipSuccess) e = colsum(dz, kHid, G + bias_off(l));
        if (e == hipSuccess)
            e = gemm(m, s, EPI_DSILU, rows, kHid, kHid, dz, kHid, 1, P + weight_off(l), kHid, 1, other, kHid, nullptr,
                     nullptr, m->Z[l - 1]);
        std::swap(dz, other);
    }
    if (e == hipSuccess) e = gemm(m, s, EPI_STORE, kHid, kIn, rows, dz, 1, kHid, X, kIn, 1, G + weight_off(0), kIn);
    if (e == hipSuccess) e = colsum(dz, kHid, G + bias_off(0));
    return e;
}

hipError_t adam(lbe_mlp* m, float lr, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    m->t++;
    const float bc1 = (float)(1 - std::pow(0.9, (double)m->t)), bc2 = (float)(1 - std::pow(0.999, (double)m->t));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, s, kParams, m->params, m->grads,
                       m->am, m->av, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

Norm5 norm_of(const lbe_mlp* m)
{
    Norm5 n;
    for (int c = 0; c < kOut; c++) {
        n.mean[c] = (float)m->out_mean[c];
        n.inv[c] = (float)(1.0 / m->out_scale[c]);
    }
    return n;
}

}  // namespace

namespace lbe {

int mlp_max_rows(const lbe_mlp* m) { return m->max_rows; }
float* mlp_input(lbe_mlp* m) { return m->Xb; }
const float* mlp_output(const lbe_mlp* m) { return m->Y; }
void mlp_scaling(const lbe_mlp* m, double* mean, double* scale)
{
    for (int c = 0; c < kOut; c++) {
        mean[c] = m->out_mean[c];
        scale[c] = m->out_scale[c];
    }
}
hipError_t mlp_forward_rows(lbe_mlp* m, const float* X, int rows, hipStream_t s) { return forward(m, X, rows, s); }

}  // namespace lbe

extern "C" {

lbe_status lbe_mlp_query(int32_t max_rows, size_t* device_bytes, int64_t* n_params)
{
    if (max_rows < 1) return LBE_EINVAL;
    if (device_bytes) *device_bytes = mlp_bytes(max_rows);
    if (n_params) *n_params = kParams;
    return LBE_OK;
}

lbe_status lbe_mlp_init(int32_t max_rows, int32_t gemm_kind, void* device_ws, size_t ws_bytes, void* hip_stream,
                        lbe_mlp** out)
{
    if (!out || !device_ws || max_rows < 1 || (gemm_kind != LBE_GEMM_BF16 && gemm_kind != LBE_GEMM_FP32))
        return LBE_EINVAL;
    if (((uintptr_t)device_ws & 255) != 0) return LBE_EINVAL;
    *out = nullptr;
    if (ws_bytes < mlp_bytes(max_rows)) return LBE_ENOMEM;
    lbe_mlp* m = new (std::nothrow) lbe_mlp;
    if (!m) return LBE_ENOMEM;
    m->gemm = gemm_kind;
    m->max_rows = max_rows;
    m->stream = (hipStream_t)hip_stream;
    char* p = (char*)device_ws;
    auto take = [&](size_t bytes) {
        char* at = p;
        p += a256(bytes);
        return at;
    };
    const size_t F = sizeof(float), R = (size_t)max_rows;
    m->params = (float*)take(kParams * F);
    m->grads = (float*)take(kParams * F);
    m->am = (float*)take(kParams * F);
    m->av = (float*)take(kParams * F);
    for (int l = 0; l < 4; l++) {
        m->Z[l] = (float*)take(R * kHid * F);
        m->H[l] = (float*)take(R * kHid * F);
    }
    m->Y = (float*)take(R * kOut * F);
    m->dY = (float*)take(R * kOut * F);
    m->dA = (float*)take(R * kHid * F);
    m->dB = (float*)take(R * kHid * F);
    m->Xb = (float*)take(R * kIn * F);
    m->Tb = (float*)take(R * kOut * F);
    m->loss = (double*)take(2 * sizeof(double));
    m->split = (float*)take((size_t)kMaxSplit * kHid * kHid * F);
    hipError_t e = hipMemsetAsync(device_ws, 0, mlp_bytes(max_rows), m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        delete m;
        return LBE_EDEVICE;
    }
    *out = m;
    return LBE_OK;
}

lbe_status lbe_mlp_init_params(lbe_mlp* m, uint64_t seed)
{
    if (!m) return LBE_EINVAL;
    std::vector<float> h(kParams, 0.f);
    uint64_t s = seed;
    for (int l = 0; l < kNL; l++) {
        const double a = std::sqrt(6.0 / (kFanIn[l] + kFanOut[l]));
        for (int64_t k = 0; k < (int64_t)kFanIn[l] * kFanOut[l]; k++) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            h[weight_off(l) + k] = (float)((2 * u - 1) * a);
        }
    }
    lbe_status st = merr(m, hipMemcpyAsync(m->params, h.data(), kParams * sizeof(float), hipMemcpyHostToDevice,
                                           m->stream),
                         "params");
    if (st == LBE_OK) st = merr(m, hipMemsetAsync(m->am, 0, kParams * sizeof(float), m->stream), "adam");
    if (st == LBE_OK) st = merr(m, hipMemsetAsync(m->av, 0, kParams * sizeof(float), m->stream), "adam");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(m->stream), "sync");
    m->t = 0;
    return st;
}

lbe_status lbe_mlp_set_params(lbe_mlp* m, const float* host, int64_t len)
{
    if (!m || !host || len != kParams) return LBE_EINVAL;
    lbe_status st = merr(m, hipMemcpyAsync(m->params, host, kParams * sizeof(float), hipMemcpyHostToDevice, m->stream),
                         "params");
    if (st == LBE_OK) st = merr(m, hipMemsetAsync(m->am, 0, kParams * sizeof(float), m->stream), "adam");
    if (st == LBE_OK) st = merr(m, hipMemsetAsync(m->av, 0, kParams * sizeof(float), m->stream), "adam");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(m->stream), "sync");
    m->t = 0;
    return st;
}

lbe_status lbe_mlp_get_params(lbe_mlp* m, float* host, int64_t cap)
{
    if (!m || !host || cap < kParams) return LBE_EINVAL;
    lbe_status st = merr(m, hipMemcpyAsync(host, m->params, kParams * sizeof(float), hipMemcpyDeviceToHost, m->stream),
                         "params");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(m->stream), "sync");
    return st;
}

lbe_status lbe_mlp_set_grads(lbe_mlp* m, const float* host, int64_t len)
{
    if (!m || !host || len != kParams) return LBE_EINVAL;
    lbe_status st = merr(m, hipMemcpyAsync(m->grads, host, kParams * sizeof(float), hipMemcpyHostToDevice, m->stream),
                         "grads");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(m->stream), "sync");
    return st;
}

lbe_status lbe_mlp_set_scaling(lbe_mlp* m, const double* mean, const double* scale)
{
    if (!m || !mean || !scale) return LBE_EINVAL;
    for (int c = 0; c < kOut; c++)
        if (!(scale[c] > 0) || !std::isfinite(mean[c])) return LBE_EINVAL;
    for (int c = 0; c < kOut; c++) {
        m->out_mean[c] = mean[c];
        m->out_scale[c] = scale[c];
    }
    return LBE_OK;
}

lbe_status lbe_mlp_get_scaling(lbe_mlp* m, double* mean, double* scale)
{
    if (!m || !mean || !scale) return LBE_EINVAL;
    lbe::mlp_scaling(m, mean, scale);
    return LBE_OK;
}

lbe_status lbe_mlp_forward(lbe_mlp* m, const float* dev_x, int32_t rows, float* dev_y)
{
    if (!m || !dev_x || !dev_y || rows < 0 || rows > m->max_rows) return LBE_EINVAL;
    if (rows == 0) return LBE_OK;
    lbe_status st = merr(m, forward(m, dev_x, rows, m->stream), "forward");
    if (st == LBE_OK)
        st = merr(m, hipMemcpyAsync(dev_y, m->Y, (size_t)rows * kOut * sizeof(float), hipMemcpyDeviceToDevice,
                                    m->stream),
                  "output copy");
    return st;
}

lbe_status lbe_mlp_loss_grad(lbe_mlp* m, const float* dev_x, const float* dev_t, int32_t rows, double* loss,
                             float* host_grad, int64_t cap)
{
    if (!m || !dev_x || !dev_t || rows < 1 || rows > m->max_rows) return LBE_EINVAL;
    if (host_grad && cap < kParams) return LBE_EINVAL;
    hipStream_t s = m->stream;
    lbe_status st = merr(m, forward(m, dev_x, rows, s), "forward");
    if (st == LBE_OK) {
        hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, rows, m->Y, dev_t, m->dY, m->loss);
        st = merr(m, hipGetLastError(), "loss");
    }
    if (st == LBE_OK) st = merr(m, backward(m, dev_x, rows, s), "backward");
    double lh[2] = {0, 0};
    if (st == LBE_OK)
        st = merr(m, hipMemcpyAsync(lh, m->loss, sizeof(lh), hipMemcpyDeviceToHost, s), "loss read");
    if (st == LBE_OK && host_grad)
        st = merr(m, hipMemcpyAsync(host_grad, m->grads, kParams * sizeof(float), hipMemcpyDeviceToHost, s),
                  "grad read");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(s), "sync");
    if (loss) *loss = lh[0];
    return st;
}

lbe_status lbe_mlp_adam_step(lbe_mlp* m, float lr)
{
    if (!m || !(lr > 0)) return LBE_EINVAL;
    lbe_status st = merr(m, adam(m, lr, m->stream), "adam");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(m->stream), "sync");
    return st;
}

lbe_status lbe_mlp_train(lbe_mlp* m, const float* dev_x, const float* dev_t, int64_t n, int32_t epochs, int32_t batch,
                         float lr, uint64_t seed, double* host_loss)
{
    if (!m || !dev_x || !dev_t || n < 2 || epochs < 1 || batch < 1 || batch > m->max_rows || !(lr > 0))
        return LBE_EINVAL;
    hipStream_t s = m->stream;
    // standardisation of the targets (per output, FP64 over the whole set)
    std::vector<float> th((size_t)n * kOut);
    lbe_status st = merr(m, hipMemcpyAsync(th.data(), dev_t, th.size() * sizeof(float), hipMemcpyDeviceToHost, s),
                         "target read");
    if (st == LBE_OK) st = merr(m, hipStreamSynchronize(s), "sync");
    if (st != LBE_OK) return st;
    for (int c = 0; c < kOut; c++) {
        double mu = 0, sq = 0;
        for (int64_t i = 0; i < n; i++) mu += th[(size_t)i * kOut + c];
        mu /= (double)n;
        for (int64_t i = 0; i < n; i++) {
            const double d = th[(size_t)i * kOut + c] - mu;
            sq += d * d;
        }
        const double sd = std::sqrt(sq / (double)n);
        m->out_mean[c] = mu;
        m->out_scale[c] = std::max(sd, 1e-6 * (std::fabs(mu) + 1e-3));
    }
    const Norm5 nm = norm_of(m);
    uint64_t rs = seed;
    const int64_t nb = (n + batch - 1) / batch;
    for (int ep = 0; ep < epochs && st == LBE_OK; ep++) {
        // affine permutation of the rows for this epoch
        uint64_t a = 1 + splitmix64(rs) % (uint64_t)(n - 1);
        while (gcd64(a, (uint64_t)n) != 1) a = 1 + (a % (uint64_t)(n - 1));
        const uint64_t b = splitmix64(rs) % (uint64_t)n;
        // learning rate: cosine from lr to lr / 10 over the epochs
        const float lr_e = (float)(lr * (0.55 + 0.45 * std::cos(M_PI * ep / (double)epochs)));
        st = merr(m, hipMemsetAsync(m->loss, 0, 2 * sizeof(double), s), "loss reset");
        for (int64_t k = 0; k < nb && st == LBE_OK; k++) {
            const int rows = (int)std::min<int64_t>(batch, n - k * batch);
            hipLaunchKernelGGL(k_gather, dim3((rows + 255) / 256), dim3(256), 0, s, n, a, b, k * batch, rows, dev_x,
                               dev_t, nm, m->Xb, m->Tb);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = forward(m, m->Xb, rows, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, rows, m->Y, m->Tb, m->dY, m->loss);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = backward(m, m->Xb, rows, s);
            if (e == hipSuccess) e = adam(m, lr_e, s);
            st = merr(m, e, "train step");
        }
        double lh[2] = {0, 0};
        if (st == LBE_OK) st = merr(m, hipMemcpyAsync(lh, m->loss, sizeof(lh), hipMemcpyDeviceToHost, s), "loss");
        if (st == LBE_OK) st = merr(m, hipStreamSynchronize(s), "sync");
        if (host_loss) host_loss[ep] = lh[1] / ((double)n * kOut);
    }
    return st;
}

const char* lbe_mlp_last_error(const lbe_mlp* m) { return m ? m->err.c_str() : "null network"; }

void lbe_mlp_free(lbe_mlp* m) { delete m; }

}  // extern "C"
