// Surrogate network kernels behind the chem_mlp_* entry points of chem.h:
// training in FP32 (GEMMs on the FP32 matrix cores, v_mfma_f32_32x32x2_f32,
// with tiles staged through LDS and fused bias + GELU epilogues, split-K
// weight gradients reduced in a fixed order, MSE, Adam, counter-based
// minibatch sampling, row gathers, feature standardisation) and inference on
// the BF16 matrix cores (v_mfma_f32_32x32x16_bf16) accumulating in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <utility>

#include "chem.h"
#include "chem_mlp.hpp"

namespace chem {
int set_error(int code, const char* msg);   // chem_lib.hip: thread-local message
}

using namespace chem;
using namespace chem::mlp;

#define MCHK(x)                                                                         \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) return set_error(CHEM_E_HIP, hipGetErrorString(e_));       \
    } while (0)

namespace {

constexpr float INV_SQRT2 = 0.70710678118654752f;
constexpr float INV_SQRT2PI = 0.39894228040143268f;

// GELU (the network's exact-erf form) and its derivative, branch free.  erf
// from Abramowitz & Stegun 7.1.26 (rational-times-Gaussian form, |error| <=
// 1.5e-7: at the FP32 rounding, far below BF16's), with the hardware
// reciprocal and exp2.  For a = |z|, erf(a/sqrt 2) = 1 - poly(t) exp(-a^2/2),
// so the normal tail Phi(-a) = (poly(t)/2) exp(-a^2/2) (the 1/2 folded into
// the coefficients); e returns exp(-a^2/2).
__device__ __forceinline__ float normal_tail(float a, float& e) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * INV_SQRT2, a, 1.0f));
    const float half_poly =
        t * (0.127414796f + t * (-0.142248368f + t * (0.7107068705f + t * (-0.7265760135f + t * 0.5307027145f))));
    e = __builtin_amdgcn_exp2f(a * a * (-0.5f * 1.4426950408889634f));
    return half_poly * e;
}

// both signs of z: GELU(z) = z Phi(z) = max(z, 0) - |z| Phi(-|z|)
__device__ __forceinline__ float gelu_fast(float z) {
    float e;
    const float a = fabsf(z);
    return fmaf(-a, normal_tail(a, e), fmaxf(z, 0.0f));
}

// GELU'(z) = Phi(z) + z phi(z), phi(z) = exp(-z^2/2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_d_fast(float z) {
    float e;
    const float tail = normal_tail(fabsf(z), e);
    const float Phi = z >= 0.0f ? 1.0f - tail : tail;
    return fmaf(z * INV_SQRT2PI, e, Phi);
}

// ------------------------------------------------------------ FP32 GEMM
// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = TA ? A[k lda + m] : A[m lda + k]
// and B(k, n) = TB ? B[n ldb + k] : B[k ldb + n], on the FP32 matrix cores
// (v_mfma_f32_32x32x2_f32: FP32 products and sums).  64 x 64 tiles, one
// 32 x 32 quadrant per wave, 128-deep K slices staged in LDS (the next slice
// is read from memory into registers while this one's products run: deep
// slices keep many loads in flight, as these GEMMs are small and latency
// bound).  gridDim.z > 1 splits K into chunks of kc (a multiple of GK) and
// writes partial z to C + z * M * ldc.
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BACK = 3 };
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int GK = 32;   // K slice
constexpr int GPT = 64 * GK / 256;   // elements of each tile per thread and slice

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int kc, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, const float* __restrict__ aux,
                                              float* __restrict__ H) {
    __shared__ float As[2][GK][64 + 1];
    __shared__ float Bs[2][GK][64 + 1];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
    C += (int64_t)blockIdx.z * M * ldc;
    // element i of this thread's share of a slice: (m or n, k) of the A and B tiles,
    // consecutive threads on consecutive addresses
    auto a_mk = [&](int i, int& am, int& ak) {
        const int idx = t + 256 * i;
        am = TA ? (idx & 63) : (idx / GK);
        ak = TA ? (idx >> 6) : (idx % GK);
    };
    auto b_nk = [&](int i, int& bn, int& bk) {
        const int idx = t + 256 * i;
        bn = TB ? (idx / GK) : (idx & 63);
        bk = TB ? (idx % GK) : (idx >> 6);
    };
    float ra[GPT], rb[GPT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < GPT; i++) {
            int am, ak, bn, bk;
            a_mk(i, am, ak);
            b_nk(i, bn, bk);
            // every load is issued, from a clamped address (the value is
            // dropped at the store to LDS), so that no branch separates them
            // and none is waited for before this slice's products
            const int cm = min(m0 + am, M - 1), cka = min(k0 + ak, kend - 1);
            const int cn = min(n0 + bn, N - 1), ckb = min(k0 + bk, kend - 1);
            ra[i] = TA ? A[(int64_t)cka * lda + cm] : A[(int64_t)cm * lda + cka];
            rb[i] = TB ? B[(int64_t)cn * ldb + ckb] : B[(int64_t)ckb * ldb + cn];
        }
    };
    auto stash = [&](int buf, int k0) {
#pragma unroll
        for (int i = 0; i < GPT; i++) {
            int am, ak, bn, bk;
            a_mk(i, am, ak);
            b_nk(i, bn, bk);
            As[buf][ak][am] = (m0 + am < M && k0 + ak < kend) ? ra[i] : 0.f;
            Bs[buf][bk][bn] = (n0 + bn < N && k0 + bk < kend) ? rb[i] : 0.f;
        }
    };
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 16; q++) acc[q] = 0.f;
    if (kbeg < kend) {
        fetch(kbeg);
        stash(0, kbeg);
        __syncthreads();
    }
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        const bool more = k0 + GK < kend;
        if (more) fetch(k0 + GK);
        // A operand: lane l holds A(m = l%32, k = kk + l/32) of the quadrant, B likewise
#pragma unroll
        for (int kk = 0; kk < GK; kk += 2) {
            const float a = As[buf][kk + (lane >> 5)][wm * 32 + (lane & 31)];
            const float b = Bs[buf][kk + (lane >> 5)][wn * 32 + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        if (more) stash(buf ^ 1, k0 + GK);
        __syncthreads();
        buf ^= 1;
    }
    // accumulator element q of lane l: row 8*(q/4) + 4*(l/32) + q%4, column l%32.
    // The epilogue's operands are all requested before any is used.
    const int n = n0 + wn * 32 + (lane & 31);
    const int mb = m0 + wm * 32 + 4 * (lane >> 5);
    auto row = [&](int q) { return mb + 8 * (q >> 2) + (q & 3); };
    const int cn = min(n, N - 1);
    const float bn = (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) ? bias[cn] : 0.f;
    float v[16], hv[16];
#pragma unroll
    for (int q = 0; q < 16; q++) {
        v[q] = acc[q] + bn;
        if (EPI == EPI_GELU_BACK) v[q] *= gelu_d_fast(aux[(int64_t)min(row(q), M - 1) * ldc + cn]);
        if (EPI == EPI_BIAS_GELU) hv[q] = gelu_fast(v[q]);
    }
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const int m = row(q);
        if (m >= M || n >= N) continue;
        const int64_t o = (int64_t)m * ldc + n;
        C[o] = v[q];
        if (EPI == EPI_BIAS_GELU) H[o] = hv[q];
    }
}

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
          const float* bias = nullptr, const float* aux = nullptr, float* H = nullptr, int splits = 1) {
    const int kc = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), dim3((N + 63) / 64, (M + 63) / 64, splits), dim3(256), 0, s, M, N, K,
                       kc, A, lda, B, ldb, C, ldc, bias, aux, H);
}

// out[i] = sum_z part[z * n + i], z in order (deterministic split-K reduction)
__global__ void k_reduce_splits(int S, int64_t n, const float* __restrict__ part, float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        // four independent sums (z mod 4), combined in a fixed order
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        int z = 0;
        for (; z + 4 <= S; z += 4)
#pragma unroll
            for (int u = 0; u < 4; u++) v[u] += part[(int64_t)(z + u) * n + i];
        for (; z < S; z++) v[0] += part[(int64_t)z * n + i];
        out[i] = (v[0] + v[1]) + (v[2] + v[3]);
    }
}

// column sums of D [rows][cols]: partial[chunk][col] over row chunks; four
// threads per column take every fourth row, combined in a fixed order
__global__ void __launch_bounds__(256) k_colsum_part(int64_t rows, int cols, int64_t rpc, const float* __restrict__ D,
                                                     float* __restrict__ part) {
    __shared__ float sh[4][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    const int64_t r0 = blockIdx.y * rpc, r1 = min(rows, r0 + rpc);
    float v0 = 0.f, v1 = 0.f;
    if (c < cols) {
        int64_t r = r0 + ph;
        for (; r + 4 < r1; r += 8) {
            v0 += D[r * cols + c];
            v1 += D[(r + 4) * cols + c];
        }
        if (r < r1) v0 += D[r * cols + c];
    }
    sh[ph][cl] = v0 + v1;
    __syncthreads();
    if (ph == 0 && c < cols) part[(int64_t)blockIdx.y * cols + c] = (sh[0][cl] + sh[1][cl]) + (sh[2][cl] + sh[3][cl]);
}

void colsum(hipStream_t s, int64_t rows, int cols, const float* D, float* part, float* out) {
    const int chunks = 64;
    const int64_t rpc = (rows + chunks - 1) / chunks;
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, chunks), dim3(256), 0, s, rows, cols, rpc, D, part);
    hipLaunchKernelGGL(k_reduce_splits, dim3((cols + 255) / 256), dim3(256), 0, s, chunks, (int64_t)cols, part, out);
}

// ------------------------------------------------------- loss and optimiser
__global__ void k_mse(int64_t n, const float* __restrict__ out, const float* __restrict__ T, float* __restrict__ dout,
                      double* __restrict__ loss) {
    __shared__ double sh[256];
    double acc = 0.0;
    const float sc = 2.0f / (float)n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = out[i] - T[i];
        dout[i] = sc * d;
        acc += (double)d * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) atomicAdd(loss, sh[0] / (double)n);
}

// 1 - beta is passed rounded from double (1.0f - 0.999f is 1.3e-5 off)
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float omb1, float omb2, float eps, float c1,
                       float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + omb1 * gi;
        const float vi = b2 * v[i] + omb2 * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// SplitMix64 finaliser (Steele, Lea and Flood, 2014) as a counter-based
// generator: sample i of step s draws row hash(seed, s, i) mod n
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_gather(int64_t n_data, const float* __restrict__ X, const float* __restrict__ T, int64_t batch,
                         uint64_t seed, int64_t step, float* __restrict__ Xb, float* __restrict__ Tb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const uint64_t h = splitmix64(splitmix64(seed ^ (uint64_t)step * 0xD1B54A32D192ED03ull) + (uint64_t)i);
    const int64_t r = (int64_t)(h % (uint64_t)n_data);
#pragma unroll
    for (int k = 0; k < NIN; k++) Xb[i * NIN + k] = X[r * NIN + k];
#pragma unroll
    for (int k = 0; k < NOUT; k++) Tb[i * NOUT + k] = T[r * NOUT + k];
}

// rows idx[i] of X [*][NIN] and T [*][NOUT] to row i of Xo and To
__global__ void k_take(int64_t n, const int64_t* __restrict__ idx, const float* __restrict__ X,
                       const float* __restrict__ T, float* __restrict__ Xo, float* __restrict__ To) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = idx[i];
#pragma unroll
    for (int k = 0; k < NIN; k++) Xo[i * NIN + k] = X[r * NIN + k];
#pragma unroll
    for (int k = 0; k < NOUT; k++) To[i * NOUT + k] = T[r * NOUT + k];
}

__global__ void k_colstats(int64_t n, int cols, const float* __restrict__ D, double* __restrict__ acc) {
    // acc[2c] += sum x, acc[2c+1] += sum x^2 over this thread's rows
    const int c = threadIdx.x % cols;
    const int lanes = blockDim.x / cols;
    const int li = threadIdx.x / cols;
    if (li >= lanes) return;
    double s = 0.0, q = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)lanes + li; r < n; r += (int64_t)gridDim.x * lanes) {
        const double x = D[r * cols + c];
        s += x;
        q += x * x;
    }
    atomicAdd(&acc[2 * c], s);
    atomicAdd(&acc[2 * c + 1], q);
}

__global__ void k_finish_stats(int64_t n, int cols, const double* __restrict__ acc, float* __restrict__ mean,
                               float* __restrict__ sd) {
    const int c = threadIdx.x;
    if (c >= cols) return;
    const double mu = acc[2 * c] / (double)n;
    const double var = fmax(acc[2 * c + 1] / (double)n - mu * mu, 0.0);
    mean[c] = (float)mu;
    sd[c] = (float)fmax(sqrt(var), 1e-12);
}

__global__ void k_fill_f64(double* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// order-preserving map of a float to an unsigned integer (for atomic min/max)
__device__ __forceinline__ unsigned int ford(float f) {
    const unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funord(unsigned int u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

__global__ void k_range_init(int cols, unsigned int* r) {
    const int c = threadIdx.x;
    if (c < cols) {
        r[2 * c] = 0xFFFFFFFFu;
        r[2 * c + 1] = 0u;
    }
}

__global__ void k_colrange(int64_t n, int cols, const float* __restrict__ D, unsigned int* __restrict__ r) {
    const int c = threadIdx.x % cols;
    const int lanes = blockDim.x / cols, li = threadIdx.x / cols;
    unsigned int lo = 0xFFFFFFFFu, hi = 0u;
    for (int64_t row = blockIdx.x * (int64_t)lanes + li; row < n; row += (int64_t)gridDim.x * lanes) {
        const unsigned int u = ford(D[row * cols + c]);
        lo = min(lo, u);
        hi = max(hi, u);
    }
    atomicMin(&r[2 * c], lo);
    atomicMax(&r[2 * c + 1], hi);
}

__global__ void k_range_finish(int cols, const unsigned int* __restrict__ r, double* __restrict__ lo,
                               double* __restrict__ hi) {
    const int c = threadIdx.x;
    if (c < cols) {
        lo[c] = funord(r[2 * c]);
        hi[c] = funord(r[2 * c + 1]);
    }
}

__global__ void k_standardize(int64_t n, int cols, float* __restrict__ D, const float* __restrict__ mean,
                              const float* __restrict__ sd) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * cols; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % cols);
        D[i] = (D[i] - mean[c]) / sd[c];
    }
}

// ------------------------------------------------------ BF16 MFMA inference
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int KB16 = NH / 16;   // K steps of the 32x32x16 products
constexpr int IW = 8;           // waves per workgroup, one 32-row tile each
constexpr int KS = 2;           // K steps per staged block of weight fragments

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Dense weights are stored in the operand order of v_mfma_f32_32x32x16_bf16
// (the A order with the layer's outputs as rows): fragment (kb, nb) holds,
// for lane l, W[nb*32 + l%32][kb*16 + 8*(l/32) + e], e = 0..7 (16 bytes per
// lane, 1 KB per fragment).
__global__ void k_to_bf16_frag(const float* __restrict__ W, int nout, int nblk, uint16_t* __restrict__ F) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // element of F
    const int64_t total = (int64_t)KB16 * nblk * 64 * 8;
    if (i >= total) return;
    const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
    const int64_t f = i >> 9;
    const int nb = (int)(f % nblk), kb = (int)(f / nblk);
    const int row = nb * 32 + (lane & 31), col = kb * 16 + 8 * (lane >> 5) + e;
    F[i] = row < nout ? f2bf(W[(int64_t)row * NH + col]) : (uint16_t)0;
}

// First-layer weights in the same order with one 16-deep K step (the 12
// inputs, zero-padded): fragment nb, lane l holds W1[nb*32 + l%32][8*(l/32) + e],
// as a BF16 high part (first NH*16 entries) and the BF16 rounding of the rest.
__global__ void k_w1_frag(const float* __restrict__ W1, uint16_t* __restrict__ F) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= NW1H / 2) return;
    const int e = (int)(i & 7), lane = (int)((i >> 3) & 63), nb = (int)(i >> 9);
    const int row = nb * 32 + (lane & 31), k = 8 * (lane >> 5) + e;
    const float w = k < NIN ? W1[(int64_t)row * NIN + k] : 0.f;
    const uint16_t hi = f2bf(w);
    F[i] = hi;
    F[NW1H / 2 + i] = f2bf(w - __uint_as_float((uint32_t)hi << 16));
}

// The products are taken transposed, D = W H^T: with the weights as the A
// operand, accumulator element q of lane l is output 8*(q/4) + 4*(l/32) + q%4
// (of the 32-output block) for row l%32 of the wave's tile.  The accumulators
// start at the bias.
template <int NB>
__device__ __forceinline__ void acc_bias(f32x16 (&acc)[NB], const float* __restrict__ b, int lane) {
    const float* bl = b + 4 * (lane >> 5);   // one base, constant offsets (16-byte aligned)
#pragma unroll
    for (int nb = 0; nb < NB; nb++)
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const float4 v = *(const float4*)(bl + nb * 32 + 8 * g);
            acc[nb][4 * g] = v.x, acc[nb][4 * g + 1] = v.y, acc[nb][4 * g + 2] = v.z, acc[nb][4 * g + 3] = v.w;
        }
}

template <class T> __device__ __forceinline__ T* opaque(T* q) {
    asm volatile("" : "+s"(q));
    return q;
}

// The activations of a wave's 32 rows stay in registers between layers, in
// the accumulator order: Hr[nb][g] is outputs nb*32 + 8g + 4h .. +3 of row r
// for lane (r = l%32, h = l/32), four BF16 in two dwords (64 registers).
typedef uint32_t HReg[NH / 32][4][2];

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

template <int NB>
__device__ __forceinline__ void gelu_to_regs(const f32x16 (&acc)[NB], HReg& Hr) {
#pragma unroll
    for (int nb = 0; nb < NB; nb++)
#pragma unroll
        for (int g = 0; g < 4; g++) {
            Hr[nb][g][0] = pack_bf16(gelu_fast(acc[nb][4 * g]), gelu_fast(acc[nb][4 * g + 1]));
            Hr[nb][g][1] = pack_bf16(gelu_fast(acc[nb][4 * g + 2]), gelu_fast(acc[nb][4 * g + 3]));
            __builtin_amdgcn_sched_barrier(0);   // one group at a time: bounded register demand
        }
}

// B operand of K step kb (inputs kb*16 + 8h + e of row r for lane (r, h)):
// with s = kb%2, lane (r, 0) holds inputs 16s + 0..3 (its Hr[kb/2][2s]) and
// lane (r, 1) inputs 16s + 4..7; the second eight are Hr[kb/2][2s+1] of the
// two lanes.  One exchange between lanes l and l+32 (lanes 32-63 of the
// first operand with lanes 0-31 of the second) gives every lane its eight.
__device__ __forceinline__ bf16x8 b_operand(const HReg& Hr, int kb) {
    const int nb = kb >> 1, s = kb & 1;
    const auto x0 = __builtin_amdgcn_permlane32_swap(Hr[nb][2 * s][0], Hr[nb][2 * s + 1][0], false, false);
    const auto x1 = __builtin_amdgcn_permlane32_swap(Hr[nb][2 * s][1], Hr[nb][2 * s + 1][1], false, false);
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 u;
    u[0] = x0[0];
    u[1] = x1[0];
    u[2] = x0[1];
    u[3] = x1[1];
    return __builtin_bit_cast(bf16x8, u);
}

// One 256 -> 32*NB dense layer for the workgroup's IW tiles of 32 rows: the
// weight fragments staged in LDS once per workgroup, KS K steps at a time
// (double-buffered: the next stage is loaded from L2 while this one's
// products run), the activations from registers, FP32 accumulators.
template <int NB>
__device__ __forceinline__ void wg_layer(const HReg& Hr, const bf16x8* __restrict__ F, bf16x8 (*Bst)[KS * 8 * 64],
                                         int tid, f32x16 (&acc)[NB]) {
    const int lane = tid & 63;
    constexpr int FS = KS * NB * 64;                       // fragments per stage
    constexpr int PER = (FS + 64 * IW - 1) / (64 * IW);   // fragments per thread and stage
    bf16x8 g[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int e = tid + 64 * IW * u;
        if (e < FS) Bst[0][e] = F[e];
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < KB16 / KS; st++) {
        if (st + 1 < KB16 / KS) {
#pragma unroll
            for (int u = 0; u < PER; u++) {
                const int e = tid + 64 * IW * u;
                if (e < FS) g[u] = F[(int64_t)(st + 1) * FS + e];
            }
        }
        const bf16x8* Bc = Bst[st & 1];
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
            const bf16x8 h = b_operand(Hr, st * KS + ks);
#pragma unroll
            for (int nb = 0; nb < NB; nb++)
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Bc[(ks * NB + nb) * 64 + lane], h, acc[nb], 0, 0, 0);
        }
        if (st + 1 < KB16 / KS) {
#pragma unroll
            for (int u = 0; u < PER; u++) {
                const int e = tid + 64 * IW * u;
                if (e < FS) Bst[(st + 1) & 1][e] = g[u];
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64 * IW, 2) k_mlp_infer(MlpDev w, int64_t rows_host, const int* __restrict__ rows_dev,
                                                          const float* __restrict__ X, float* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) bf16x8 Bst[2][KS * 8 * 64];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int64_t rows = rows_dev ? (int64_t)*rows_dev : rows_host;
    const int64_t ntile = (rows + 32 * IW - 1) / (32 * IW);
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        // the weight and bias pointers made opaque per tile, so that their
        // loads are not hoisted out of the loop to stay live in registers
        const float* p = opaque(w.p);
        const bf16x8* W1f = opaque((const bf16x8*)w.w1h);
        const int64_t r0 = tile * (32 * IW) + 32 * wv;   // this wave's rows
        const int64_t row = r0 + (lane & 31);
        HReg Hr;
        {   // layer 1 on the matrix cores: inputs and weights as hi + lo BF16 parts
            // (16 significant bits each), the lo x lo product dropped.  Lane
            // (row r, half h) reads inputs 8h .. 8h+7 of its row (rows are 48 bytes).
            const int h = lane >> 5;
            float x[8];
            if (row < rows) {
                const float4* xr = (const float4*)(X + row * NIN + 8 * h);
                const float4 u = xr[0];
                x[0] = u.x, x[1] = u.y, x[2] = u.z, x[3] = u.w;
                if (h == 0) {
                    const float4 v = xr[1];
                    x[4] = v.x, x[5] = v.y, x[6] = v.z, x[7] = v.w;
                } else {
                    x[4] = x[5] = x[6] = x[7] = 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++) x[e] = 0.f;
            }
            bf16x8 xh, xl;
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const __bf16 hb = (__bf16)x[e];
                xh[e] = hb;
                xl[e] = (__bf16)(x[e] - (float)hb);
            }
            f32x16 acc[NH / 32];
            acc_bias<NH / 32>(acc, p + OB1, lane);
#pragma unroll
            for (int nb = 0; nb < NH / 32; nb++) {
                const bf16x8 wh = W1f[nb * 64 + lane], wl = W1f[(NH / 32 + nb) * 64 + lane];
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, xh, acc[nb], 0, 0, 0);
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, xl, acc[nb], 0, 0, 0);
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, xh, acc[nb], 0, 0, 0);
                if (nb & 1) __builtin_amdgcn_sched_barrier(0);   // fragments of two blocks in flight
            }
            gelu_to_regs<NH / 32>(acc, Hr);
        }
#pragma unroll 1
        for (int layer = 0; layer < 2; layer++) {
            f32x16 acc[NH / 32];
            acc_bias<NH / 32>(acc, p + (layer == 0 ? OB2 : OB3), lane);
            wg_layer<NH / 32>(Hr, (const bf16x8*)(layer == 0 ? w.w2h : w.w3h), Bst, tid, acc);
            gelu_to_regs<NH / 32>(acc, Hr);
        }
        // output layer (10 of 32 outputs used): lane (r, h) holds outputs
        // 4h .. 4h+3 (q < 4) and 8 + 4h .. (q 4..7) of row r
        f32x16 acc[1];
#pragma unroll
        for (int q = 0; q < 16; q++) acc[0][q] = 0.f;
        wg_layer<1>(Hr, (const bf16x8*)w.w4h, Bst, tid, acc);
        if (row < rows) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int j = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                if (j < NOUT) out[row * NOUT + j] = acc[0][q] + p[OB4 + j];
            }
        }
    }
}

int g_ncu = 0;

int num_cu() {
    if (g_ncu > 0) return g_ncu;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    g_ncu = prop.multiProcessorCount;
    return g_ncu;
}

// training workspace layout (floats) for a batch of B rows
struct Ws {
    float *Z[3], *H[3], *G0, *G1, *part, *cpart;
    uint16_t* bf;
};
constexpr int SPLITS = 16;

Ws carve(float* ws, int64_t B) {
    Ws w;
    float* q = ws;
    w.bf = (uint16_t*)q;
    q += (NBF16 + 1) / 2;
    q = (float*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    for (int l = 0; l < 3; l++) {
        w.Z[l] = q;
        q += B * NH;
        w.H[l] = q;
        q += B * NH;
    }
    w.G0 = q;
    q += B * NH;
    w.G1 = q;
    q += B * NH;
    w.part = q;
    q += (int64_t)SPLITS * NH * NH;
    w.cpart = q;
    return w;
}

int64_t ws_floats(int64_t B) { return (NBF16 + 1) / 2 + 64 + 8 * B * NH + (int64_t)SPLITS * NH * NH + 64 * NH; }

}  // namespace

namespace chem {
namespace mlp {

int convert_bf16(hipStream_t s, const float* params, uint16_t* bf) {
    const int64_t n23 = NW2H, n4 = NW4H;   // fragment elements of one 256 x 256 layer and of the padded output layer
    hipLaunchKernelGGL(k_to_bf16_frag, dim3((n23 + 255) / 256), dim3(256), 0, s, params + OW2, NH, NH / 32, bf);
    hipLaunchKernelGGL(k_to_bf16_frag, dim3((n23 + 255) / 256), dim3(256), 0, s, params + OW3, NH, NH / 32, bf + NW2H);
    hipLaunchKernelGGL(k_to_bf16_frag, dim3((n4 + 255) / 256), dim3(256), 0, s, params + OW4, NOUT, 1,
                       bf + NW2H + NW3H);
    hipLaunchKernelGGL(k_w1_frag, dim3((NW1H / 2 + 255) / 256), dim3(256), 0, s, params + OW1, bf + NW2H + NW3H + NW4H);
    MCHK(hipGetLastError());
    return 0;
}

int launch_infer(hipStream_t s, const MlpDev& w, int64_t rows_host, const int* rows_dev, int64_t max_rows,
                 const float* X, float* out, int ncu) {
    const int64_t tiles = (max_rows + 32 * IW - 1) / (32 * IW);
    if (tiles == 0) return 0;
    const int64_t grid = std::min<int64_t>(tiles, (int64_t)ncu * 2);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(64 * IW), 0, s, w, rows_host, rows_dev, X, out);
    MCHK(hipGetLastError());
    return 0;
}

}  // namespace mlp
}  // namespace chem

extern "C" {

int64_t chem_mlp_nparams(void) { return NPARAM; }

int64_t chem_mlp_workspace_floats(int64_t batch) { return batch < 0 ? -1 : ws_floats(batch); }

int chem_mlp_forward(void* stream, int64_t batch, const float* params, const float* X, float* out, float* ws,
                     int mode) {
    if (batch < 0 || !params || !ws || (batch > 0 && (!X || !out))) return set_error(CHEM_E_INVAL, "bad argument");
    if (mode != 0 && mode != 1) return set_error(CHEM_E_INVAL, "mode must be 0 (FP32) or 1 (BF16 MFMA)");
    if (batch > INT32_MAX / NH) return set_error(CHEM_E_INVAL, "batch too large");
    if (batch == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    Ws w = carve(ws, batch);
    const int B = (int)batch;
    if (mode == 1) {
        if (((uintptr_t)X | (uintptr_t)params) & 15)
            return set_error(CHEM_E_INVAL, "X and params must be 16-byte aligned for the BF16 kernel");
        int rc = convert_bf16(s, params, w.bf);
        if (rc) return rc;
        MlpDev d{params, w.bf, w.bf + NW2H, w.bf + NW2H + NW3H, w.bf + NW2H + NW3H + NW4H};
        return launch_infer(s, d, batch, nullptr, batch, X, out, num_cu());
    }
    gemm<false, true, EPI_BIAS_GELU>(s, B, NH, NIN, X, NIN, params + OW1, NIN, w.Z[0], NH, params + OB1, nullptr, w.H[0]);
    gemm<false, true, EPI_BIAS_GELU>(s, B, NH, NH, w.H[0], NH, params + OW2, NH, w.Z[1], NH, params + OB2, nullptr, w.H[1]);
    gemm<false, true, EPI_BIAS_GELU>(s, B, NH, NH, w.H[1], NH, params + OW3, NH, w.Z[2], NH, params + OB3, nullptr, w.H[2]);
    gemm<false, true, EPI_BIAS>(s, B, NOUT, NH, w.H[2], NH, params + OW4, NH, out, NOUT, params + OB4);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_backward(void* stream, int64_t batch, const float* params, const float* X, const float* ws,
                      const float* dout, float* grads) {
    if (batch <= 0 || !params || !X || !ws || !dout || !grads) return set_error(CHEM_E_INVAL, "bad argument");
    if (batch > INT32_MAX / NH) return set_error(CHEM_E_INVAL, "batch too large");
    hipStream_t s = (hipStream_t)stream;
    Ws w = carve((float*)ws, batch);
    const int B = (int)batch;
    // output layer: dW4 = dout^T H3, db4 = colsum(dout), dZ3 = (dout W4) * gelu'(Z3)
    gemm<true, false, EPI_STORE>(s, NOUT, NH, B, dout, NOUT, w.H[2], NH, w.part, NH, nullptr, nullptr, nullptr, SPLITS);
    hipLaunchKernelGGL(k_reduce_splits, dim3(16), dim3(256), 0, s, SPLITS, (int64_t)NOUT * NH, w.part, grads + OW4);
    colsum(s, batch, NOUT, dout, w.cpart, grads + OB4);
    gemm<false, false, EPI_GELU_BACK>(s, B, NH, NOUT, dout, NOUT, params + OW4, NH, w.G0, NH, nullptr, w.Z[2]);
    // hidden layers 3, 2 (weights W3, W2) then the input layer W1
    float* dz = w.G0;
    float* nxt = w.G1;
    for (int l = 2; l >= 0; l--) {
        const float* hin = l > 0 ? w.H[l - 1] : X;
        const int kin = l > 0 ? NH : NIN;
        const int64_t ow = l == 2 ? OW3 : (l == 1 ? OW2 : OW1), ob = l == 2 ? OB3 : (l == 1 ? OB2 : OB1);
        gemm<true, false, EPI_STORE>(s, NH, kin, B, dz, NH, hin, kin, w.part, kin, nullptr, nullptr, nullptr, SPLITS);
        hipLaunchKernelGGL(k_reduce_splits, dim3(256), dim3(256), 0, s, SPLITS, (int64_t)NH * kin, w.part, grads + ow);
        colsum(s, batch, NH, dz, w.cpart, grads + ob);
        if (l > 0) {
            gemm<false, false, EPI_GELU_BACK>(s, B, NH, NH, dz, NH, params + ow, NH, nxt, NH, nullptr, w.Z[l - 1]);
            std::swap(dz, nxt);
        }
    }
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_mse(void* stream, int64_t n, const float* out, const float* target, float* dout, double* loss) {
    if (n <= 0 || !out || !target || !dout) return set_error(CHEM_E_INVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    if (loss) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, loss, 1);
    const int64_t grid = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_mse, dim3(grid), dim3(256), 0, s, n, out, target, dout, loss);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_adam(void* stream, int64_t n, float* params, const float* grads, float* m, float* v, double lr,
                  double beta1, double beta2, double eps, int step) {
    if (n <= 0 || !params || !grads || !m || !v || step < 1) return set_error(CHEM_E_INVAL, "bad argument");
    const float c1 = (float)(1.0 / (1.0 - std::pow(beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(beta2, step)));
    const int64_t grid = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_adam, dim3(grid), dim3(256), 0, (hipStream_t)stream, n, params, grads, m, v, (float)lr,
                       (float)beta1, (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps, c1, c2);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_gather(void* stream, int64_t n_data, const float* X, const float* T, int64_t batch, uint64_t seed,
                    int64_t step, float* Xb, float* Tb) {
    if (n_data <= 0 || batch <= 0 || !X || !T || !Xb || !Tb) return set_error(CHEM_E_INVAL, "bad argument");
    hipLaunchKernelGGL(k_gather, dim3((batch + 255) / 256), dim3(256), 0, (hipStream_t)stream, n_data, X, T, batch,
                       seed, step, Xb, Tb);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_take(void* stream, int64_t n, const int64_t* idx, const float* X, const float* T, float* Xo, float* To) {
    if (n < 0 || (n > 0 && (!idx || !X || !T || !Xo || !To))) return set_error(CHEM_E_INVAL, "bad argument");
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_take, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, idx, X, T, Xo,
                       To);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_colstats(void* stream, int64_t n, int cols, const float* data, double* acc, float* mean, float* sd) {
    if (n <= 0 || cols <= 0 || cols > 64 || !data || !acc || !mean || !sd) return set_error(CHEM_E_INVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(128), 0, s, acc, 2 * cols);
    const int threads = (256 / cols) * cols;
    hipLaunchKernelGGL(k_colstats, dim3(1024), dim3(threads), 0, s, n, cols, data, acc);
    hipLaunchKernelGGL(k_finish_stats, dim3(1), dim3(64), 0, s, n, cols, acc, mean, sd);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_colrange(void* stream, int64_t n, int cols, const float* data, unsigned int* scratch, double* lo,
                      double* hi) {
    if (n <= 0 || cols <= 0 || cols > 64 || !data || !scratch || !lo || !hi) return set_error(CHEM_E_INVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_range_init, dim3(1), dim3(64), 0, s, cols, scratch);
    const int threads = (256 / cols) * cols;
    hipLaunchKernelGGL(k_colrange, dim3(1024), dim3(threads), 0, s, n, cols, data, scratch);
    hipLaunchKernelGGL(k_range_finish, dim3(1), dim3(64), 0, s, cols, scratch, lo, hi);
    MCHK(hipGetLastError());
    return 0;
}

int chem_mlp_standardize(void* stream, int64_t n, int cols, float* data, const float* mean, const float* sd) {
    if (n < 0 || cols <= 0 || !data || !mean || !sd) return set_error(CHEM_E_INVAL, "bad argument");
    if (n == 0) return 0;
    const int64_t grid = std::min<int64_t>((n * cols + 255) / 256, 4096);
    hipLaunchKernelGGL(k_standardize, dim3(grid), dim3(256), 0, (hipStream_t)stream, n, cols, data, mean, sd);
    MCHK(hipGetLastError());
    return 0;
}

}  // extern "C"
