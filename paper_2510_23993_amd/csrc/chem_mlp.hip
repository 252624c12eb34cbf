// Surrogate network kernels behind the chem_mlp_* entry points of chem.h:
// training in FP32 (tiled GEMMs through LDS, fused bias + GELU epilogues,
// split-K weight gradients reduced in a fixed order, MSE, Adam, counter-based
// minibatch sampling, feature standardisation) and inference with BF16 MFMA
// (v_mfma_f32_32x32x8bf16_1k) accumulating in FP32.
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

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * INV_SQRT2)); }
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * INV_SQRT2)) + z * expf(-0.5f * z * z) * INV_SQRT2PI;
}

// ------------------------------------------------------------ FP32 GEMM
// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = TA ? A[k lda + m] : A[m lda + k]
// and B(k, n) = TB ? B[n ldb + k] : B[k ldb + n]; 64 x 64 tiles, 16-deep K
// slices staged in LDS, 4 x 4 outputs per thread.  gridDim.z > 1 splits K
// into chunks of kc and writes partial z to C + z * M * ldc.
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BACK = 3 };

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int kc, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, const float* __restrict__ aux,
                                              float* __restrict__ H) {
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
    C += (int64_t)blockIdx.z * M * ldc;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0.f;
    for (int k0 = kbeg; k0 < kend; k0 += 16) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int idx = t + 256 * i;
            const int am = TA ? (idx & 63) : (idx >> 4), ak = TA ? (idx >> 6) : (idx & 15);
            const int gm = m0 + am, gk = k0 + ak;
            float v = 0.f;
            if (gm < M && gk < kend) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[ak][am] = v;
            const int bn = TB ? (idx >> 4) : (idx & 63), bk = TB ? (idx & 15) : (idx >> 6);
            const int gn = n0 + bn, gk2 = k0 + bk;
            float w = 0.f;
            if (gn < N && gk2 < kend) w = TB ? B[(int64_t)gn * ldb + gk2] : B[(int64_t)gk2 * ldb + gn];
            Bs[bk][bn] = w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk++) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; i++) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; j++) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int m = m0 + ty + 16 * i, n = n0 + tx + 16 * j;
            if (m >= M || n >= N) continue;
            const int64_t o = (int64_t)m * ldc + n;
            float v = acc[i][j];
            if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) v += bias[n];
            if (EPI == EPI_GELU_BACK) v *= gelu_d(aux[o]);
            C[o] = v;
            if (EPI == EPI_BIAS_GELU) H[o] = gelu(v);
        }
}

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
          const float* bias = nullptr, const float* aux = nullptr, float* H = nullptr, int splits = 1) {
    const int kc = ((K + splits - 1) / splits + 15) / 16 * 16;
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), dim3((N + 63) / 64, (M + 63) / 64, splits), dim3(256), 0, s, M, N, K,
                       kc, A, lda, B, ldb, C, ldc, bias, aux, H);
}

// out[i] = sum_z part[z * n + i], z in order (deterministic split-K reduction)
__global__ void k_reduce_splits(int S, int64_t n, const float* __restrict__ part, float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int z = 0; z < S; z++) v += part[(int64_t)z * n + i];
        out[i] = v;
    }
}

// column sums of D [rows][cols]: partial[chunk][col] over row chunks
__global__ void k_colsum_part(int64_t rows, int cols, int64_t rpc, const float* __restrict__ D,
                              float* __restrict__ part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const int64_t r0 = blockIdx.y * rpc, r1 = min(rows, r0 + rpc);
    float v = 0.f;
    for (int64_t r = r0; r < r1; r++) v += D[r * cols + c];
    part[(int64_t)blockIdx.y * cols + c] = v;
}

void colsum(hipStream_t s, int64_t rows, int cols, const float* D, float* part, float* out) {
    const int chunks = 64;
    const int64_t rpc = (rows + chunks - 1) / chunks;
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, chunks), dim3(64), 0, s, rows, cols, rpc, D, part);
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
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int HS = NH + 4;   // LDS row stride (bf16 elements): 130 dwords, spreads rows over banks

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Dense weights are stored in MFMA B-fragment order: fragment (kb, nb) holds,
// for lane l, W[nb*32 + l%32][kb*8 + 4*(l/32) + e], e = 0..3, so each
// fragment is one coalesced 512-byte load.
__global__ void k_to_bf16_frag(const float* __restrict__ W, int nout, int nblk, uint16_t* __restrict__ F) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // element of F
    const int64_t total = (int64_t)(NH / 8) * nblk * 64 * 4;
    if (i >= total) return;
    const int e = (int)(i & 3), lane = (int)((i >> 2) & 63);
    const int64_t f = i >> 8;
    const int nb = (int)(f % nblk), kb = (int)(f / nblk);
    const int row = nb * 32 + (lane & 31), col = kb * 8 + 4 * (lane >> 5) + e;
    F[i] = row < nout ? f2bf(W[(int64_t)row * NH + col]) : (uint16_t)0;
}

// One 32-row tile through a 256 -> 32*NB dense layer: A from the LDS tile,
// B fragments from global memory (L2-resident weights), FP32 accumulators.
// The fragments of the next k-step are in flight while the current step's
// products run, which hides most of the L2 latency of a wave.
template <int NB>
__device__ __forceinline__ void tile_mfma(const uint16_t* __restrict__ Hs, const uint16_t* __restrict__ F, int lane,
                                          f32x16 (&acc)[NB]) {
    const int r = lane & 31, kh = 4 * (lane >> 5);
    const bf16x4* Fv = (const bf16x4*)F;
#pragma unroll
    for (int nb = 0; nb < NB; nb++)
#pragma unroll
        for (int q = 0; q < 16; q++) acc[nb][q] = 0.f;
    bf16x4 bn[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) bn[nb] = Fv[nb * 64 + lane];
    for (int kb = 0; kb < NH / 8; kb++) {
        const bf16x4 a = *(const bf16x4*)(Hs + r * HS + kb * 8 + kh);
        bf16x4 bc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++) bc[nb] = bn[nb];
        if (kb + 1 < NH / 8) {
#pragma unroll
            for (int nb = 0; nb < NB; nb++) bn[nb] = Fv[((int64_t)(kb + 1) * NB + nb) * 64 + lane];
        }
#pragma unroll
        for (int nb = 0; nb < NB; nb++) acc[nb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bc[nb], acc[nb], 0, 0, 0);
    }
}

// accumulator element q of lane l is row 8*(q/4) + 4*(l/32) + q%4, column l%32
__device__ __forceinline__ int acc_row(int lane, int q) { return 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3); }

__global__ void __launch_bounds__(64) k_mlp_infer(MlpDev w, int64_t rows_host, const int* __restrict__ rows_dev,
                                                  const float* __restrict__ X, float* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) uint16_t Hs[32 * HS];
    __shared__ float Xs[32 * NIN];
    const int lane = threadIdx.x;
    const int64_t rows = rows_dev ? (int64_t)*rows_dev : rows_host;
    const int64_t ntile = (rows + 31) / 32;
    const float* p = w.p;
    // first-layer weights and biases of this lane's outputs, loaded once
    float w1[4][NIN], b1[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int j = lane + 64 * q;
#pragma unroll
        for (int k = 0; k < NIN; k++) w1[q][k] = p[OW1 + j * NIN + k];
        b1[q] = p[OB1 + j];
    }
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t r0 = tile * 32;
        for (int e = lane; e < 32 * NIN; e += 64) {
            const int64_t r = r0 + e / NIN;
            Xs[e] = r < rows ? X[r * NIN + e % NIN] : 0.f;
        }
        __syncthreads();
        // layer 1 on the FP32 units: lane owns outputs lane + 64 q
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int j = lane + 64 * q;
            for (int r = 0; r < 32; r++) {
                float z = b1[q];
#pragma unroll
                for (int k = 0; k < NIN; k++) z = fmaf(w1[q][k], Xs[r * NIN + k], z);
                Hs[r * HS + j] = f2bf(gelu(z));
            }
        }
        __syncthreads();
        // layers 2 and 3 in place: all reads of the tile finish before the
        // epilogue overwrites it
#pragma unroll 1
        for (int layer = 0; layer < 2; layer++) {
            const uint16_t* F = layer == 0 ? w.w2h : w.w3h;
            const float* b = p + (layer == 0 ? OB2 : OB3);
            f32x16 acc[NH / 32];
            tile_mfma<NH / 32>(Hs, F, lane, acc);
            __syncthreads();
#pragma unroll
            for (int nb = 0; nb < NH / 32; nb++) {
                const int j = nb * 32 + (lane & 31);
                const float bj = b[j];
#pragma unroll
                for (int q = 0; q < 16; q++) Hs[acc_row(lane, q) * HS + j] = f2bf(gelu(acc[nb][q] + bj));
            }
            __syncthreads();
        }
        // output layer (10 of 32 columns used)
        f32x16 acc[1];
        tile_mfma<1>(Hs, w.w4h, lane, acc);
        const int j = lane & 31;
        if (j < NOUT) {
            const float bj = p[OB4 + j];
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int64_t r = r0 + acc_row(lane, q);
                if (r < rows) out[r * NOUT + j] = acc[0][q] + bj;
            }
        }
        __syncthreads();
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
    const int64_t n23 = NW2H, n4 = NW4H;
    hipLaunchKernelGGL(k_to_bf16_frag, dim3((n23 + 255) / 256), dim3(256), 0, s, params + OW2, NH, NH / 32, bf);
    hipLaunchKernelGGL(k_to_bf16_frag, dim3((n23 + 255) / 256), dim3(256), 0, s, params + OW3, NH, NH / 32, bf + NW2H);
    hipLaunchKernelGGL(k_to_bf16_frag, dim3((n4 + 255) / 256), dim3(256), 0, s, params + OW4, NOUT, 1,
                       bf + NW2H + NW3H);
    MCHK(hipGetLastError());
    return 0;
}

int launch_infer(hipStream_t s, const MlpDev& w, int64_t rows_host, const int* rows_dev, int64_t max_rows,
                 const float* X, float* out, int ncu) {
    const int64_t tiles = (max_rows + 31) / 32;
    if (tiles == 0) return 0;
    const int64_t grid = std::min<int64_t>(tiles, (int64_t)ncu * 8);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(64), 0, s, w, rows_host, rows_dev, X, out);
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
        int rc = convert_bf16(s, params, w.bf);
        if (rc) return rc;
        MlpDev d{params, w.bf, w.bf + NW2H, w.bf + NW2H + NW3H};
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
