// Stoichiometric contractions of the matrix-form rate evaluation, as a batch
// operation over many states: for every reaction j,
//   zf_j = sum_k nu'_kj ln|C_k|   and   zr_j = sum_k nu''_kj ln|C_k|,
// the two products of the stoichiometric matrices with the log-concentration
// vector that precede the exponentials (forward and reverse rates of
// progress are exp(ln k_f + zf) and exp(ln k_f - ln K_c + zr)).  Three
// arithmetic variants:
//   - FP64 and FP32 sparse loops over each reaction's participants (the
//     integrator's own form, one state per thread);
//   - dense BF16 matrix cores (v_mfma_f32_16x16x32_bf16): ln C is split into
//     three BF16 terms hi + mid + lo (about 24 significant bits together),
//     the integer coefficients are exact in BF16, products accumulate in
//     FP32.  One wave multiplies 16 states by the whole padded matrix
//     (species padded to a multiple of 32, the 2 nr columns zf_0, zr_0,
//     zf_1, ... padded to a multiple of 16), whose fragments are staged in
//     LDS once per workgroup.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace chem {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CONTRACT_KTMAX = 4;   // up to 128 species on the matrix cores

struct ContractTables {
    int ns, nr;
    const int* ptr;       // [2 nr + 1]: participants of column c (2j: nu'_.j, 2j+1: nu''_.j)
    const int* sp;        // their species
    const int* nu;        // and coefficients
    const bf16x8* frag;   // [kt][nt][64] B fragments: lane l holds rows kb*32 + 8 (l/16) + e, column nb*16 + l%16
    int kt, nt;           // 32-species K tiles, 16-column N tiles
};

template <class T>
__global__ void __launch_bounds__(256) k_contract_sparse(ContractTables t, int64_t n, const double* __restrict__ lnC,
                                                         double* __restrict__ zf, double* __restrict__ zr) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        for (int c = 0; c < 2 * t.nr; c++) {
            T s = 0;
            for (int p = t.ptr[c]; p < t.ptr[c + 1]; p++) s += (T)t.nu[p] * (T)lnC[(int64_t)t.sp[p] * n + i];
            ((c & 1) ? zr : zf)[(int64_t)(c >> 1) * n + i] = (double)s;
        }
    }
}

__device__ __forceinline__ void split3(double x, __bf16& hi, __bf16& mid, __bf16& lo) {
    hi = (__bf16)(float)x;
    const double r1 = x - (double)(float)hi;
    mid = (__bf16)(float)r1;
    const double r2 = r1 - (double)(float)mid;
    lo = (__bf16)(float)r2;
}

// 256 threads = 4 waves, each 16 consecutive states per pass.
__global__ void __launch_bounds__(256) k_contract_mfma(ContractTables t, int64_t n, const double* __restrict__ lnC,
                                                       double* __restrict__ zf, double* __restrict__ zr) {
    extern __shared__ bf16x8 Bs[];
    const int nfrag = t.kt * t.nt * 64;
    for (int e = threadIdx.x; e < nfrag; e += 256) Bs[e] = t.frag[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = lane & 15, kq = 8 * (lane >> 4);
    for (int64_t s0 = ((int64_t)blockIdx.x * 4 + w) * 16; s0 < n; s0 += (int64_t)gridDim.x * 64) {
        const int64_t st = s0 + row;
        bf16x8 A[3][CONTRACT_KTMAX];
#pragma unroll
        for (int kb = 0; kb < CONTRACT_KTMAX; kb++) {
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int k = kb * 32 + kq + e;
                const double x = (kb < t.kt && k < t.ns && st < n) ? lnC[(int64_t)k * n + st] : 0.0;
                __bf16 h, m, l;
                split3(x, h, m, l);
                A[0][kb][e] = h;
                A[1][kb][e] = m;
                A[2][kb][e] = l;
            }
        }
        for (int nb0 = 0; nb0 < t.nt; nb0 += 8) {
            f32x4 acc[8];
#pragma unroll
            for (int q = 0; q < 8; q++) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < CONTRACT_KTMAX; kb++) {
                if (kb < t.kt) {
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        if (nb0 + q < t.nt) {
                            const bf16x8 b = Bs[(kb * t.nt + nb0 + q) * 64 + lane];
#pragma unroll
                            for (int p = 0; p < 3; p++)
                                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[p][kb], b, acc[q], 0, 0, 0);
                        }
                    }
                }
            }
            // D: lane l holds rows 4 (l/16) + r, column l%16 of each tile
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int col = (nb0 + q) * 16 + (lane & 15);
                if (nb0 + q < t.nt && col < 2 * t.nr) {
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int64_t s = s0 + 4 * (lane >> 4) + r;
                        if (s < n) ((col & 1) ? zr : zf)[(int64_t)(col >> 1) * n + s] = (double)acc[q][r];
                    }
                }
            }
        }
    }
}

}  // namespace chem
