// Learned-surrogate pass of the chemistry step (one cell per lane, FP64
// checks): features of the compacted active cells, the network (BF16 MFMA),
// and a trust check that accepts a predicted increment or hands the cell to
// the implicit integrator.
//
// Trust check, all in FP64.  Every prediction is decoded, projected onto
// element conservation (weighted by |Y0| + 1e-12) and must keep every mass
// fraction >= -10 atol and a temperature, recovered from the fixed internal
// energy, within 0.5 K of the predicted one; every feature vector must lie in
// the training envelope.  The accuracy test is the semigroup property of the
// exact flow: the one-step prediction y1 = N(y0, dt) must agree with the
// two-step y1' = N(N(y0, dt/2), dt/2) in the weighted RMS norm with weights
// 1/(rtol_s max(|y1|, |y1'|) + atol).  (A one-step defect test such as the
// trapezoidal rule is not usable here: the exact increment itself fails it
// whenever fast radical modes relax within dt.)
#pragma once
#include <hip/hip_runtime.h>

#include "chem_coop.hpp"
#include "chem_device.hpp"
#include "chem_kernels.hpp"
#include "chem_mlp.hpp"
#include "chem_types.hpp"

namespace chem {

constexpr int SURR_NS = 9;       // species of the network's input and output
constexpr int SURR_NEMAX = 4;    // elements handled by the projection
constexpr double SURR_ATM = 101325.0;
constexpr double SURR_YCLIP = 1e-20;
constexpr double SURR_SREL = 1e-4, SURR_SABS = 1e-14;   // increment scales of the targets
constexpr double SURR_DT_TOL = 0.5;                     // K, predicted vs recovered T
enum { SURR_OK = 1, SURR_WHY_ENV = 0, SURR_WHY_NEG = 2, SURR_WHY_T = 3 };

struct SurrTables {
    float mean_x[mlp::NIN], sd_x[mlp::NIN], mean_t[mlp::NOUT], sd_t[mlp::NOUT];
    double env_lo[mlp::NIN], env_hi[mlp::NIN];   // raw-feature training envelope
    double A[SURR_NEMAX][SURR_NS];               // element count / molar mass
    int ne;
};

// standardised features of (y, dt) into X[12]; true if inside the envelope
template <class M>
__device__ __forceinline__ bool surr_features(const Params<M>& P, const SurrTables* __restrict__ tb, const double* y,
                                              double rho, double dt, float* __restrict__ X) {
    double x[mlp::NIN], sw = 0.0;
#pragma unroll
    for (int k = 0; k < SURR_NS; k++) {
        sw += y[k] * P.invW[k];
        x[2 + k] = log(fmax(y[k], SURR_YCLIP));
    }
    x[0] = y[SURR_NS];
    x[1] = log(rho * RGAS * y[SURR_NS] * sw / SURR_ATM);
    x[11] = log(dt);
    bool in = true;
#pragma unroll
    for (int c = 0; c < mlp::NIN; c++) {
        in = in && x[c] >= tb->env_lo[c] && x[c] <= tb->env_hi[c];
        X[c] = (float)((x[c] - tb->mean_x[c]) / tb->sd_x[c]);
    }
    return in;
}

// network output row -> end state y1 (projected, T from e); returns SURR_OK or a reason
template <class M>
__device__ __forceinline__ int surr_decode(const Params<M>& P, const SurrTables* __restrict__ tb,
                                           const float* __restrict__ o, const double* y0, double e0, double atol,
                                           double* y1) {
    constexpr int NS = SURR_NS;
    double dY[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const double raw = (double)o[k] * tb->sd_t[k] + tb->mean_t[k];
        dY[k] = sinh(raw) * (SURR_SREL * fabs(y0[k]) + SURR_SABS);
    }
    const double rawT = (double)o[NS] * tb->sd_t[NS] + tb->mean_t[NS];
    const double Tpred = y0[NS] + sinh(rawT) * SURR_SREL * y0[NS];
    // element conservation: dY -= D A^T (A D A^T)^-1 A dY, D = |Y0| + 1e-12
    const int ne = tb->ne;
    double Mm[SURR_NEMAX][SURR_NEMAX + 1];
#pragma unroll
    for (int a = 0; a < SURR_NEMAX; a++) {
#pragma unroll
        for (int b = 0; b <= SURR_NEMAX; b++) Mm[a][b] = (a == b && a >= ne) ? 1.0 : 0.0;
        if (a < ne) {
#pragma unroll
            for (int k = 0; k < NS; k++) {
                const double Dk = fabs(y0[k]) + 1e-12;
                Mm[a][SURR_NEMAX] += tb->A[a][k] * dY[k];
#pragma unroll
                for (int b = 0; b < SURR_NEMAX; b++)
                    if (b < ne) Mm[a][b] += tb->A[a][k] * tb->A[b][k] * Dk;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < SURR_NEMAX; c++) {   // Gauss-Jordan, symmetric positive definite
        const double piv = 1.0 / Mm[c][c];
#pragma unroll
        for (int b = 0; b <= SURR_NEMAX; b++) Mm[c][b] *= piv;
#pragma unroll
        for (int a = 0; a < SURR_NEMAX; a++)
            if (a != c) {
                const double f = Mm[a][c];
#pragma unroll
                for (int b = 0; b <= SURR_NEMAX; b++) Mm[a][b] -= f * Mm[c][b];
            }
    }
    bool pos = true;
#pragma unroll
    for (int k = 0; k < NS; k++) {
        double corr = 0.0;
#pragma unroll
        for (int a = 0; a < SURR_NEMAX; a++)
            if (a < ne) corr += tb->A[a][k] * Mm[a][SURR_NEMAX];
        y1[k] = y0[k] + dY[k] - (fabs(y0[k]) + 1e-12) * corr;
        pos = pos && isfinite(y1[k]) && y1[k] >= -10.0 * atol;
    }
    if (!pos) return SURR_WHY_NEG;
    double T1 = Tpred;
    if (!(isfinite(Tpred) && T_from_e(P, e0, y1, Tpred, T1) && fabs(T1 - Tpred) <= SURR_DT_TOL)) return SURR_WHY_T;
    y1[NS] = T1;
    return SURR_OK;
}

template <class M>
__device__ __forceinline__ void surr_load(const DevBox* __restrict__ boxes, int nbox, int64_t g, double* y, double& rho,
                                          double& e0, double& dt, const DevBox*& Bp, int64_t& i) {
    const DevBox& B = boxes[find_box(boxes, nbox, g)];
    i = g - B.off;
#pragma unroll
    for (int k = 0; k < SURR_NS; k++) y[k] = B.Y[k * B.ldY + i];
    y[SURR_NS] = B.T[i];
    rho = B.rho[i];
    e0 = B.e[i];
    dt = B.dt;
    Bp = &B;
}

// stage 1: features of (y0, dt) into rows [0, n) and (y0, dt/2) into rows [cap, cap + n)
template <class M>
__global__ void __launch_bounds__(256) k_surr_prep(const Params<M>* __restrict__ Pp, const SurrTables* __restrict__ tb,
                                                   const DevBox* __restrict__ boxes, int nbox,
                                                   const int* __restrict__ ids, const int* __restrict__ n_act,
                                                   int64_t cap, float* __restrict__ X, uint8_t* __restrict__ ok) {
    const Params<M>& P = *Pp;
    const int n = *n_act;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        double y[M::N], rho, e0, dt;
        const DevBox* B;
        int64_t i;
        surr_load<M>(boxes, nbox, ids[s], y, rho, e0, dt, B, i);
        const bool a = surr_features(P, tb, y, rho, dt, X + (int64_t)s * mlp::NIN);
        const bool b = surr_features(P, tb, y, rho, 0.5 * dt, X + (cap + s) * mlp::NIN);
        ok[s] = (a && b) ? SURR_OK : SURR_WHY_ENV;
    }
}

// stage 2: half-step state from rows [cap, cap + n) of the output, its
// features (dt/2) into rows [2 cap, 2 cap + n)
template <class M>
__global__ void __launch_bounds__(64) k_surr_mid(const Params<M>* __restrict__ Pp, const SurrTables* __restrict__ tb,
                                                 const DevBox* __restrict__ boxes, int nbox,
                                                 const int* __restrict__ ids, const int* __restrict__ n_act,
                                                 int64_t cap, const float* __restrict__ out, float* __restrict__ X,
                                                 double* __restrict__ yh, uint8_t* __restrict__ ok, double atol) {
    constexpr int N = M::N;
    const Params<M>& P = *Pp;
    const int n = *n_act;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        double y0[N], y1[N], rho, e0, dt;
        const DevBox* B;
        int64_t i;
        surr_load<M>(boxes, nbox, ids[s], y0, rho, e0, dt, B, i);
        int r = ok[s];
        if (r == SURR_OK) r = surr_decode(P, tb, out + (cap + s) * mlp::NOUT, y0, e0, atol, y1);
        if (r == SURR_OK) {
#pragma unroll
            for (int k = 0; k < N; k++) yh[(int64_t)k * cap + s] = y1[k];
            if (!surr_features(P, tb, y1, rho, 0.5 * dt, X + (2 * cap + s) * mlp::NIN)) r = SURR_WHY_ENV;
        } else {
#pragma unroll
            for (int c = 0; c < mlp::NIN; c++) X[(2 * cap + s) * mlp::NIN + c] = 0.f;
        }
        ok[s] = (uint8_t)r;
    }
}

// stage 3: decide.  One-step prediction from rows [0, n), two-step from rows
// [2 cap, 2 cap + n) applied to the half-step state.
template <class M>
__global__ void __launch_bounds__(64) k_surr_accept(const Params<M>* __restrict__ Pp, const SurrTables* __restrict__ tb,
                                                    const DevBox* __restrict__ boxes, int nbox,
                                                    const int* __restrict__ ids, const int* __restrict__ n_act,
                                                    int64_t cap, const float* __restrict__ out,
                                                    const double* __restrict__ yh, const uint8_t* __restrict__ ok,
                                                    uint8_t* __restrict__ flag, uint8_t* __restrict__ st_int,
                                                    double rtol_s, double atol, Counters* __restrict__ ct) {
    constexpr int NS = M::NS, N = M::N;
    static_assert(NS == SURR_NS, "the surrogate network is built for 9 species");
    const Params<M>& P = *Pp;
    const int n = *n_act;
    unsigned long long n_ok = 0, n_rej = 0, why[4] = {0, 0, 0, 0};
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        const int64_t g = ids[s];
        double y0[N], y1[N], ym[N], y2[N], rho, e0, dt;
        const DevBox* B;
        int64_t i;
        surr_load<M>(boxes, nbox, g, y0, rho, e0, dt, B, i);
        int r = ok[s];
        if (r == SURR_OK) r = surr_decode(P, tb, out + (int64_t)s * mlp::NOUT, y0, e0, atol, y1);
        if (r == SURR_OK) {
#pragma unroll
            for (int k = 0; k < N; k++) ym[k] = yh[(int64_t)k * cap + s];
            r = surr_decode(P, tb, out + (2 * cap + s) * mlp::NOUT, ym, e0, atol, y2);
        }
        bool acc = r == SURR_OK;
        if (acc) {
            double ss = 0.0;
#pragma unroll
            for (int k = 0; k < N; k++) {
                const double d = y1[k] - y2[k];
                const double w = rtol_s * fmax(fabs(y1[k]), fabs(y2[k])) + atol;
                ss += (d / w) * (d / w);
            }
            acc = isfinite(ss) && ss <= (double)N;
            if (!acc) why[3]++;
        } else {
            why[r == SURR_WHY_ENV ? 0 : (r == SURR_WHY_NEG ? 1 : 2)]++;
        }
        if (acc) {
#pragma unroll
            for (int k = 0; k < NS; k++) B->Y[k * B->ldY + i] = y1[k];
            B->T[i] = y1[NS];
            if (B->status) B->status[i] = ST_SURR_OK;
            st_int[g] = ST_SURR_OK;
            flag[s] = 2;
            n_ok++;
        } else {
            st_int[g] = ST_SURR_REJ;
            n_rej++;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        n_ok += __shfl_xor(n_ok, o);
        n_rej += __shfl_xor(n_rej, o);
#pragma unroll
        for (int r = 0; r < 4; r++) why[r] += __shfl_xor(why[r], o);
    }
    if (threadIdx.x == 0) {
        atomicAdd(&ct->surr_ok, n_ok);
        atomicAdd(&ct->surr_rej, n_rej);
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (why[r]) atomicAdd(&ct->surr_why[r], why[r]);
    }
}

// Training pairs: raw features of (rho, Y0, T0, dt) and raw targets of the
// increment to (Y1, T1), written as FP32 rows; the arithmetic is FP64.
__global__ void __launch_bounds__(256) k_surr_pairs(CoopMech M, int64_t n, const double* __restrict__ rho,
                                                    const double* __restrict__ Y0, const double* __restrict__ T0,
                                                    const double* __restrict__ Y1, const double* __restrict__ T1,
                                                    const double* __restrict__ dt, float* __restrict__ X,
                                                    float* __restrict__ Tg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double T = T0[i];
        double sw = 0.0;
        for (int k = 0; k < SURR_NS; k++) {
            const double y = Y0[k * n + i], y1 = Y1[k * n + i];
            sw += y * M.sp[(size_t)k * SPS + SP_INVW];
            X[i * mlp::NIN + 2 + k] = (float)log(fmax(y, SURR_YCLIP));
            Tg[i * mlp::NOUT + k] = (float)asinh((y1 - y) / (SURR_SREL * fabs(y) + SURR_SABS));
        }
        X[i * mlp::NIN + 0] = (float)T;
        X[i * mlp::NIN + 1] = (float)log(rho[i] * RGAS * T * sw / SURR_ATM);
        X[i * mlp::NIN + 11] = (float)log(dt[i]);
        Tg[i * mlp::NOUT + SURR_NS] = (float)asinh((T1[i] - T) / (SURR_SREL * T));
    }
}

}  // namespace chem
