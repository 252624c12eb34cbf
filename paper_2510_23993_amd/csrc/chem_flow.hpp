// The minimal compressible flow step around the chemistry (Sec. 2.1: HLLC
// convective fluxes, second-order SSP Runge-Kutta, operator splitting of the
// chemical source), one dimension, for the Strang-split coupling
// flow dt/2 -> chemistry dt -> flow dt/2.
//
// State per cell, SoA over cells (U[v*ldU + i]):
//   U = (rho, rho u, rho E, rho Y_1 .. rho Y_ns),  E = e + u^2/2,
// e the mass-specific internal energy including formation energy (the same
// e as the chemistry's).  Piecewise-linear reconstruction of (rho, u, p, Y)
// with the minmod limiter, HLLC with the direct wave-speed estimates
// S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R) (Toro,
// Riemann Solvers and Numerical Methods for Fluid Dynamics, Sec. 10.4-10.6),
// frozen sound speed c^2 = gamma p / rho, species carried with the contact,
// transmissive ends (cells outside the tube take the end cell's values).
// All three kernels are HBM-bound streaming passes: one lane per cell or
// face, coalesced component-major loads.
#pragma once
#include <hip/hip_runtime.h>

#include "chem_device.hpp"

namespace chem {

// Per cell: U -> primitive Q = (rho, u, p, Y_1..Y_ns) and T (Newton on e
// with the previous T as the guess).  Cells whose inversion fails (a state
// outside the thermo's bracket) keep the guess and are counted in *bad.
template <class M>
__global__ void __launch_bounds__(256) k_flow_prim(const Params<M>* __restrict__ Pp, int64_t n,
                                                   const double* __restrict__ U, int64_t ldU,
                                                   double* __restrict__ Q, double* __restrict__ T,
                                                   int* __restrict__ bad) {
    const Params<M>& P = *Pp;
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const double rho = U[i], irho = 1.0 / rho;
    const double u = U[ldU + i] * irho;
    const double e = U[2 * ldU + i] * irho - 0.5 * u * u;
    double Y[M::NS], sw = 0.0;
#pragma unroll
    for (int k = 0; k < M::NS; k++) {
        Y[k] = U[(3 + k) * ldU + i] * irho;
        sw += Y[k] * P.invW[k];
    }
    double Tn;
    if (!(rho > 0.0) || !T_from_e(P, e, Y, T[i], Tn)) {
        atomicAdd(bad, 1);
        Tn = T[i];
    }
    T[i] = Tn;
    Q[i] = rho;
    Q[n + i] = u;
    Q[2 * n + i] = rho * RGAS * Tn * sw;
#pragma unroll
    for (int k = 0; k < M::NS; k++) Q[(3 + k) * n + i] = Y[k];
}

__device__ __forceinline__ double minmod(double a, double b) {
    return (a * b > 0.0) ? (fabs(a) < fabs(b) ? a : b) : 0.0;
}

// Face state thermo from (rho, p, Y): e and the frozen sound speed.
template <class M>
__device__ __forceinline__ void face_thermo(const Params<M>& P, double rho, double p, const double* Y, double& e,
                                            double& c) {
    double sw = 0.0;
#pragma unroll
    for (int k = 0; k < M::NS; k++) sw += Y[k] * P.invW[k];
    const double T = p / (rho * RGAS * sw);
    double cv;
    e_cv(P, T, Y, e, cv);
    const double cp = cv + RGAS * sw;
    c = sqrt(cp / cv * p / rho);
}

// Per face f = 0..n (between cells f-1 and f): MUSCL-minmod states and the
// HLLC flux, F[v*(n+1) + f].
template <class M>
__global__ void __launch_bounds__(256) k_flow_flux(const Params<M>* __restrict__ Pp, int64_t n,
                                                   const double* __restrict__ Q, double* __restrict__ F) {
    constexpr int NQ = 3 + M::NS;
    const Params<M>& P = *Pp;
    const int64_t f = blockIdx.x * 256ll + threadIdx.x;
    if (f > n) return;
    auto cl = [&](int64_t j) { return j < 0 ? 0 : (j >= n ? n - 1 : j); };
    const int64_t a = cl(f - 2), b = cl(f - 1), c = cl(f), d = cl(f + 1);
    double qL[NQ], qR[NQ];
#pragma unroll
    for (int v = 0; v < NQ; v++) {
        const double qa = Q[v * n + a], qb = Q[v * n + b], qc = Q[v * n + c], qd = Q[v * n + d];
        qL[v] = qb + 0.5 * minmod(qb - qa, qc - qb);
        qR[v] = qc - 0.5 * minmod(qc - qb, qd - qc);
    }
    const double rL = qL[0], uL = qL[1], pL = qL[2], rR = qR[0], uR = qR[1], pR = qR[2];
    double eL, cL, eR, cR;
    face_thermo(P, rL, pL, qL + 3, eL, cL);
    face_thermo(P, rR, pR, qR + 3, eR, cR);
    const double EL = rL * (eL + 0.5 * uL * uL), ER = rR * (eR + 0.5 * uR * uR);
    const double SL = fmin(uL - cL, uR - cR), SR = fmax(uL + cL, uR + cR);
    const double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR));
    // the upwind side of the contact; inside the wave fan the flux is
    // F_K + S_K (U*_K - U_K) with the star state U*_K of that side
    const bool left = 0.0 <= Ss;
    const double r = left ? rL : rR, u = left ? uL : uR, p = left ? pL : pR, E = left ? EL : ER;
    const double S = left ? SL : SR;
    const double* Yk = left ? qL + 3 : qR + 3;
    const bool outside = left ? (0.0 <= SL) : (SR <= 0.0);
    double dU[3] = {0.0, 0.0, 0.0}, dr = 0.0;
    if (!outside) {
        const double fs = r * (S - u) / (S - Ss);
        dr = S * (fs - r);
        dU[0] = dr;
        dU[1] = S * (fs * Ss - r * u);
        dU[2] = S * (fs * (E / r + (Ss - u) * (Ss + p / (r * (S - u)))) - E);
    }
    const double Fk[3] = {r * u, r * u * u + p, u * (E + p)};
    const int64_t ld = n + 1;
#pragma unroll
    for (int v = 0; v < 3; v++) F[v * ld + f] = Fk[v] + dU[v];
#pragma unroll
    for (int k = 0; k < M::NS; k++) F[(3 + k) * ld + f] = (r * u + dr) * Yk[k];
}

// U_out = a U_base + b (U_cur - dt/dx (F_{i+1/2} - F_{i-1/2})) for nv
// components (every pointer valid; the three arrays have their own strides)
__global__ void __launch_bounds__(256) k_flow_update(int64_t n, int nv, double dt_dx, double a, double b,
                                                     const double* Ubase, int64_t ldb, const double* Ucur,
                                                     int64_t ldc, const double* __restrict__ F, double* Uout,
                                                     int64_t ldo) {
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const int64_t ld = n + 1;
    for (int v = 0; v < nv; v++) {
        const double L = Ucur[v * ldc + i] - dt_dx * (F[v * ld + i + 1] - F[v * ld + i]);
        Uout[v * ldo + i] = a * Ubase[v * ldb + i] + b * L;
    }
}

// Chemistry inputs from U: rho, e and Y (the T guess is already in T).
__global__ void __launch_bounds__(256) k_flow_to_chem(int64_t n, int ns, const double* __restrict__ U, int64_t ldU,
                                                      double* __restrict__ rho, double* __restrict__ e,
                                                      double* __restrict__ Y) {
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const double r = U[i], ir = 1.0 / r, u = U[ldU + i] * ir;
    rho[i] = r;
    e[i] = U[2 * ldU + i] * ir - 0.5 * u * u;
    for (int k = 0; k < ns; k++) Y[k * n + i] = U[(3 + k) * ldU + i] * ir;
}

// After the chemistry (rho and e unchanged): rho Y_k from the new Y.
__global__ void __launch_bounds__(256) k_chem_to_flow(int64_t n, int ns, const double* __restrict__ Y,
                                                      double* __restrict__ U, int64_t ldU) {
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const double r = U[i];
    for (int k = 0; k < ns; k++) U[(3 + k) * ldU + i] = r * Y[k * n + i];
}

}  // namespace chem
