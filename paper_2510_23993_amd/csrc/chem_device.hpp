// Device building blocks for one reactor cell per lane (gfx950, FP64):
// NASA-7 thermo, log-form (matrix) rates of progress, the reactor
// right-hand side, its analytic Jacobian, an LU with partial pivoting kept
// in LDS, and the temperature inversion.  Templated on a generated
// mechanism-structure type M (species indices and stoichiometry are
// compile-time constants; numbers come from Params<M> in device memory).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "chem_math.hpp"
#include "chem_types.hpp"

namespace chem {

// Mechanism type with the mixed-precision rate evaluation: the same structure
// and parameter layout, exponentials of the rates on the FP32 units.
template <class B>
struct MixedOf : B {
    static constexpr int PREC = 1;
};

template <class M>
__device__ __forceinline__ double mexp(double x) {
    if constexpr (M::PREC) return exp32(x);
    else return exp(x);
}

template <class M>
__device__ __forceinline__ double mlog(double x) {
    if constexpr (M::PREC) return log32(x);
    else return log(x);
}

// The parameter block as seen by one evaluation.  The kernels run their
// evaluations inside loops; without this the compiler hoists every
// parameter load out of those loops and keeps hundreds of uniform values
// live across them (spilled to vector registers and scratch).  Passing the
// block's address through an empty asm makes it opaque, so each evaluation
// reloads its parameters through the scalar cache where it uses them.
template <class T>
__device__ __forceinline__ const T& fresh(const T& p) {
#if defined(__HIP_DEVICE_COMPILE__) && !defined(CHEM_NO_OPAQUE)
    // read-only for the whole kernel (constant address space): loads through
    // it go through the scalar cache
    const __attribute__((address_space(4))) T* q = (const __attribute__((address_space(4))) T*)&p;
    asm volatile("" : "+s"(q));
    return *(const T*)q;
#else
    return p;
#endif
}

// ---------------------------------------------------------------- thermo
// NASA-7 with pre-divided coefficients (host packs them):
//   h/RT = H0 + T(H1 + T(H2 + T(H3 + T H4))) + H5/T
//   s/R  = S0 lnT + T(S1 + T(S2 + T(S3 + T S4))) + S5
//   cp/R = C0 + T(C1 + T(C2 + T(C3 + T C4)))
// The low set applies iff T < Tmid (the polynomials are not clamped).
template <class M>
__device__ __forceinline__ void thermo_hg(const Params<M>& P, double T, double lnT, double invT,
                                          double* h_RT, double* g_RT) {
#pragma unroll
    for (int k = 0; k < M::NS; k++) {
        const bool lo = T < P.Tmid[k];
        double H[6], S[6];
#pragma unroll
        for (int a = 0; a < 6; a++) {
            H[a] = lo ? P.hlo[k][a] : P.hhi[k][a];
            S[a] = lo ? P.slo[k][a] : P.shi[k][a];
        }
        const double h = H[0] + T * (H[1] + T * (H[2] + T * (H[3] + T * H[4]))) + H[5] * invT;
        const double s = S[0] * lnT + T * (S[1] + T * (S[2] + T * (S[3] + T * S[4]))) + S[5];
        h_RT[k] = h;
        g_RT[k] = h - s;
    }
}

template <class M>
__device__ __forceinline__ double cp_R(const Params<M>& P, int k, double T) {
    const bool lo = T < P.Tmid[k];
    double c[5];
#pragma unroll
    for (int a = 0; a < 5; a++) c[a] = lo ? P.clo[k][a] : P.chi[k][a];
    return c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4])));
}

template <class M>
__device__ __forceinline__ double dcp_R_dT(const Params<M>& P, int k, double T) {
    const bool lo = T < P.Tmid[k];
    double c[5];
#pragma unroll
    for (int a = 0; a < 5; a++) c[a] = lo ? P.clo[k][a] : P.chi[k][a];
    return c[1] + T * (2.0 * c[2] + T * (3.0 * c[3] + T * 4.0 * c[4]));
}

template <class M>
__device__ __forceinline__ double h_RT_one(const Params<M>& P, int k, double T, double invT) {
    const bool lo = T < P.Tmid[k];
    double H[6];
#pragma unroll
    for (int a = 0; a < 6; a++) H[a] = lo ? P.hlo[k][a] : P.hhi[k][a];
    return H[0] + T * (H[1] + T * (H[2] + T * (H[3] + T * H[4]))) + H[5] * invT;
}

// e(T, Y) and c_v(T, Y), mass based
template <class M>
__device__ __forceinline__ void e_cv(const Params<M>& P, double T, const double* Y, double& e,
                                     double& cv) {
    const double invT = 1.0 / T;
    double se = 0.0, sc = 0.0;
#pragma unroll
    for (int k = 0; k < M::NS; k++) {
        const double w = Y[k] * P.invW[k];
        se += w * (h_RT_one(P, k, T, invT) - 1.0);
        sc += w * (cp_R(P, k, T) - 1.0);
    }
    e = se * RGAS * T;
    cv = sc * RGAS;
}

// Newton on e(T, Y) = e0 with a bisection guard in [100, 6000] K.
// Returns false if e0 is outside [e(100), e(6000)].
template <class M>
__device__ __forceinline__ bool T_from_e(const Params<M>& P, double e0, const double* Y, double Tg, double& Tout) {
    double lo = 100.0, hi = 6000.0, elo, ehi, cv;
    e_cv(P, lo, Y, elo, cv);
    e_cv(P, hi, Y, ehi, cv);
    if (!(elo <= e0 && ehi >= e0)) return false;
    double T = (Tg > lo && Tg < hi) ? Tg : 1500.0;
    for (int it = 0; it < 100; it++) {
        double e;
        e_cv(P, T, Y, e, cv);
        const double fT = e - e0;
        if (fT == 0.0) break;
        if (fT < 0.0) lo = T;
        else hi = T;
        double Tn = T - fT / cv;
        if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
        const double dT = fabs(Tn - T);
        T = Tn;
        if (dT <= 1e-12 * T || hi - lo <= 1e-12 * T) break;
    }
    Tout = T;
    return true;
}

// --------------------------------------------------------------- kinetics
constexpr double LN10 = 2.302585092994045684;
constexpr double INV_LN10 = 0.434294481903251828;
constexpr double LN_PREF_OVER_R = 9.408091968961747;  // ln(101325 / 8.314462618)

// Per-reaction log-space quantities: ln kf (falloff included) and, for
// falloff reactions, d ln kf / d ln [M] and d ln kf / dT.
struct RxnK {
    double lnkf, dlnkf_dT, dlnkf_dlnM, M;
};

template <class M, int j>
__device__ __forceinline__ void rxn_k(const Params<M>& P, double lnT, double invT, const double* C,
                                      RxnK& r, bool want_deriv) {
    constexpr int TY = M::TYPE[j];
    // Arrhenius as a contraction of (ln A, b, Ea/R) with (1, ln T, -1/T)
    double lnkinf = P.lnA[j] + P.b[j] * lnT - P.EaR[j] * invT;
    double dlnkinf = (P.b[j] + P.EaR[j] * invT) * invT;
    r.M = 0.0;
    if (TY != RX_ELEM) {
#pragma unroll
        for (int k = 0; k < M::NS; k++) r.M += P.eff[j][k] * C[k];
    }
    r.lnkf = lnkinf;
    r.dlnkf_dT = dlnkinf;
    r.dlnkf_dlnM = 0.0;
    if (TY == RX_FO) {
        const double lnk0 = P.lnA0[j] + P.b0[j] * lnT - P.Ea0R[j] * invT;
        const double dlnk0 = (P.b0[j] + P.Ea0R[j] * invT) * invT;
        const double Pr = fmax(mexp<M>(lnk0 - lnkinf) * r.M, 1e-300);
        const double lnPr = mlog<M>(Pr);
        double lnF = 0.0, dlnF_dlnPr = 0.0, dlnF_dT = 0.0;
        if (M::TROE[j] > 0) {
            const double a = P.troe[j][0], T = 1.0 / invT;
            const double e3 = mexp<M>(-T / P.troe[j][1]), e1 = mexp<M>(-T / P.troe[j][2]);
            double Fc = (1.0 - a) * e3 + a * e1;
            double dFc = -(1.0 - a) / P.troe[j][1] * e3 - a / P.troe[j][2] * e1;
            if (M::TROE[j] == 4) {
                const double e2 = mexp<M>(-P.troe[j][3] * invT);
                Fc += e2;
                dFc += P.troe[j][3] * invT * invT * e2;
            }
            const double phi = mlog<M>(Fc) * INV_LN10;
            const double c = -0.4 - 0.67 * phi, nn = 0.75 - 1.27 * phi;
            const double u = lnPr * INV_LN10 + c;
            const double den = nn - 0.14 * u;
            const double f1 = u / den;
            const double q = 1.0 + f1 * f1;
            lnF = LN10 * phi / q;
            if (want_deriv) {
                const double iq2 = 1.0 / (q * q), iden2 = 1.0 / (den * den);
                const double df1_dx = nn * iden2;
                const double df1_dphi = (-0.67 * den + u * (1.27 - 0.14 * 0.67)) * iden2;
                dlnF_dlnPr = -phi * 2.0 * f1 * df1_dx * iq2;
                const double dlog10F_dphi = 1.0 / q - phi * 2.0 * f1 * df1_dphi * iq2;
                dlnF_dT = dlog10F_dphi * dFc / Fc;
            }
        }
        const double ip = 1.0 / (1.0 + Pr);
        r.lnkf = lnkinf + lnPr + mlog<M>(ip) + lnF;   // ln(kinf Pr/(1+Pr) F)
        if (want_deriv) {
            const double dlnPr_dT = dlnk0 - dlnkinf;
            r.dlnkf_dlnM = ip + dlnF_dlnPr;
            r.dlnkf_dT = dlnkinf + dlnPr_dT * ip + dlnF_dT + dlnF_dlnPr * dlnPr_dT;
        }
    }
}

// Shared per-cell quantities for one evaluation.
template <class M>
struct CellEval {
    double C[M::NS], lnC[M::NS], h_RT[M::NS], g_RT[M::NS];
    double lnT, invT, lnPref;
    uint64_t neg;   // bit k set: C_k < 0
};

template <class M>
__device__ __forceinline__ void cell_eval(const Params<M>& P, double rho, const double* y,
                                          CellEval<M>& E) {
    const double T = y[M::NS];
    E.lnT = log(T);
    E.invT = 1.0 / T;
    E.lnPref = LN_PREF_OVER_R - E.lnT;
    // ln|C| with the sign kept aside: negative concentrations then give the
    // signed integer powers of the plain mass-action product
    static_assert(M::NS <= 64, "sign mask holds 64 species");
    E.neg = 0;
#pragma unroll
    for (int k = 0; k < M::NS; k++) {
        E.C[k] = rho * y[k] * P.invW[k];
        E.lnC[k] = log(fmax(fabs(E.C[k]), C_FLOOR));
        E.neg |= (uint64_t)(E.C[k] < 0.0) << k;
    }
    thermo_hg(P, T, E.lnT, E.invT, E.h_RT, E.g_RT);
}

// ln qf and ln qr of reaction j: stoichiometric contractions against ln C
// (forward: nu'; reverse: nu'' minus the ln Kc row).
template <class M, int j>
__device__ __forceinline__ void rxn_lnq(const CellEval<M>& E, double lnkf, double& lnqf,
                                        double& lnqr, double& sf, double& sr) {
    lnqf = lnkf;
    uint64_t pf = 0, pr = 0;   // parity of the negative factors with odd exponents
#pragma unroll
    for (int i = 0; i < M::NRE[j]; i++) {
        lnqf += M::RNU[j][i] * E.lnC[M::RSP[j][i]];
        if (M::RNU[j][i] & 1) pf ^= E.neg >> M::RSP[j][i];
    }
#pragma unroll
    for (int i = 0; i < M::NPR[j]; i++)
        if (M::PNU[j][i] & 1) pr ^= E.neg >> M::PSP[j][i];
    sf = (pf & 1) ? -1.0 : 1.0;
    sr = (pr & 1) ? -1.0 : 1.0;
    lnqr = -1e300;
    if (M::REV[j]) {
        double sg = 0.0;  // sum_k nu_kj g_k/RT
#pragma unroll
        for (int i = 0; i < M::NPR[j]; i++) sg += M::PNU[j][i] * E.g_RT[M::PSP[j][i]];
#pragma unroll
        for (int i = 0; i < M::NRE[j]; i++) sg -= M::RNU[j][i] * E.g_RT[M::RSP[j][i]];
        const double lnKc = -sg + M::DNU[j] * E.lnPref;
        lnqr = lnkf - lnKc;
#pragma unroll
        for (int i = 0; i < M::NPR[j]; i++) lnqr += M::PNU[j][i] * E.lnC[M::PSP[j][i]];
    }
}

// Net rate of progress of reaction j (times [M] for a third-body reaction).
template <class M, int j>
__device__ __forceinline__ double rxn_net(const Params<M>& P, const CellEval<M>& E) {
    RxnK r;
    rxn_k<M, j>(P, E.lnT, E.invT, E.C, r, false);
    double lnqf, lnqr, sf, sr;
    rxn_lnq<M, j>(E, r.lnkf, lnqf, lnqr, sf, sr);
    double q;
    if constexpr (M::PREC) {
        // FP32 exponentials: near equilibrium the net rate is -qf expm1(d)
        // with the FP64 log ratio d, not a difference of two rounded q's
        const double Ef = exp32(lnqf);
        q = sf * Ef;
        if (M::REV[j]) {
            const double d = lnqr - lnqf;
            if (sf == sr && fabs(d) < 0.35) q = -q * expm1_small(d);
            else q -= sr * exp32(lnqr);
        }
    } else {
        q = sf * exp(lnqf);
        if (M::REV[j]) q -= sr * exp(lnqr);
    }
    if (M::TYPE[j] == RX_TB) q *= r.M;
    return q;
}

template <class M, int j>
__device__ __forceinline__ void rxn_scatter(double q, double* om) {
#pragma unroll
    for (int i = 0; i < M::NRE[j]; i++) om[M::RSP[j][i]] -= M::RNU[j][i] * q;
#pragma unroll
    for (int i = 0; i < M::NPR[j]; i++) om[M::PSP[j][i]] += M::PNU[j][i] * q;
}

// Reactions are evaluated CHEM_RXN_GROUP at a time between scheduling
// barriers: the exp/log sequences of a group are independent and can
// interleave, while the barriers keep the scheduler from interleaving the
// whole reaction list (whose live ranges would overflow the register file).
#ifndef CHEM_RXN_GROUP
#define CHEM_RXN_GROUP 1
#endif

template <class M, int j>
__device__ __forceinline__ void rhs_loop(const Params<M>& P, const CellEval<M>& E, double* om) {
    if constexpr (j < M::NR) {
        constexpr int G = CHEM_RXN_GROUP;
        double q[G];
        q[0] = rxn_net<M, j>(P, E);
        if constexpr (G > 1 && j + 1 < M::NR) q[1] = rxn_net<M, (j + 1 < M::NR ? j + 1 : j)>(P, E);
        if constexpr (G > 2 && j + 2 < M::NR) q[2] = rxn_net<M, (j + 2 < M::NR ? j + 2 : j)>(P, E);
        rxn_scatter<M, j>(q[0], om);
        if constexpr (G > 1 && j + 1 < M::NR) rxn_scatter<M, (j + 1 < M::NR ? j + 1 : j)>(q[1], om);
        if constexpr (G > 2 && j + 2 < M::NR) rxn_scatter<M, (j + 2 < M::NR ? j + 2 : j)>(q[2], om);
        __builtin_amdgcn_sched_barrier(0);
        rhs_loop<M, j + G>(P, E, om);
    }
}

// f = dy/dt for y = (Y_1..Y_NS, T) at constant rho and e.
template <class M>
__device__ __forceinline__ void rhs(const Params<M>& Pin, double rho, const double* y, double* f) {
    const Params<M>& P = fresh(Pin);
    CellEval<M> E;
    cell_eval(P, rho, y, E);
    double om[M::NS];
#pragma unroll
    for (int k = 0; k < M::NS; k++) om[k] = 0.0;
    rhs_loop<M, 0>(P, E, om);
    const double T = y[M::NS];
    double cvs = 0.0, S = 0.0;
    const double irho = 1.0 / rho;
#pragma unroll
    for (int k = 0; k < M::NS; k++) {
        f[k] = P.W[k] * om[k] * irho;
        cvs += y[k] * P.invW[k] * (cp_R(P, k, T) - 1.0);
        S += (E.h_RT[k] - 1.0) * om[k];
    }
    // -sum u_k om_k/(rho cv) with u_k = (h_RT - 1) R T and cv = R cvs
    f[M::NS] = -S * T * irho / cvs;
}

// ---------------------------------------------------------------- Jacobian
// Analytic Jacobian of the reactor RHS, organised for registers: one pass
// over the reactions keeps each reaction's forward and reverse rates of
// progress (times [M] for third-body reactions) and the dense third-body /
// falloff factor, together with the production rates and their temperature
// derivatives; a second pass builds dω/dC one column at a time,
//   G[k][m] = (1/C_m) Σ_j ν_kj (ν'_mj qf_j − ν''_mj qr_j) + Σ_j ν_kj α_jm g_j,
// whose stoichiometric products are compile-time constants, and hands each
// finished entry over scaled, J[k][m] = (W_k / W_m) G[k][m], through
// store(i, j, v) (every entry of the n x n Jacobian exactly once, the
// species block by columns, then the temperature column).
template <class M, int j>
__device__ __forceinline__ void jc_rates(const Params<M>& P, const CellEval<M>& E, double* QF, double* QR,
                                         double* G, double* om, double* dwT) {
    if constexpr (j < M::NR) {
        constexpr int TY = M::TYPE[j];
        RxnK r;
        rxn_k<M, j>(P, E.lnT, E.invT, E.C, r, true);
        double lnqf, lnqr, sf, sr;
        rxn_lnq<M, j>(E, r.lnkf, lnqf, lnqr, sf, sr);
        const double qf = sf * mexp<M>(lnqf);
        const double qr = M::REV[j] ? sr * mexp<M>(lnqr) : 0.0;
        const double mul = (TY == RX_TB) ? r.M : 1.0;
        double dlnKc = 0.0;
        if (M::REV[j]) {
            double sh = 0.0;
#pragma unroll
            for (int i = 0; i < M::NPR[j]; i++) sh += M::PNU[j][i] * E.h_RT[M::PSP[j][i]];
#pragma unroll
            for (int i = 0; i < M::NRE[j]; i++) sh -= M::RNU[j][i] * E.h_RT[M::RSP[j][i]];
            dlnKc = (sh - M::DNU[j]) * E.invT;
        }
        const double net = qf - qr;
        const double q = mul * net;
        const double dqdT = mul * (qf * r.dlnkf_dT - qr * (r.dlnkf_dT - dlnKc));
        QF[j] = mul * qf;
        QR[j] = mul * qr;
        G[j] = (TY == RX_TB) ? net : ((TY == RX_FO) ? net * r.dlnkf_dlnM / fmax(r.M, 1e-300) : 0.0);
#pragma unroll
        for (int i = 0; i < M::NRE[j]; i++) {
            om[M::RSP[j][i]] -= M::RNU[j][i] * q;
            dwT[M::RSP[j][i]] -= M::RNU[j][i] * dqdT;
        }
#pragma unroll
        for (int i = 0; i < M::NPR[j]; i++) {
            om[M::PSP[j][i]] += M::PNU[j][i] * q;
            dwT[M::PSP[j][i]] += M::PNU[j][i] * dqdT;
        }
        __builtin_amdgcn_sched_barrier(0);
        jc_rates<M, j + 1>(P, E, QF, QR, G, om, dwT);
    }
}

// signed stoichiometric coefficient of species k in reaction j (products
// positive, reactants negative), summed over the participant lists
template <class M>
__device__ __forceinline__ constexpr int nu_of(int j, int k) {
    int v = 0;
    for (int i = 0; i < M::NPR[j]; i++)
        if (M::PSP[j][i] == k) v += M::PNU[j][i];
    for (int i = 0; i < M::NRE[j]; i++)
        if (M::RSP[j][i] == k) v -= M::RNU[j][i];
    return v;
}

template <class M>
__device__ __forceinline__ constexpr int nuf_of(int j, int k) {   // reactant coefficient
    int v = 0;
    for (int i = 0; i < M::NRE[j]; i++)
        if (M::RSP[j][i] == k) v += M::RNU[j][i];
    return v;
}

template <class M>
__device__ __forceinline__ constexpr int nur_of(int j, int k) {   // product coefficient
    int v = 0;
    for (int i = 0; i < M::NPR[j]; i++)
        if (M::PSP[j][i] == k) v += M::PNU[j][i];
    return v;
}

template <class M, class Store>
__device__ __forceinline__ void jac_cols(const Params<M>& Pin, double rho, const double* y, Store store) {
    const Params<M>& P = fresh(Pin);
    constexpr int NS = M::NS, NR = M::NR;
    CellEval<M> E;
    cell_eval(P, rho, y, E);
    const double T = y[NS];
    double invC[NS], om[NS], dwT[NS], QF[NR], QR[NR], G[NR];
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const double aC = fmax(fabs(E.C[k]), C_FLOOR);
        invC[k] = (E.C[k] < 0.0) ? -1.0 / aC : 1.0 / aC;
        om[k] = dwT[k] = 0.0;
    }
    jc_rates<M, 0>(P, E, QF, QR, G, om, dwT);
    double uk[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) uk[k] = (E.h_RT[k] - 1.0) * T;   // u_k / R (molar)
    const double irho = 1.0 / rho;
    double cvs = 0.0, dcvs = 0.0, S = 0.0;
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const double cvk = cp_R(P, k, T) - 1.0;   // c_v,k / R (molar)
        cvs += y[k] * P.invW[k] * cvk;
        dcvs += y[k] * P.invW[k] * dcp_R_dT(P, k, T);
        S += uk[k] * om[k];
    }
    const double fT = -S * irho / cvs;
    const double icvs = 1.0 / cvs;
    // species columns
#pragma unroll
    for (int m = 0; m < NS; m++) {
        double col[NS];
#pragma unroll
        for (int k = 0; k < NS; k++) col[k] = 0.0;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const int af = nuf_of<M>(j, m), ar = M::REV[j] ? nur_of<M>(j, m) : 0;
            if (af != 0 || ar != 0) {
                const double d = (af != 0 ? af * QF[j] : 0.0) - (ar != 0 ? ar * QR[j] : 0.0);
#pragma unroll
                for (int k = 0; k < NS; k++) {
                    const int nk = nu_of<M>(j, k);
                    if (nk != 0) col[k] += nk * d;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NS; k++) col[k] *= invC[m];
#pragma unroll
        for (int j = 0; j < NR; j++) {
            if (M::TYPE[j] != RX_ELEM) {
                const double d = P.eff[j][m] * G[j];
#pragma unroll
                for (int k = 0; k < NS; k++) {
                    const int nk = nu_of<M>(j, k);
                    if (nk != 0) col[k] += nk * d;
                }
            }
        }
        double dS = 0.0;
#pragma unroll
        for (int k = 0; k < NS; k++) {
            dS += uk[k] * col[k];
            store(k, m, (P.W[k] * P.invW[m]) * col[k]);
        }
        const double cvm = cp_R(P, m, T) - 1.0;
        store(NS, m, -P.invW[m] * icvs * (dS + fT * cvm));
        __builtin_amdgcn_sched_barrier(0);
    }
    // temperature column
    double dS = 0.0;
#pragma unroll
    for (int k = 0; k < NS; k++) {
        dS += (cp_R(P, k, T) - 1.0) * om[k] + uk[k] * dwT[k];
        store(k, NS, P.W[k] * irho * dwT[k]);
    }
    store(NS, NS, -dS * irho * icvs - fT * dcvs * icvs);
}

// Lanes of a 64-lane workgroup that carry a cell.  Each carries its NN x NN
// Newton matrix in LDS; the register file allows 4 such waves per CU, so the
// workgroup uses fewer than 64 lanes when that lets a fourth one fit in the
// CU's 160 KB (9 x 9 FP64 per lane: 63 lanes; 10 x 10: 51).
template <class M>
constexpr int lanes_per_wave() {
    constexpr int per_lane = M::NN * M::NN * 8;
    constexpr int lw = (160 * 1024 / 4) / per_lane;
    return lw >= 64 ? 64 : lw;
}

// Newton matrix A = I - c J over the Newton system (species that react, then
// T; inert species are left out) written to LDS: element (r, c) at
// A[(r*NN + c)*LW].
template <class M>
__device__ __forceinline__ void newton_matrix(const Params<M>& P, double rho, const double* y,
                                              double c, double* A) {
    constexpr int NN = M::NN, LW = lanes_per_wave<M>();
    jac_cols<M>(P, rho, y, [&](int i, int j, double v) {
        const int si = M::SYS[i], sj = M::SYS[j];
        if (si >= 0 && sj >= 0) A[(si * NN + sj) * LW] = (si == sj ? 1.0 : 0.0) - c * v;
    });
}

// --------------------------------------------------------------- dense LU
// In-place LU with partial pivoting of the lane's N x N matrix in LDS
// (element (r, c) at A[(r*N + c)*LW]).  The diagonal is replaced by its
// reciprocal; pivot rows go to piv[].  Rows are swapped only from column k
// on, and solves replay the same sequence of interchanges.  Returns false
// if a pivot is zero or not finite.
template <int N, int LW>
__device__ __forceinline__ bool lu_factor(double* A, int* piv) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < N; k++) {
        int p = k;
        double best = fabs(A[(k * N + k) * LW]);
#pragma unroll
        for (int i = k + 1; i < N; i++) {
            const double v = fabs(A[(i * N + k) * LW]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        piv[k] = p;
        if (!(best > 0.0) || !isfinite(best)) ok = false;
        if (p != k) {
#pragma unroll
            for (int c = k; c < N; c++) {
                const double t = A[(k * N + c) * LW];
                A[(k * N + c) * LW] = A[(p * N + c) * LW];
                A[(p * N + c) * LW] = t;
            }
        }
        double rowk[N];
#pragma unroll
        for (int c = k; c < N; c++) rowk[c] = A[(k * N + c) * LW];
        const double inv = 1.0 / rowk[k];
        A[(k * N + k) * LW] = inv;
#pragma unroll
        for (int i = k + 1; i < N; i++) {
            const double l = A[(i * N + k) * LW] * inv;
            A[(i * N + k) * LW] = l;
#pragma unroll
            for (int c = k + 1; c < N; c++) A[(i * N + c) * LW] -= l * rowk[c];
        }
    }
    return ok;
}

template <int N, int LW>
__device__ __forceinline__ void lu_solve(const double* A, const int* piv, double* b) {
#pragma unroll
    for (int k = 0; k < N; k++) {
        // interchange b[k] <-> b[piv[k]] (piv[k] >= k) with selects: b stays in registers
        const int p = piv[k];
#pragma unroll
        for (int i = k + 1; i < N; i++) {
            const bool s = (p == i);
            const double bk = b[k], bi = b[i];
            b[k] = s ? bi : bk;
            b[i] = s ? bk : bi;
        }
        const double bk = b[k];
#pragma unroll
        for (int i = k + 1; i < N; i++) b[i] -= A[(i * N + k) * LW] * bk;
    }
#pragma unroll
    for (int i = N - 1; i >= 0; i--) {
        double s = b[i];
#pragma unroll
        for (int c = i + 1; c < N; c++) s -= A[(i * N + c) * LW] * b[c];
        b[i] = s * A[(i * N + i) * LW];
    }
}

}  // namespace chem
