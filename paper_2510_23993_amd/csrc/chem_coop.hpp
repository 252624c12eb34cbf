// Cooperative schedule: a group of G lanes integrates one reactor cell
// (64/G cells per wave).  Component i of the state (Y_1..Y_ns, T) and row i
// of the Newton matrix live in registers of lane i % G, slot i / G.  The
// mechanism is data driven (runtime tables), so one kernel family serves any
// mechanism up to G*R components:
//   - species phase: each lane evaluates its species' thermo and ln C and
//     publishes ln C, C, 1/C, g/RT in the group's LDS area;
//   - reaction phase: lane l evaluates reactions l, l+G, ... (ln k_f as a
//     contraction of (ln A, b, Ea/R) with (1, ln T, -1/T); ln q_f / ln q_r as
//     contractions of nu', nu'' against ln C and of nu against g/RT; exp) and
//     writes the rates of progress to LDS;
//   - production / Jacobian rows: each lane gathers over its species'
//     reaction lists (fixed order: deterministic, no atomics);
//   - group reductions (butterfly shuffles) give every lane of the group the
//     same bits, so all lanes take the same control path.
// The LU uses implicit partial pivoting: rows never move; the pivot row of
// step k is broadcast through LDS and its index recorded.
#pragma once
#include <hip/hip_runtime.h>

#include "chem_kernels.hpp"

namespace chem {

constexpr int CMP = 4;   // participants per side supported by the tables

// Device tables of one mechanism (data driven).
struct CoopMech {
    int ns, nr, n;
    int prec;              // 0: FP64 transcendentals; 1: FP32 exp/log with FP64 range reduction
    const double* sp;      // [ns][SPS]
    const double* rx;      // [nr][RXS]
    const int* rxi;        // [nr][RXI]
    const int* eff_sp;     // enhanced third-body efficiencies: species
    const double* eff_am1; //   and (alpha - 1)
    const int* csr_ptr;    // [ns+1] species -> (reaction, signed nu) list
    const int* csr_rx;
    const double* csr_nu;
};
// species record
enum { SP_W = 0, SP_INVW, SP_TMID, SP_HLO, SP_HHI = SP_HLO + 6, SP_SLO = SP_HHI + 6, SP_SHI = SP_SLO + 6,
       SP_CLO = SP_SHI + 6, SP_CHI = SP_CLO + 5, SPS = SP_CHI + 5 };
// reaction record (doubles)
enum { RX_LNA = 0, RX_B, RX_EAR, RX_LNA0, RX_B0, RX_EA0R, RX_TROE, RXS = RX_TROE + 4 };
// reaction record (ints)
enum { RI_TYPE = 0, RI_REV, RI_TROEN, RI_DNU, RI_NRE, RI_NPR, RI_RSP, RI_RNU = RI_RSP + CMP,
       RI_PSP = RI_RNU + CMP, RI_PNU = RI_PSP + CMP, RI_EB = RI_PNU + CMP, RI_EE, RXI };

// LDS doubles of one group, for nsp species slots, nr reactions, nc columns
__host__ __device__ inline int group_lds_doubles(int nsp, int nr, int nc) { return 6 * nsp + 5 * nr + 2 * nc + 8; }

// Partner exchange for the group reductions, combining level o = 1, 2, 4, ...
// bottom-up: DPP within 16-lane rows (quad permutes for o = 1, 2; half-row and
// row mirrors for o = 4, 8, which pair the already reduced quads and halves),
// a swizzle for o = 16 and a permute across the wave halves for o = 32.  Each
// pair of partners combines the same two values, so every lane of a group
// ends with bit-identical results.
template <int O>
__device__ __forceinline__ int xchg32(int v) {
    if constexpr (O == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    else if constexpr (O == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    else if constexpr (O == 4) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    else if constexpr (O == 8) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    else if constexpr (O == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);                  // lane ^ 16
    else return __shfl_xor(v, 32);
}

template <int O>
__device__ __forceinline__ double xchg(double v) {
    const int lo = xchg32<O>(__double2loint(v));
    const int hi = xchg32<O>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

template <int G, int O = 1>
__device__ __forceinline__ double gsum(double v) {
    if constexpr (O < G) {
        v += xchg<O>(v);
        return gsum<G, 2 * O>(v);
    } else {
        return v;
    }
}

// group argmax of (value, index): larger value wins, ties -> smaller index
template <int G, int O = 1>
__device__ __forceinline__ void gargmax(double& v, int& idx) {
    if constexpr (O < G) {
        const double v2 = xchg<O>(v);
        const int i2 = xchg32<O>(idx);
        if (v2 > v || (v2 == v && i2 < idx)) {
            v = v2;
            idx = i2;
        }
        gargmax<G, 2 * O>(v, idx);
    }
}

// value of lane `src` of the group (src: lane index in the wave)
template <int G>
__device__ __forceinline__ double gbcast(double v, int src) {
    if constexpr (G == 64) {   // one group per wave: src is wave-uniform
        const int s = __builtin_amdgcn_readfirstlane(src);
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), s);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), s);
        return __hiloint2double(hi, lo);
    } else {
        return __shfl(v, src);
    }
}

__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// select element s (runtime, s < R) of a register array without dynamic indexing
template <int R>
__device__ __forceinline__ double rsel(const double* a, int s) {
    double v = a[0];
#pragma unroll
    for (int q = 1; q < R; q++) v = (s == q) ? a[q] : v;
    return v;
}

// Transcendentals of the rate evaluation.  prec = 1 uses the FP32 hardware
// units (v_exp_f32 / v_log_f32) on a range-reduced argument and keeps the
// range and the reduction in FP64: relative error ~1e-7 instead of ~1e-16.
__device__ __forceinline__ double rexp(double x, int prec) { return prec ? exp32(x) : exp(x); }
__device__ __forceinline__ double rlog(double c, int prec) { return prec ? log32(c) : log(c); }   // c > 0

// ------------------------------------------------------------------ thermo
__device__ __forceinline__ void coop_thermo(const double* sp, double T, double lnT, double invT,
                                            double& h_RT, double& s_R, double& cp_R, double& dcp) {
    const bool lo = T < sp[SP_TMID];
    const double* H = sp + (lo ? SP_HLO : SP_HHI);
    const double* S = sp + (lo ? SP_SLO : SP_SHI);
    const double* C = sp + (lo ? SP_CLO : SP_CHI);
    h_RT = H[0] + T * (H[1] + T * (H[2] + T * (H[3] + T * H[4]))) + H[5] * invT;
    s_R = S[0] * lnT + T * (S[1] + T * (S[2] + T * (S[3] + T * S[4]))) + S[5];
    cp_R = C[0] + T * (C[1] + T * (C[2] + T * (C[3] + T * C[4])));
    dcp = C[1] + T * (2.0 * C[2] + T * (3.0 * C[3] + T * 4.0 * C[4]));
}

// Group LDS layout: per species ln C, C, 1/C, g/RT, h/RT, c_v/R; per reaction
// [qf*mul, qr*mul, dense third-body factor, dq/dT, net*mul]; pivot row; pivot order.
struct GL {
    double *lnC, *C, *iC, *g, *h, *cv, *q, *prow;
    int* perm;
    __device__ GL(double* base, int nsp, int nr, int nc) {
        lnC = base;
        C = lnC + nsp;
        iC = C + nsp;
        g = iC + nsp;
        h = g + nsp;
        cv = h + nsp;
        q = cv + nsp;
        prow = q + 5 * nr;
        perm = (int*)(prow + nc);
    }
};

constexpr double C_LN10 = 2.302585092994045684;
constexpr double C_INV_LN10 = 0.434294481903251828;
constexpr double C_LN_PREF_OVER_R = 9.408091968961747;  // ln(101325 / 8.314462618)

// Species phase: own species' thermo; publish ln C, C, 1/C, g/RT, h/RT, c_v/R.
// Returns the group sums needed by the RHS: C_tot, c_v-mix/R and d(c_v)/dT/R.
template <int G, int R>
__device__ __forceinline__ void coop_species(const CoopMech& M, const GL& gl, int l, double rho,
                                             const double* y, double T, double lnT, double invT,
                                             double& Ctot, double& cvs, double& dcvs) {
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
    for (int s = 0; s < R; s++) {
        const int k = l + G * s;
        if (k < M.ns) {
            const double* sp = M.sp + (size_t)k * SPS;
            double h, sR, cp, dcp;
            coop_thermo(sp, T, lnT, invT, h, sR, cp, dcp);
            // ln|C| (FP64 in every mode: near equilibrium the net rates
            // depend on differences of these logarithms); the sign of C is
            // carried separately so that negative concentrations give the
            // same signed powers as the plain mass-action product
            const double C = rho * y[s] * sp[SP_INVW];
            const double aC = fmax(fabs(C), C_FLOOR);
            gl.lnC[k] = log(aC);
            gl.C[k] = C;
            gl.iC[k] = (C < 0.0) ? -1.0 / aC : 1.0 / aC;
            gl.g[k] = h - sR;
            gl.h[k] = h;
            gl.cv[k] = cp - 1.0;
            c0 += C;
            c1 += y[s] * sp[SP_INVW] * (cp - 1.0);
            c2 += y[s] * sp[SP_INVW] * dcp;
        }
    }
    Ctot = gsum<G>(c0);
    cvs = gsum<G>(c1);
    dcvs = gsum<G>(c2);
}

// Reaction phase: lane l evaluates reactions l, l+G, ...; writes net rates
// (and, with JAC, the derivative data) to LDS.
template <int G, bool JAC>
__device__ __forceinline__ void coop_reactions(const CoopMech& M, const GL& gl, int l, double lnT,
                                               double invT, double Ctot) {
    const double lnPref = C_LN_PREF_OVER_R - lnT;
    for (int j = l; j < M.nr; j += G) {
        const double* rx = M.rx + (size_t)j * RXS;
        const int* ri = M.rxi + (size_t)j * RXI;
        const int type = ri[RI_TYPE];
        const double lnkinf = rx[RX_LNA] + rx[RX_B] * lnT - rx[RX_EAR] * invT;
        const double dlnkinf = (rx[RX_B] + rx[RX_EAR] * invT) * invT;
        double lnkf = lnkinf, dlnkf = dlnkinf, dlnkf_dlnM = 0.0, Mc = 0.0;
        if (type != RX_ELEM) {   // [M] = C_tot + sum (alpha - 1) C over enhanced species
            Mc = Ctot;
            for (int e = ri[RI_EB]; e < ri[RI_EE]; e++) Mc += M.eff_am1[e] * gl.C[M.eff_sp[e]];
        }
        if (type == RX_FO) {
            const double lnk0 = rx[RX_LNA0] + rx[RX_B0] * lnT - rx[RX_EA0R] * invT;
            const double dlnk0 = (rx[RX_B0] + rx[RX_EA0R] * invT) * invT;
            const double Pr = fmax(rexp(lnk0 - lnkinf, M.prec) * Mc, 1e-300);
            const double lnPr = rlog(Pr, M.prec);
            double lnF = 0.0, dlnF_dlnPr = 0.0, dlnF_dT = 0.0;
            const int tn = ri[RI_TROEN];
            if (tn > 0) {
                const double a = rx[RX_TROE], T3 = rx[RX_TROE + 1], T1 = rx[RX_TROE + 2];
                const double T = 1.0 / invT;
                const double e3 = rexp(-T / T3, M.prec), e1 = rexp(-T / T1, M.prec);
                double Fc = (1.0 - a) * e3 + a * e1;
                double dFc = -(1.0 - a) / T3 * e3 - a / T1 * e1;
                if (tn == 4) {
                    const double T2 = rx[RX_TROE + 3];
                    const double e2 = rexp(-T2 * invT, M.prec);
                    Fc += e2;
                    dFc += T2 * invT * invT * e2;
                }
                const double phi = rlog(Fc, M.prec) * C_INV_LN10;
                const double c = -0.4 - 0.67 * phi, nn = 0.75 - 1.27 * phi;
                const double u = lnPr * C_INV_LN10 + c;
                const double den = nn - 0.14 * u;
                const double f1 = u / den;
                const double qq = 1.0 + f1 * f1;
                lnF = C_LN10 * phi / qq;
                if (JAC) {
                    const double iq2 = 1.0 / (qq * qq), iden2 = 1.0 / (den * den);
                    const double df1_dx = nn * iden2;
                    const double df1_dphi = (-0.67 * den + u * (1.27 - 0.14 * 0.67)) * iden2;
                    dlnF_dlnPr = -phi * 2.0 * f1 * df1_dx * iq2;
                    dlnF_dT = (1.0 / qq - phi * 2.0 * f1 * df1_dphi * iq2) * dFc / Fc;
                }
            }
            const double ip = 1.0 / (1.0 + Pr);
            lnkf = lnkinf + lnPr - rlog(1.0 + Pr, M.prec) + lnF;   // ln(kinf Pr/(1+Pr) F)
            if (JAC) {
                const double dlnPr_dT = dlnk0 - dlnkinf;
                dlnkf_dlnM = ip + dlnF_dlnPr;
                dlnkf = dlnkinf + dlnPr_dT * ip + dlnF_dT + dlnF_dlnPr * dlnPr_dT;
            }
        }
        const int nre = ri[RI_NRE], npr = ri[RI_NPR];
        double lnqf = lnkf;   // ln|qf| = ln kf + nu' . ln|C|; sign = parity of negative factors
        int negf = 0;
        for (int i = 0; i < nre; i++) {
            const int k = ri[RI_RSP + i], nu = ri[RI_RNU + i];
            lnqf += nu * gl.lnC[k];
            negf ^= (nu & 1) & (gl.C[k] < 0.0);
        }
        const double qf = negf ? -rexp(lnqf, M.prec) : rexp(lnqf, M.prec);
        double qr = 0.0, dlnKc = 0.0, net = qf;
        if (ri[RI_REV]) {
            // ln Kc = -nu . g/RT + dnu ln(Pref/RT);  ln|qr| = ln kf - ln Kc + nu'' . ln|C|
            double sg = 0.0, sh = 0.0, lnqr = lnkf;
            int negr = 0;
            for (int i = 0; i < npr; i++) {
                const int k = ri[RI_PSP + i], inu = ri[RI_PNU + i];
                const double nu = inu;
                sg += nu * gl.g[k];
                sh += nu * gl.h[k];
                lnqr += nu * gl.lnC[k];
                negr ^= (inu & 1) & (gl.C[k] < 0.0);
            }
            for (int i = 0; i < nre; i++) {
                const int k = ri[RI_RSP + i];
                const double nu = ri[RI_RNU + i];
                sg -= nu * gl.g[k];
                sh -= nu * gl.h[k];
            }
            const double lnKc = -sg + ri[RI_DNU] * lnPref;
            lnqr -= lnKc;
            qr = negr ? -rexp(lnqr, M.prec) : rexp(lnqr, M.prec);
            dlnKc = (sh - ri[RI_DNU]) * invT;   // d(g/RT)/dT = -h/(R T^2)
            net = qf - qr;
            // FP32 exponentials carry ~1e-7 relative error each, which the
            // difference would amplify near equilibrium: there the net rate is
            // formed as -qf expm1(ln qr - ln qf) with the FP64 log ratio
            if (M.prec != 0 && negf == negr) {
                const double d = lnqr - lnqf;
                if (fabs(d) < 0.35) net = -qf * expm1_small(d);
            }
        }
        const double mul = (type == RX_TB) ? Mc : 1.0;
        double* qj = gl.q + 5 * j;
        qj[4] = mul * net;
        if (JAC) {
            qj[0] = mul * qf;
            qj[1] = mul * qr;
            double g = 0.0;   // d q / d C_m = ... + alpha_m g
            if (type == RX_TB) g = net;
            if (type == RX_FO) g = net * dlnkf_dlnM / fmax(Mc, 1e-300);
            qj[2] = g;
            qj[3] = mul * (qf * dlnkf - qr * (dlnkf - dlnKc));
        }
    }
}

template <int G, int R>
__device__ __forceinline__ double group_T(const double* y, int ns, int base) {
    return gbcast<G>(rsel<R>(y, ns / G), base + ns % G);
}

// f = dy/dt of the group's cell, distributed like y.
template <int G, int R>
__device__ __forceinline__ void coop_rhs(const CoopMech& M, const GL& gl, int l, int base, double rho, const double* y,
                         double* f) {
    const double T = group_T<G, R>(y, M.ns, base);
    const double lnT = log(T), invT = 1.0 / T;
    double Ctot, cvs, dcvs;
    coop_species<G, R>(M, gl, l, rho, y, T, lnT, invT, Ctot, cvs, dcvs);
    lds_fence();
    coop_reactions<G, false>(M, gl, l, lnT, invT, Ctot);
    lds_fence();
    double Sp = 0.0;
#pragma unroll
    for (int s = 0; s < R; s++) {
        const int k = l + G * s;
        f[s] = 0.0;
        if (k < M.ns) {
            double om = 0.0;
            for (int p = M.csr_ptr[k]; p < M.csr_ptr[k + 1]; p++) om += M.csr_nu[p] * gl.q[5 * M.csr_rx[p] + 4];
            f[s] = M.sp[(size_t)k * SPS + SP_W] * om / rho;
            Sp += (gl.h[k] - 1.0) * om;
        }
    }
    const double S = gsum<G>(Sp);
    const double fT = -S * T / (rho * cvs);
#pragma unroll
    for (int s = 0; s < R; s++)
        if (l + G * s == M.ns) f[s] = fT;
    lds_fence();   // the LDS area is reused by the next phase
}

// Newton matrix rows A = I - c J of the group's cell, left in the group's LDS
// matrix: row k = l + G*s, column col at jb[col*n + G*s] (jb points at the
// lane's row 0; column-major over the n rows, rows of lanes k >= n are not
// stored).
template <int G, int R>
__device__ __forceinline__ void coop_newton_matrix(const CoopMech& M, const GL& gl, int l, int base, double rho,
                                   const double* y, double c, double* jb) {
    const int ns = M.ns, n = M.n;
    const double T = group_T<G, R>(y, ns, base);
    const double lnT = log(T), invT = 1.0 / T;
    double Ctot, cvs, dcvs;
    coop_species<G, R>(M, gl, l, rho, y, T, lnT, invT, Ctot, cvs, dcvs);
    lds_fence();
    coop_reactions<G, true>(M, gl, l, lnT, invT, Ctot);
    lds_fence();
    // species rows into the LDS buffer: J[k][m] = (W_k/W_m) d omega_k / d C_m
    double omk[R], dwTk[R];
    double Sp = 0.0, Ep = 0.0;
#pragma unroll
    for (int s = 0; s < R; s++) {
        const int k = l + G * s;
        omk[s] = dwTk[s] = 0.0;
        if (k < ns) {
            for (int col = 0; col < ns; col++) jb[col * n + G * s] = 0.0;
            const double Wk = M.sp[(size_t)k * SPS + SP_W];
            double om = 0.0, dwT = 0.0, gd = 0.0;
            for (int p = M.csr_ptr[k]; p < M.csr_ptr[k + 1]; p++) {
                const int j = M.csr_rx[p];
                const double nu = M.csr_nu[p];
                const double* qj = gl.q + 5 * j;
                const int* ri = M.rxi + (size_t)j * RXI;
                om += nu * qj[4];
                dwT += nu * qj[3];
                for (int i = 0; i < ri[RI_NRE]; i++) {
                    const int m = ri[RI_RSP + i];
                    jb[m * n + G * s] += Wk * M.sp[(size_t)m * SPS + SP_INVW] * nu * ri[RI_RNU + i] * qj[0] * gl.iC[m];
                }
                for (int i = 0; i < ri[RI_NPR]; i++) {
                    const int m = ri[RI_PSP + i];
                    jb[m * n + G * s] -= Wk * M.sp[(size_t)m * SPS + SP_INVW] * nu * ri[RI_PNU + i] * qj[1] * gl.iC[m];
                }
                if (ri[RI_TYPE] != RX_ELEM) {   // alpha_m g: ones part (below) + enhanced part
                    const double v = nu * qj[2];
                    gd += v;
                    for (int e = ri[RI_EB]; e < ri[RI_EE]; e++) {
                        const int m = M.eff_sp[e];
                        jb[m * n + G * s] += Wk * M.sp[(size_t)m * SPS + SP_INVW] * v * M.eff_am1[e];
                    }
                }
            }
            if (gd != 0.0) {
                for (int col = 0; col < ns; col++) jb[col * n + G * s] += Wk * M.sp[(size_t)col * SPS + SP_INVW] * gd;
            }
            omk[s] = om;
            dwTk[s] = dwT;
            Sp += (gl.h[k] - 1.0) * T * om;                  // u_k om_k / R
            Ep += gl.cv[k] * om + (gl.h[k] - 1.0) * T * dwT; // d(sum u om)/dT / R
        }
    }
    const double S = gsum<G>(Sp), E = gsum<G>(Ep);
    const double irho = 1.0 / rho;
    const double fT = -S * irho / cvs;
    // temperature row needs dS_m = sum_k u_k d omega_k/dC_m = W_m sum_k u_k J[k][m] / W_k,
    // reduced over the group column by column while the own rows are assembled
    // rolled: an unrolled loop over 64 columns (each with a group reduction)
    // makes the kernel larger than the instruction cache
#pragma unroll 1
    for (int col = 0; col < n; col++) {
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int k = l + G * s;
            if (k < ns && col < ns) v += (gl.h[k] - 1.0) * T * M.sp[(size_t)k * SPS + SP_INVW] * jb[col * n + G * s];
        }
        const double dS = (col < ns) ? gsum<G>(v) : 0.0;
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int k = l + G * s;
            double J = 0.0;
            if (k < ns) {
                if (col < ns) J = jb[col * n + G * s];
                else if (col == ns) J = M.sp[(size_t)k * SPS + SP_W] * irho * dwTk[s];
            } else if (k == ns) {
                if (col < ns) {
                    const double Wm = M.sp[(size_t)col * SPS + SP_W];
                    J = -(1.0 / (Wm * cvs)) * (dS * Wm + fT * gl.cv[col]);
                } else if (col == ns) {
                    J = -E * irho / cvs - fT * dcvs / cvs;
                }
            }
            if (k < n) jb[col * n + G * s] = ((k == col) ? 1.0 : 0.0) - c * J;   // the Newton matrix, in place
        }
    }
    lds_fence();
}

// LU with implicit partial pivoting of the group's matrix (own rows in the
// group's LDS matrix A, element (s, col) at A[col*n + G*s]).  After
// the call: pstep[s] = elimination step at which own row became pivot;
// gl.perm[k] = pivot row of step k; the pivot row stores 1/pivot on its
// diagonal and U to its right, other rows keep their multipliers in the
// columns of the steps that eliminated them.  Loops over steps and columns
// run to n (not unrolled), which keeps the kernel within the instruction cache.
template <int G, int R>
__device__ __forceinline__ bool coop_lu(const GL& gl, int l, int n, double* A, int* pstep) {
    bool ok = true;
#pragma unroll
    for (int s = 0; s < R; s++) pstep[s] = -1;
#pragma unroll 1
    for (int k = 0; k < n; k++) {
        double best = -1.0;
        int bidx = 1 << 30;
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int i = l + G * s;
            if (i < n && pstep[s] < 0) {
                const double v = fabs(A[k * n + G * s]);
                if (v > best) {
                    best = v;
                    bidx = i;
                }
            }
        }
        gargmax<G>(best, bidx);
        if (!(best > 0.0) || !isfinite(best)) ok = false;
        const int p = bidx;
        const bool own = (p % G) == l;
        const int sp = p / G;
        if (own) {
#pragma unroll 4
            for (int col = k; col < n; col++) gl.prow[col] = A[col * n + G * sp];
        }
        lds_fence();
        const double inv = 1.0 / gl.prow[k];
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int i = l + G * s;
            if (own && s == sp) {
                pstep[s] = k;
                A[k * n + G * s] = inv;
            } else if (i < n && pstep[s] < 0) {
                const double m = A[k * n + G * s] * inv;
                A[k * n + G * s] = m;
#pragma unroll 4
                for (int col = k + 1; col < n; col++) A[col * n + G * s] -= m * gl.prow[col];
            }
        }
        if (l == 0) gl.perm[k] = p;
        lds_fence();
    }
    return ok;
}

// Solve with the implicit-pivot LU: b (own rows, distributed) -> x (own
// components).  Forward: step k eliminates the broadcast pivot value from the
// rows that became pivots later; back: column-oriented substitution.
template <int G, int R>
__device__ __forceinline__ void coop_solve(const GL& gl, int l, int base, int n, const double* A, const int* pstep,
                                           double* b) {
#pragma unroll 1
    for (int k = 0; k < n; k++) {
        const int p = gl.perm[k];
        const double z = gbcast<G>(rsel<R>(b, p / G), base + p % G);
#pragma unroll
        for (int s = 0; s < R; s++)
            if (pstep[s] > k) b[s] -= A[k * n + G * s] * z;
    }
    double x[R];
#pragma unroll
    for (int s = 0; s < R; s++) x[s] = 0.0;
#pragma unroll 1
    for (int k = n - 1; k >= 0; k--) {
        const int p = gl.perm[k];
        // the owner of row p holds b_p (fully reduced) and 1/pivot on (sp, k)
        double cand = 0.0;
#pragma unroll
        for (int s = 0; s < R; s++)
            if (pstep[s] == k) cand = b[s] * A[k * n + G * s];
        const double xk = gbcast<G>(cand, base + p % G);
#pragma unroll
        for (int s = 0; s < R; s++) {
            if (pstep[s] >= 0 && pstep[s] < k) b[s] -= A[k * n + G * s] * xk;
            if (l + G * s == k) x[s] = xk;
        }
    }
#pragma unroll
    for (int s = 0; s < R; s++) b[s] = x[s];
}

// ---------------------------------------------------------------- BDF (group)
// The same variable-order BDF as the one-lane stepper (Shampine & Reichelt
// 1997, kappa = 0), with each component's differences in the registers of
// the lane that owns it.  Newton convergence test, difference update and
// order selection follow SciPy's BDF (scipy/integrate/_ivp/bdf.py,
// BSD-3-Clause).
template <int G, int R>
struct CLane {
    static constexpr int NC = G * R;
    double D[ND][R];
    int pstep[R];   // the matrix rows live in the group's LDS matrix
    double t, tend, h, c_lu, rho;
    int k, neq, att, round_att;
    bool lu_ok, jac_fresh;
    unsigned long long n_steps, n_att, n_rhs, n_jac, n_lu, n_solve;
};

template <int G, int R>
__device__ __forceinline__ double cwrms(const double* v, const double* isc, int n) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < R; q++) {
        const double r = v[q] * isc[q];
        s += r * r;
    }
    return sqrt(gsum<G>(s) / n);
}

__device__ __forceinline__ double c_gamma(int k) {
    double g = 0.0;
    g = (k == 1) ? 1.0 : g;
    g = (k == 2) ? 1.5 : g;
    g = (k == 3) ? 11.0 / 6.0 : g;
    g = (k == 4) ? 25.0 / 12.0 : g;
    g = (k == 5) ? 137.0 / 60.0 : g;
    return g;
}

// D_j <- the differences of the interpolating polynomial on the grid of
// spacing r*h (j = 1..k), as in the one-lane stepper.
template <int G, int R>
__device__ __forceinline__ void crescale(CLane<G, R>& L, int k, double r) {
    double Tm[MAXORD + 1][MAXORD + 1];
#pragma unroll
    for (int j = 1; j <= MAXORD; j++) {
#pragma unroll
        for (int i = 0; i <= MAXORD; i++) {
            double s = 0.0, binom = 1.0;
#pragma unroll
            for (int m = 0; m <= j; m++) {
                double b = 1.0;
                const double x = m * r;
#pragma unroll
                for (int q = 1; q <= i; q++) b *= (q - 1 - x) * (1.0 / q);
                s += ((m & 1) ? -binom : binom) * b;
                binom = binom * (j - m) / (m + 1);
            }
            Tm[j][i] = s;
        }
    }
#pragma unroll
    for (int c = 0; c < R; c++) {
        double d[MAXORD + 1];
#pragma unroll
        for (int i = 0; i <= MAXORD; i++) d[i] = (i <= k) ? L.D[i][c] : 0.0;
#pragma unroll
        for (int j = 1; j <= MAXORD; j++) {
            if (j <= k) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i <= MAXORD; i++) s += Tm[j][i] * d[i];
                L.D[j][c] = s;
            }
        }
    }
}

template <int G, int R>
__device__ __forceinline__ int cbdf_attempt(const CoopMech& M, const GL& gl, int l, int base, CLane<G, R>& L,
                            double* jb, double rtol, double atol) {
    const int n = M.n;
    constexpr double EPS = 2.220446049250313e-16;
    L.att++;
    L.round_att++;
    L.n_att++;
    if (!(L.h >= 10.0 * EPS * fabs(L.t))) return SR_FAIL;
    bool last = false;
    if (L.t + L.h >= L.tend || L.h >= L.tend - L.t) {   // rounding of t + h cannot hide the end
        const double hn = L.tend - L.t;
        crescale<G, R>(L, L.k, hn / L.h);
        L.h = hn;
        L.neq = 0;
        last = true;
    }
    const double tn = last ? L.tend : L.t + L.h;
    const int k = L.k;
    const double gk = c_gamma(k);
    double yp[R], psi[R], isc[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        double a = 0.0, b = 0.0, gj = 0.0;
#pragma unroll
        for (int j = 0; j <= MAXORD; j++) {
            if (j <= k) {
                const double dj = L.D[j][q];
                a += dj;
                if (j >= 1) {
                    gj += 1.0 / j;
                    b += gj * dj;
                }
            }
        }
        yp[q] = a;
        psi[q] = b / gk;
        isc[q] = (l + G * q < n) ? 1.0 / (atol + rtol * fabs(a)) : 0.0;
    }
    const double c = L.h / gk;
    if (!L.lu_ok || fabs(c - L.c_lu) > 0.3 * L.c_lu) {
        coop_newton_matrix<G, R>(M, gl, l, base, L.rho, yp, c, jb);
        L.n_jac++;
        L.n_lu++;
        L.jac_fresh = true;
        L.lu_ok = coop_lu<G, R>(gl, l, n, jb, L.pstep);
        L.c_lu = c;
        if (!L.lu_ok) {
            crescale<G, R>(L, k, 0.25);
            L.h *= 0.25;
            L.neq = 0;
            return SR_RETRY;
        }
    }
    const double tol = fmax(10.0 * EPS / rtol, fmin(0.03, sqrt(rtol)));
    double d[R];
#pragma unroll
    for (int q = 0; q < R; q++) d[q] = 0.0;
    bool conv = false;
    double dn_old = -1.0;
    for (int it = 0; it < 4; it++) {
        double yn[R], f[R];
#pragma unroll
        for (int q = 0; q < R; q++) yn[q] = yp[q] + d[q];
        coop_rhs<G, R>(M, gl, l, base, L.rho, yn, f);
        L.n_rhs++;
        int fin = 1;
#pragma unroll
        for (int q = 0; q < R; q++) {
            f[q] = c * f[q] - psi[q] - d[q];
            if (l + G * q >= n) f[q] = 0.0;
            fin &= isfinite(f[q]) ? 1 : 0;
        }
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) fin &= __shfl_xor(fin, o);
        if (!fin) break;
        coop_solve<G, R>(gl, l, base, n, jb, L.pstep, f);
        L.n_solve++;
        const double dn = cwrms<G, R>(f, isc, n);
        const double rate = dn_old > 0.0 ? dn / dn_old : -1.0;
        if (rate >= 0.0) {
            double rp = 1.0;
            for (int q = 0; q < 4 - it; q++) rp *= rate;
            if (rate >= 1.0 || rp / (1.0 - rate) * dn > tol) break;
        }
#pragma unroll
        for (int q = 0; q < R; q++) d[q] += f[q];
        if (dn == 0.0 || (rate >= 0.0 && rate / (1.0 - rate) * dn < tol)) {
            conv = true;
            break;
        }
        dn_old = dn;
    }
    if (!conv) {
        if (!L.jac_fresh) {
            L.lu_ok = false;
            return SR_RETRY;
        }
        crescale<G, R>(L, k, 0.5);
        L.h *= 0.5;
        L.neq = 0;
        return SR_RETRY;
    }
    double ise[R], e1[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        ise[q] = (l + G * q < n) ? 1.0 / (atol + rtol * fabs(yp[q] + d[q])) : 0.0;
        e1[q] = d[q] * (1.0 / (k + 1));
    }
    const double en = cwrms<G, R>(e1, ise, n);
    if (en > 1.0) {
        const double fac = fmax(0.2, 0.9 * ctl_pow(en, -1.0 / (k + 1)));
        crescale<G, R>(L, k, fac);
        L.h *= fac;
        L.neq = 0;
        return SR_RETRY;
    }
    L.n_steps++;
    L.t = tn;
    L.jac_fresh = false;
    // D_{k+2} = d - D_{k+1}, D_{k+1} = d, D_j += D_{j+1} for j = k..0
#pragma unroll
    for (int q = 0; q < R; q++) {
        double dv[ND];
#pragma unroll
        for (int j = 0; j < ND; j++) dv[j] = L.D[j][q];
        const double dk1 = rsel<ND>(dv, k + 1);
        double acc = d[q];
#pragma unroll
        for (int j = ND - 1; j >= 0; j--) {
            if (j == k + 2) L.D[j][q] = d[q] - dk1;
            else if (j == k + 1) L.D[j][q] = d[q];
            else if (j <= k) {
                acc = dv[j] + acc;
                L.D[j][q] = acc;
            }
        }
    }
    L.neq++;
    if (last) return SR_DONE;
    if (L.neq < k + 1) return SR_ACCEPT;
    double em = 0.0, ep = 0.0;
    {
        double v[R];
        if (k > 1) {
#pragma unroll
            for (int q = 0; q < R; q++) {
                double dk = 0.0;
#pragma unroll
                for (int j = 0; j < ND; j++) dk = (j == k) ? L.D[j][q] : dk;
                v[q] = dk * (1.0 / k);
            }
            em = cwrms<G, R>(v, ise, n);
        }
        if (k < MAXORD) {
#pragma unroll
            for (int q = 0; q < R; q++) {
                double dk = 0.0;
#pragma unroll
                for (int j = 0; j < ND; j++) dk = (j == k + 2) ? L.D[j][q] : dk;
                v[q] = dk * (1.0 / (k + 2));
            }
            ep = cwrms<G, R>(v, ise, n);
        }
    }
    const double f0 = ctl_pow(en, -1.0 / (k + 1));
    const double fm = (k > 1) ? ctl_pow(em, -1.0 / k) : 0.0;
    const double fp = (k < MAXORD) ? ctl_pow(ep, -1.0 / (k + 2)) : 0.0;
    int dk = 0;
    double best = f0;
    if (fm > best) {
        best = fm;
        dk = -1;
    }
    if (fp > best) {
        best = fp;
        dk = 1;
    }
    L.k = k + dk;
    const double fac = fmin(10.0, 0.9 * best);
    crescale<G, R>(L, L.k, fac);
    L.h *= fac;
    L.neq = 0;
    return SR_ACCEPT;
}

template <int G, int R>
__device__ __forceinline__ void cbdf_init(const CoopMech& M, const GL& gl, int l, int base, CLane<G, R>& L,
                          const double* y0, double rtol, double atol) {
    const int n = M.n;
    double f0[R], isc[R], y1[R], f1[R];
    coop_rhs<G, R>(M, gl, l, base, L.rho, y0, f0);
#pragma unroll
    for (int q = 0; q < R; q++) isc[q] = (l + G * q < n) ? 1.0 / (atol + rtol * fabs(y0[q])) : 0.0;
    const double d0 = cwrms<G, R>(y0, isc, n), d1 = cwrms<G, R>(f0, isc, n);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, L.tend);
#pragma unroll
    for (int q = 0; q < R; q++) y1[q] = y0[q] + h0 * f0[q];
    coop_rhs<G, R>(M, gl, l, base, L.rho, y1, f1);
    L.n_rhs += 2;
#pragma unroll
    for (int q = 0; q < R; q++) f1[q] -= f0[q];
    const double d2 = cwrms<G, R>(f1, isc, n) / h0;
    const double mx = fmax(d1, d2);
    const double h1 = (mx <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : sqrt(0.01 / mx);
    L.h = fmin(fmin(100.0 * h0, h1), L.tend);
#pragma unroll
    for (int q = 0; q < R; q++) {
#pragma unroll
        for (int j = 0; j < ND; j++) L.D[j][q] = 0.0;
        L.D[0][q] = y0[q];
        L.D[1][q] = L.h * f0[q];
    }
    L.t = 0.0;
    L.k = 1;
    L.neq = 0;
    L.att = 0;
    L.lu_ok = false;
    L.jac_fresh = false;
    L.c_lu = 0.0;
}

// ------------------------------------------------- data-driven thermo kernels
__device__ __forceinline__ void coop_e_cv(const CoopMech& M, double T, const double* Y, int64_t ldY,
                                          double& e, double& cv) {
    const double lnT = log(T), invT = 1.0 / T;
    double se = 0.0, sc = 0.0;
    for (int k = 0; k < M.ns; k++) {
        const double* sp = M.sp + (size_t)k * SPS;
        double h, sR, cp, dcp;
        coop_thermo(sp, T, lnT, invT, h, sR, cp, dcp);
        const double w = Y[k * ldY] * sp[SP_INVW];
        se += w * (h - 1.0);
        sc += w * (cp - 1.0);
    }
    e = se * RGAS * T;
    cv = sc * RGAS;
}

// Newton on e(T, Y) = e0 guarded by bisection in [100, 6000] K
__device__ __forceinline__ bool coop_T_from_e(const CoopMech& M, double e0, const double* Y, int64_t ldY, double Tg,
                              double& Tout) {
    double lo = 100.0, hi = 6000.0, elo, ehi, cv;
    coop_e_cv(M, lo, Y, ldY, elo, cv);
    coop_e_cv(M, hi, Y, ldY, ehi, cv);
    if (!(elo <= e0 && ehi >= e0)) return false;
    double T = (Tg > lo && Tg < hi) ? Tg : 1500.0;
    for (int it = 0; it < 100; it++) {
        double e;
        coop_e_cv(M, T, Y, ldY, e, cv);
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

// same contract as k_screen, for data-driven mechanisms
__global__ void __launch_bounds__(256) k_screen_coop(CoopMech M, const DevBox* __restrict__ boxes,
                                                     int nbox, int64_t total, double t_react_min,
                                                     uint8_t* __restrict__ st_int, int* __restrict__ block_cnt) {
    __shared__ int sh[4];
    const int64_t g = blockIdx.x * 256ll + threadIdx.x;
    bool active = false;
    if (g < total) {
        const DevBox& B = boxes[find_box(boxes, nbox, g)];
        const int64_t i = g - B.off;
        uint8_t st;
        if (B.mask && B.mask[i]) {
            st = ST_SKIPPED;
        } else {
            const double rho = B.rho[i], e = B.e[i];
            double T0;
            if (!(rho > 0.0) || !isfinite(rho) || !isfinite(e) ||
                !coop_T_from_e(M, e, B.Y + i, B.ldY, B.T[i], T0)) {
                st = ST_TINV;
            } else {
                B.T[i] = T0;
                st = (T0 < t_react_min) ? ST_SKIPPED : ST_ACTIVE;
            }
        }
        st_int[g] = st;
        if (st != ST_ACTIVE && B.status) B.status[i] = st;
        active = (st == ST_ACTIVE);
    }
    int tot;
    block_prefix_256(active, sh, tot);
    if (threadIdx.x == 0) block_cnt[blockIdx.x] = tot;
}

__global__ void k_prepare_coop(CoopMech M, int64_t n, const double* __restrict__ T,
                               const double* __restrict__ p, const double* __restrict__ Y, int64_t ldY,
                               double* __restrict__ rho, double* __restrict__ e) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sw = 0.0;
    for (int k = 0; k < M.ns; k++) sw += Y[k * ldY + i] * M.sp[(size_t)k * SPS + SP_INVW];
    double ee, cv;
    coop_e_cv(M, T[i], Y + i, ldY, ee, cv);
    rho[i] = p[i] / (RGAS * T[i] * sw);
    e[i] = ee;
}

// ------------------------------------------------------------------ kernels
struct CoopSave {          // per active slot, [field][slot]
    double* D;             // ND*n fields (the n components)
    double* A;             // n*n fields
    double* scal;          // t, h, c_lu
    int* ints;             // pstep[NC], k, neq, att, flags
    int64_t ld;
};

struct CoopArgs {
    CoopMech M;
    const DevBox* boxes;
    int nbox;
    uint8_t* st_int;
    const int* active_ids;
    const int* items;
    const int* n_items_dev;
    int64_t n_items_host;
    int* queue;
    int* unfinished;
    int* rounds;
    const int* gate;
    const int* gate_prev;  // the count one round earlier (decay gate)
    double keep;           // stop the rounds once a round keeps more than keep of its cells
    int nstar;
    uint8_t* flag;
    CoopSave sv;
    int kmax;
    double rtol, atol;
    Counters* ctr;
    int gl_stride;         // doubles per group area
    int nsp;               // species slots in the group area
};

template <int G, int R, int MODE>
__global__ void __launch_bounds__(64, 2) k_integrate_coop(CoopArgs a) {
    constexpr int NC = G * R, NGRP = 64 / G;
    extern __shared__ double lds[];
    const CoopMech& M = a.M;
    const int lane = threadIdx.x, grp0 = lane / G;
    if (MODE == BULK) {
        if (*a.n_items_dev == 0) return;
        if (a.gate && *a.gate <= a.nstar) return;
        if (a.gate_prev && (double)*a.gate > a.keep * (double)*a.gate_prev) return;
        if (blockIdx.x == 0 && lane == 0) atomicAdd(a.rounds, 1);
    }
    const int64_t n_items = (MODE == PLAIN) ? a.n_items_host : (int64_t)*a.n_items_dev;
    CLane<G, R> L;
    L.n_steps = L.n_att = L.n_rhs = L.n_jac = L.n_lu = L.n_solve = 0;
    unsigned long long max_att = 0, incomplete = 0, unfinished = 0;
    int64_t cur = -1, g = -1;
    int slot = -1, bidx = 0;
    bool exhausted = false, static_taken = false;
    const int n = M.n, ns = M.ns;
    for (;;) {
        if (MODE == PLAIN) {
            if (cur < 0 && !static_taken) {
                static_taken = true;
                const int64_t it = blockIdx.x * (int64_t)NGRP + grp0;
                if (it < n_items && a.st_int[it] == ST_ACTIVE) cur = it;
            }
        } else {
            for (;;) {
                const bool need = cur < 0 && !exhausted;           // uniform within a group
                const unsigned long long m = __ballot(need && (lane % G) == 0);
                if (!m) break;
                const int cnt = __popcll(m);
                const int leader = __ffsll((long long)m) - 1;
                int b0 = 0;
                if (lane == leader) b0 = atomicAdd(a.queue, cnt);
                b0 = __shfl(b0, leader);
                const int rank = __popcll(m & ((1ull << (grp0 * G)) - 1ull));
                if (need) {
                    const int my = b0 + rank;
                    if (my < n_items) {
                        const int s = (MODE == SPARSE) ? a.items[my] : my;
                        if (a.flag[s] != 2) {
                            cur = my;
                            slot = s;
                        }
                    } else {
                        exhausted = true;
                    }
                }
            }
        }
        if (__ballot(cur >= 0) == 0) break;
        if (cur < 0) continue;
        // lane-derived indices and LDS addresses are recomputed every iteration from
        // an opaque copy of the lane id, so the compiler cannot hoist hundreds of
        // them out of the persistent loop and keep them live across it
        int lv = lane;
        asm volatile("" : "+v"(lv));
        const int l = lv % G, grp = lv / G, base = grp * G;
        GL gl(lds + grp * a.gl_stride, a.nsp, M.nr, NC);
        double* jb = lds + NGRP * a.gl_stride + grp * n * n + l;
        if (g < 0) {
            g = (MODE == PLAIN) ? cur : (int64_t)a.active_ids[slot];
            bidx = find_box(a.boxes, a.nbox, g);
            const DevBox& B = a.boxes[bidx];
            const int64_t i = g - B.off;
            L.rho = B.rho[i];
            L.tend = B.dt;
            L.round_att = 0;
            if (MODE != PLAIN && a.flag[slot] == 1) {
                const CoopSave& S = a.sv;
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int c = l + G * q;
#pragma unroll
                    for (int j = 0; j < ND; j++) L.D[j][q] = c < n ? S.D[(j * n + c) * S.ld + slot] : 0.0;
                    if (c < n)
                        for (int col = 0; col < n; col++) jb[col * n + G * q] = S.A[(c * n + col) * S.ld + slot];
                    L.pstep[q] = S.ints[c * S.ld + slot];
                    if (L.pstep[q] >= 0) gl.perm[L.pstep[q]] = c;
                }
                L.t = S.scal[0 * S.ld + slot];
                L.h = S.scal[1 * S.ld + slot];
                L.c_lu = S.scal[2 * S.ld + slot];
                L.k = S.ints[(NC + 0) * S.ld + slot];
                L.neq = S.ints[(NC + 1) * S.ld + slot];
                L.att = S.ints[(NC + 2) * S.ld + slot];
                const int fl = S.ints[(NC + 3) * S.ld + slot];
                L.lu_ok = fl & 1;
                L.jac_fresh = (fl >> 1) & 1;
                lds_fence();
            } else {
                double y0[R];
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int c = l + G * q;
                    y0[q] = (c < ns) ? B.Y[c * B.ldY + i] : (c == ns ? B.T[i] : 0.0);
                }
                cbdf_init<G, R>(M, gl, l, base, L, y0, a.rtol, a.atol);
            }
        }
        const int r = cbdf_attempt<G, R>(M, gl, l, base, L, jb, a.rtol, a.atol);
        bool finished = false, save = false;
        uint8_t st = ST_DONE;
        if (r == SR_DONE) finished = true;
        else if (r == SR_FAIL) {
            finished = true;
            st = ST_FAIL;
        } else if (L.round_att >= a.kmax) {
            if (MODE == BULK) save = true;
            else {
                finished = true;
                st = ST_KMAX;
            }
        }
        if (finished || save) {
            if (l == 0) max_att = max(max_att, (unsigned long long)L.att);
            if (finished) {
                const DevBox& B = a.boxes[bidx];
                const int64_t i = g - B.off;
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int c = l + G * q;
                    if (c < ns) B.Y[c * B.ldY + i] = L.D[0][q];
                    else if (c == ns) B.T[i] = L.D[0][q];
                }
                if (l == 0) {
                    const uint8_t fin = (st == ST_DONE && a.st_int[g] == ST_SURR_REJ) ? (uint8_t)ST_SURR_REJ : st;
                    a.st_int[g] = fin;
                    if (B.status) B.status[i] = fin;
                    if (MODE != PLAIN) a.flag[slot] = 2;
                    if (st != ST_DONE) incomplete++;
                }
            } else {
                const CoopSave& S = a.sv;
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int c = l + G * q;
                    if (c < n) {
#pragma unroll
                        for (int j = 0; j < ND; j++) S.D[(j * n + c) * S.ld + slot] = L.D[j][q];
                        for (int col = 0; col < n; col++) S.A[(c * n + col) * S.ld + slot] = jb[col * n + G * q];
                    }
                    S.ints[c * S.ld + slot] = L.pstep[q];
                }
                if (l == 0) {
                    S.scal[0 * S.ld + slot] = L.t;
                    S.scal[1 * S.ld + slot] = L.h;
                    S.scal[2 * S.ld + slot] = L.c_lu;
                    S.ints[(NC + 0) * S.ld + slot] = L.k;
                    S.ints[(NC + 1) * S.ld + slot] = L.neq;
                    S.ints[(NC + 2) * S.ld + slot] = L.att;
                    S.ints[(NC + 3) * S.ld + slot] = (L.lu_ok ? 1 : 0) | (L.jac_fresh ? 2 : 0);
                    a.flag[slot] = 1;
                    unfinished++;
                }
            }
            cur = -1;
            g = -1;
            slot = -1;
        }
    }
    if (lane % G != 0) L.n_steps = L.n_att = L.n_rhs = L.n_jac = L.n_lu = L.n_solve = 0;
    auto wsum = [&](unsigned long long v) {
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        return v;
    };
    auto wmax = [&](unsigned long long v) {
        for (int o = 32; o >= 1; o >>= 1) v = max(v, (unsigned long long)__shfl_xor(v, o));
        return v;
    };
    const unsigned long long s0 = wsum(L.n_steps), s1 = wsum(L.n_att), s2 = wsum(L.n_rhs),
                             s3 = wsum(L.n_jac), s4 = wsum(L.n_lu), s5 = wsum(L.n_solve),
                             s6 = wmax(max_att), s7 = wsum(incomplete), s8 = wsum(unfinished);
    if (lane == 0) {
        Counters* ct = a.ctr + (MODE == BULK ? 1 : 0);   // [0] sparse or plain, [1] bulk rounds
        atomicAdd(&ct->steps, s0);
        atomicAdd(&ct->attempts, s1);
        atomicAdd(&ct->rhs, s2);
        atomicAdd(&ct->jac, s3);
        atomicAdd(&ct->lu, s4);
        atomicAdd(&ct->solves, s5);
        atomicMax(&ct->max_attempts, s6);
        atomicAdd(&ct->incomplete, s7);
        if (MODE == BULK && s8) atomicAdd(a.unfinished, (int)s8);
    }
}

// RHS and Jacobian of many states with the cooperative building blocks
// (test entry point): one group per state.
template <int G, int R>
__global__ void __launch_bounds__(64) k_eval_coop(CoopMech M, int gl_stride, int nsp, int64_t ncell,
                                                  const double* __restrict__ rho, const double* __restrict__ y,
                                                  double* __restrict__ f, double* __restrict__ J) {
    constexpr int NC = G * R, NGRP = 64 / G;
    extern __shared__ double lds[];
    const int lane = threadIdx.x, l = lane % G, grp = lane / G, base = grp * G;
    GL gl(lds + grp * gl_stride, nsp, M.nr, NC);
    const int n = M.n;
    double* jb = lds + NGRP * gl_stride + grp * n * n + l;
    const int64_t c = blockIdx.x * (int64_t)NGRP + grp;
    if (c >= ncell) return;   // whole groups exit together
    double yy[R], ff[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int i = l + G * q;
        yy[q] = (i < n) ? y[i * ncell + c] : 0.0;
    }
    coop_rhs<G, R>(M, gl, l, base, rho[c], yy, ff);
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int i = l + G * q;
        if (i < n) f[i * ncell + c] = ff[q];
    }
    if (J) {
        // c = -1 gives A = I + J in the group's LDS matrix
        coop_newton_matrix<G, R>(M, gl, l, base, rho[c], yy, -1.0, jb);
#pragma unroll
        for (int q = 0; q < R; q++) {
            const int i = l + G * q;
            if (i < n) {
                for (int col = 0; col < n; col++)
                    J[(i * n + col) * ncell + c] = jb[col * n + G * q] - (i == col ? 1.0 : 0.0);
            }
        }
    }
}

}  // namespace chem
