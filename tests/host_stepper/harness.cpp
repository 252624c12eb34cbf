// Host build of the library's one-lane BDF stepper (test harness; never part
// of the library).  The device functions of the stepper are compiled for the
// CPU so that its step-size control can be exercised on the CPU: the cell
// loop of the integration kernel (init, attempts until done, failed or the
// attempt limit) runs here over arrays of cells, with the power used by the
// step-size controllers selectable:
//   0  the library's power (FP32 log2f/exp2f),
//   1  an emulation of the bare FP32 hardware log2/exp2 instructions
//      (denormal inputs and results flushed to zero),
//   2  the FP64 pow,
//   3  as 1, with results moved by up to 2 ulp (a deterministic hash of the
//      input), as instructions that are not correctly rounded may give.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <string>

// device functions of the stepper become host-and-device functions
#undef __device__
#define __device__ __attribute__((host)) __attribute__((device))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#include "chem_math.hpp"

// the stepper's calls of the controllers' power go to the harness's version
namespace chem {
double harness_ctl_pow(double x, double y);
using std::isfinite;   // HIP's isfinite(double) is a device function
}
#define ctl_pow harness_ctl_pow
#include "chem_kernels.hpp"
#include "chem_params.hpp"
#include "gen/mech_list.hpp"

namespace chem {

static int g_pow_mode = 0;

static float flush(float v) { return std::fpclassify(v) == FP_SUBNORMAL ? std::copysign(0.0f, v) : v; }

double harness_ctl_pow(double x, double y) {
    if (g_pow_mode == 2) return std::pow(x, y);
    if (g_pow_mode == 1 || g_pow_mode == 3) {
        const float l = flush(std::log2(flush((float)x)));
        float r = flush(std::exp2(flush(l * (float)y)));
        if (g_pow_mode == 3 && std::isfinite(r) && r != 0.0f) {
            // results off by up to 2 ulp (the hardware instructions are not
            // correctly rounded): a deterministic hash of the input bits
            uint64_t b;
            memcpy(&b, &x, 8);
            b ^= b >> 29;
            b *= 0xbf58476d1ce4e5b9ull;
            b ^= b >> 32;
            const int k = (int)(b % 5) - 2;
            for (int i = 0; i < (k < 0 ? -k : k); i++) r = std::nextafter(r, k < 0 ? 0.0f : INFINITY);
        }
        return (double)r;
    }
    return (ctl_pow)(x, y);   // the library's own function
}

}  // namespace chem

using namespace chem;
using M = Mech_m9;

template <int N>
static int lu_n(const double* A, double* b) {
    double a[N * N], x[N];
    int piv[N];
    for (int i = 0; i < N * N; i++) a[i] = A[i];
    if (!lu_factor<N, 1>(a, piv)) return 0;
    for (int i = 0; i < N; i++) x[i] = b[i];
    lu_solve<N, 1>(a, piv, x);
    for (int i = 0; i < N; i++) b[i] = x[i];
    return 1;
}

extern "C" {

// Integrates n cells (Y[ns][n] column-major and T[n] in/out) over dt with the
// one-lane stepper; status[i] as the library's codes, attempts[i] the
// attempts used.  Returns 0, or -1 if the mechanism is not the compiled one.
int hs_integrate(const char* mech_path, int pow_mode, int64_t n, const double* rho, double* Y, double* T, double dt,
                 double rtol, double atol, int kmax, uint8_t* status, int64_t* attempts) {
    HostMech h = parse_mechanism(mech_path);
    if (h.hash != M::HASH) return -1;
    auto P = std::make_unique<Params<M>>();
    pack_params<M>(h, *P);
    g_pow_mode = pow_mode;
    constexpr int N = M::N, NN = M::NN, LW = lanes_per_wave<M>();
    static double A[NN * NN * LW];
    double D[ND][M::NN];
    for (int64_t i = 0; i < n; i++) {
        Lane<M> L{};
        L.rho = rho[i];
        L.tend = dt;
        L.round_att = 0;
        double y0[N];
        for (int k = 0; k < M::NS; k++) y0[k] = Y[k * n + i];
        y0[M::NS] = T[i];
        bdf_init(*P, L, D, y0, rtol, atol);
        uint8_t st = ST_KMAX;
        for (;;) {
            const int r = bdf_attempt(*P, L, D, A, rtol, atol);
            if (r == SR_DONE) {
                st = ST_DONE;
                break;
            }
            if (r == SR_FAIL) {
                st = ST_FAIL;
                break;
            }
            if (L.att >= kmax) break;
        }
        for (int k = 0; k < M::NS; k++)
            if (M::SYS[k] >= 0) Y[k * n + i] = D[0][M::SYS[k]];
        T[i] = D[0][M::SYS[M::NS]];
        status[i] = st;
        attempts[i] = L.att;
    }
    return 0;
}

// The step-size planning at the end of an attempt, on its own: from (t, h,
// t_end, fac) returns 1 if the next attempt is the last one, 0 if not, -1
// if the step is below the resolution of t; hn and the clamped fac out.
int hs_next_step(double t, double h, double tend, double fac, double* hn, double* fac_out) {
    Lane<M> L{};
    L.t = t;
    L.h = h;
    L.tend = tend;
    if (!next_step(L, fac, *hn)) return -1;
    *fac_out = fac;
    return L.last ? 1 : 0;
}

// The library's dense LU (partial pivoting, reciprocal diagonal) and solve
// on an n x n row-major matrix: b is overwritten by the solution.  Returns 1,
// 0 if the factorisation reports a zero or non-finite pivot, -1 for an n
// with no instantiation here.
int hs_lu(int n, const double* A, double* b) {
    switch (n) {
        case 1: return lu_n<1>(A, b);
        case 2: return lu_n<2>(A, b);
        case 3: return lu_n<3>(A, b);
        case 5: return lu_n<5>(A, b);
        case 9: return lu_n<9>(A, b);
        case 10: return lu_n<10>(A, b);
        case 16: return lu_n<16>(A, b);
        default: return -1;
    }
}

}  // extern "C"
