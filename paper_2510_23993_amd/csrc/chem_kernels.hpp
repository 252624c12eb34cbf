// Kernels of the chemistry hot path (gfx950, wave64).  One reactor cell per
// lane; the per-lane Newton matrix / LU lives in LDS, the BDF backward
// differences in the lane's registers.
//
// Pipeline of the bulk-sparse algorithm (Alg. 3):
//   k_screen    T from (e, Y), skip cold / masked cells, per-block counts
//   k_scan      exclusive scan of the block counts (one workgroup)
//   k_scatter   deterministic compaction of active cells -> active_ids
//   k_integrate<BULK>    up to kmax_bulk steps per cell per round; gated on
//                        the device while more than nactive_star cells remain
//   k_count_unfinished / k_scan / k_scatter_unfinished -> sparse slot list
//   k_integrate<SPARSE>  persistent kernel: lanes pull cells from a queue and
//                        integrate them to completion
// The plain algorithm (Alg. 2) is k_screen + k_integrate<PLAIN>: one thread
// per cell, integrate to completion, no refill.
#pragma once
#include <hip/hip_runtime.h>

#include "chem_device.hpp"

namespace chem {

enum Mode { PLAIN = 0, BULK = 1, SPARSE = 2 };

__device__ __forceinline__ int find_box(const DevBox* boxes, int nbox, int64_t g) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// --------------------------------------------------------------- utilities
__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i32(int* p, int64_t n, int v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// block of 256 threads = 4 waves; returns the block total in every thread and
// each thread's exclusive prefix within the block.
__device__ __forceinline__ int block_prefix_256(bool pred, int* sh, int& total) {
    const unsigned long long m = wave_ballot(pred);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int within = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) sh[w] = __popcll(m);
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (i < w) before += sh[i];
        total += sh[i];
    }
    __syncthreads();
    return before + within;
}

// One workgroup of 1024 threads: exclusive scan of cnt[0..nb) into off[],
// total into *total.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ cnt, int nb,
                                               int* __restrict__ off, int* __restrict__ total) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per, b1 = min(nb, b0 + per);
    int s = 0;
    for (int i = b0; i < b1; i++) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {   // Hillis-Steele inclusive scan of the partials
        const int v = (t >= d) ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int i = b0; i < b1; i++) {
        off[i] = run;
        run += cnt[i];
    }
    if (t == 1023) *total = part[1023];
}

// Exclusive scan of cnt[0..n) for large n, in three launches: k_scan_tiles
// scans tiles of 2048 counts (256 threads, 8 contiguous counts each) into
// off[] and writes each tile's total; k_scan (one workgroup) scans the tile
// totals; k_scan_add adds each tile's offset.
constexpr int SCAN_TILE = 2048;

__global__ void __launch_bounds__(256) k_scan_tiles(const int* __restrict__ cnt, int64_t n, int* __restrict__ off,
                                                    int* __restrict__ tsum) {
    __shared__ int sh[256];
    const int t = threadIdx.x;
    const int64_t base = blockIdx.x * (int64_t)SCAN_TILE + t * 8;
    int v[8], s = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        v[i] = base + i < n ? cnt[base + i] : 0;
        s += v[i];
    }
    sh[t] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {   // inclusive scan of the thread sums
        const int x = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    int run = sh[t] - s;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        if (base + i < n) off[base + i] = run;
        run += v[i];
    }
    if (t == 255) tsum[blockIdx.x] = sh[255];
}

__global__ void __launch_bounds__(256) k_scan_add(int* __restrict__ off, int64_t n, const int* __restrict__ toff) {
    const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
    const int add = toff[blockIdx.x];
    for (int64_t i = base + threadIdx.x; i < base + SCAN_TILE && i < n; i += 256) off[i] += add;
}

// --------------------------------------------------------------- screening
// status_int[g] <- ST_ACTIVE for cells to integrate, else a final code.
// T[i] <- T0 = T(e, Y) for every cell with a valid state.
template <class M>
__global__ void __launch_bounds__(256) k_screen(const Params<M>* __restrict__ Pp,
                                                const DevBox* __restrict__ boxes, int nbox,
                                                int64_t total, double t_react_min,
                                                uint8_t* __restrict__ st_int,
                                                int* __restrict__ block_cnt) {
    __shared__ int sh[4];
    const Params<M>& P = *Pp;
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
            double Y[M::NS];
#pragma unroll
            for (int k = 0; k < M::NS; k++) Y[k] = B.Y[k * B.ldY + i];
            double T0;
            if (!(rho > 0.0) || !isfinite(rho) || !isfinite(e) || !T_from_e(P, e, Y, B.T[i], T0)) {
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

// active_ids[off[b] + rank] = g for ST_ACTIVE cells, in increasing g.
__global__ void __launch_bounds__(256) k_scatter(const uint8_t* __restrict__ st_int, int64_t total,
                                                 const int* __restrict__ off,
                                                 int* __restrict__ ids) {
    __shared__ int sh[4];
    const int64_t g = blockIdx.x * 256ll + threadIdx.x;
    const bool a = g < total && st_int[g] == ST_ACTIVE;
    int tot;
    const int r = block_prefix_256(a, sh, tot);
    if (a) ids[off[blockIdx.x] + r] = (int)g;
}

// unfinished slots (flag != 2) among [0, *n)
__global__ void __launch_bounds__(256) k_count_unfinished(const uint8_t* __restrict__ flag,
                                                          const int* __restrict__ n,
                                                          int* __restrict__ block_cnt) {
    __shared__ int sh[4];
    const int64_t s = blockIdx.x * 256ll + threadIdx.x;
    const bool a = s < *n && flag[s] != 2;
    int tot;
    block_prefix_256(a, sh, tot);
    if (threadIdx.x == 0) block_cnt[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scatter_unfinished(const uint8_t* __restrict__ flag,
                                                            const int* __restrict__ n,
                                                            const int* __restrict__ off,
                                                            int* __restrict__ ids) {
    __shared__ int sh[4];
    const int64_t s = blockIdx.x * 256ll + threadIdx.x;
    const bool a = s < *n && flag[s] != 2;
    int tot;
    const int r = block_prefix_256(a, sh, tot);
    if (a) ids[off[blockIdx.x] + r] = (int)s;
}

// ------------------------------------------- cost-ordered compaction
// Per-cell completion prediction for the order in which lanes take cells:
// the number of tolerance units the state moves per dt at the start,
// s = dt max_i |f_i(y0)| / (rtol |y0_i| + atol) (one RHS per active cell),
// ranks cells by the work the integrator will spend on them.  Cells are
// taken longest first (bucket 0 = largest s, one bucket per factor 2^(1/4) of s),
// so long cells do not start last and leave a tail of idle lanes.  Results
// do not depend on the order: each cell is integrated by itself.
constexpr int COST_BUCKETS = 256;

template <class M>
__global__ void __launch_bounds__(256) k_cost_key(const Params<M>* __restrict__ Pp,
                                                  const DevBox* __restrict__ boxes, int nbox,
                                                  const int* __restrict__ ids, const int* __restrict__ n_items,
                                                  double rtol, double atol, uint8_t* __restrict__ key,
                                                  int* __restrict__ bcnt, int nb) {
    __shared__ int hist[COST_BUCKETS];
    const Params<M>& P = *Pp;
    const int n = *n_items;
    const int64_t slot = blockIdx.x * 256ll + threadIdx.x;
    if (threadIdx.x < COST_BUCKETS) hist[threadIdx.x] = 0;
    __syncthreads();
    if (slot < n) {
        const int64_t g = ids[slot];
        const DevBox& B = boxes[find_box(boxes, nbox, g)];
        const int64_t i = g - B.off;
        double y[M::N], f[M::N];
#pragma unroll
        for (int k = 0; k < M::NS; k++) y[k] = B.Y[k * B.ldY + i];
        y[M::NS] = B.T[i];
        rhs(P, B.rho[i], y, f);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < M::N; k++) s = fmax(s, fabs(f[k]) / (rtol * fabs(y[k]) + atol));
        s *= B.dt;
        // s that is not finite (a state the integrator will reject) goes first
        const int lg = isfinite(s) ? (int)fmin(floor(4.0 * log2(fmax(s, 1.0))), (double)(COST_BUCKETS - 1)) : COST_BUCKETS - 1;
        const int b = COST_BUCKETS - 1 - lg;
        key[slot] = (uint8_t)b;
        atomicAdd(&hist[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < COST_BUCKETS) bcnt[threadIdx.x * nb + blockIdx.x] = hist[threadIdx.x];
}

// ids_out[off[b * nb + block] + rank] = ids_in[slot], rank = the slot's
// position among the block's slots of bucket b (in slot order): a stable
// counting sort by bucket.
__global__ void __launch_bounds__(256) k_bucket_scatter(const uint8_t* __restrict__ key,
                                                        const int* __restrict__ ids_in,
                                                        const int* __restrict__ n_items,
                                                        const int* __restrict__ off, int nb,
                                                        int* __restrict__ ids_out) {
    __shared__ int wc[4][COST_BUCKETS];
    const int n = *n_items;
    const int64_t slot = blockIdx.x * 256ll + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = slot < n ? (int)key[slot] : -1;
    for (int i = threadIdx.x; i < 4 * COST_BUCKETS; i += 256) wc[i / COST_BUCKETS][i % COST_BUCKETS] = 0;
    __syncthreads();
    // one pass per bucket present in the wave (the first pending lane's):
    // each lane's rank among the wave's lanes of its bucket, and the counts
    int within = 0;
    bool pending = b >= 0;
    for (;;) {
        const unsigned long long pm = wave_ballot(pending);
        if (!pm) break;
        const int bb = __shfl(b, __ffsll((long long)pm) - 1);
        const unsigned long long m = wave_ballot(pending && b == bb);
        if (pending && b == bb) {
            within = __popcll(m & ((1ull << lane) - 1ull));
            pending = false;
        }
        if (lane == 0) wc[w][bb] = __popcll(m);
    }
    __syncthreads();
    if (b >= 0) {
        int before = 0;
        for (int q = 0; q < w; q++) before += wc[q][b];
        ids_out[off[b * nb + blockIdx.x] + before + within] = ids_in[slot];
    }
}

// --------------------------------------------------------- state preparation
template <class M>
__global__ void k_prepare(const Params<M>* __restrict__ Pp, int64_t n, const double* __restrict__ T,
                          const double* __restrict__ p, const double* __restrict__ Y, int64_t ldY,
                          double* __restrict__ rho, double* __restrict__ e) {
    const Params<M>& P = *Pp;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y[M::NS], sw = 0.0;
#pragma unroll
    for (int k = 0; k < M::NS; k++) {
        y[k] = Y[k * ldY + i];
        sw += y[k] * P.invW[k];
    }
    double ee, cv;
    e_cv(P, T[i], y, ee, cv);
    rho[i] = p[i] / (RGAS * T[i] * sw);
    e[i] = ee;
}

template <class M>
__global__ void k_eval_rhs(const Params<M>* __restrict__ Pp, int64_t n, const double* __restrict__ rho,
                           const double* __restrict__ y, double* __restrict__ f,
                           double* __restrict__ J) {
    const Params<M>& P = *Pp;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n) return;
    double yy[M::N], ff[M::N];
#pragma unroll
    for (int i = 0; i < M::N; i++) yy[i] = y[i * n + c];
    rhs(P, rho[c], yy, ff);
#pragma unroll
    for (int i = 0; i < M::N; i++) f[i * n + c] = ff[i];
    if (J) jac_cols<M>(P, rho[c], yy, [&](int i, int j, double v) { J[(i * M::N + j) * n + c] = v; });
}

// ------------------------------------------------------------ BDF stepper
// Variable-order (1-5) BDF in backward-difference form on a quasi-constant
// step (Shampine & Reichelt 1997, kappa = 0): predictor y0 = sum_{j<=k} D_j,
// correction d solving d = (h/gamma_k) f(y0 + d) - psi by modified Newton
// with M = I - c_lu J (LU in LDS; J and LU refreshed together when the
// step-size coefficient drifts by more than 30% or Newton fails with a
// Jacobian from an earlier step), local error d/(k+1), WRMS norm with
// weights 1/(rtol |y| + atol).  The Newton convergence test, the update of
// the differences on acceptance and the order selection follow SciPy's BDF
// implementation (scipy/integrate/_ivp/bdf.py, BSD-3-Clause), except that
// the first Newton iteration may already converge on the contraction
// estimate carried from earlier attempts (Hairer & Wanner's RADAU5 rule).  The
// differences D[j][i] (j = 0..MAXORD+2) live in the lane's registers: every
// access below uses indices that are compile-time constants once the loops
// are unrolled (the order k only selects among them).

__device__ __forceinline__ double gamma_k(int k) {  // sum_{i<=k} 1/i
    double g = 0.0;
    g = (k == 1) ? 1.0 : g;
    g = (k == 2) ? 1.5 : g;
    g = (k == 3) ? 11.0 / 6.0 : g;
    g = (k == 4) ? 25.0 / 12.0 : g;
    g = (k == 5) ? 137.0 / 60.0 : g;
    return g;
}

template <class M>
struct Lane {
    static constexpr int N = M::N;
    double t, tend, h, c_lu, rho;
    double eta;   // Newton contraction estimate theta/(1 - theta) carried between attempts
    double yin[M::N > M::NN ? M::N - M::NN : 1];   // species in no reaction: constant over the step
    int k, neq, att, round_att;
    bool lu_ok, jac_fresh, last;   // last: the next attempt ends on t_end
    int piv[M::NN];
    // per-lane statistics
    unsigned long long n_steps, n_att, n_rhs, n_jac, n_lu, n_solve;
};

// Weight 1/x of the error norms; the weights only scale tolerances, so the
// FP32 reciprocal (one instruction, ~1 ulp of FP32) is enough.
__device__ __forceinline__ double inv_weight(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (double)__builtin_amdgcn_rcpf((float)x);
#else
    return (double)(1.0f / (float)x);
#endif
}

// weighted mean square (the square of wrms) over the first N entries, as a
// mean over DIV components (the integrated components are the state less
// its constant inert species, whose entries are zero in every norm)
template <int N, int DIV = N>
__device__ __forceinline__ double wms(const double* v, const double* isc) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const double r = v[i] * isc[i];
        s += r * r;
    }
    return s * (1.0 / DIV);
}

template <int N, int DIV = N>
__device__ __forceinline__ double wrms(const double* v, const double* isc) {
    return sqrt(wms<N, DIV>(v, isc));
}

// full state y (N components) from the integrated components yr (the
// Newton system's order) and the constant inert species
template <class M>
__device__ __forceinline__ void expand_state(const double* yr, const double* yin, double* y) {
    int q = 0;
#pragma unroll
    for (int i = 0; i < M::N; i++) {
        if (M::SYS[i] >= 0) {
            y[i] = yr[M::SYS[i]];
        } else {
            y[i] = yin[q];
            q++;
        }
    }
}

// D_j <- nabla'^j P(t_n) on the grid of spacing rho*h (j = 1..k; D_0 unchanged):
// T_ji = sum_m (-1)^m C(j,m) b_i(m rho), b_i(x) = prod_{l=1..i} (l - 1 - x)/l.
// b_i(m rho) does not depend on j: one table of them, then the alternating
// binomial sums with compile-time coefficients.
template <int N>
__device__ __forceinline__ void rescale(double (&D)[ND][N], int k, double r) {
    double B[MAXORD + 1][MAXORD + 1];   // B[m][i] = b_i(m r)
#pragma unroll
    for (int m = 0; m <= MAXORD; m++) {
        const double x = m * r;
        double b = 1.0;
        B[m][0] = 1.0;
#pragma unroll
        for (int l = 1; l <= MAXORD; l++) {
            b *= (l - 1 - x) * (1.0 / l);
            B[m][l] = b;
        }
    }
    double Tm[MAXORD + 1][MAXORD + 1];
#pragma unroll
    for (int j = 1; j <= MAXORD; j++) {
#pragma unroll
        for (int i = 0; i <= MAXORD; i++) {
            double s = 0.0, binom = 1.0;
#pragma unroll
            for (int m = 0; m <= j; m++) {
                s += ((m & 1) ? -binom : binom) * B[m][i];
                binom = binom * (j - m) / (m + 1);
            }
            Tm[j][i] = s;
        }
    }
#pragma unroll
    for (int c = 0; c < N; c++) {
        double d[MAXORD + 1];
#pragma unroll
        for (int i = 0; i <= MAXORD; i++) d[i] = (i <= k) ? D[i][c] : 0.0;
#pragma unroll
        for (int j = 1; j <= MAXORD; j++) {
            if (j <= k) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i <= MAXORD; i++) s += Tm[j][i] * d[i];
                D[j][c] = s;
            }
        }
    }
}

enum StepResult { SR_RETRY = 0, SR_ACCEPT = 1, SR_DONE = 2, SR_FAIL = 3 };

// Step size hn = h fac of the next attempt, clamped onto t_end (fac is then
// the clamped ratio).  A step reaches t_end when t + hn rounds to it or when
// hn covers the remaining interval: after a clamp h = t_end - t exactly, but
// t + h may round below t_end, and a retry at that size must still land on
// t_end.  Returns false when hn is below the resolution of t.
template <class M>
__device__ __forceinline__ bool next_step(Lane<M>& L, double& fac, double& hn) {
    constexpr double EPS = 2.220446049250313e-16;
    hn = L.h * fac;
    if (!(hn >= 10.0 * EPS * fabs(L.t))) return false;
    L.last = L.t + hn >= L.tend || hn >= L.tend - L.t;
    if (L.last) {
        fac = (L.tend - L.t) / L.h;
        hn = L.tend - L.t;
    }
    return true;
}

// Every change of step size (rejections, order and step selection, the
// clamp of the last step onto t_end) goes through one rescale of D at the
// end of the attempt: the ratios of successive changes multiply, since each
// re-samples the same interpolating polynomial.  The last step is flagged
// there, so the next attempt lands exactly on t_end.
template <class M>
__device__ __forceinline__ int bdf_attempt(const Params<M>& P, Lane<M>& L, double (&D)[ND][M::NN], double* A,
                           double rtol, double atol) {
    // the integrated components: the Newton system's (species that react,
    // then T); norms are means over all N components (inert entries are 0)
    constexpr int N = M::N, NI = M::NN;
    constexpr double EPS = 2.220446049250313e-16;
    L.att++;
    L.round_att++;
    L.n_att++;
    const bool last = L.last;
    const double tn = last ? L.tend : L.t + L.h;
    const int k = L.k;
    const double gk = gamma_k(k);
    int res = SR_RETRY;
    bool resc = false;     // the step size changes by fac for the next attempt
    double fac = 1.0;
    double ise[NI];
    const double c = L.h / gk;
    bool lu_ready = true;
    if (!L.lu_ok || fabs(c - L.c_lu) > 0.3 * L.c_lu) {
        // the predicted state is formed here and again below, so that no
        // per-component vector stays live across the Jacobian
        double yr[NI], yj[N];
#pragma unroll
        for (int i = 0; i < NI; i++) {
            double a = 0.0;
#pragma unroll
            for (int j = 0; j <= MAXORD; j++)
                if (j <= k) a += D[j][i];
            yr[i] = a;
        }
        expand_state<M>(yr, L.yin, yj);
        newton_matrix<M>(P, L.rho, yj, c, A);
        L.n_jac++;
        L.n_lu++;
        L.jac_fresh = true;
        L.lu_ok = lu_factor<M::NN, lanes_per_wave<M>()>(A, L.piv);
        L.c_lu = c;
        if (!L.lu_ok) {   // singular even with a fresh Jacobian: shrink the step
            fac = 0.25;
            resc = true;
        }
        lu_ready = L.lu_ok;
    }
    double yp[NI], psi[NI], isc[NI];
#pragma unroll
    for (int i = 0; i < NI; i++) {
        double a = 0.0, b = 0.0, gj = 0.0;
#pragma unroll
        for (int j = 0; j <= MAXORD; j++) {
            if (j <= k) {
                const double dj = D[j][i];
                a += dj;
                if (j >= 1) {
                    gj += 1.0 / j;
                    b += gj * dj;
                }
            }
        }
        yp[i] = a;
        psi[i] = b / gk;
        isc[i] = inv_weight(atol + rtol * fabs(a));
    }
    if (lu_ready) {
        const double tol = fmax(10.0 * EPS / rtol, fmin(0.03, sqrt(rtol)));
        double d[NI], yn[NI];
#pragma unroll
        for (int i = 0; i < NI; i++) {
            d[i] = 0.0;
            yn[i] = yp[i];
        }
        bool conv = false;
        double dn_old = -1.0;
        for (int it = 0; it < 4; it++) {
            double f[NI];
            {
                double y[N], ff[N];
                expand_state<M>(yn, L.yin, y);
                rhs(P, L.rho, y, ff);
#pragma unroll
                for (int s = 0; s < NI; s++) f[s] = ff[M::ISYS[s]];
            }
            L.n_rhs++;
            bool fin = true;
#pragma unroll
            for (int i = 0; i < NI; i++) {
                f[i] = c * f[i] - psi[i] - d[i];
                fin = fin && isfinite(f[i]);
            }
            if (!fin) break;
            lu_solve<M::NN, lanes_per_wave<M>()>(A, L.piv, f);
            L.n_solve++;
            const double dn = wrms<NI, N>(f, isc);
            const double rate = dn_old > 0.0 ? dn / dn_old : -1.0;
            if (rate >= 0.0) {
                double rp = 1.0;
                for (int q = 0; q < 4 - it; q++) rp *= rate;
                if (rate >= 1.0 || rp / (1.0 - rate) * dn > tol) break;
            }
#pragma unroll
            for (int i = 0; i < NI; i++) {
                yn[i] += f[i];
                d[i] += f[i];
            }
            // the first iteration may converge on the contraction estimate of
            // the previous attempts, eta^0.8 (the rule of Hairer & Wanner's
            // RADAU5); later ones on this attempt's own rate
            const double eta = rate >= 0.0 ? rate / (1.0 - rate) : exp2(0.8 * log2(fmax(L.eta, 1e-16)));
            if (rate >= 0.0) L.eta = eta;
            if (dn == 0.0 || eta * dn < tol) {
                conv = true;
                break;
            }
            dn_old = dn;
        }
        double en = 0.0;
        if (!conv) {
            if (!L.jac_fresh) {   // refresh J and LU, same step size
                L.lu_ok = false;
            } else {
                fac = 0.5;
                resc = true;
            }
        } else {
            // error test
            double e1[NI];
#pragma unroll
            for (int i = 0; i < NI; i++) {
                ise[i] = inv_weight(atol + rtol * fabs(yn[i]));
                e1[i] = d[i] * (1.0 / (k + 1));
            }
            en = wms<NI, N>(e1, ise);   // squared: the powers below take half exponents
            if (en > 1.0) {
                fac = fmax(0.2, 0.9 * ctl_pow(en, -0.5 / (k + 1)));
                resc = true;
            }
        }
        if (conv && en <= 1.0) {
            // accept: D_{k+2} = d - D_{k+1}, D_{k+1} = d, D_j += D_{j+1} for j = k..0
            L.n_steps++;
            L.t = tn;
            L.jac_fresh = false;
            // written with selects only: no branches on the order
#pragma unroll
            for (int i = 0; i < NI; i++) {
                double dk1 = 0.0;   // D_{k+1}
#pragma unroll
                for (int j = 1; j <= MAXORD + 1; j++) dk1 = (j == k + 1) ? D[j][i] : dk1;
                double acc = d[i];
#pragma unroll
                for (int j = ND - 1; j >= 0; j--) {
                    const double upd = D[j][i] + acc;
                    const double nv = (j == k + 2) ? d[i] - dk1 : ((j == k + 1) ? d[i] : ((j <= k) ? upd : D[j][i]));
                    acc = (j <= k) ? upd : acc;
                    D[j][i] = nv;
                }
            }
            L.neq++;
            res = last ? SR_DONE : SR_ACCEPT;
            if (!last && L.neq >= k + 1) {
                // order and step-size selection
                double em = 0.0, ep = 0.0;
                {
                    double v[NI];
                    if (k > 1) {
#pragma unroll
                        for (int i = 0; i < NI; i++) {
                            double a = 0.0;
#pragma unroll
                            for (int j = 2; j <= MAXORD; j++)
                                if (j == k) a = D[j][i];
                            v[i] = a * (1.0 / k);
                        }
                        em = wms<NI, N>(v, ise);
                    }
                    if (k < MAXORD) {
#pragma unroll
                        for (int i = 0; i < NI; i++) {
                            double a = 0.0;
#pragma unroll
                            for (int j = 3; j <= MAXORD + 1; j++)
                                if (j == k + 2) a = D[j][i];
                            v[i] = a * (1.0 / (k + 2));
                        }
                        ep = wms<NI, N>(v, ise);
                    }
                }
                const double f0 = ctl_pow(en, -0.5 / (k + 1));
                const double fm = (k > 1) ? ctl_pow(em, -0.5 / k) : 0.0;
                const double fp = (k < MAXORD) ? ctl_pow(ep, -0.5 / (k + 2)) : 0.0;
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
                fac = fmin(10.0, 0.9 * best);
                resc = true;
            }
        }
    }
    if (res == SR_DONE) return res;
    double hn;
    if (!next_step(L, fac, hn)) return SR_FAIL;
    resc = resc || L.last;
    if (resc) {
        rescale<NI>(D, L.k, fac);
        L.h = hn;
        L.neq = 0;
    }
    return res;
}

// Initial state of a fresh cell from its full state y0 (N components):
// D_0 = y0, D_1 = h f(y0) over the integrated components, the inert species
// kept aside, order 1, with the starting step of Hairer, Norsett & Wanner
// (Solving ODEs I, Sec. II.4).
template <class M>
__device__ __forceinline__ void bdf_init(const Params<M>& P, Lane<M>& L, double (&D)[ND][M::NN], const double* y0,
                         double rtol, double atol) {
    constexpr int N = M::N, NI = M::NN;
    {
        int q = 0;
#pragma unroll
        for (int i = 0; i < N; i++)
            if (M::SYS[i] < 0) L.yin[q++] = y0[i];
    }
    double r0[NI], f0[NI], isc[NI], y1[N], f1[NI];
    double d1 = 0.0, h0 = 0.0;
#pragma unroll
    for (int s = 0; s < NI; s++) {
        r0[s] = y0[M::ISYS[s]];
        isc[s] = inv_weight(atol + rtol * fabs(r0[s]));
    }
#pragma unroll
    for (int i = 0; i < N; i++) y1[i] = y0[i];
    // f(y0), then f(y0 + h0 f(y0)): one evaluation site for both
#pragma unroll 1
    for (int pass = 0; pass < 2; pass++) {
        {
            double ff[N];
            rhs(P, L.rho, y1, ff);
#pragma unroll
            for (int s = 0; s < NI; s++) f1[s] = ff[M::ISYS[s]];
        }
        if (pass == 0) {
#pragma unroll
            for (int s = 0; s < NI; s++) f0[s] = f1[s];
            const double d0 = wrms<NI, N>(r0, isc);
            d1 = wrms<NI, N>(f0, isc);
            h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
            h0 = fmin(h0, L.tend);
#pragma unroll
            for (int s = 0; s < NI; s++) y1[M::ISYS[s]] = r0[s] + h0 * f0[s];
        }
    }
    L.n_rhs += 2;
#pragma unroll
    for (int s = 0; s < NI; s++) f1[s] -= f0[s];
    const double d2 = wrms<NI, N>(f1, isc) / h0;
    const double mx = fmax(d1, d2);
    const double h1 = (mx <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : sqrt(0.01 / mx);
    L.h = fmin(fmin(100.0 * h0, h1), L.tend);
#pragma unroll
    for (int s = 0; s < NI; s++) {
        D[0][s] = r0[s];
        D[1][s] = L.h * f0[s];
#pragma unroll
        for (int j = 2; j < ND; j++) D[j][s] = 0.0;
    }
    L.t = 0.0;
    L.k = 1;
    L.neq = 0;
    L.att = 0;
    L.lu_ok = false;
    L.jac_fresh = false;
    L.c_lu = 0.0;
    L.eta = 1.0;
    L.last = L.h >= L.tend;   // t = 0: the first step covers the interval
}

// ------------------------------------------------------- integration kernel
struct SaveArea {             // per active slot, lane-major [field][slot]
    double* D;                // ND * NN rows (the integrated components)
    double* LU;               // N * N rows
    double* scal;             // 4 rows: t, h, c_lu, eta
    int* ints;                // 4 rows: k, neq, att, flags(lu_ok | jac_fresh<<1 | last<<2)
    int8_t* piv;              // N rows
    int64_t ld;               // capacity (slots)
};

struct IntArgs {
    const DevBox* boxes;
    int nbox;
    uint8_t* st_int;
    const int* active_ids;    // slot -> global cell (BULK, SPARSE)
    const int* items;         // SPARSE: item -> slot
    const int* n_items_dev;   // BULK: n_active, SPARSE: n_sparse
    int64_t n_items_host;     // PLAIN: total cells
    int* queue;               // refill counter of this launch
    int* unfinished;          // BULK: cells left unfinished by this round
    int* rounds;              // BULK: number of rounds that passed the gate
    const int* gate;          // BULK round > 0: previous round's unfinished count
    const int* gate_prev;     // BULK round > 0: the count one round earlier (decay gate)
    double keep;              // stop the rounds once a round keeps more than keep of its cells
    int nstar;
    uint8_t* flag;            // per slot: 0 fresh, 1 saved, 2 done
    SaveArea sv;
    int kmax;
    double rtol, atol;
    Counters* ctr;
    const int* kmax_dev;      // BULK: this round's step limit on the device (adaptive rounds), or null
    unsigned* rem_hist;       // BULK: histogram of predicted remaining attempts of the saved cells, or null
    uint8_t* rem_key;         // BULK: per saved slot, REM_BINS - 1 - its predicted-remaining bin, or null
};

// Completion prediction of a cell that stops at a round's step limit: the
// attempts the rest of its interval would take at the pace of this round,
// att_round (t_end - t) / (t - t_round_start), as a log2 bin (0 .. 31).
constexpr int REM_BINS = 32;
__device__ __forceinline__ int remaining_bin(int att_round, double t0, double t, double tend) {
    const double prog = t - t0;
    const double rem = prog > 0.0 ? att_round * (tend - t) / prog : 1e30;
    return (int)fmin(ceil(log2(1.0 + rem)), (double)(REM_BINS - 1));
}

// Completion key of an unfinished slot: the key its last round saved
// (flag 1), or bucket 0 (most work first) for a cell no round has taken yet.
__device__ __forceinline__ int slot_key(const uint8_t* flag, const uint8_t* key, int64_t slot) {
    return flag[slot] == 1 ? (key[slot] < REM_BINS ? key[slot] : REM_BINS - 1) : 0;
}

// Per-block counts of the unfinished cells (flag != 2) by their completion
// key, bucket-major: bcnt[key * nb + block].  With `ran`, nothing is done
// unless bulk round r ran (the counts of the last build stay valid).
__global__ void __launch_bounds__(256) k_key_count(const uint8_t* __restrict__ flag, const uint8_t* __restrict__ key,
                                                   const int* __restrict__ n_items, int* __restrict__ bcnt, int nb,
                                                   const int* __restrict__ ran, int r) {
    __shared__ int hist[REM_BINS];
    if (ran && *ran <= r) return;
    const int64_t slot = blockIdx.x * 256ll + threadIdx.x;
    if (threadIdx.x < REM_BINS) hist[threadIdx.x] = 0;
    __syncthreads();
    if (slot < *n_items && flag[slot] != 2) atomicAdd(&hist[slot_key(flag, key, slot)], 1);
    __syncthreads();
    if (threadIdx.x < REM_BINS) bcnt[threadIdx.x * nb + blockIdx.x] = hist[threadIdx.x];
}

// items[off[key * nb + block] + rank] = slot for the unfinished cells, rank
// = the slot's position among the block's unfinished slots of that key: a
// stable counting sort, most remaining work first.
__global__ void __launch_bounds__(256) k_key_scatter(const uint8_t* __restrict__ flag, const uint8_t* __restrict__ key,
                                                     const int* __restrict__ n_items, const int* __restrict__ off,
                                                     int nb, int* __restrict__ items, const int* __restrict__ ran,
                                                     int r) {
    __shared__ int wc[4][REM_BINS];
    if (ran && *ran <= r) return;
    const int64_t slot = blockIdx.x * 256ll + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = (slot < *n_items && flag[slot] != 2) ? slot_key(flag, key, slot) : -1;
    int within = 0;
    for (int bb = 0; bb < REM_BINS; bb++) {
        const unsigned long long m = wave_ballot(b == bb);
        if (b == bb) within = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wc[w][bb] = __popcll(m);
    }
    __syncthreads();
    if (b >= 0) {
        int before = 0;
        for (int q = 0; q < w; q++) before += wc[q][b];
        items[off[b * nb + blockIdx.x] + before + within] = (int)slot;
    }
}

// Step limit of the next bulk round from the predictions of the cells the
// last round saved: the smallest 2^b that covers a fraction q of them,
// clamped to [kmin, kcap] (kmin when no cell was saved).
__global__ void k_next_kmax(const unsigned* __restrict__ hist, const int* __restrict__ saved, double q, int kmin,
                            int kcap, int* __restrict__ kmax) {
    if (threadIdx.x != 0) return;
    const double need = q * (double)*saved;
    double cum = 0.0;
    int b = REM_BINS - 1;
    for (int i = 0; i < REM_BINS; i++) {
        cum += hist[i];
        if (cum >= need) {
            b = i;
            break;
        }
    }
    const double k = *saved > 0 ? ldexp(1.0, b) : (double)kmin;
    *kmax = (int)fmin(fmax(k, (double)kmin), (double)kcap);
}

// a wave refills once this many of its LW cell-carrying lanes are free (7/8:
// on the detonation patch with LW = 63 every value from 48 to 60 was within
// noise of the best, 3-4% faster than 24; on the AMR boxes 9%).  The sparse
// phase waits for the whole wave: 1.5-2% faster again when it runs alone
template <int LW> constexpr int refill_min() { return LW * 7 / 8; }

template <class M, int MODE>
__global__ void __launch_bounds__(64) k_integrate(const Params<M>* __restrict__ Pp, IntArgs a) {
    constexpr int N = M::N, NS = M::NS;
    constexpr int NN = M::NN, LW = lanes_per_wave<M>();
    __shared__ double lds[NN * NN * LW];
    const Params<M>& P = *Pp;
    const int lane = threadIdx.x;
    double* A = lds + lane;   // lanes >= LW carry no cell and never touch it
    if (MODE == BULK) {
        const int nact = *a.n_items_dev;
        if (nact == 0) return;
        if (a.gate && *a.gate <= a.nstar) return;
        if (a.gate_prev && (double)*a.gate > a.keep * (double)*a.gate_prev) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.rounds, 1);
    }
    const int kmax = (MODE == BULK && a.kmax_dev) ? *a.kmax_dev : a.kmax;
    const int64_t n_items = (MODE == PLAIN) ? a.n_items_host : (int64_t)*a.n_items_dev;
    double D[ND][NN];

    Lane<M> L;
    L.n_steps = L.n_att = L.n_rhs = L.n_jac = L.n_lu = L.n_solve = 0;
    double t_round0 = 0.0;   // the cell's time when this round took it
    unsigned long long max_att = 0, incomplete = 0, unfinished = 0;
    int64_t cur = -1;     // current item
    int slot = -1;
    int64_t g = -1;
    int bidx = 0;
    bool exhausted = lane >= LW;
    bool static_taken = false;

    for (;;) {
        // ---- pick up work
        if (MODE == PLAIN) {
            if (cur < 0 && !static_taken) {
                static_taken = true;
                const int64_t it = blockIdx.x * (int64_t)LW + lane;   // LW cells per workgroup
                if (lane < LW && it < n_items && a.st_int[it] == ST_ACTIVE) cur = it;
            }
        } else {
            // lanes refill together: a wave takes new cells once refill_min of
            // its lanes are free (or none is busy; in the sparse phase, whose
            // cells come in cost order, only then), so the starting steps of
            // new cells, which every lane of the wave executes, run for many
            // cells at once instead of for one or two per attempt
            const bool refill = wave_ballot(cur >= 0) == 0 ||
                                __popcll(wave_ballot(cur < 0 && !exhausted)) >= (MODE == SPARSE ? LW : refill_min<LW>());
            for (; refill;) {
                const bool need = cur < 0 && !exhausted;
                const unsigned long long m = wave_ballot(need);
                if (!m) break;
                const int cnt = __popcll(m);
                const int leader = __ffsll((long long)m) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(a.queue, cnt);
                base = __shfl(base, leader);
                if (need) {
                    const int my = base + __popcll(m & ((1ull << lane) - 1ull));
                    if (my < n_items) {
                        const int s = (MODE == SPARSE || a.items) ? a.items[my] : my;
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
        if (wave_ballot(cur >= 0) == 0) break;
        if (cur < 0) continue;
        // ---- a cell was just taken: load it
        if (g < 0) {
            g = (MODE == PLAIN) ? cur : (int64_t)a.active_ids[slot];
            bidx = find_box(a.boxes, a.nbox, g);
            const DevBox& B = a.boxes[bidx];
            const int64_t i = g - B.off;
            L.rho = B.rho[i];
            L.tend = B.dt;
            L.round_att = 0;
            if (MODE != PLAIN && a.flag[slot] == 1) {
                const SaveArea& S = a.sv;
#pragma unroll
                for (int r = 0; r < ND * NN; r++) D[r / NN][r % NN] = S.D[r * S.ld + slot];
#pragma unroll 4
                for (int r = 0; r < NN * NN; r++) A[r * LW] = S.LU[r * S.ld + slot];
#pragma unroll
                for (int r = 0; r < NN; r++) L.piv[r] = S.piv[r * S.ld + slot];
                L.t = S.scal[0 * S.ld + slot];
                L.h = S.scal[1 * S.ld + slot];
                L.c_lu = S.scal[2 * S.ld + slot];
                L.eta = S.scal[3 * S.ld + slot];
                L.k = S.ints[0 * S.ld + slot];
                L.neq = S.ints[1 * S.ld + slot];
                L.att = S.ints[2 * S.ld + slot];
                const int fl = S.ints[3 * S.ld + slot];
                L.lu_ok = fl & 1;
                L.jac_fresh = (fl >> 1) & 1;
                L.last = (fl >> 2) & 1;
                int q = 0;   // inert species: unchanged in Y until the write-back
#pragma unroll
                for (int k = 0; k < NS; k++)
                    if (M::SYS[k] < 0) L.yin[q++] = B.Y[k * B.ldY + i];
            } else {
                double y0[N];
#pragma unroll
                for (int k = 0; k < NS; k++) y0[k] = B.Y[k * B.ldY + i];
                y0[NS] = B.T[i];
                bdf_init(P, L, D, y0, a.rtol, a.atol);
            }
            t_round0 = L.t;
        }
        // ---- one step attempt
        const int r = bdf_attempt(P, L, D, A, a.rtol, a.atol);
        bool finished = false, save = false;
        uint8_t st = ST_DONE;
        if (r == SR_DONE) {
            finished = true;
        } else if (r == SR_FAIL) {
            finished = true;
            st = ST_FAIL;
        } else if (L.round_att >= kmax) {
            if (MODE == BULK) save = true;
            else {
                finished = true;
                st = ST_KMAX;
            }
        }
        if (finished || save) {
            max_att = max(max_att, (unsigned long long)L.att);
            if (finished) {
                const DevBox& B = a.boxes[bidx];
                const int64_t i = g - B.off;
#pragma unroll
                for (int k = 0; k < NS; k++)
                    if (M::SYS[k] >= 0) B.Y[k * B.ldY + i] = D[0][M::SYS[k]];   // inert species unchanged
                B.T[i] = D[0][M::SYS[NS]];
                // a cell the surrogate handed over reports that it was integrated instead
                const uint8_t fin = (st == ST_DONE && a.st_int[g] == ST_SURR_REJ) ? (uint8_t)ST_SURR_REJ : st;
                a.st_int[g] = fin;
                if (B.status) B.status[i] = fin;
                if (MODE != PLAIN) a.flag[slot] = 2;
                if (st != ST_DONE) incomplete++;
            } else {
                const SaveArea& S = a.sv;
#pragma unroll
                for (int rr = 0; rr < ND * NN; rr++) S.D[rr * S.ld + slot] = D[rr / NN][rr % NN];
#pragma unroll 4
                for (int rr = 0; rr < NN * NN; rr++) S.LU[rr * S.ld + slot] = A[rr * LW];
#pragma unroll
                for (int rr = 0; rr < NN; rr++) S.piv[rr * S.ld + slot] = (int8_t)L.piv[rr];
                S.scal[0 * S.ld + slot] = L.t;
                S.scal[1 * S.ld + slot] = L.h;
                S.scal[2 * S.ld + slot] = L.c_lu;
                S.scal[3 * S.ld + slot] = L.eta;
                S.ints[0 * S.ld + slot] = L.k;
                S.ints[1 * S.ld + slot] = L.neq;
                S.ints[2 * S.ld + slot] = L.att;
                S.ints[3 * S.ld + slot] = (L.lu_ok ? 1 : 0) | (L.jac_fresh ? 2 : 0) | (L.last ? 4 : 0);
                a.flag[slot] = 1;
                unfinished++;
                if (MODE == BULK && (a.rem_hist || a.rem_key)) {
                    const int bin = remaining_bin(L.round_att, t_round0, L.t, L.tend);
                    if (a.rem_hist) atomicAdd(&a.rem_hist[bin], 1u);
                    if (a.rem_key) a.rem_key[slot] = (uint8_t)(REM_BINS - 1 - bin);
                }
            }
            cur = -1;
            g = -1;
            slot = -1;
        }
    }
    // ---- statistics: one atomic per wave and counter
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

// --------------------------------------------- explicit scheme (Sec. 2.1)
// The paper's first-order kinetics steps: Y <- Y + h S with S = dY/dt
// (Eq. 5) and h the largest step for which no mass fraction changes by more
// than frac of max(|Y_k|, y_floor); T follows from the fixed e by Newton
// after every step (Alg. 2); the last step ends exactly at dt.  One lane per
// cell over the compacted active list, refilled from a device queue.
struct ExpArgs {
    const DevBox* boxes;
    int nbox;
    uint8_t* st_int;
    const int* active_ids;
    const int* n_items_dev;
    const uint8_t* flag;      // per slot: 2 = taken by the surrogate pass
    int* queue;               // refill counter (zero at launch)
    int kmax;
    double frac, y_floor;
    Counters* ctr;
};

template <class M>
__global__ void __launch_bounds__(64) k_explicit(const Params<M>* __restrict__ Pp, ExpArgs a) {
    constexpr int N = M::N, NS = M::NS;
    const Params<M>& P = *Pp;
    const int n = *a.n_items_dev;
    const int lane = threadIdx.x;
    unsigned long long steps = 0, max_steps = 0, incomplete = 0;
    // one step per lane and iteration; a lane whose cell is done takes the
    // next one from the queue, so long and short cells mix within a wave
    int cur = -1, k = 0;
    bool exhausted = false;
    int64_t g = 0, i = 0;
    const DevBox* B = nullptr;
    double y[N], rho = 0.0, e0 = 0.0, dt = 0.0, t = 0.0;
    for (;;) {
        for (;;) {
            const bool need = cur < 0 && !exhausted;
            const unsigned long long m = wave_ballot(need);
            if (!m) break;
            const int cnt = __popcll(m);
            const int leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(a.queue, cnt);
            base = __shfl(base, leader);
            if (need) {
                const int my = base + __popcll(m & ((1ull << lane) - 1ull));
                if (my < n) {
                    if (a.flag[my] != 2) cur = my;
                } else {
                    exhausted = true;
                }
            }
        }
        if (wave_ballot(cur >= 0) == 0) break;
        if (cur < 0) continue;
        if (k == 0 && t == 0.0) {   // a cell was just taken: load it
            g = a.active_ids[cur];
            B = &a.boxes[find_box(a.boxes, a.nbox, g)];
            i = g - B->off;
            rho = B->rho[i];
            e0 = B->e[i];
            dt = B->dt;
#pragma unroll
            for (int q = 0; q < NS; q++) y[q] = B->Y[q * B->ldY + i];
            y[NS] = B->T[i];   // from the screen's inversion of e
        }
        uint8_t st = ST_DONE;
        bool done = false;
        if (k >= a.kmax) {
            st = ST_KMAX;
            done = true;
        } else {
            double f[N];
            rhs(P, rho, y, f);
            double h = dt - t;
#pragma unroll
            for (int q = 0; q < NS; q++)
                if (f[q] != 0.0) h = fmin(h, a.frac * fmax(fabs(y[q]), a.y_floor) / fabs(f[q]));
            const bool last = h >= dt - t;
#pragma unroll
            for (int q = 0; q < NS; q++) y[q] += h * f[q];
            t = last ? dt : t + h;
            k++;
            double Tn;
            if (!T_from_e(P, e0, y, y[NS], Tn)) {
                st = ST_TINV;
                done = true;
            } else {
                y[NS] = Tn;
                done = last;
            }
        }
        if (done) {
#pragma unroll
            for (int q = 0; q < NS; q++) B->Y[q * B->ldY + i] = y[q];
            B->T[i] = y[NS];
            const uint8_t fin = (st == ST_DONE && a.st_int[g] == ST_SURR_REJ) ? (uint8_t)ST_SURR_REJ : st;
            a.st_int[g] = fin;
            if (B->status) B->status[i] = fin;
            steps += k;
            max_steps = max(max_steps, (unsigned long long)k);
            if (st != ST_DONE) incomplete++;
            cur = -1;
            k = 0;
            t = 0.0;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        steps += __shfl_xor(steps, o);
        incomplete += __shfl_xor(incomplete, o);
        max_steps = max(max_steps, (unsigned long long)__shfl_xor(max_steps, o));
    }
    if (lane == 0) {
        Counters* ct = a.ctr;
        atomicAdd(&ct->steps, steps);
        atomicAdd(&ct->attempts, steps);
        atomicAdd(&ct->rhs, steps);
        atomicMax(&ct->max_attempts, max_steps);
        atomicAdd(&ct->incomplete, incomplete);
    }
}

}  // namespace chem
