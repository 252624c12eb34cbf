/*
 * chem.h -- C ABI of the MI355X stiff-chemistry library (libchem.so).
 *
 * The operation: every cell is an independent constant-volume ideal-gas
 * reactor whose density rho and mass-specific internal energy e stay fixed
 * while its composition Y and temperature T are advanced from t = 0 to
 * t = dt, the chemistry substep of a Strang-split reacting-flow step
 * (paper Sec. 2.1, Eq. 5-6: dY_k/dt = W_k Omega_k / rho, and the
 * temperature equation read as dT/dt = -sum_k u_k Omega_k / (rho c_v) with
 * the mass-based mixture c_v and molar internal energies u_k).  The initial
 * temperature is recovered from (e, Y) by Newton iteration at constant rho
 * and e (Sec. 2.1).  Cells colder than a threshold, or masked as solid,
 * are not integrated (Alg. 2 and Alg. 3, "T < T_reaction_min or
 * is_solid").
 *
 * Rates use the matrix form: every reaction's forward and reverse rate of
 * progress is a stoichiometric contraction against log-concentrations
 * followed by exp (Sec. 2.1, kinetics adapted from a matrix-based solver).
 * The contraction runs on ln|C| (|C| floored at 1e-300 mol/m^3) and the sign
 * of a rate of progress is the parity of its negative factors with odd
 * exponents, so negative concentrations give the plain mass-action product.
 * Integration is implicit (variable-order BDF, modified Newton with an
 * analytic Jacobian and LU with partial pivoting, FP64).  With the
 * bulk-sparse algorithm (Alg. 3) every active cell first runs rounds of at
 * most kmax_bulk steps while more than nactive_star cells remain active;
 * the remaining stiff cells are then compacted through an index map and
 * integrated to completion (Sec. 3.2).
 *
 * Units: SI (kg, m, s, mol, J, K); e includes formation energy (NASA-7
 * absolute enthalpy basis).  Mechanism files use CHEMKIN units
 * (cm, mol, s, cal/mol, g/mol); see the mechanism file format in the
 * package documentation.
 *
 * Memory and streams: every state array passed to the integration calls is
 * caller-owned DEVICE memory (hipMalloc'd or a torch CUDA tensor) and stays
 * owned by the caller; the library never frees or reallocates it.  The
 * library owns its workspace (grown on demand, reused across calls).  All
 * work is enqueued on the context's stream, in order; calls return as soon
 * as the work is enqueued unless a chem_stats pointer is passed, in which
 * case the call synchronises the stream and fills it.
 *
 * Errors: 0 = CHEM_OK; negative = hard error (nothing enqueued, message in
 * chem_last_error(), thread-local); positive CHEM_W_INCOMPLETE = the work
 * ran but at least one cell did not reach dt (only reported when a
 * chem_stats pointer forces a synchronisation; per-cell status says which).
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CHEM_OK = 0,
    CHEM_W_INCOMPLETE = 1,
    CHEM_E_INVAL = -1,   /* NULL pointer, ncell < 0, dt <= 0, rtol <= 0, ldY < ncell, bad key */
    CHEM_E_HIP = -2,     /* HIP runtime error */
    CHEM_E_NOMEM = -3,   /* device allocation failed */
    CHEM_E_MECH = -4,    /* parse error, unbalanced reaction, or no compiled kernel for it */
    CHEM_E_STATE = -5    /* object used in a wrong state */
};

/* per-cell status codes written to the status array */
enum {
    CHEM_ST_DONE = 0,        /* reached dt */
    CHEM_ST_SKIPPED = 1,     /* cold (T < t_react_min) or masked: not integrated, Y unchanged */
    CHEM_ST_KMAX = 2,        /* step limit reached; Y, T hold the last accepted state */
    CHEM_ST_FAIL = 3,        /* Newton / step-size failure; last accepted state kept */
    CHEM_ST_TINV = 4,        /* T inversion failed or rho/e not finite or rho <= 0 */
    CHEM_ST_SURR_OK = 5,     /* surrogate increment accepted */
    CHEM_ST_SURR_REJ = 6     /* surrogate rejected, cell integrated implicitly instead */
};

typedef struct chem_mech_s* chem_mech_t; /* immutable after load; shareable across contexts */
typedef struct chem_ctx_s* chem_ctx_t;   /* owns workspace + stream binding; not thread-safe */

typedef struct {
    int64_t ncell;              /* cells handed in */
    int64_t n_active0;          /* cells integrated (after screening) */
    int64_t n_active_after_bulk;/* cells still unfinished when the bulk phase stopped */
    int64_t n_bulk_rounds;      /* bulk rounds that ran */
    int64_t n_sparse;           /* cells handed to the sparse phase */
    int64_t n_incomplete;       /* cells that did not reach dt */
    int64_t n_fallback;         /* surrogate: cells sent back to the implicit path */
    int64_t steps_total;        /* accepted BDF steps */
    int64_t attempts_total;     /* attempted steps (accepted + rejected + retried) */
    int64_t rhs_evals, jac_evals, lu_facts, lin_solves;
    int64_t max_steps_cell;     /* most attempts spent by one cell */
    double t_total_ms;          /* device time of the call (events on the context stream) */
    /* phase split (eager calls only; zero when the call replayed a graph):
     * screening + compaction, bulk rounds, sparse phase (or the plain path) */
    double t_screen_ms, t_bulk_ms, t_sparse_ms;
    /* the part of rhs_evals .. lin_solves spent in the bulk rounds */
    int64_t bulk_rhs_evals, bulk_jac_evals, bulk_lu_facts, bulk_lin_solves;
    /* surrogate pass: cells whose predicted increment was accepted (the
     * cells it handed to the integrator are n_fallback) and its device time */
    int64_t n_surrogate;
    double t_surrogate_ms;
    /* surrogate rejections by the first check that failed: features outside
     * the training envelope, a mass fraction below -10 atol, temperature
     * mismatch, one-step vs two-step disagreement */
    int64_t surr_reject[4];
    /* chem_strang_step: device time of the two flow half steps, and cells
     * whose temperature inversion failed in the flow's primitive pass */
    double t_flow_ms;
    int64_t flow_bad_cells;
} chem_stats;

/* One AMR box (a separately allocated grid): device pointers, column-major
 * Y[k * ldY + i], its own dt.  status and mask may be NULL. */
typedef struct {
    int64_t ncell;
    const double* rho;
    const double* e;
    double* Y;
    int64_t ldY;
    double* T;
    const uint8_t* mask;
    uint8_t* status;
    double dt;
    int level;
} chem_box;

/* Parse a mechanism file (host), check element balance, select the kernels
 * compiled for its reaction structure, and upload its parameters to the
 * current device.  Errors: CHEM_E_INVAL (NULL), CHEM_E_MECH (parse error,
 * unbalanced reaction, structure without compiled kernels), CHEM_E_HIP. */
int chem_load_mechanism(const char* path, chem_mech_t* out);
/* Species / reaction counts and molecular weights [kg/mol] (host array owned
 * by the mechanism). */
int chem_mech_info(chem_mech_t m, int* nspec, int* nreac, const double** W_host);
int chem_species_name(chem_mech_t m, int k, const char** name);
void chem_free_mechanism(chem_mech_t m);

/* Create a context on `device` bound to `hip_stream` (a hipStream_t; NULL =
 * the default stream).  Allocates nothing large until the first call. */
int chem_ctx_create(chem_mech_t m, int device, void* hip_stream, chem_ctx_t* out);
void chem_ctx_destroy(chem_ctx_t c);

/* Options (all numeric):
 *   algorithm     0 = plain (Alg. 2: every unmasked cell, one thread per cell,
 *                 no temperature skip), 1 = bulk-sparse (Alg. 3), default 1
 *   t_react_min   K, cells colder than this are skipped (bulk-sparse), default 500
 *   kmax_bulk     steps per bulk round (Alg. 3 Sec. 2), default 5
 *   nactive_star  bulk rounds continue while more cells than this are active, default 1e4
 *   kmax_sparse   step limit of the sparse phase / plain path, default 1e5
 *   max_rounds    bulk-round launches enqueued per call (device decides how many run), default 24
 *   grid_waves    waves per CU of the persistent integration kernel, default 0 (auto)
 *   precision     0 = FP64 rates (default); 1 = the exponentials of the rate evaluation
 *                 (and the falloff logarithms) on the FP32 units with FP64 range
 *                 reduction; ln C, the contractions, near-equilibrium net rates
 *                 (-q_f expm1 of the FP64 log ratio), Newton, LU and the T inversion
 *                 stay FP64.  Available on every schedule
 *   group         lanes per cell: 0 = compiled one-lane kernel (if the mechanism's
 *                 structure was compiled in), 4/8/16/32/64 = cooperative kernels,
 *                 -1 = automatic (default)
 *   cells_per_wave the same choice counted in cells per 64-lane wave: 64 = one
 *                 lane per cell (group 0; the one-lane kernel's workgroups hold
 *                 63 or 64 cells, by the mechanism's LDS need), 16/8/4/2/1 =
 *                 group 4/8/16/32/64, 0 = automatic
 *   use_graph     1 = capture the enqueued pipeline of chem_integrate_boxes in a
 *                 hipGraph and replay it while the box table is unchanged, default 1
 *   surrogate     1 = run the learned surrogate on the active cells before the
 *                 implicit integration (needs chem_load_surrogate and algorithm 1);
 *                 cells failing its trust check are integrated, default 0
 *   round_decay   0 .. 0.99, default 0 (off): besides the N* gate, the bulk
 *                 rounds stop once a round retires less than this fraction of
 *                 the cells it started with (the active count's decay decides
 *                 the number of rounds); results do not depend on it
 *   order         0 (default) or 1: lanes take the cells longest first.  The
 *                 first round orders the active cells by a predicted cost, the
 *                 number of tolerance units the state moves per dt at the start,
 *                 dt max_i |f_i(y0)| / (rtol |y0_i| + atol), in factor-2^(1/4) buckets;
 *                 later rounds and the sparse phase take the cells the last
 *                 round saved by their predicted remaining attempts, the round's
 *                 pace extrapolated to t_end, att (dt - t) / (t - t_start), in
 *                 factor-2 buckets (the per-cell completion prediction the
 *                 paper's App. B names as the way to adapt the bulk phase).
 *                 Results do not depend on it.  Compiled mechanisms only
 *   kmax_adapt    0 (default, off) .. 1: each bulk round after the first takes its
 *                 step limit from the completion predictions of the cells the
 *                 previous round saved: the smallest power of two that covers
 *                 this fraction of them (at least 2).  Results do not depend on
 *                 it.  Compiled mechanisms only; ignored by the cooperative kernels
 *   method        0 = variable-order BDF (default); 1 = the paper's explicit
 *                 first-order scheme (Sec. 2.1, Alg. 2): Y <- Y + h dY/dt with h
 *                 the largest step that changes no mass fraction by more than
 *                 explicit_frac of max(|Y_k|, 1e-10), T from e by Newton after
 *                 every step, the last step ending at dt; rtol and atol are
 *                 not used, kmax_sparse bounds the steps per cell.  Runs one
 *                 lane per cell (compiled mechanisms only, CHEM_E_INVAL
 *                 otherwise), after the same screen and compaction
 *   explicit_frac largest relative change per explicit step, 1e-6 .. 0.05,
 *                 default 0.01
 *   surr_rtol     relative tolerance of the surrogate's consistency check, default
 *                 1e-6: the check does not see network errors that scale with
 *                 the step (they cancel between the one-step and two-step
 *                 predictions), and on the 8.4M-cell evaluation field it
 *                 accepted cells 10-200x over their tolerance at 1e-4, so the
 *                 default is two orders below a 1e-4 error budget
 * Returns CHEM_E_INVAL for an unknown key or out-of-range value. */
int chem_set_option(chem_ctx_t c, const char* key, double value);
int chem_get_option(chem_ctx_t c, const char* key, double* value);

/* Integrate ncell cells over [0, dt].
 *   rho, e   [ncell] device, read only
 *   Y        [nspec][ldY] device, column-major (Y[k*ldY + i]), in/out
 *   T        [ncell] device, in: temperature guess (values outside
 *            (100, 6000) K mean none), out: final temperature
 *   skip_mask[ncell] device or NULL: nonzero = solid cell, not integrated
 *   status   [ncell] device or NULL: per-cell CHEM_ST_* code
 *   rtol, atol: BDF tolerances, error weights 1/(rtol |y| + atol) on (Y, T)
 *   stats    NULL (asynchronous) or a host struct filled after a stream sync
 * Returns CHEM_OK, CHEM_W_INCOMPLETE (only with stats), or a negative error. */
int chem_integrate(chem_ctx_t c, int64_t ncell, const double* rho, const double* e, double* Y,
                   int64_t ldY, double* T, const uint8_t* skip_mask, uint8_t* status, double dt,
                   double rtol, double atol, chem_stats* stats);

/* Allocation-free variant of chem_integrate, for callers that cannot
 * allocate device memory: code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, layout and per-cell
 * results as chem_integrate with the cooperative schedule and no bulk rounds
 * (option group > 0, or 16 lanes per cell for up to 16 state components and
 * 64 above; screen, compaction, integration to completion); the other
 * options apply as there.  Its workspace is one file-scope device array of
 * about 10.5 MB per GPU, held until the process ends, so
 *   - ncell is at most 1048576 (CHEM_E_INVAL above);
 *   - every call on a GPU uses that GPU's one array: calls that overlap on
 *     one GPU (on different streams or from different threads) race and
 *     give wrong results; calls in one stream are ordered and safe;
 *   - it needs surrogate 0 and method 0 (CHEM_E_STATE otherwise).
 * The call calls no hipMalloc / hipFree and returns without synchronising;
 * it never fills statistics (check status[] for cells that did not finish).
 * Errors as chem_integrate (negative codes only). */
int chem_integrate_noalloc(chem_ctx_t c, int64_t ncell, const double* rho, const double* e, double* Y,
                           int64_t ldY, double* T, const uint8_t* skip_mask, uint8_t* status, double dt,
                           double rtol, double atol);

/* Integrate many separately allocated boxes, each over its own dt, in one
 * enqueued pipeline (one screening pass, one compaction, persistent
 * integration kernels over all boxes; Sec. 3.2.1 multigrid fusion with an
 * index map).  The box table is copied; pointers must stay valid until the
 * work completes.  Same return conventions as chem_integrate. */
int chem_integrate_boxes(chem_ctx_t c, int nbox, const chem_box* boxes, double rtol, double atol,
                         chem_stats* stats);

/* One step of the minimal one-dimensional compressible flow around the
 * chemistry (Sec. 2.1: HLLC convective fluxes, second-order SSP Runge-Kutta):
 * MUSCL reconstruction of (rho, u, p, Y) with the minmod limiter, HLLC with
 * the direct wave-speed estimates, Heun's SSP-RK2, transmissive ends.
 *   U   [3 + nspec][ldU] device, in/out, component-major: rho, rho u, rho E,
 *       rho Y_1 .. rho Y_nspec per cell (E = e + u^2/2, e the chemistry's
 *       mass-specific internal energy including formation energy)
 *   T   [ncell] device, in: temperature guess of the Newton inversion of e
 *       (values outside (100, 6000) K mean none), out: T of the new state
 *   dx  cell size [m], dt step [s] (the caller keeps dt within the CFL limit)
 * Compiled mechanisms only (CHEM_E_INVAL otherwise).  Synchronises the
 * stream; CHEM_E_STATE if a cell's state left the thermo's bracket. */
int chem_flow_step(chem_ctx_t c, int64_t ncell, double dx, double dt, double* U, int64_t ldU, double* T);

/* One Strang-split reacting step (Sec. 2.1 operator splitting): flow over
 * dt/2, the chemistry of chem_integrate over dt (constant rho and e per cell,
 * so only rho Y changes), flow over dt/2.  U, T as chem_flow_step; status
 * [ncell] or NULL as chem_integrate.  With stats the call synchronises and
 * also reports the flow half steps' device time (t_flow_ms) next to the
 * chemistry's phases; without, it is asynchronous.  Returns as
 * chem_integrate; CHEM_E_STATE if the flow's temperature inversion failed
 * (stats only). */
int chem_strang_step(chem_ctx_t c, int64_t ncell, double dx, double dt, double* U, int64_t ldU, double* T,
                     uint8_t* status, double rtol, double atol, chem_stats* stats);

/* (T, p, Y) -> (rho, e) on the device for ncell cells (ideal gas, NASA-7):
 * a convenience to build reactor inputs from primitive states.  T, p
 * [ncell], Y [nspec][ldY]; rho, e [ncell] outputs.  Asynchronous. */
int chem_prepare_state(chem_ctx_t c, int64_t ncell, const double* T, const double* p,
                       const double* Y, int64_t ldY, double* rho, double* e);

/* Right-hand side and analytic Jacobian of the reactor ODE for ncell states
 * (device arrays): y [nspec+1][ncell] column-major (Y then T), rho [ncell];
 * f [nspec+1][ncell]; J [(nspec+1)^2][ncell] with J[(i*(nspec+1)+j)*ncell + c]
 * = d f_i / d y_j (J may be NULL).  Asynchronous.  For testing the kernels'
 * building blocks against the oracle. */
int chem_eval_rhs(chem_ctx_t c, int64_t ncell, const double* rho, const double* y, double* f,
                  double* J);

/* Stoichiometric contractions of the matrix-form rate evaluation (Sec. 2.1,
 * rates of progress as contractions of the stoichiometric matrices with
 * log-concentrations, then exp) as a batch operation: for n states given as
 * lnC [nspec][n] (ln|C_k| in ln(mol/m^3), column-major, device),
 *   zf[j][i] = sum_k nu'_kj lnC[k][i],  zr[j][i] = sum_k nu''_kj lnC[k][i]
 * for every reaction j (outputs [nreac][n] each, device, FP64).
 *   precision 0: FP64 loops over each reaction's participants;
 *             1: the same loops in FP32;
 *             2: dense BF16 matrix cores, ln C split into three BF16 terms
 *                (about 24 significant bits), integer coefficients exact,
 *                FP32 accumulation; at most 128 species.
 * Asynchronous.  CHEM_E_INVAL for bad arguments, CHEM_E_MECH when the
 * mechanism is too large for the matrix-core variant. */
int chem_eval_contractions(chem_ctx_t c, int64_t n, const double* lnC, double* zf, double* zr, int precision);

/* Autotuner: times candidate schedules (lanes per cell, bulk phase on/off,
 * N*, steps per bulk round, persistent grid size) on the given boxes and sets the fastest as the
 * context's options.  Y and T of every box are restored afterwards (the call
 * synchronises the stream).  The choice is cached as a JSON line keyed by
 * (GPU arch, mechanism structure hash, box count, cell count, rtol, atol,
 * precision) in cache_path (NULL = no cache); a cache hit runs nothing.
 * best_ms (may be NULL) receives the winning call time.  Errors as
 * chem_integrate_boxes. */
int chem_autotune(chem_ctx_t c, int nbox, const chem_box* boxes, double rtol, double atol,
                  const char* cache_path, double* best_ms);

/* Learned surrogate of the chemistry step (an addition to the method: the
 * paper has no learned component).  A network 12 -> 256 -> 256 -> 256 -> 10
 * with GELU maps (T, ln(p/atm), ln max(Y_k, 1e-20) for 9 species, ln dt),
 * z-scored, to z-scored asinh-scaled increments (dY_k / (1e-4 |Y_k| + 1e-14),
 * dT / (1e-4 T)); inference runs in BF16 on the matrix cores with FP32
 * accumulation.  A cell's prediction is accepted only if the features of
 * every network evaluation lie in the training envelope, every decoded
 * increment (projected onto element conservation) keeps each Y >= -10 atol
 * and a temperature recovered from the fixed e within 0.5 K of the predicted
 * one, and the one-step prediction N(y0, dt) agrees with the two-step
 * N(N(y0, dt/2), dt/2) (a property of the exact flow) in the weighted RMS
 * norm with weights 1/(surr_rtol |y| + atol); other cells are
 * integrated implicitly.  Weights file (little endian): "CHEMSURR", int32
 * version 1, nin 12, nh 256, nout 10, nspec 9, uint64 mechanism structure
 * hash, float32 parameters (chem_mlp layout), float32 feature mean[12] and
 * std[12], target mean[10] and std[10], float64 raw-feature envelope
 * low[12] and high[12].  Errors: CHEM_E_INVAL (file), CHEM_E_STATE (the
 * context's mechanism is not the compiled 9-species structure it was trained
 * for), CHEM_E_HIP / CHEM_E_NOMEM. */
int chem_load_surrogate(chem_ctx_t c, const char* weights_path);
/* Training pairs of the surrogate for n cells on the device: raw features
 * X [n][12] of (rho, Y0, T0, dt) and raw targets [n][10] (asinh-scaled
 * increments to Y1, T1) as float32, before standardisation.  Y0, Y1 are
 * [9][n] column major; rho, T0, T1, dt [n].  CHEM_E_STATE unless the
 * mechanism has 9 species. */
int chem_surrogate_pairs(chem_ctx_t c, int64_t n, const double* rho, const double* Y0, const double* T0,
                         const double* Y1, const double* T1, const double* dt, float* X, float* targets);
/* Structure hash of a mechanism (what surrogate files and tuning caches key on). */
int chem_mech_hash(chem_mech_t m, uint64_t* hash);

/* Network kernels (training and inference of the surrogate), on device
 * buffers, enqueued on `stream` (a hipStream_t, NULL = default stream).
 * Parameters are one FP32 vector of chem_mlp_nparams() = 137482 entries:
 * W1[256][12], b1[256], W2[256][256], b2, W3[256][256], b3, W4[10][256],
 * b4[10] (W[out][in]).  X is [batch][12] and out [batch][10], row major.
 * ws is a caller-owned workspace of chem_mlp_workspace_floats(batch) floats;
 * chem_mlp_forward with mode 0 (FP32) leaves there the activations that
 * chem_mlp_backward reads; mode 1 is BF16 matrix-core inference (X and
 * params then 16-byte aligned).  Errors: CHEM_E_INVAL for NULL, misaligned or
 * out-of-range arguments, CHEM_E_HIP. */
int64_t chem_mlp_nparams(void);
int64_t chem_mlp_workspace_floats(int64_t batch);
int chem_mlp_forward(void* stream, int64_t batch, const float* params, const float* X, float* out, float* ws,
                     int mode);
/* grads (same layout as params) of the loss whose output gradient is dout
 * [batch][10], after a mode-0 forward of the same batch into ws. */
int chem_mlp_backward(void* stream, int64_t batch, const float* params, const float* X, const float* ws,
                      const float* dout, float* grads);
/* mean squared error over n values: dout = 2 (out - target) / n; loss (device
 * double, may be NULL) receives the mean. */
int chem_mlp_mse(void* stream, int64_t n, const float* out, const float* target, float* dout, double* loss);
/* Adam with bias correction, step counted from 1; m and v start at zero. */
int chem_mlp_adam(void* stream, int64_t n, float* params, const float* grads, float* m, float* v, double lr,
                  double beta1, double beta2, double eps, int step);
/* Minibatch of `batch` rows drawn with replacement from X [n_data][12] and
 * T [n_data][10] by a counter-based generator (SplitMix64 of seed, step, row). */
int chem_mlp_gather(void* stream, int64_t n_data, const float* X, const float* T, int64_t batch, uint64_t seed,
                    int64_t step, float* Xb, float* Tb);
/* Column mean and standard deviation of data [n][cols] (cols <= 64); acc is
 * a device scratch of 2 cols doubles. */
/* Rows idx[0..n) of X [*][12] and T [*][10] copied to rows 0..n) of Xo and To
 * (device buffers; idx is int64 on the device, every entry a valid row: the
 * kernel does not check).  The training driver's data split and the
 * compaction of integrated pairs use it.  CHEM_E_INVAL for NULL pointers or
 * n < 0. */
int chem_mlp_take(void* stream, int64_t n, const int64_t* idx, const float* X, const float* T, float* Xo, float* To);
int chem_mlp_colstats(void* stream, int64_t n, int cols, const float* data, double* acc, float* mean, float* sd);
/* Column minimum and maximum of data [n][cols] (cols <= 64) into lo, hi
 * (device doubles); scratch is 2 cols unsigned ints of device memory. */
int chem_mlp_colrange(void* stream, int64_t n, int cols, const float* data, unsigned int* scratch, double* lo,
                      double* hi);
/* data = (data - mean) / sd, column-wise, in place. */
int chem_mlp_standardize(void* stream, int64_t n, int cols, float* data, const float* mean, const float* sd);
int chem_synchronize(chem_ctx_t c);
const char* chem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
