// Types shared by the host side and the kernels of libchem.
#pragma once
#include <cstdint>

namespace chem {

constexpr double RGAS = 8.314462618;
constexpr double PREF = 101325.0;
constexpr double C_FLOOR = 1e-300;   // floor of concentrations inside logarithms [mol/m^3]
constexpr int MAXORD = 5;            // BDF orders 1..5
constexpr int ND = MAXORD + 3;       // backward differences kept per component

enum RxType { RX_ELEM = 0, RX_TB = 1, RX_FO = 2 };

enum : uint8_t {
    ST_DONE = 0,
    ST_SKIPPED = 1,
    ST_KMAX = 2,
    ST_FAIL = 3,
    ST_TINV = 4,
    ST_SURR_OK = 5,
    ST_SURR_REJ = 6,
    ST_ACTIVE = 7,   // internal: selected for integration, not finished
};

// Numerical mechanism parameters, SI, laid out for uniform (scalar) loads.
template <class M>
struct Params {
    double W[M::NS], invW[M::NS], Tmid[M::NS];
    double hlo[M::NS][6], hhi[M::NS][6];   // h/RT coefficients (pre-divided)
    double slo[M::NS][6], shi[M::NS][6];   // s/R coefficients (pre-divided)
    double clo[M::NS][5], chi[M::NS][5];   // cp/R coefficients
    double lnA[M::NR], b[M::NR], EaR[M::NR];
    double lnA0[M::NR], b0[M::NR], Ea0R[M::NR];
    double troe[M::NR][4];
    double eff[M::NR][M::NS];
};

// Device-side box descriptor (one per AMR box; a single box for chem_integrate).
struct DevBox {
    const double* rho;
    const double* e;
    double* Y;
    double* T;
    const uint8_t* mask;
    uint8_t* status;
    int64_t ncell, ldY, off;  // off = first global cell index of the box
    double dt;
};

// Device counters (one set per context).
struct Counters {
    unsigned long long steps, attempts, rhs, jac, lu, solves, max_attempts, incomplete;
    unsigned long long surr_ok, surr_rej;   // surrogate pass: accepted, handed to the integrator
    unsigned long long surr_why[4];         // first failed check: envelope, Y >= -10 atol, T, one-step vs two-step
};

}  // namespace chem
