// Packing of a parsed mechanism's numbers into the parameter block Params<M>
// that the compiled one-lane kernels read (host side): NASA-7 coefficients
// pre-divided for Horner evaluation of h/RT and s/R, Arrhenius triples as
// (ln A, b, Ea/R), Troe constants and third-body efficiencies.
#pragma once
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "chem_host_mech.hpp"
#include "chem_types.hpp"

namespace chem {

template <class M>
void pack_params(const HostMech& h, Params<M>& P) {
    if (h.ns != M::NS || (int)h.rx.size() != M::NR) throw std::runtime_error("size mismatch");
    memset(&P, 0, sizeof(Params<M>));
    for (int k = 0; k < M::NS; k++) {
        P.W[k] = h.W[k];
        P.invW[k] = 1.0 / h.W[k];
        P.Tmid[k] = h.Tmid[k];
        const double* src[2] = {&h.alo[7 * k], &h.ahi[7 * k]};
        double(*H[2])[6] = {P.hlo, P.hhi};
        double(*S[2])[6] = {P.slo, P.shi};
        double(*Cc[2])[5] = {P.clo, P.chi};
        for (int r = 0; r < 2; r++) {
            const double* a = src[r];
            const double hc[6] = {a[0], a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5, a[5]};
            const double sc[6] = {a[0], a[1], a[2] / 2, a[3] / 3, a[4] / 4, a[6]};
            for (int q = 0; q < 6; q++) {
                H[r][k][q] = hc[q];
                S[r][k][q] = sc[q];
            }
            for (int q = 0; q < 5; q++) Cc[r][k][q] = a[q];
        }
    }
    for (int j = 0; j < M::NR; j++) {
        const HostReaction& r = h.rx[j];
        P.lnA[j] = std::log(r.A);
        P.b[j] = r.b;
        P.EaR[j] = r.Ea / RGAS;
        P.lnA0[j] = r.type == 2 ? std::log(r.A0) : 0.0;
        P.b0[j] = r.b0;
        P.Ea0R[j] = r.Ea0 / RGAS;
        for (int q = 0; q < 4; q++) P.troe[j][q] = r.troe[q];
        for (int k = 0; k < M::NS; k++) P.eff[j][k] = r.eff[k];
    }
}

}  // namespace chem
