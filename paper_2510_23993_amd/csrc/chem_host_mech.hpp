// Host-side mechanism representation and parser of the library (separate
// from any test code).  Converts CHEMKIN units (cm, mol, s, cal/mol, g/mol)
// to SI and computes the structure hash that selects compiled kernels.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <sstream>
#include <stdexcept>
#include <string>
#include <vector>

namespace chem {

struct HostReaction {
    int type = 0, rev = 1, troe_n = 0;
    std::vector<std::pair<int, int>> re, pr;  // (species, nu)
    double A = 0, b = 0, Ea = 0;              // SI, Ea in J/mol
    double A0 = 0, b0 = 0, Ea0 = 0;
    double troe[4] = {0, 0, 0, 0};
    std::vector<double> eff;                  // [ns], default 1
};

struct HostMech {
    std::string name;
    int ns = 0, ne = 0;
    std::vector<std::string> elements, species;
    std::vector<double> W;                    // kg/mol
    std::vector<int> comp;                    // ns * ne
    std::vector<double> Tlo, Tmid, Thi;
    std::vector<double> alo, ahi;             // ns * 7
    std::vector<HostReaction> rx;
    uint64_t hash = 0;
};

inline uint64_t fnv1a64(const std::string& s) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 0x100000001b3ull;
    }
    return h;
}

inline std::string structure_string(const HostMech& m) {
    std::ostringstream o;
    o << "ns=" << m.ns << ";nr=" << m.rx.size() << ";";
    for (const auto& r : m.rx) {
        o << r.type << "," << r.rev << "," << r.troe_n << ":";
        for (size_t i = 0; i < r.re.size(); i++) o << (i ? "." : "") << r.re[i].first << "^" << r.re[i].second;
        o << ">";
        for (size_t i = 0; i < r.pr.size(); i++) o << (i ? "." : "") << r.pr[i].first << "^" << r.pr[i].second;
        o << ";";
    }
    return o.str();
}

inline HostMech parse_mechanism(const std::string& path) {
    std::ifstream f(path);
    if (!f) throw std::runtime_error("cannot open mechanism file " + path);
    std::vector<std::string> tok;
    std::string line;
    while (std::getline(f, line)) {
        auto p = line.find('#');
        if (p != std::string::npos) line.resize(p);
        std::istringstream ls(line);
        std::string t;
        while (ls >> t) tok.push_back(t);
    }
    size_t pos = 0;
    auto next = [&]() -> const std::string& {
        if (pos >= tok.size()) throw std::runtime_error("unexpected end of mechanism file");
        return tok[pos++];
    };
    auto expect = [&](const char* kw) {
        if (next() != kw) throw std::runtime_error(std::string("expected ") + kw + " at token " + std::to_string(pos));
    };
    auto geti = [&]() {
        const std::string& s = next();
        size_t k;
        int v = std::stoi(s, &k);
        if (k != s.size()) throw std::runtime_error("bad integer '" + s + "'");
        return v;
    };
    auto getd = [&]() {
        const std::string& s = next();
        size_t k;
        double v = std::stod(s, &k);
        if (k != s.size()) throw std::runtime_error("bad number '" + s + "'");
        return v;
    };
    HostMech m;
    expect("MECHANISM");
    m.name = next();
    expect("UNITS");
    expect("CM-MOL-S");
    expect("CAL/MOL");
    expect("ELEMENTS");
    m.ne = geti();
    if (m.ne <= 0) throw std::runtime_error("bad element count");
    for (int e = 0; e < m.ne; e++) m.elements.push_back(next());
    expect("SPECIES");
    m.ns = geti();
    if (m.ns <= 0) throw std::runtime_error("bad species count");
    m.comp.assign((size_t)m.ns * m.ne, 0);
    for (int k = 0; k < m.ns; k++) {
        m.species.push_back(next());
        double w = getd();
        if (!(w > 0)) throw std::runtime_error("bad molecular weight");
        m.W.push_back(w * 1e-3);
        for (int e = 0; e < m.ne; e++) m.comp[k * m.ne + e] = geti();
        for (int j = 0; j < k; j++)
            if (m.species[j] == m.species[k]) throw std::runtime_error("duplicate species " + m.species[k]);
    }
    auto find = [&](const std::string& s) {
        for (int k = 0; k < m.ns; k++)
            if (m.species[k] == s) return k;
        return -1;
    };
    expect("THERMO");
    m.Tlo.assign(m.ns, 0);
    m.Tmid.assign(m.ns, 0);
    m.Thi.assign(m.ns, 0);
    m.alo.assign(7 * m.ns, 0);
    m.ahi.assign(7 * m.ns, 0);
    std::vector<int> seen(m.ns, 0);
    for (int q = 0; q < m.ns; q++) {
        int k = find(next());
        if (k < 0 || seen[k]) throw std::runtime_error("bad THERMO species");
        seen[k] = 1;
        m.Tlo[k] = getd();
        m.Tmid[k] = getd();
        m.Thi[k] = getd();
        for (int a = 0; a < 7; a++) m.alo[7 * k + a] = getd();
        for (int a = 0; a < 7; a++) m.ahi[7 * k + a] = getd();
    }
    expect("REACTIONS");
    int nr = geti();
    if (nr < 0) throw std::runtime_error("bad reaction count");
    for (int j = 0; j < nr; j++) {
        expect("REACTION");
        HostReaction r;
        const std::string ty = next(), rv = next();
        if (ty == "ELEMENTARY") r.type = 0;
        else if (ty == "THREEBODY") r.type = 1;
        else if (ty == "FALLOFF") r.type = 2;
        else throw std::runtime_error("unknown reaction type " + ty);
        if (rv == "REV") r.rev = 1;
        else if (rv == "IRREV") r.rev = 0;
        else throw std::runtime_error("expected REV or IRREV");
        r.eff.assign(m.ns, 1.0);
        bool arr = false, low = false;
        for (;;) {
            const std::string kw = next();
            if (kw == "END") break;
            if (kw == "REACTANTS" || kw == "PRODUCTS") {
                int c = geti();
                if (c <= 0 || c > 6) throw std::runtime_error("bad participant count");
                auto& side = (kw[0] == 'R') ? r.re : r.pr;
                for (int i = 0; i < c; i++) {
                    int k = find(next());
                    int nu = geti();
                    if (k < 0 || nu <= 0 || nu > 3) throw std::runtime_error("bad participant");
                    for (auto& pq : side)
                        if (pq.first == k) throw std::runtime_error("repeated species on one side");
                    side.push_back({k, nu});
                }
            } else if (kw == "ARRHENIUS") {
                r.A = getd();
                r.b = getd();
                r.Ea = getd();
                arr = true;
            } else if (kw == "EFFICIENCIES") {
                int c = geti();
                for (int i = 0; i < c; i++) {
                    int k = find(next());
                    double v = getd();
                    if (k >= 0) r.eff[k] = v;
                }
            } else if (kw == "LOW") {
                r.A0 = getd();
                r.b0 = getd();
                r.Ea0 = getd();
                low = true;
            } else if (kw == "TROE") {
                int c = geti();
                if (c != 3 && c != 4) throw std::runtime_error("bad TROE count");
                r.troe_n = c;
                for (int i = 0; i < c; i++) r.troe[i] = getd();
            } else {
                throw std::runtime_error("unknown keyword " + kw);
            }
        }
        if (!arr || r.re.empty() || r.pr.empty()) throw std::runtime_error("incomplete reaction");
        if (r.type == 2 && !low) throw std::runtime_error("FALLOFF without LOW");
        for (int e = 0; e < m.ne; e++) {
            long bal = 0;
            for (auto& pq : r.re) bal -= (long)pq.second * m.comp[pq.first * m.ne + e];
            for (auto& pq : r.pr) bal += (long)pq.second * m.comp[pq.first * m.ne + e];
            if (bal != 0) throw std::runtime_error("reaction " + std::to_string(j + 1) + " is not element-balanced");
        }
        int order = 0;
        for (auto& pq : r.re) order += pq.second;
        const int oinf = order + (r.type == 1 ? 1 : 0);
        r.A *= std::pow(1e-6, oinf - 1);
        r.Ea *= 4.184;
        if (r.type == 2) {
            r.A0 *= std::pow(1e-6, order);
            r.Ea0 *= 4.184;
        }
        m.rx.push_back(r);
    }
    expect("END");
    m.hash = fnv1a64(structure_string(m));
    return m;
}

}  // namespace chem
