// Clifford synthesis on the binary tableau: the paper's steps (i)-(iv) and its
// appendix algorithm for linearly independent terms.
//
// Readings of the printed algorithms (the paper is silent or inconsistent):
//  * CNOT update of the Z block: z_c ^= z_t (the printed z_t ^= z_c contradicts
//    the two-qubit conjugation table, e.g. I1 Z2 -> Z1 Z2 under CNOT(1,2)).
//  * Step (i) visits qubits from the highest to the lowest; this order is the
//    one that reproduces the worked example (Hadamards on qubits 3 and 4).
//  * Independent-set elimination clears the pivot column in the rows *below*
//    the pivot row (as the text and the worked appendix example do).
//  * Steps (ii)/(iii) use pivots: row i takes column i when some row j >= i
//    has a 1 there (the paper's row swap), else the lowest unpivoted column
//    holding a 1; CNOT/CZ targets are the unpivoted / other columns.  This is
//    the printed algorithm whenever the X block has full rank, and it also
//    handles the zero-padded rows of rank-deficient groups.
//  * Skip rule: a pre-pass; {I,Z}-only qubits leave the tableau, {I,X}-only
//    qubits get H first and then leave it.
#include <algorithm>
#include <cstring>

#include "sd_internal.h"

namespace sd {

uint64_t Echelon::reduce(uint64_t v, uint64_t *used) const {
    uint64_t u = 0;
    for (size_t i = 0; i < vec.size(); ++i)
        if ((v >> piv[i]) & 1) {
            v ^= vec[i];
            u ^= comb[i];
        }
    if (used) *used = u;
    return v;
}

bool Echelon::insert(uint64_t v) {
    uint64_t cm = 0;
    uint64_t r = reduce(v, &cm);
    int idx = inserted++;
    if (r == 0) return false;
    cm ^= (idx < 64) ? (1ull << idx) : 0ull;
    int p = high_pivot ? 63 - __builtin_clzll(r) : ctz(r);
    for (size_t i = 0; i < vec.size(); ++i)
        if ((vec[i] >> p) & 1) {
            vec[i] ^= r;
            comb[i] ^= cm;
        }
    vec.push_back(r);
    comb.push_back(cm);
    piv.push_back(p);
    return true;
}

int gf2_rank(std::vector<uint64_t> rows) {
    Echelon e;
    for (uint64_t r : rows) e.insert(r);
    return e.dim();
}

// ---------------------------------------------------------------------------
// gate table
// ---------------------------------------------------------------------------
void apply_gate(Row &w, const Gate &g) {
    const uint64_t A = 1ull << g.a;
    switch (g.kind) {
        case SD_GATE_H: {
            int xa = (w.x & A) != 0, za = (w.z & A) != 0;
            w.r ^= xa & za;
            w.x = (w.x & ~A) | (za ? A : 0);
            w.z = (w.z & ~A) | (xa ? A : 0);
            break;
        }
        case SD_GATE_S: {
            int xa = (w.x & A) != 0, za = (w.z & A) != 0;
            w.r ^= xa & za;
            if (xa) w.z ^= A;
            break;
        }
        case SD_GATE_CNOT: {
            const uint64_t T = 1ull << g.b;
            int xc = (w.x & A) != 0, zc = (w.z & A) != 0;
            int xt = (w.x & T) != 0, zt = (w.z & T) != 0;
            w.r ^= xc & zt & (xt ^ zc ^ 1);
            if (xc) w.x ^= T;
            if (zt) w.z ^= A;
            break;
        }
        case SD_GATE_CZ: {
            const uint64_t T = 1ull << g.b;
            int xc = (w.x & A) != 0, zc = (w.z & A) != 0;
            int xt = (w.x & T) != 0, zt = (w.z & T) != 0;
            w.r ^= xc & xt & (zt ^ zc);
            if (xc) w.z ^= T;
            if (xt) w.z ^= A;
            break;
        }
    }
}

// ---------------------------------------------------------------------------
// appendix algorithm (independent rows)
// ---------------------------------------------------------------------------
static inline int colbit(const Row &r, const std::vector<int> &act, int c) {
    const int na = (int)act.size();
    return c < na ? (int)((r.x >> act[c]) & 1) : (int)((r.z >> act[c - na]) & 1);
}

std::vector<int64_t> independent_rows(const std::vector<Row> &in,
                                      const std::vector<int> &act) {
    const int N = (int)in.size();
    const int na = (int)act.size();
    std::vector<Row> t(in);
    std::vector<int64_t> id(N);
    for (int i = 0; i < N; ++i) id[i] = i;
    int ir = 0, ic = 0;
    while (ir < N && ic < 2 * na) {
        if (!colbit(t[ir], act, ic)) {
            int j = ir + 1;
            while (j < N && !colbit(t[j], act, ic)) ++j;
            if (j == N) {
                ++ic;
                continue;
            }
            std::swap(t[ir], t[j]);
            std::swap(id[ir], id[j]);
        }
        for (int k = ir + 1; k < N; ++k)
            if (colbit(t[k], act, ic)) {
                t[k].x ^= t[ir].x;
                t[k].z ^= t[ir].z;
            }
        ++ir;
        ++ic;
    }
    uint64_t actmask = 0;
    for (int q : act) actmask |= 1ull << q;
    std::vector<int64_t> out;
    for (int i = 0; i < N; ++i)
        if ((t[i].x | t[i].z) & actmask) out.push_back(id[i]);
    return out;
}

// ---------------------------------------------------------------------------
// steps (i)-(iv)
// ---------------------------------------------------------------------------
static int xrank(const std::vector<Row> &tab) {
    std::vector<uint64_t> r;
    for (auto &w : tab) r.push_back(w.x);
    return gf2_rank(r);
}

SynthResult synthesize(int n, const std::vector<Row> &terms, const SynthOptions &opt) {
    SynthResult res;
    std::vector<Gate> &gates = res.gates;
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);

    // tableau of all terms, used to follow every gate
    std::vector<Row> full(terms);
    for (auto &w : full) w.r = 0;
    auto emit = [&](Gate g, std::vector<Row> *tab) {
        gates.push_back(g);
        for (auto &w : full) apply_gate(w, g);
        if (tab)
            for (auto &w : *tab) apply_gate(w, g);
    };

    // skip-rule pre-pass
    uint64_t hasX = 0, hasY = 0, hasZ = 0;
    for (auto &w : terms) {
        hasX |= w.x & ~w.z;
        hasY |= w.x & w.z;
        hasZ |= ~w.x & w.z;
    }
    std::vector<int> act;
    for (int q = 0; q < n; ++q) {
        const uint64_t Q = 1ull << q;
        bool used = (hasX | hasY | hasZ) & Q;
        if (!used) continue;
        if (opt.skip_rule) {
            bool zonly = !((hasX | hasY) & Q);
            bool xonly = !((hasZ | hasY) & Q);
            if (zonly) continue;
            if (xonly) {
                emit({SD_GATE_H, q, -1}, nullptr);
                ++res.n_h_first;
                continue;
            }
        }
        act.push_back(q);
    }
    uint64_t actmask = 0;
    for (int q : act) actmask |= 1ull << q;

    // restricted tableau of the independent terms (zero padding is implicit)
    std::vector<Row> rest;
    for (auto &w : full) rest.push_back({w.x & actmask, w.z & actmask, 0});
    res.independent = independent_rows(rest, act);
    std::vector<Row> tab;
    for (int64_t k : res.independent) tab.push_back(rest[k]);
    std::vector<int64_t> rowid(res.independent);  // row identities through swaps
    const int r = (int)tab.size();

    // (i) maximise the rank of the X block with H, qubits from high to low
    if (opt.step_i) {
        for (int ai = (int)act.size() - 1; ai >= 0; --ai) {
            const int q = act[ai];
            const uint64_t Q = 1ull << q;
            int before = xrank(tab);
            std::vector<Row> trial(tab);
            for (auto &w : trial) {
                uint64_t xq = w.x & Q, zq = w.z & Q;
                w.x = (w.x & ~Q) | zq;
                w.z = (w.z & ~Q) | xq;
            }
            if (xrank(trial) > before) {
                emit({SD_GATE_H, q, -1}, &tab);
                ++res.n_h_first;
            }
        }
    }

    // (ii) clear the X block above the pivots with CNOT(p_i, j)
    std::vector<int> piv(r, -1);
    uint64_t pivoted = 0;
    int last_control = -1;
    for (int i = 0; i < r; ++i) {
        int p = -1;
        const int ci = (i < (int)act.size()) ? act[i] : -1;
        auto find_row = [&](int col) {
            for (int j = i; j < r; ++j)
                if ((tab[j].x >> col) & 1) return j;
            return -1;
        };
        if (ci >= 0 && !((pivoted >> ci) & 1)) {
            int j = find_row(ci);
            if (j >= 0) {
                std::swap(tab[i], tab[j]);
                std::swap(rowid[i], rowid[j]);
                p = ci;
            }
        }
        if (p < 0) {
            for (int q : act) {
                if ((pivoted >> q) & 1) continue;
                int j = find_row(q);
                if (j >= 0) {
                    std::swap(tab[i], tab[j]);
                    std::swap(rowid[i], rowid[j]);
                    p = q;
                    break;
                }
            }
        }
        if (p < 0) {
            res.error = "X block rank below tableau rank after step (i)";
            return res;
        }
        piv[i] = p;
        pivoted |= 1ull << p;
        for (int q : act) {
            if (q == p || ((pivoted >> q) & 1)) continue;
            if ((tab[i].x >> q) & 1) {
                emit({SD_GATE_CNOT, p, q}, &tab);
                if (p != last_control) {
                    ++res.n_cnot_controls;
                    last_control = p;
                }
            }
        }
    }

    // (iii) clear the Z block with CZ(p_i, j) and S(p_i)
    for (int i = 0; i < r; ++i) {
        const int p = piv[i];
        for (int q : act) {
            if (q == p) continue;
            if ((tab[i].z >> q) & 1) {
                emit({SD_GATE_CZ, p, q}, &tab);
                res.n_diag = 1;
            }
        }
        if ((tab[i].z >> p) & 1) {
            emit({SD_GATE_S, p, -1}, &tab);
            res.n_diag = 1;
        }
    }

    // (iv) turn X components into Z components with H
    uint64_t xcols = 0;
    for (auto &w : tab) xcols |= w.x;
    for (int q : act)
        if ((xcols >> q) & 1) {
            emit({SD_GATE_H, q, -1}, &tab);
            ++res.n_h_last;
        }

    // every term of the group must now be a signed Z-string
    res.zmask.resize(full.size());
    res.sign.resize(full.size());
    for (size_t k = 0; k < full.size(); ++k) {
        if (full[k].x & all) {
            res.error = "term not diagonalised by the synthesised Clifford";
            return res;
        }
        res.zmask[k] = full[k].z;
        res.sign[k] = (int8_t)full[k].r;
    }
    res.ok = true;
    return res;
}

}  // namespace sd
