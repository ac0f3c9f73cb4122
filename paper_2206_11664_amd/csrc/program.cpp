// Compilation of the commuting groups into device tile programs.
//
// The unitary of a commuting group, exp(-i tau sum_k c_k P_k), maps a basis
// state |x> only into x ^ span{x_k} (every P_k flips the bits of its X part).
// So it acts independently on every coset of the X span V of the group.  A
// tile is one such coset, widened by the lowest address bits so that every
// global access covers whole cache lines; it is staged on chip, transformed,
// and written back: one HBM read and one write per group application.
//
// Inside a tile, with coordinates tau relative to a basis b_0..b_{D-1} of the
// tile space (the first rho = dim V vectors span V), a term acts as
//     P_k = i^{|x_k & z_k| - |alpha_k & omega_k|} (-1)^{z_k . x_T} X^alpha_k Z^omega_k
// (alpha_k: coordinates of x_k; omega_k,i = z_k . b_i; x_T: the tile's base
// address).  The paper's steps (i)-(iv) are run on this D-qubit tableau.
// Because the X-span basis is made of terms' own X parts, the independent
// set is those basis terms, step (i) finds full X rank (no H), step (ii) finds
// an identity X block (no CNOT): the CNOT network of the physical-coordinate
// circuit is exactly the change to tile coordinates, which costs nothing at
// run time since it only changes which address lands in which on-chip slot.
// Step (iii) gives the CZ/S layer and step (iv) H on all rho coordinates.
//
// A group whose tile would exceed the on-chip limit is split into commuting
// sub-groups (any split is exact: the terms commute), each with its own tile.
#include <algorithm>
#include <cmath>

#include "device_types.h"
#include "sd_internal.h"

namespace sd {

namespace {

// coordinates of v in basis b (v must lie in span b); result bit i <-> b[i]
struct Coords {
    Echelon e;
    explicit Coords(const std::vector<uint64_t> &b) {
        for (uint64_t v : b) e.insert(v);
    }
    bool solve(uint64_t v, uint32_t *out) const {
        uint64_t used = 0;
        uint64_t r = e.reduce(v, &used);
        if (r) return false;
        *out = (uint32_t)used;
        return true;
    }
};

// ---------------------------------------------------------------------------
// Canonical form of the CZ/S layer.
//
// The layer multiplies tile coordinate y (span part) by i^{q(y)} with
// q(y) = sum_i y_i popcount(B_i & y) mod 4: S on the diagonal, CZ off it.
// q is a Z4-valued quadratic form, q(x ^ y) = q(x) + q(y) + 2 beta(x, y) with
// the GF(2) bilinear form beta(x, y) = x^T B y.  A change of the span basis
// (new coordinates y' with y = M y') is free at run time: it only relabels
// on-chip slots, like the CNOT network.  In the new basis
//     q(M y') = sum_a d_a y'_a + 2 sum_{a<b} beta(f_a, f_b) y'_a y'_b   (mod 4)
// with f_a the columns of M and d_a = q(f_a) in Z4.  Symplectic Gram-Schmidt
// over GF(2) splits the span into mutually orthogonal odd vectors
// (beta(v, v) = 1), hyperbolic pairs (beta(v, x) = 1, both even) and a
// radical; odd vectors are then traded for pairs until at most one is left.
// The chunk layout keeps the two vectors of every pair in different register
// chunks and puts the odd vector first in the last chunk.  The kernel needs
// no per-amplitude phase multiply then: the one S (d_a odd) becomes a
// butterfly with an i twiddle in the Lambda round, and every Z (d_a >= 2) and
// cross-chunk CZ becomes a relabelling of butterfly outputs (see the
// register-round kernel).
namespace {

int bil(const std::vector<uint32_t> &B, uint32_t x, uint32_t y) {
    int t = 0;
    for (uint32_t v = x; v; v &= v - 1) t ^= popc(B[ctz(v)] & y) & 1;
    return t;
}

int qform(const std::vector<uint32_t> &B, uint32_t x) {
    int q = 0;
    for (uint32_t v = x; v; v &= v - 1) q += popc(B[ctz(v)] & x);
    return q & 3;
}

// new span basis f (old coordinates, in final order) and chunk sizes
void canonical_basis(const std::vector<uint32_t> &B, int rho, std::vector<uint32_t> *f,
                     std::vector<int> *chunks) {
    std::vector<uint32_t> W, dg, rad;
    std::vector<std::pair<uint32_t, uint32_t>> pairs;
    for (int i = 0; i < rho; ++i) W.push_back(1u << i);
    while (!W.empty()) {
        size_t odd = W.size();
        for (size_t i = 0; i < W.size(); ++i)
            if (bil(B, W[i], W[i])) {
                odd = i;
                break;
            }
        if (odd < W.size()) {
            const uint32_t e = W[odd];
            W.erase(W.begin() + (long)odd);
            for (uint32_t &w : W)
                if (bil(B, w, e)) w ^= e;
            dg.push_back(e);
            continue;
        }
        size_t pi = W.size(), pj = W.size();
        for (size_t i = 0; i < W.size() && pi == W.size(); ++i)
            for (size_t j = i + 1; j < W.size(); ++j)
                if (bil(B, W[i], W[j])) {
                    pi = i;
                    pj = j;
                    break;
                }
        if (pi == W.size()) {
            rad = W;
            break;
        }
        const uint32_t v = W[pi], x = W[pj];
        W.erase(W.begin() + (long)pj);
        W.erase(W.begin() + (long)pi);
        for (uint32_t &w : W) {
            const int bx = bil(B, w, x), bv = bil(B, w, v);
            if (bx) w ^= v;
            if (bv) w ^= x;
        }
        pairs.push_back({v, x});
    }
    // At most one odd vector: three mutually orthogonal odd vectors e1, e2,
    // e3 become the hyperbolic pair (e1+e2, e1+e3) and the odd e1+e2+e3
    // (orthogonal to the pair); two become the odd e2 and the even e1+e2,
    // whose only nonzero product is with e2 (its "partner").
    while (dg.size() >= 3) {
        const uint32_t e3 = dg.back();
        dg.pop_back();
        const uint32_t e2 = dg.back();
        dg.pop_back();
        const uint32_t e1 = dg.back();
        dg.pop_back();
        pairs.push_back({e1 ^ e2, e1 ^ e3});
        dg.push_back(e1 ^ e2 ^ e3);
    }
    uint32_t odd = 0, partner = 0;
    if (dg.size() == 2) {
        odd = dg[1];
        partner = dg[0] ^ dg[1];
    } else if (dg.size() == 1) {
        odd = dg[0];
    }
    // even vectors: the partner, first vectors of the pairs, the radical,
    // second vectors of the pairs; packed greedily into chunks of up to
    // kRegBits mutually orthogonal vectors
    std::vector<uint32_t> ev;
    if (partner) ev.push_back(partner);
    for (auto &pr : pairs) ev.push_back(pr.first);
    ev.insert(ev.end(), rad.begin(), rad.end());
    for (auto &pr : pairs) ev.push_back(pr.second);
    std::vector<std::vector<uint32_t>> ch;
    for (uint32_t u : ev) {
        bool fits = !ch.empty() && (int)ch.back().size() < kRegBits;
        if (fits)
            for (uint32_t w : ch.back())
                if (bil(B, u, w)) fits = false;
        if (!fits) ch.push_back({});
        ch.back().push_back(u);
    }
    // the odd vector opens the last chunk (the Lambda round): its S is the
    // only i twiddle of the pass
    if (odd) {
        bool fits = !ch.empty() && (int)ch.back().size() < kRegBits;
        if (fits)
            for (uint32_t w : ch.back())
                if (bil(B, odd, w)) fits = false;
        if (fits)
            ch.back().insert(ch.back().begin(), odd);
        else
            ch.push_back({odd});
    }
    f->clear();
    chunks->clear();
    for (auto &c : ch) {
        f->insert(f->end(), c.begin(), c.end());
        chunks->push_back((int)c.size());
    }
}

}  // namespace

// Re-express the pass in the canonical span basis: slots, Lambda masks, the
// CZ/S form and the exported basis all change together.
sd_status canonicalize(PassHost *ps) {
    PassHost &p = *ps;
    const int rho = p.rho;
    p.zq = 0;
    p.chunk.clear();
    if (rho == 0) return SD_OK;
    std::vector<uint32_t> f;
    canonical_basis(p.B, rho, &f, &p.chunk);
    if ((int)f.size() != rho) return fail(SD_ERR_INTERNAL, "canonical basis size");
    std::vector<uint64_t> f64(f.begin(), f.end());
    Coords cf(f64);
    const uint32_t rmask = (rho >= 32) ? ~0u : ((1u << rho) - 1);
    auto to_new = [&](uint32_t y, uint32_t *out) -> bool {
        uint32_t yn = 0;
        if (!cf.solve(y & rmask, &yn)) return false;
        *out = (y & ~rmask) | yn;
        return true;
    };
    std::vector<uint32_t> Bn(rho, 0u);
    for (int a = 0; a < rho; ++a) {
        const int d = qform(p.B, f[a]);
        if (d & 1) Bn[a] |= 1u << a;
        if (d & 2) p.zq |= 1u << a;
        for (int b = 0; b < rho; ++b)
            if (b != a && bil(p.B, f[a], f[b])) Bn[a] |= 1u << b;
    }
    // every chunk must be free of CZ inside it
    int off = 0;
    for (int s : p.chunk) {
        const uint32_t cm = ((1u << s) - 1) << off;
        for (int a = off; a < off + s; ++a)
            if (Bn[a] & cm & ~(1u << a)) return fail(SD_ERR_INTERNAL, "CZ inside a register chunk");
        off += s;
    }
    for (uint32_t &z : p.zeta)
        if (!to_new(z, &z)) return fail(SD_ERR_INTERNAL, "Lambda mask outside the tile");
    for (uint32_t &m : p.mr)
        if (!to_new(m, &m)) return fail(SD_ERR_INTERNAL, "pivot coordinates outside the tile");
    std::vector<uint64_t> nb(p.basis);
    for (int a = 0; a < rho; ++a) {
        uint64_t v = 0;
        for (uint32_t w = f[a]; w; w &= w - 1) v ^= p.basis[ctz(w)];
        nb[a] = v;
    }
    p.basis = nb;
    p.B = Bn;
    return SD_OK;
}

// Register-round schedule for the on-chip transform of a tile with D
// coordinates (span coordinates 0..rho-1, spectators rho..D-1).  A thread
// holds 2^kRegBits amplitudes: the kRegBits tile coordinates of the current
// round vary over them, the remaining coordinates are the thread index (lowest
// first, so consecutive lanes touch consecutive on-chip slots).  Chunk r takes
// the next chunk[r] span coordinates; a short chunk is filled with the highest
// other coordinates, which are carried without butterflies.  Lambda is
// applied in the round of the last chunk, between the two transforms.
sd_status plan_rounds(PassHost *ps) {
    PassHost &p = *ps;
    const int D = p.D, rho = p.rho;
    p.nr = 0;
    p.full_rounds = true;
    for (int r = 0; r < 4; ++r) p.bmask[r] = p.iflag[r] = p.dflag[r] = p.later[r] = 0;
    const int RB = kRegBits;
    if (D < 2 * RB) {  // tiny tile: handled by the generic kernel only
        p.lam_round = 0;
    } else {
        auto fill = [&](int r, std::vector<int> bits, uint32_t bm) {
            for (int b = D - 1; (int)bits.size() < RB && b >= 0; --b)
                if (std::find(bits.begin(), bits.end(), b) == bits.end()) bits.push_back(b);
            for (int i = 0; i < RB; ++i) p.reg[r][i] = (uint8_t)bits[i];
            p.bmask[r] = bm;
        };
        if (rho == 0) {
            fill(0, {}, 0u);
            p.lam_round = 0;
        } else {
            p.nr = (int)p.chunk.size();
            if (p.nr > 4) return fail(SD_ERR_INTERNAL, "too many register rounds");
            int off = 0;
            for (int r = 0; r < p.nr; ++r) {
                std::vector<int> bits;
                for (int b = off; b < off + p.chunk[r]; ++b) bits.push_back(b);
                fill(r, bits, (1u << bits.size()) - 1);
                for (int l = 0; l < p.chunk[r]; ++l) {
                    const int a = off + l;
                    if ((p.B[a] >> a) & 1) p.iflag[r] |= 1u << l;
                    if ((p.zq >> a) & 1) p.dflag[r] |= 1u << l;
                }
                off += p.chunk[r];
                for (int b = off; b < rho; ++b) p.later[r] |= 1u << b;
            }
            p.lam_round = p.nr - 1;
            p.full_rounds = true;
            for (int r = 0; r < p.lam_round; ++r)
                if (p.chunk[r] != RB) p.full_rounds = false;
            // the kernel twiddles only register slot 0 of the Lambda round
            for (int r = 0; r < p.nr; ++r)
                if (p.iflag[r] & ~(r == p.lam_round ? 1u : 0u))
                    return fail(SD_ERR_INTERNAL, "S outside slot 0 of the Lambda round");
        }
    }
    // sort the Lambda terms by their pattern on the Lambda round's registers
    const int L = p.lam_round;
    auto pattern = [&](uint32_t z) {
        uint32_t w = 0;
        if (D >= 2 * RB)
            for (int i = 0; i < RB; ++i) w |= ((z >> p.reg[L][i]) & 1u) << i;
        return w;
    };
    const size_t m = p.zeta.size();
    std::vector<size_t> idx(m);
    for (size_t i = 0; i < m; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](size_t a, size_t b) { return pattern(p.zeta[a]) < pattern(p.zeta[b]); });
    std::vector<int64_t> t2;
    std::vector<uint32_t> z2;
    std::vector<uint64_t> zt2;
    std::vector<double> c2;
    for (size_t i : idx) {
        t2.push_back(p.terms[i]);
        z2.push_back(p.zeta[i]);
        zt2.push_back(p.ztile[i]);
        c2.push_back(p.coef[i]);
    }
    p.terms.swap(t2);
    p.zeta.swap(z2);
    p.ztile.swap(zt2);
    p.coef.swap(c2);
    p.bucket.assign(33, 0);
    for (size_t i = 0; i < m; ++i) p.bucket[pattern(p.zeta[i]) + 1]++;
    for (int w = 0; w < 32; ++w) p.bucket[w + 1] += p.bucket[w];
    p.coef_abs_sum = 0;
    for (double c : p.coef) p.coef_abs_sum += std::fabs(c);
    return SD_OK;
}

sd_status build_pass(int n, const std::vector<Term> &T, int32_t group,
                     const std::vector<int64_t> &ids, int D_target, int c_req,
                     PassHost *ps) {
    PassHost &p = *ps;
    p.group = group;
    p.terms = ids;
    const int c = std::min(c_req, n);
    // X-span basis from the terms' own X parts, in term order
    Echelon vx;
    std::vector<uint64_t> vbasis;
    std::vector<int64_t> gen;  // generator term per basis vector
    for (int64_t k : ids)
        if (T[k].x && vx.insert(T[k].x)) {
            vbasis.push_back(T[k].x);
            gen.push_back(k);
        }
    p.rho = (int)vbasis.size();
    // tile space: X span + low bits (coalescing) + more low bits up to D_target
    Echelon w = vx;
    std::vector<uint64_t> spect;
    for (int q = 0; q < n; ++q) {
        if (q >= c && w.dim() >= D_target) break;
        uint64_t e = 1ull << q;
        if (w.insert(e)) spect.push_back(e);
    }
    p.basis = vbasis;
    p.basis.insert(p.basis.end(), spect.begin(), spect.end());
    p.D = (int)p.basis.size();
    if (p.D > 31) return fail(SD_ERR_INTERNAL, "tile dimension above 31");

    // pivots: low bits 0..c-1 first (unit vectors), then for every further
    // vector its highest remaining bit.  High pivots leave the low address bits
    // to the tile index, so tiles with consecutive indices (processed at the
    // same time by neighbouring blocks) touch neighbouring cache lines.
    Echelon piv;
    piv.high_pivot = true;
    for (int q = 0; q < c; ++q) piv.insert(1ull << q);
    for (uint64_t b : p.basis) piv.insert(b);
    if (piv.dim() != p.D) return fail(SD_ERR_INTERNAL, "tile basis rank mismatch");
    std::vector<int> order(p.D);
    for (int i = 0; i < p.D; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return piv.piv[a] < piv.piv[b]; });
    uint64_t pivmask = 0;
    p.u.clear();
    p.upiv.clear();
    for (int i : order) {
        p.u.push_back(piv.vec[i]);
        p.upiv.push_back(piv.piv[i]);
        pivmask |= 1ull << piv.piv[i];
    }
    p.c = c;
    for (int q = 0; q < c; ++q)
        if (p.upiv[q] != q || p.u[q] != (1ull << q))
            return fail(SD_ERR_INTERNAL, "low pivots are not unit vectors");
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    p.free_mask = all & ~pivmask;

    Coords co(p.basis);
    p.mr.resize(p.D);
    for (int i = 0; i < p.D; ++i)
        if (!co.solve(p.u[i], &p.mr[i]))
            return fail(SD_ERR_INTERNAL, "echelon vector outside the tile space");

    // virtual tableau: generator rows first, then the group's terms in order
    std::vector<Row> vrows;
    std::vector<int64_t> vterm;
    auto vrow = [&](int64_t k, Row *out, int *e) -> bool {
        uint32_t alpha = 0;
        if (!co.solve(T[k].x, &alpha)) return false;
        uint32_t omega = 0;
        for (int i = 0; i < p.D; ++i) omega |= (uint32_t)parity(T[k].z & p.basis[i]) << i;
        *e = ((popc(T[k].x & T[k].z) - popc((uint64_t)(alpha & omega))) % 4 + 4) % 4;
        *out = {alpha, omega, 0};
        return true;
    };
    std::vector<int> ephase;
    for (int64_t k : gen) {
        Row r;
        int e;
        if (!vrow(k, &r, &e)) return fail(SD_ERR_INTERNAL, "generator outside tile space");
        vrows.push_back(r);
        vterm.push_back(k);
        ephase.push_back(e);
    }
    for (int64_t k : ids) {
        if (std::find(gen.begin(), gen.end(), k) != gen.end()) continue;
        Row r;
        int e;
        if (!vrow(k, &r, &e)) return fail(SD_ERR_INTERNAL, "term outside tile space");
        vrows.push_back(r);
        vterm.push_back(k);
        ephase.push_back(e);
    }
    for (int e : ephase)
        if (e != 0 && e != 2) return fail(SD_ERR_INTERNAL, "non-Hermitian tile phase");

    SynthOptions so;
    so.skip_rule = true;
    so.step_i = true;
    SynthResult sr = synthesize(p.D, vrows, so);
    if (!sr.ok) return fail(SD_ERR_INTERNAL, "tile synthesis: " + sr.error);
    // expected shape: CZ/S on coordinates < rho, then H on every coordinate < rho
    // (X-only coordinates may get their H first; it commutes with the CZ/S layer
    // because such coordinates never appear in it).
    p.B.assign(p.rho, 0u);
    uint32_t hset = 0;
    for (const Gate &g : sr.gates) {
        if (g.kind == SD_GATE_CNOT) return fail(SD_ERR_INTERNAL, "tile synthesis emitted CNOT");
        if (g.a >= p.rho || (g.b >= p.rho))
            return fail(SD_ERR_INTERNAL, "tile gate outside the X span");
        if (g.kind == SD_GATE_H) {
            if ((hset >> g.a) & 1) return fail(SD_ERR_INTERNAL, "repeated tile H");
            hset |= 1u << g.a;
        } else {
            if ((hset >> g.a) & 1 || (g.b >= 0 && ((hset >> g.b) & 1)))
                return fail(SD_ERR_INTERNAL, "CZ/S after H in tile circuit");
            if (g.kind == SD_GATE_S) {
                p.B[g.a] ^= 1u << g.a;
            } else {
                p.B[g.a] ^= 1u << g.b;
                p.B[g.b] ^= 1u << g.a;
            }
        }
    }
    const uint32_t rmask = (p.rho >= 32) ? ~0u : ((1u << p.rho) - 1);
    if (hset != rmask) return fail(SD_ERR_INTERNAL, "tile H layer does not cover the X span");


    // Lambda terms in the order of the group (vterm order is fine: they commute)
    p.zeta.clear();
    p.ztile.clear();
    p.coef.clear();
    p.terms = vterm;
    for (size_t i = 0; i < vterm.size(); ++i) {
        const int64_t k = vterm[i];
        p.zeta.push_back((uint32_t)sr.zmask[i]);
        p.ztile.push_back(T[k].z);
        double s = (sr.sign[i] ? -1.0 : 1.0) * (ephase[i] == 2 ? -1.0 : 1.0);
        p.coef.push_back(T[k].c * s);
    }
    sd_status st = canonicalize(&p);
    if (st != SD_OK) return st;
    return plan_rounds(&p);
}

}  // namespace

sd_status compile_program(int n, const std::vector<Term> &T,
                          const std::vector<std::vector<int64_t>> &groups,
                          int D_max, int c, Program *out) {
    Program &P = *out;
    P.D_max = D_max;
    P.c = c;
    P.passes.clear();
    P.group_first.assign(1, 0);
    const int cc = std::min(c, n);
    const int Dcap = std::min(D_max, n);
    for (size_t g = 0; g < groups.size(); ++g) {
        // Split into sub-groups whose tile space (X span + low bits) fits.
        // Sub-groups are grown one at a time: first every remaining term whose
        // X part already lies in the span joins (no growth), then the term
        // whose addition lets the most remaining terms in for free is added.
        std::vector<std::vector<int64_t>> subs;
        std::vector<int64_t> rest(groups[g].begin(), groups[g].end());
        while (!rest.empty()) {
            Echelon span;
            for (int q = 0; q < cc; ++q) span.insert(1ull << q);
            std::vector<int64_t> cur;
            while (true) {
                std::vector<int64_t> keep;
                for (int64_t k : rest) {
                    if ((int)cur.size() < kMaxPassTerms && span.contains(T[k].x))
                        cur.push_back(k);
                    else
                        keep.push_back(k);
                }
                rest.swap(keep);
                if (rest.empty() || span.dim() >= Dcap || (int)cur.size() >= kMaxPassTerms) break;
                size_t best = 0;
                int best_score = -1;
                for (size_t a = 0; a < rest.size(); ++a) {
                    Echelon t2 = span;
                    t2.insert(T[rest[a]].x);
                    int score = 0;
                    for (int64_t k : rest)
                        if (t2.contains(T[k].x)) ++score;
                    if (score > best_score) {
                        best_score = score;
                        best = a;
                    }
                }
                span.insert(T[rest[best]].x);
                cur.push_back(rest[best]);
                rest.erase(rest.begin() + (long)best);
            }
            subs.push_back(std::move(cur));
        }
        for (auto &s : subs) {
            PassHost ps;
            sd_status st = build_pass(n, T, (int32_t)g, s, Dcap, cc, &ps);
            if (st != SD_OK) return st;
            P.passes.push_back(std::move(ps));
        }
        P.group_first.push_back((int32_t)P.passes.size());
    }
    return SD_OK;
}

}  // namespace sd
