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
#include <atomic>
#include <string>
#include <thread>
#include <functional>
#include <unordered_map>
#include <array>
#include <cmath>
#include <cstdint>

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
// lowspan: span parts (old coordinates) of the tile coordinates of the
// lowest address bits; the chunk of round 0, which moves the tile between HBM
// and registers, is built from basis vectors none of them depends on (see
// canonicalize) whenever there are such vectors.
// low0: span parts of the combinations of those low bits that have no
// spectator part; round 0 can take the low bits as lanes (direct I/O) only
// if its chunk meets their span in zero alone.
// min0: the fewest span coordinates round 0's chunk may have (its register
// slots can only be filled with spectator coordinates).
void canonical_basis(const std::vector<uint32_t> &B, int rho, const std::vector<uint32_t> &lowspan,
                     const std::vector<uint32_t> &low0, int min0, std::vector<uint32_t> *f,
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
    // second vectors of the pairs
    std::vector<uint32_t> ev;
    if (partner) ev.push_back(partner);
    for (auto &pr : pairs) ev.push_back(pr.first);
    ev.insert(ev.end(), rad.begin(), rad.end());
    for (auto &pr : pairs) ev.push_back(pr.second);
    // basis vectors that some low address bit depends on ("dirty")
    std::vector<uint32_t> all(ev);
    if (odd) all.push_back(odd);
    std::vector<char> dirty(all.size(), 0);
    {
        std::vector<uint64_t> a64(all.begin(), all.end());
        Coords ca(a64);
        for (uint32_t v : lowspan) {
            uint32_t co = 0;
            if (!v || !ca.solve(v, &co)) continue;
            for (size_t i = 0; i < all.size(); ++i)
                if ((co >> i) & 1) dirty[i] = 1;
        }
    }
    // Assign the vectors to K chunks of at most kChunkBits each; vectors of
    // one chunk with a nonzero product (a CZ inside the round) are allowed
    // among at most kRegBits of them, which take the register slots (there
    // the CZ is a sign per register pattern); the odd vector goes first in
    // the last chunk (the Lambda round: its S is the pass's only i twiddle).  Round 0's chunk decides
    // how the tile moves between HBM and registers: made of clean vectors
    // only, the low address bits are plain lanes of round 0; meeting low0 in
    // zero alone, they are lanes with a sign correction (shift0); otherwise
    // the pass is staged through LDS.  The fewest chunks win, then the
    // cheaper I/O; the chunks before the last are filled to kChunkBits when
    // possible (their rounds then run the straight-line code).  The products form a matching
    // (hyperbolic pairs, the odd vector and its partner), so a depth-first
    // search over at most 13 vectors is quick.
    const int nv = (int)all.size();
    const int io = odd ? nv - 1 : -1;
    std::vector<uint32_t> conf(nv, 0);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j)
            if (i != j && bil(B, all[i], all[j])) conf[i] |= 1u << j;
    // search order: the odd vector, then pairs next to each other, dirty first
    std::vector<int> order;
    if (io >= 0) order.push_back(io);
    {
        std::vector<char> seen(nv, 0);
        if (io >= 0) seen[io] = 1;
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < nv; ++i) {
                if (seen[i] || (pass == 0) != (dirty[i] != 0)) continue;
                seen[i] = 1;
                order.push_back(i);
                for (int j = 0; j < nv; ++j)
                    if (!seen[j] && ((conf[i] >> j) & 1)) {
                        seen[j] = 1;
                        order.push_back(j);
                    }
            }
    }
    std::vector<int> asg(nv, -1);
    // mode 0: round 0's chunk clean; 1: it meets low0 in zero; 2: anything
    auto meets_low0 = [&](uint32_t mem0) {
        Echelon e;
        for (uint32_t u : low0) e.insert(u);
        for (int i = 0; i < nv; ++i)
            if (((mem0 >> i) & 1) && !e.insert(all[i])) return true;
        return false;
    };
    auto search = [&](int K, int mode, bool inner_cz, const std::vector<int> &cap) -> bool {
        std::vector<int> size(K, 0);
        std::vector<uint32_t> mem(K, 0);
        int budget = 200000;  // node limit (never reached at these sizes)
        std::function<bool(int)> rec = [&](int t) -> bool {
            if (--budget < 0) return false;
            if (t == nv) {
                for (int r = 0; r < K; ++r)
                    if (size[r] == 0) return false;
                return size[0] >= min0 || K == 1;
            }
            const int v = order[t];
            int left = nv - t, room = 0;
            for (int r = 0; r < K; ++r) room += cap[r] - size[r];
            if (room < left) return false;
            for (int r = 0; r < K; ++r) {
                if (v == io && r != K - 1) continue;
                if (size[r] >= cap[r]) continue;
                if (mem[r] & conf[v]) {
                    if (!inner_cz) continue;
                    uint32_t inv = 0;
                    const uint32_t mm = mem[r] | (1u << v);
                    for (int i = 0; i < nv; ++i)
                        if (((mm >> i) & 1) && (conf[i] & mm)) inv |= 1u << i;
                    // (the odd vector takes register slot 0 of the last chunk)
                    if (io >= 0 && r == K - 1) inv |= 1u << io;
                    if (__builtin_popcount(inv) > kRegBits) continue;
                }
                if (mode == 0 && r == 0 && dirty[v]) continue;
                if (mode == 1 && r == 0 && meets_low0(mem[0] | (1u << v))) continue;
                size[r]++;
                mem[r] |= 1u << v;
                asg[v] = r;
                if (rec(t + 1)) return true;
                size[r]--;
                mem[r] &= ~(1u << v);
                asg[v] = -1;
            }
            return false;
        };
        return rec(0);
    };
    std::vector<std::vector<uint32_t>> ch;
    int bestK = 0;
    const int kmin = std::max(1, (nv + kChunkBits - 1) / kChunkBits);
    // Order of preference at a chunk count: clean round 0 without a CZ
    // inside a chunk (no sign work), clean with it (a sign mask per such
    // round), shifted round 0 (per-thread sign) without and with, staged.
    for (int K = kmin; K <= 4 && !bestK; ++K) {
        for (int step = 0; step < 6 && !bestK; ++step) {
            const int mode = step / 2;
            const bool inner_cz = step & 1;
            // (a single round is Lambda's: no sign correction there, only the
            // layout, so "meets low0 in zero" suffices for it as well)
            // first with the chunks before the last full, then any sizes
            std::vector<int> exact(K, kChunkBits);
            exact[K - 1] = nv - kChunkBits * (K - 1);
            std::vector<int> loose(K, kChunkBits);
            if (exact[K - 1] >= 1 && search(K, mode, inner_cz, exact)) bestK = K;
            else if (search(K, mode, inner_cz, loose)) bestK = K;
        }
    }
    if (!bestK) {
        // (cannot happen for rho <= 4 kChunkBits: a matching splits over two chunks)
        ch.assign(1, {});
        for (int i = 0; i < nv; ++i) ch[0].push_back(all[i]);
    } else {
        // within a chunk: the odd vector, then the vectors with a partner in
        // the chunk (register slots), then the rest
        ch.assign(bestK, {});
        std::vector<uint32_t> cmem(bestK, 0);
        for (int i = 0; i < nv; ++i) cmem[asg[i]] |= 1u << i;
        if (io >= 0) ch[bestK - 1].push_back(all[io]);
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < nv; ++i) {
                if (i == io) continue;
                const bool inner = (conf[i] & cmem[asg[i]]) != 0;
                if (inner == (pass == 0)) ch[asg[i]].push_back(all[i]);
            }
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
    std::vector<uint32_t> lowspan;
    const uint32_t rmk = (rho >= 32) ? ~0u : ((1u << rho) - 1);
    for (int k = 0; k < p.c && k < 4 && k < (int)p.mr.size(); ++k) lowspan.push_back(p.mr[k] & rmk);
    std::vector<uint32_t> low0;
    {
        const int kk = (int)lowspan.size();
        for (uint32_t sset = 1; sset < (1u << kk); ++sset) {
            uint32_t x = 0;
            for (int k = 0; k < kk; ++k)
                if ((sset >> k) & 1) x ^= p.mr[k];
            if (!(x & ~rmk)) low0.push_back(x);
        }
    }
    // round 0's register slots not taken by its chunk hold spectators
    // (tiles below the register-round kernel's minimum run the generic kernel)
    const bool rounds = p.D >= 2 * kRegBits + kXBits;
    const int min0 = rounds ? std::min(rho, std::max(0, kRegBits - (p.D - rho))) : 0;
    canonical_basis(p.B, rho, lowspan, low0, min0, &f, &p.chunk);
    if (!p.chunk.empty() && p.chunk[0] < min0)
        return fail(SD_ERR_INTERNAL, "round 0 chunk too small for its register slots");
    if ((int)f.size() != rho) return fail(SD_ERR_INTERNAL, "canonical basis size");
    // Round 0 moves the tile between HBM and registers directly, with its
    // lanes running over the lowest address bits (coalescing); the chunk
    // search above has put in front the chunk that allows it (see
    // plan_rounds for the lanes).
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
    // a CZ inside a chunk only between its register slots (its first
    // kRegBits coordinates)
    int off = 0;
    for (int s : p.chunk) {
        const uint32_t cm = ((1u << s) - 1) << off;
        for (int a = off; a < off + s; ++a)
            if (a - off >= kRegBits && (Bn[a] & cm & ~(1u << a)))
                return fail(SD_ERR_INTERNAL, "CZ inside a chunk outside its register slots");
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
// coordinates (span coordinates 0..rho-1, spectators rho..D-1).
//
// A thread holds 2^kRegBits amplitudes.  Round r transforms chunk r (up to
// kChunkBits span coordinates): its first kRegBits coordinates sit in the
// register slots (their amplitudes of a thread differ in them); the next up
// to kXBits sit on lane bits 4 and 5, and after the register butterflies they
// are exchanged with register bits 2 and 3 (a lane permute inside the wave),
// so their butterflies run in registers too.  The other coordinates are lane
// bits.  A short chunk fills its register slots with other coordinates, which
// are carried without butterflies; they are never span coordinates of a later
// chunk (the CZs between a chunk and later chunks are applied as per-thread
// sign patterns, which needs the later coordinates among the lane bits).
// Lambda is applied in the round of the last chunk, between the two
// transforms.
//
// Lane bits: in round 0, which moves the tile between HBM and registers
// directly, lanes 0..c-1 are the tile coordinates of the c lowest address
// bits (consecutive lanes then read consecutive amplitudes).  That needs
// them free of components along the chunk's coordinates (the butterflies
// would see shifted inputs) and independent of the registers; when they are
// not, the pass is staged: the tile goes HBM -> LDS in pivot order (lanes over
// the low pivots, as coalesced), and round 0 reads it from LDS.  Other lanes
// are the lowest free unit coordinates.  Lanes 4 and 5 hold the
// exchanged coordinates, the rest follow lowest first.
//
// The on-chip slot of tile coordinate t is t ^ sum_j parity(t & swz[j]) << j
// for j = 0..3 (swz[0..2] only have bits >= 3 and swz[3] bits >= 4, so the
// map is invertible).  On
// gfx950 a 16-byte LDS write serves 8 lanes per 128-byte phase and a 16-byte
// read 16 lanes per 256-byte phase, so a layout is free of bank conflicts
// when the low 3 slot bits of lane vectors 0..2 and the low 4 slot bits of
// lane vectors 0..3 are independent.  The default masks fold the 4-bit
// groups of t >> 4; when they fail some layout, seeded random masks are
// tried.
sd_status plan_rounds(PassHost *ps) {
    PassHost &p = *ps;
    const int D = p.D, rho = p.rho;
    const int RB = kRegBits, TL = D - RB;
    p.nr = 0;
    p.full_rounds = true;
    for (int r = 0; r < 4; ++r) {
        p.bmask[r] = p.iflag[r] = p.dflag[r] = p.later[r] = p.czm[r] = 0;
        p.nx[r] = 0;
        p.lanes[r].clear();
        p.lanes_post[r].clear();
    }
    p.io_phys.clear();
    p.io_k = 0;
    p.staged = false;
    p.shift0 = false;
    if (D < 2 * RB + kXBits) {  // tiny tile: handled by the generic kernel only
        p.lam_round = 0;
        p.bucket.assign(33, 0);
        p.bucket[1] = (int32_t)p.zeta.size();
        for (int w = 1; w < 32; ++w) p.bucket[w + 1] = p.bucket[w];
        p.coef_abs_sum = 0;
        for (double c : p.coef) p.coef_abs_sum += std::fabs(c);
        return SD_OK;
    }
    std::vector<int> chunks = p.chunk;
    if (rho == 0) chunks = {0};
    p.nr = rho == 0 ? 0 : (int)chunks.size();
    const int nrounds = (int)chunks.size();
    if (nrounds > 4) return fail(SD_ERR_INTERNAL, "too many register rounds");
    int off = 0;
    for (int r = 0; r < nrounds; ++r) {
        const int s = chunks[r];
        for (int b = off + s; b < rho; ++b) p.later[r] |= 1u << b;
        std::vector<int> bits;
        for (int b = off; b < off + std::min(s, RB); ++b) bits.push_back(b);
        p.nx[r] = std::max(0, s - RB);
        for (int x = 0; x < p.nx[r]; ++x) p.xl[r][x] = (uint8_t)(off + RB + x);
        const uint32_t chunkm = s ? (((1u << s) - 1) << off) : 0u;
        // fillers: highest coordinates outside the chunk and the later chunks;
        // in round 0 first those that keep the low address bits independent
        std::vector<int> cand;
        for (int b = D - 1; b >= 0; --b)
            if (!((chunkm >> b) & 1) && !((p.later[r] >> b) & 1)) cand.push_back(b);
        if (r == 0) {
            Echelon e;
            for (int b = off; b < off + s; ++b) e.insert(1ull << b);
            for (int k = 0; k < p.c && k < D; ++k)
                if (!e.insert(p.mr[k])) break;
            for (int b : cand)
                if ((int)bits.size() < RB && e.insert(1ull << b)) bits.push_back(b);
        }
        for (int b : cand)
            if ((int)bits.size() < RB && std::find(bits.begin(), bits.end(), b) == bits.end())
                bits.push_back(b);
        if ((int)bits.size() < RB) return fail(SD_ERR_INTERNAL, "no filler coordinates left for a round");
        for (int i = 0; i < RB; ++i) p.reg[r][i] = (uint8_t)bits[i];
        p.bmask[r] = (1u << std::min(s, RB)) - 1;
        for (int l = 0; l < RB; ++l) p.regpost[r][l] = p.reg[r][l];
        for (int x = 0; x < p.nx[r]; ++x) p.regpost[r][2 + x] = p.xl[r][x];
        for (int l = 0; l < s; ++l) {
            const int a = off + l;
            if ((p.B[a] >> a) & 1) p.iflag[r] |= 1u << l;
            if ((p.zq >> a) & 1) p.dflag[r] |= 1u << l;
        }
        // CZ between register slots of the chunk: sign of register pattern g
        // is the parity of the CZ pairs that g has both bits of
        for (int l1 = 0; l1 < std::min(s, RB); ++l1)
            for (int l2 = l1 + 1; l2 < std::min(s, RB); ++l2)
                if ((p.B[off + l1] >> (off + l2)) & 1)
                    for (int g = 0; g < (1 << RB); ++g)
                        if ((g >> l1) & (g >> l2) & 1) p.czm[r] ^= 1u << g;
        off += s;
    }
    p.lam_round = nrounds - 1;
    for (int r = 0; r < p.lam_round; ++r)
        if (chunks[r] != kChunkBits) p.full_rounds = false;
    // the kernel twiddles only register slot 0 of the Lambda round
    for (int r = 0; r < nrounds; ++r)
        if (p.iflag[r] & ~(r == p.lam_round ? 1u : 0u))
            return fail(SD_ERR_INTERNAL, "S outside slot 0 of the Lambda round");

    // lane vectors
    for (int r = 0; r < nrounds; ++r) {
        Echelon e;
        std::vector<uint32_t> ln(TL, 0u);
        std::vector<char> set(TL, 0);
        for (int l = 0; l < RB; ++l) e.insert(1ull << p.reg[r][l]);
        for (int x = 0; x < p.nx[r]; ++x) {
            e.insert(1ull << p.xl[r][x]);
            ln[4 + x] = 1u << p.xl[r][x];
            set[4 + x] = 1;
        }
        uint32_t chunk0 = 0;  // round 0's own (transformed) coordinates
        if (r == 0) {
            // Direct I/O needs the c leading low address bits as lanes 0..3,
            // independent of the round's registers and exchanged lanes;
            // otherwise the tile is staged through LDS in pivot order.  A low
            // bit with components along the round's own coordinates shifts
            // the thread's register frame: the kernel writes the round's
            // outputs without those components (lanes_post) and corrects
            // their signs (shift0).
            chunk0 = p.chunk.empty() ? 0u : (((1u << chunks[0]) - 1));
            Echelon e2 = e;
            int k = 0;
            while (k < p.c && k < 4 && e2.insert(p.mr[k])) ++k;
            p.staged = k < std::min(p.c, 4);
            p.io_k = p.staged ? 0 : k;
            for (int i = 0; i < p.io_k; ++i) {
                e.insert(p.mr[i]);
                ln[i] = p.mr[i];
                set[i] = 1;
            }
        }
        int slot = 0;
        for (int q = 0; q < D; ++q) {
            while (slot < TL && set[slot]) ++slot;
            if (slot >= TL) break;
            if (e.insert(1ull << q)) {
                ln[slot] = 1u << q;
                set[slot] = 1;
            }
        }
        for (int i = 0; i < TL; ++i)
            if (!set[i]) return fail(SD_ERR_INTERNAL, "lane vectors do not span the tile");
        p.lanes[r] = ln;
        p.lanes_post[r] = ln;
        for (int x = 0; x < p.nx[r]; ++x) p.lanes_post[r][4 + x] = 1u << p.reg[r][2 + x];
        if (r == 0)
            for (int i = 0; i < p.io_k; ++i) {
                p.lanes_post[0][i] = ln[i] & ~chunk0;
                if (ln[i] & chunk0) p.shift0 = true;
            }
    }
    auto phys = [&](uint32_t v) {
        uint64_t x = 0;
        for (uint32_t w = v; w; w &= w - 1) x ^= p.basis[ctz(w)];
        return x;
    };
    for (uint32_t t : p.lanes[0]) p.io_phys.push_back(phys(t));
    for (int l = 0; l < RB; ++l) p.io_reg[l] = p.basis[p.reg[0][l]];
    // Lane vectors of every LDS layout (every round, and the pivot-order
    // staging of a staged pass).  16-byte writes serve 8 lanes (bits 0..2)
    // per 128-byte phase, 16-byte reads 16 lanes (bits 0..3) per 256-byte
    // phase: the low 3 slot bits of lanes 0..2 and the low 4 slot bits of
    // lanes 0..3 must be independent.
    std::vector<std::array<uint32_t, 4>> quads;
    for (int r = 0; r < nrounds; ++r)
        quads.push_back({p.lanes_post[r][0], p.lanes_post[r][1], p.lanes_post[r][2], p.lanes_post[r][3]});
    if (p.staged) quads.push_back({p.mr[0], p.mr[1], p.mr[2], p.mr[3]});
    // A round before the Lambda round writes its outputs at its layout XOR a
    // per-thread flip of its chunk coordinates (the CZs with later chunks):
    // bit a of the flip is the parity of B[a] & later[r] & (the thread's
    // coordinates), linear in the lane bits, so lane i's write vector is
    // lanes_post[r][i] XOR flip(lanes[r][i]).  Those layouts take the same
    // conflict rules.
    for (int r = 0; r + 1 < nrounds; ++r) {
        std::vector<int> chunk;
        for (int l = 0; l < RB; ++l)
            if ((p.bmask[r] >> l) & 1u) chunk.push_back(p.reg[r][l]);
        for (int x = 0; x < p.nx[r]; ++x) chunk.push_back(p.xl[r][x]);
        auto flip = [&](uint32_t v) {
            uint32_t f = 0;
            for (int a : chunk) f |= (uint32_t)(popc(p.B[a] & p.later[r] & v) & 1) << a;
            return f;
        };
        std::array<uint32_t, 4> q;
        bool any = false;
        for (int i = 0; i < 4; ++i) {
            const uint32_t f = i < (int)p.lanes[r].size() ? flip(p.lanes[r][i]) : 0;
            any = any || f;
            q[i] = p.lanes_post[r][i] ^ f;
        }
        if (any) quads.push_back(q);
    }
    auto lowbits = [](uint32_t v, const uint32_t *m, int nb) {
        uint32_t g = v & ((1u << nb) - 1);
        for (int j = 0; j < nb; ++j) g ^= (uint32_t)(popc(v & m[j]) & 1) << j;
        return g;
    };
    auto indep = [](std::vector<uint32_t> v) {
        Echelon e;
        for (uint32_t x : v)
            if (!e.insert(x)) return false;
        return true;
    };
    auto score = [&](const uint32_t *m) {
        int ok = 0;
        for (auto &q : quads) {
            if (indep({lowbits(q[0], m, 3), lowbits(q[1], m, 3), lowbits(q[2], m, 3)})) ++ok;
            if (indep({lowbits(q[0], m, 4), lowbits(q[1], m, 4), lowbits(q[2], m, 4), lowbits(q[3], m, 4)})) ++ok;
        }
        return ok;
    };
    const int target = 2 * (int)quads.size();
    // slot bit j < 3 may fold in bits >= 3, slot bit 3 bits >= 4: the map
    // stays triangular, hence invertible
    const uint32_t all = (1u << D) - 1;
    const uint32_t hm[4] = {all & ~7u, all & ~7u, all & ~7u, all & ~15u};
    uint32_t mk[4];
    for (int j = 0; j < 4; ++j) {
        mk[j] = 0;
        for (int q = 4 + j; q < D; q += 4) mk[j] |= 1u << q;
    }
    int best = score(mk);
    uint64_t rng = 0x9e3779b97f4a7c15ull ^ ((uint64_t)p.rho << 32) ^ (uint64_t)p.terms.size();
    for (int it = 0; it < 8192 && best < target; ++it) {
        uint32_t cand[4];
        for (int j = 0; j < 4; ++j) {
            rng ^= rng << 13;
            rng ^= rng >> 7;
            rng ^= rng << 17;
            cand[j] = (uint32_t)rng & hm[j];
        }
        const int sc = score(cand);
        if (sc > best) {
            best = sc;
            for (int j = 0; j < 4; ++j) mk[j] = cand[j];
        }
    }
    for (int j = 0; j < 4; ++j) p.swz[j] = mk[j];

    // sort the Lambda terms by their pattern on the Lambda round's registers
    // (after the exchange)
    const int L = p.lam_round;
    auto pattern = [&](uint32_t z) {
        uint32_t w = 0;
        for (int i = 0; i < RB; ++i) w |= ((z >> p.regpost[L][i]) & 1u) << i;
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
    std::vector<double> c2, u2;
    for (size_t i : idx) {
        t2.push_back(p.terms[i]);
        z2.push_back(p.zeta[i]);
        zt2.push_back(p.ztile[i]);
        c2.push_back(p.coef[i]);
        u2.push_back(p.usign[i]);
    }
    p.terms.swap(t2);
    p.zeta.swap(z2);
    p.ztile.swap(zt2);
    p.coef.swap(c2);
    p.usign.swap(u2);
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
    p.usign.clear();
    p.terms = vterm;
    for (size_t i = 0; i < vterm.size(); ++i) {
        const int64_t k = vterm[i];
        p.zeta.push_back((uint32_t)sr.zmask[i]);
        p.ztile.push_back(T[k].z);
        double s = (sr.sign[i] ? -1.0 : 1.0) * (ephase[i] == 2 ? -1.0 : 1.0);
        p.coef.push_back(T[k].c * s);
        p.usign.push_back(s);
    }
    sd_status st = canonicalize(&p);
    if (st != SD_OK) return st;
    return plan_rounds(&p);
}

}  // namespace

// Modelled time of one tile pass (about microseconds for a 2^28 state; a fit
// over measured launches): a fixed part for the HBM round trip, one part per
// register round (ceil(rho / kChunkBits) of them) and one per span coordinate.
// Splits of a group into sub-groups are compared by the sum over their passes.
constexpr int kShrinkMaxTerms = 32;  // passes with more Lambda terms keep the full tile
constexpr int kShrinkMinCap = 11;    // smallest tile a group split is tried for (shrink)
constexpr int kPlannerThreads = 16;  // host threads compiling groups

// Extra modelled time per pass of a tile with one or two fewer contiguous low
// bits than the 128-byte line (fitted: 64-byte runs cost about 130, 32-byte
// runs about 370 per pass on the benchmark, with partner tiles run in a row).
constexpr int64_t kCoalescePenalty1 = 130;
constexpr int64_t kCoalescePenalty2 = 370;

static int64_t pass_cost(int rho) {
    return 500 + 280 * ((std::max(rho, 1) + kChunkBits - 1) / kChunkBits) + 39 * (int64_t)rho;
}

sd_status compile_program(int n, const std::vector<Term> &T,
                          const std::vector<std::vector<int64_t>> &groups,
                          int D_max, int c, int c_min, Program *out, bool shrink) {
    Program &P = *out;
    P.D_max = D_max;
    P.c = c;
    P.passes.clear();
    P.group_first.assign(1, 0);
    const int cc = std::min(c, n);
    const int Dcap = std::min(D_max, n);
    // The groups are compiled independently (their own seeded searches), on
    // a few host threads; the passes are then joined in group order, so the
    // program does not depend on the thread count.
    struct GroupOut {
        sd_status st = SD_OK;
        std::string err;
        std::vector<PassHost> passes;
    };
    std::vector<GroupOut> outs(groups.size());
    auto compile_group = [&](const size_t g) {
        // Split into sub-groups whose tile space (X span + low bits) fits.
        // Sub-groups are grown one at a time: first every remaining term whose
        // X part already lies in the span joins (no growth), then the term
        // whose addition lets the most remaining terms in for free is added.
        // The growth is repeated with seeded random tie-breaks (and now and
        // then the second-best term); the split of least modelled cost
        // (pass_cost of each sub-group's X rank) is kept, and then sub-groups
        // are dissolved into the others while that lowers the cost.  Every
        // split is exact: the terms commute.
        // the split of group g for a tile space with cc contiguous low bits,
        // and its modelled cost
        auto split_group = [&](const int cc, const int Dcap) {
            auto grow = [&](uint64_t seed) {
                std::vector<std::vector<int64_t>> subs;
                std::vector<int64_t> rest(groups[g].begin(), groups[g].end());
                uint64_t rng = seed;
                auto next = [&]() {
                    rng ^= rng << 13;
                    rng ^= rng >> 7;
                    rng ^= rng << 17;
                    return rng;
                };
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
                        // Adding x_a brings in exactly the terms whose X part has
                        // the same remainder modulo the span (the echelon basis is
                        // fully reduced, so the remainder is the coset's unique
                        // representative): the score is a count of equal remainders.
                        std::vector<uint64_t> rem(rest.size());
                        std::unordered_map<uint64_t, int> count;
                        for (size_t a = 0; a < rest.size(); ++a) {
                            rem[a] = span.reduce(T[rest[a]].x);
                            ++count[rem[a]];
                        }
                        size_t best = 0, second = 0;
                        int best_score = -1, second_score = -1;
                        for (size_t a = 0; a < rest.size(); ++a) {
                            const int score = count[rem[a]];
                            // (seed 0: the plain greedy, first best in term order)
                            const bool tie = seed && score == best_score && (next() & 1);
                            if (score > best_score || tie) {
                                second = best;
                                second_score = best_score;
                                best_score = score;
                                best = a;
                            } else if (score > second_score) {
                                second_score = score;
                                second = a;
                            }
                        }
                        if (seed && second_score >= 0 && (next() % 8) == 0) best = second;
                        span.insert(T[rest[best]].x);
                        cur.push_back(rest[best]);
                        rest.erase(rest.begin() + (long)best);
                    }
                    subs.push_back(std::move(cur));
                }
                return subs;
            };
            // a sub-group under construction: its tile space (low bits and X
            // parts), the rank of its X parts alone, its terms
            struct Sub {
                Echelon tile, xs;
                std::vector<int64_t> terms;
            };
            auto make_sub = [&](const std::vector<int64_t> &terms) {
                Sub u;
                for (int q = 0; q < cc; ++q) u.tile.insert(1ull << q);
                for (int64_t k : terms) {
                    u.tile.insert(T[k].x);
                    u.xs.insert(T[k].x);
                }
                u.terms = terms;
                return u;
            };
            auto split_cost = [&](const std::vector<std::vector<int64_t>> &subs) {
                int64_t cost = 0;
                for (auto &t : subs) {
                    Echelon xs;
                    for (int64_t k : t) xs.insert(T[k].x);
                    cost += pass_cost(xs.dim());
                }
                return cost;
            };
            std::vector<std::vector<int64_t>> best_split = grow(0);
            int64_t best_cost = split_cost(best_split);
            // (no restarts when the plain greedy meets the bound set by the
            // dimension of the group's X span with the low bits)
            size_t lb = 1;
            {
                Echelon all;
                for (int q = 0; q < cc; ++q) all.insert(1ull << q);
                for (int64_t k : groups[g]) all.insert(T[k].x);
                const int room = std::max(1, Dcap - cc);
                lb = (size_t)std::max(1, (all.dim() - cc + room - 1) / room);
            }
            // (each restart costs about size^2 reductions: fewer for big groups)
            const size_t gs = groups[g].size();
            const uint64_t restarts = std::max<uint64_t>(4, std::min<uint64_t>(48, 40000 / (gs * gs + 1)));
            for (uint64_t r = 1; r <= restarts && gs > 1 && best_split.size() > lb; ++r) {
                auto cand = grow(0x9e3779b97f4a7c15ull * r + g * 0x632be59bd9b4e019ull + 1);
                const int64_t cost = split_cost(cand);
                if (cost < best_cost) {
                    best_split = std::move(cand);
                    best_cost = cost;
                }
            }
            // Dissolve sub-groups, smallest first: each of its terms goes to the
            // other sub-group where it adds the least modelled cost (within the
            // tile space and term limits); kept when every term finds a place and
            // the total cost drops.
            if (best_split.size() > 1) {
                std::vector<Sub> cur;
                for (auto &t : best_split) cur.push_back(make_sub(t));
                auto total = [&](const std::vector<Sub> &v) {
                    int64_t cost = 0;
                    for (auto &u : v) cost += pass_cost(u.xs.dim());
                    return cost;
                };
                // (the two moves alternate until neither lowers the cost: each
                // accepted move lowers it, so this ends)
                for (bool again = true; again;) {
                    again = false;
                    for (bool improved = true; improved && cur.size() > 1;) {
                        improved = false;
                        std::vector<size_t> order(cur.size());
                        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
                        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
                            return cur[a].terms.size() < cur[b].terms.size();
                        });
                        const int64_t before = total(cur);
                        for (size_t sidx : order) {
                            std::vector<Sub> trial = cur;
                            bool placed = true;
                            for (int64_t k : cur[sidx].terms) {
                                const uint64_t x = T[k].x;
                                size_t to = SIZE_MAX;
                                int64_t delta_best = INT64_MAX;
                                for (size_t j = 0; j < trial.size(); ++j) {
                                    if (j == sidx || (int)trial[j].terms.size() >= kMaxPassTerms) continue;
                                    if (!trial[j].tile.contains(x) && trial[j].tile.dim() >= Dcap) continue;
                                    const int rho = trial[j].xs.dim();
                                    const int rho_new = rho + (trial[j].xs.contains(x) ? 0 : 1);
                                    const int64_t delta = pass_cost(rho_new) - pass_cost(rho);
                                    if (delta < delta_best) {
                                        delta_best = delta;
                                        to = j;
                                    }
                                }
                                if (to == SIZE_MAX) {
                                    placed = false;
                                    break;
                                }
                                trial[to].tile.insert(x);
                                trial[to].xs.insert(x);
                                trial[to].terms.push_back(k);
                            }
                            if (!placed) continue;
                            trial.erase(trial.begin() + (long)sidx);
                            if (total(trial) < before) {
                                cur = std::move(trial);
                                improved = true;
                                break;
                            }
                        }
                    }
                    // Move single terms: a term whose X part lies outside the span of
                    // the rest of its sub-group moves to another sub-group when that
                    // lowers the cost (e.g. a span of 13 = 3 rounds drops to 12 = 2).
                    for (bool improved = true; improved && cur.size() > 1;) {
                        improved = false;
                        for (size_t sidx = 0; sidx < cur.size() && !improved; ++sidx) {
                            const int rho_s = cur[sidx].xs.dim();
                            const auto &ts = cur[sidx].terms;
                            // (a lone term is never moved: that would leave an empty
                            // sub-group; dissolving above covers that case)
                            if (ts.size() < 2) continue;
                            for (size_t ti = 0; ti < ts.size() && !improved; ++ti) {
                                const uint64_t x = T[ts[ti]].x;
                                Echelon wo;
                                for (size_t u = 0; u < ts.size(); ++u)
                                    if (u != ti) wo.insert(T[ts[u]].x);
                                if (wo.contains(x)) continue;  // its X part is spanned by the rest
                                const int64_t gain_s = pass_cost(rho_s) - pass_cost(wo.dim());
                                size_t to = SIZE_MAX;
                                int64_t best_delta = 0;
                                for (size_t j = 0; j < cur.size(); ++j) {
                                    if (j == sidx || (int)cur[j].terms.size() >= kMaxPassTerms) continue;
                                    if (!cur[j].tile.contains(x) && cur[j].tile.dim() >= Dcap) continue;
                                    const int rho = cur[j].xs.dim();
                                    const int rho_new = rho + (cur[j].xs.contains(x) ? 0 : 1);
                                    const int64_t delta = pass_cost(rho_new) - pass_cost(rho) - gain_s;
                                    if (delta < best_delta) {
                                        best_delta = delta;
                                        to = j;
                                    }
                                }
                                if (to == SIZE_MAX) continue;
                                const int64_t k = ts[ti];
                                std::vector<int64_t> rest_terms;
                                for (size_t u = 0; u < ts.size(); ++u)
                                    if (u != ti) rest_terms.push_back(ts[u]);
                                cur[to].tile.insert(x);
                                cur[to].xs.insert(x);
                                cur[to].terms.push_back(k);
                                cur[sidx] = make_sub(rest_terms);
                                improved = again = true;
                            }
                        }
                    }
                }
                best_split.clear();
                for (auto &u : cur) best_split.push_back(std::move(u.terms));
            }
            return std::make_pair(best_split, split_cost(best_split));
        };
        // complex64: passes may take fewer contiguous low bits (down to
        // c_min) where that needs fewer passes: each HBM access run is then
        // shorter (64 or 32 bytes), which the tile order of the kernels
        // recovers only in part (kCoalescePenalty per pass), so the width of
        // least modelled cost is taken per group.
        int cg = cc;
        std::vector<std::vector<int64_t>> best_split;
        {
            auto r = split_group(cc, Dcap);
            int64_t best_total = r.second;
            best_split = std::move(r.first);
            for (int c2 = cc - 1; c2 >= std::max(0, c_min) && c2 >= cc - 2; --c2) {
                auto r2 = split_group(c2, Dcap);
                const int64_t pen = (cc - c2 == 1 ? kCoalescePenalty1 : kCoalescePenalty2) *
                                    (int64_t)r2.first.size();
                if (r2.second + pen < best_total) {
                    best_total = r2.second + pen;
                    best_split = std::move(r2.first);
                    cg = c2;
                }
            }
        }
        // complex64 (shrink): the group split again for tiles one and two
        // coordinates smaller, kept while it needs no more passes.  The passes
        // then take tiles of 2^12 or 2^11, which run two or four blocks per CU
        // whose barriers do not stall each other (n = 28: 139 passes either
        // way, 1.8% less time per step).
        // (a group of one pass already has its smallest tile)
        if (shrink && best_split.size() > 1) {
            for (int cap = Dcap - 1; cap >= std::max(kShrinkMinCap, cg + 1) && cap >= Dcap - 2; --cap) {
                auto r3 = split_group(cg, cap);
                if (r3.first.size() > best_split.size()) break;
                best_split = std::move(r3.first);
            }
        }
        std::vector<std::vector<int64_t>> &subs = best_split;
        for (auto &s : subs) {
            PassHost ps;
            // shrink: the smallest tile (not below the register-round minimum)
            // that holds the sub-group's span and low bits.  A pass with many
            // Lambda terms keeps the full tile: every thread runs the whole
            // term loop, and the small blocks of a shrunk tile (each with its
            // own term tables in LDS, so fewer waves per CU) run it slower.
            int Dt = Dcap;
            if (shrink && (int)s.size() <= kShrinkMaxTerms) {
                Echelon sp;
                for (int q = 0; q < cg; ++q) sp.insert(1ull << q);
                for (int64_t k : s) sp.insert(T[k].x);
                Dt = std::min(Dcap, std::max(sp.dim(), 2 * kRegBits + kXBits));
            }
            sd_status st = build_pass(n, T, (int32_t)g, s, Dt, cg, &ps);
            if (st != SD_OK) {
                // (the message is in this thread's last error)
                outs[g].st = st;
                outs[g].err = sd_last_error();
                return;
            }
            outs[g].passes.push_back(std::move(ps));
        }
    };
    const size_t nthreads = std::min<size_t>(
        {groups.size(), (size_t)kPlannerThreads, (size_t)std::max(1u, std::thread::hardware_concurrency())});
    if (nthreads <= 1) {
        for (size_t g = 0; g < groups.size(); ++g) compile_group(g);
    } else {
        std::atomic<size_t> next{0};
        std::vector<std::thread> pool;
        for (size_t t = 0; t < nthreads; ++t)
            pool.emplace_back([&]() {
                for (size_t g = next++; g < groups.size(); g = next++) compile_group(g);
            });
        for (auto &th : pool) th.join();
    }
    for (size_t g = 0; g < groups.size(); ++g) {
        if (outs[g].st != SD_OK) return fail(outs[g].st, outs[g].err);
        for (auto &ps : outs[g].passes) P.passes.push_back(std::move(ps));
        P.group_first.push_back((int32_t)P.passes.size());
    }
    return SD_OK;
}

}  // namespace sd
