// Device execution for gfx950: tile-pass kernels, reductions and the
// sd_evolve / sd_expectation / sd_norm2 / sd_inner entry points.
//
// One tile pass applies the exponential of one commuting (sub-)group:
//   load a tile (a coset of the group's X span, widened by low address bits)
//   -> multiply by i^{q(y)}                     (CZ/S layer, step (iii))
//   -> Walsh-Hadamard over the rho span coords  (H layer, step (iv))
//   -> multiply by exp(-i tau Lambda)           (diagonal operator, FP64 angle)
//   -> Walsh-Hadamard, multiply by i^{-q(y)} 2^{-rho}   (C^dagger)
//   -> store.
// The CNOT network of steps (ii) is the affine map between physical addresses
// and tile coordinates, applied while loading and storing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "device_types.h"
#include "sd_internal.h"

namespace sd {

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
int64_t pack_size(const Program &P) {
    int64_t s = (int64_t)P.passes.size() * (int64_t)sizeof(PassDev);
    for (auto &p : P.passes) s += (term_bytes((int)p.terms.size()) + 255) / 256 * 256;
    return s;
}

static void pack_program(const Program &P, int n, int64_t base_off, std::vector<uint8_t> &buf) {
    const int64_t total = pack_size(P);
    buf.assign((size_t)total, 0);
    int64_t toff = (int64_t)P.passes.size() * (int64_t)sizeof(PassDev);
    for (size_t i = 0; i < P.passes.size(); ++i) {
        const PassHost &p = P.passes[i];
        PassDev d;
        std::memset(&d, 0, sizeof(d));
        d.n = n;
        d.D = p.D;
        d.rho = p.rho;
        d.c = p.c;
        d.m = (int32_t)p.terms.size();
        d.n_free = n - p.D;
        d.n_tiles = (int64_t)1 << (n - p.D);
        d.term_off = base_off + toff;
        d.scale = std::ldexp(1.0, -p.rho);
        {
            // (exact: the scale is a power of two)
            const double kc[7] = {1.0, -1.0 / 2.0, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0,
                                  -1.0 / 3628800.0, 1.0 / 479001600.0};
            const double ks[7] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0,
                                  -1.0 / 39916800.0, 1.0 / 6227020800.0};
            for (int i = 0; i < 7; ++i) {
                d.kcos[i] = d.scale * kc[i];
                d.ksin[i] = d.scale * ks[i];
            }
        }
        for (int j = p.c; j < p.D; ++j) d.u_hi[j - p.c] = p.u[j];
        for (int j = 0; j < p.D; ++j) d.mr[j] = p.mr[j];
        for (int j = 0; j < p.rho; ++j) d.B[j] = p.B[j];
        d.zq = p.zq;
        int f = 0;
        for (int q = 0; q < n; ++q)
            if ((p.free_mask >> q) & 1) d.free_pos[f++] = q;
        d.nr = p.nr;
        d.lam_round = p.lam_round;
        for (int r = 0; r < 4; ++r) {
            for (int b = 0; b < 4; ++b) {
                d.reg[r][b] = p.reg[r][b];
                d.regpost[r][b] = p.regpost[r][b];
            }
            for (int x = 0; x < 2; ++x) d.xl[r][x] = p.xl[r][x];
            d.nx[r] = p.nx[r];
            d.bmask[r] = p.bmask[r];
            d.iflag[r] = p.iflag[r];
            d.dflag[r] = p.dflag[r];
            d.later[r] = p.later[r];
            d.czm[r] = p.czm[r];
            for (size_t i = 0; i < p.lanes[r].size() && i < (size_t)kMaxD; ++i) {
                d.lanes[r][i] = p.lanes[r][i];
                d.lanes_post[r][i] = p.lanes_post[r][i];
            }
        }
        for (int w = 0; w < 33; ++w) d.bucket[w] = p.bucket.empty() ? 0 : p.bucket[w];
        d.coef_abs_sum = p.coef_abs_sum;
        for (size_t i = 0; i < p.io_phys.size() && i < (size_t)kMaxD; ++i) d.io_phys[i] = p.io_phys[i];
        for (int l = 0; l < 4; ++l) d.io_reg[l] = p.io_reg[l];
        for (int j = 0; j < 4; ++j) d.swz[j] = p.swz[j];
        d.staged = p.staged ? 1 : 0;
        d.shift0 = p.shift0 ? 1 : 0;
        std::memcpy(buf.data() + i * sizeof(PassDev), &d, sizeof(d));
        uint8_t *t = buf.data() + toff;
        const int m = d.m;
        std::memcpy(t, p.zeta.data(), 4 * (size_t)m);
        int64_t o2 = ((int64_t)m * 4 + 7) / 8 * 8;
        std::memcpy(t + o2, p.ztile.data(), 8 * (size_t)m);
        std::memcpy(t + o2 + 8 * m, p.coef.data(), 8 * (size_t)m);
        std::memcpy(t + o2 + 16 * m, p.usign.data(), 8 * (size_t)m);
        toff += (term_bytes(m) + 255) / 256 * 256;
    }
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 ld_amp(const float2 *p, int64_t i) {
    float2 v = p[i];
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 ld_amp(const double2 *p, int64_t i) { return p[i]; }
__device__ __forceinline__ void st_amp(float2 *p, int64_t i, double2 v) {
    p[i] = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ void st_amp(double2 *p, int64_t i, double2 v) { p[i] = v; }

// a * i^q
__device__ __forceinline__ double2 mul_ipow(double2 a, int q) {
    switch (q & 3) {
        case 0: return a;
        case 1: return make_double2(-a.y, a.x);
        case 2: return make_double2(-a.x, -a.y);
        default: return make_double2(a.y, -a.x);
    }
}

// exponent of the CZ/S layer's phase i^{q(y)} (-1)^{popcount(y & zq)}
__device__ __forceinline__ int quad_form(const uint32_t *B, uint32_t zq, int rho, uint32_t y) {
    int q = 2 * __popc(zq & y);
    for (int i = 0; i < rho; ++i)
        if ((y >> i) & 1) q += __popc(B[i] & y);
    return q;
}

__device__ void wht_lds(double2 *tile, int D, int rho) {
    const int64_t half = (int64_t)1 << (D - 1);
    for (int b = 0; b < rho; ++b) {
        __syncthreads();
        const uint32_t lowm = (1u << b) - 1;
        for (int64_t j = threadIdx.x; j < half; j += blockDim.x) {
            const uint32_t lo = (((uint32_t)j >> b) << (b + 1)) | ((uint32_t)j & lowm);
            const uint32_t hi = lo | (1u << b);
            const double2 a = tile[lo], c = tile[hi];
            tile[lo] = make_double2(a.x + c.x, a.y + c.y);
            tile[hi] = make_double2(a.x - c.x, a.y - c.y);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

constexpr int kBlock = 256;

// MODE 0: evolve in place.  MODE 1: accumulate <psi|H_pass|psi> into partial[blockIdx].
// MODE 2: <psi|P_k|psi> of every term k of the pass: the probabilities of the
// transformed tile go through a full Walsh-Hadamard transform in LDS, whose
// entry at term k's Lambda mask (times its sign) is the tile's share; thread
// k keeps term k's running sum, written to partial[blockIdx * kMaxPassTerms + k].
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock)
k_pass(T *__restrict__ state, const PassDev *__restrict__ pdp, const uint8_t *__restrict__ ws,
       double tau, double *__restrict__ partial) {
    extern __shared__ double2 tile[];
    __shared__ double cks[kMaxPassTerms];
    __shared__ uint32_t zs[kMaxPassTerms];
    __shared__ double red[kBlock];
    const PassDev &pd = *pdp;
    const int D = pd.D, rho = pd.rho, c = pd.c, m = pd.m;
    const int64_t size = (int64_t)1 << D;
    const uint8_t *tb = ws + pd.term_off;
    const uint32_t *zeta = (const uint32_t *)tb;
    const int64_t o2 = ((int64_t)m * 4 + 7) / 8 * 8;
    const uint64_t *ztile = (const uint64_t *)(tb + o2);
    const double *coef = (const double *)(tb + o2 + 8 * (int64_t)m);
    const double *usgn = (const double *)(tb + o2 + 16 * (int64_t)m);
    const uint32_t rmask = (rho >= 32) ? ~0u : ((1u << rho) - 1);
    const uint64_t cmask = ((uint64_t)1 << c) - 1;
    const double scale = pd.scale;
    double acc = 0.0;

    for (int64_t ti = blockIdx.x; ti < pd.n_tiles; ti += gridDim.x) {
        uint64_t xT = 0;
        for (int i = 0; i < pd.n_free; ++i)
            if ((ti >> i) & 1) xT |= (uint64_t)1 << pd.free_pos[i];
        for (int k = threadIdx.x; k < m; k += blockDim.x) {
            const double v = MODE == 2 ? usgn[k] : coef[k];
            cks[k] = (__popcll(ztile[k] & xT) & 1) ? -v : v;
            zs[k] = zeta[k];
        }
        for (int64_t p = threadIdx.x; p < size; p += blockDim.x) {
            uint64_t off = (uint64_t)p & cmask;
            uint32_t tc = 0;
            for (int i = 0; i < D; ++i)
                if ((p >> i) & 1) {
                    tc ^= pd.mr[i];
                    if (i >= c) off ^= pd.u_hi[i - c];
                }
            tile[tc] = ld_amp(state, (int64_t)(xT ^ off));
        }
        __syncthreads();
        if (rho > 0) {
            for (int64_t t = threadIdx.x; t < size; t += blockDim.x)
                tile[t] = mul_ipow(tile[t], quad_form(pd.B, pd.zq, rho, (uint32_t)t & rmask));
            wht_lds(tile, D, rho);
        }
        if (MODE == 0) {
            for (int64_t t = threadIdx.x; t < size; t += blockDim.x) {
                double phi = 0.0;
                for (int k = 0; k < m; ++k)
                    phi += (__popc(zs[k] & (uint32_t)t) & 1) ? -cks[k] : cks[k];
                double sn, cs;
                sincos(-tau * phi, &sn, &cs);
                const double2 a = tile[t];
                tile[t] = make_double2((a.x * cs - a.y * sn) * scale, (a.x * sn + a.y * cs) * scale);
            }
            if (rho > 0) {
                wht_lds(tile, D, rho);
                for (int64_t t = threadIdx.x; t < size; t += blockDim.x)
                    tile[t] = mul_ipow(tile[t], -quad_form(pd.B, pd.zq, rho, (uint32_t)t & rmask));
            }
            __syncthreads();
            for (int64_t p = threadIdx.x; p < size; p += blockDim.x) {
                uint64_t off = (uint64_t)p & cmask;
                uint32_t tc = 0;
                for (int i = 0; i < D; ++i)
                    if ((p >> i) & 1) {
                        tc ^= pd.mr[i];
                        if (i >= c) off ^= pd.u_hi[i - c];
                    }
                st_amp(state, (int64_t)(xT ^ off), tile[tc]);
            }
        } else if (MODE == 1) {
            for (int64_t t = threadIdx.x; t < size; t += blockDim.x) {
                double phi = 0.0;
                for (int k = 0; k < m; ++k)
                    phi += (__popc(zs[k] & (uint32_t)t) & 1) ? -cks[k] : cks[k];
                const double2 a = tile[t];
                acc += (a.x * a.x + a.y * a.y) * phi * scale;
            }
        } else {
            __syncthreads();
            for (int64_t t = threadIdx.x; t < size; t += blockDim.x) {
                const double2 a = tile[t];
                tile[t] = make_double2((a.x * a.x + a.y * a.y) * scale, 0.0);
            }
            wht_lds(tile, D, D);
            if ((int)threadIdx.x < m) acc += cks[threadIdx.x] * tile[zs[threadIdx.x] & (uint32_t)(size - 1)].x;
        }
        __syncthreads();
    }
    if (MODE == 1) {
        double s = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] += s;
    }
    if (MODE == 2 && (int)threadIdx.x < m) partial[(int64_t)blockIdx.x * kMaxPassTerms + threadIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// k_tile: register-round tile pass (tiles of 2^D amplitudes, D >= kTileMinD)
// ---------------------------------------------------------------------------
// A block of 2^(D-kLE) threads owns one tile at a time; every thread holds
// kE = 2^kLE amplitudes in FP64 registers.  In the round of chunk r the kE
// amplitudes of a thread differ in the kLE tile coordinates reg[r] and share
// the others (taken from the thread index), so the butterflies of those
// coordinates run in registers; between rounds the tile is exchanged through
// LDS.  The LDS slot of tile coordinate t is t ^ sum_j parity(t & swz[j]) << j
// with per-pass masks that the planner picks so that, in every round, the
// lanes served together hit distinct banks: 8 lanes per 128-byte phase for
// 16-byte writes, 16 lanes per 256-byte phase for 16-byte reads on gfx950.  The slot map is linear
// over GF(2), so every address is a per-thread base XOR a uniform offset; the
// tile sits at LDS address 0 and addresses are plain byte offsets (no static
// LDS in these kernels).
//
// The CZ/S layer costs no per-amplitude work.  The planner puts its quadratic
// form in a basis where no chunk has a CZ inside it, so the layer factors
// into: an S on a chunk coordinate, applied as an i twiddle inside that
// coordinate's butterfly; a Z on a chunk coordinate and the CZs between a
// chunk coordinate and a coordinate of a later chunk (a thread-index bit in
// this round), which are sign patterns (-1)^{l.j} on the register index j
// before the butterflies, i.e. an XOR l on their output index.  That XOR is
// folded into the address the round writes to, and into the address the
// mirrored inverse round reads from (a Walsh-Hadamard transform of the
// permuted data applies the inverse sign pattern by itself).  In the Lambda
// round, the XOR is folded into the signs of Lambda's terms instead.
constexpr int kLE = 4;
constexpr int kE = 1 << kLE;
constexpr int kTileMinD = 10;
constexpr int kMaxThreads = 1 << (kMaxTileLog2 - kLE);

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) dvec2 lds_c2;
__device__ __forceinline__ double2 lds_ld(uint32_t a) {
    const dvec2 v = *(const lds_c2 *)(size_t)a;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void lds_st(uint32_t a, double2 v) {
    dvec2 w;
    w.x = v.x;
    w.y = v.y;
    *(lds_c2 *)(size_t)a = w;
}

// Dynamic LDS of k_tile, in bytes from 0: the tile (16 B per amplitude); per
// thread and round the pair of round addresses (8 B); per term the record
// {signed coefficient of the current tile, Lambda mask} (16 B) and the record
// {coefficient, physical Z mask for the tile sign} (16 B); the register
// offsets of the rounds before and after the lane exchange (128 B); the 17
// bucket bounds (80 B); 8 block-sum slots (64 B).
struct TileLds {
    uint32_t thr, trec, tsrc, rs, bk, red, total;
};
__host__ __device__ inline TileLds tile_lds(int D, int threads, int nrounds, int m) {
    TileLds l;
    l.thr = 16u << D;
    l.trec = l.thr + 8u * (uint32_t)(nrounds * threads);
    l.tsrc = l.trec + 16u * (uint32_t)m;
    l.rs = l.tsrc + 16u * (uint32_t)m;
    l.bk = l.rs + 128u;
    l.red = l.bk + 80u;
    l.total = l.red + 64u;
    return l;
}
// the largest layout any pass can ask for (attribute setup)
constexpr size_t kTileLdsMax =
    ((size_t)16 << kMaxTileLog2) + 8 * 4 * (size_t)kMaxThreads + 32 * (size_t)kMaxPassTerms + 128 + 80 + 64;

// e^{i theta}: Taylor polynomials of cos and sin at x = theta / 2^halv
// (|x| <= 1/4), then halv double-angle steps.  FULL: degrees 12/13 (truncation
// below 1e-17, for complex128 states); otherwise degrees 8/9 (below 3e-13,
// far under the complex64 rounding of the result).
template <bool FULL>
__device__ __forceinline__ void cis(double th, int halv, double &c, double &s) {
    const double x = ldexp(th, -halv);
    const double x2 = x * x;
    double pc, ps;
    if (FULL) {
        pc = 1.0 / 479001600.0;
        pc = fma(pc, x2, -1.0 / 3628800.0);
        pc = fma(pc, x2, 1.0 / 40320.0);
        ps = 1.0 / 6227020800.0;
        ps = fma(ps, x2, -1.0 / 39916800.0);
        ps = fma(ps, x2, 1.0 / 362880.0);
    } else {
        pc = 1.0 / 40320.0;
        ps = 1.0 / 362880.0;
    }
    pc = fma(pc, x2, -1.0 / 720.0);
    pc = fma(pc, x2, 1.0 / 24.0);
    pc = fma(pc, x2, -0.5);
    c = fma(pc, x2, 1.0);
    ps = fma(ps, x2, -1.0 / 5040.0);
    ps = fma(ps, x2, 1.0 / 120.0);
    ps = fma(ps, x2, -1.0 / 6.0);
    s = fma(x * x2, ps, x);
    for (int i = 0; i < halv; ++i) {
        const double c2 = fma(c, c, -s * s);
        s = 2.0 * c * s;
        c = c2;
    }
}

// 2^-rho e^{i x} for |x| <= 1/4 and no double-angle steps: the polynomials
// of cis with every coefficient multiplied by 2^-rho (kc, ks from the pass
// record, constant term first; exact, the factor being a power of two), so
// the result needs no separate scaling.  FULL: degrees 12/13, else 8/9.
template <bool FULL, typename CP>
__device__ __forceinline__ void cis_scaled(double x, CP kc, CP ks, double &c, double &s) {
    constexpr int N = FULL ? 7 : 5;
    const double x2 = x * x;
    double pc = kc[N - 1], ps = ks[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) {
        pc = fma(pc, x2, kc[i]);
        ps = fma(ps, x2, ks[i]);
    }
    c = pc;
    s = ps * x;
}

// Sum of v over the 64 lanes of a wave (every lane active), the same value
// in every lane: within each 16-lane row by DPP moves (lane i ^ 1, lane
// i ^ 2, then the mirrored lane of its half-row and of its row: after each
// step every lane holds the sum over its pair, quad, half-row, row), then
// the four row sums read out of lanes 0, 16, 32, 48 and added in that order.
__device__ __forceinline__ double wave_sum_f64(double v) {
    auto dpp = [](double x, auto ctrl) {
        const uint64_t u = (uint64_t)__double_as_longlong(x);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, decltype(ctrl)::value, 0xF, 0xF, false);
        const uint32_t hi =
            (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), decltype(ctrl)::value, 0xF, 0xF, false);
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    };
    v += dpp(v, std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
    v += dpp(v, std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
    v += dpp(v, std::integral_constant<int, 0x141>{});  // row_half_mirror
    v += dpp(v, std::integral_constant<int, 0x140>{});  // row_mirror
    auto row = [&](int l) {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    };
    return ((row(0) + row(16)) + row(32)) + row(48);
}

// butterflies on register bit L.  Forward: (a, c) -> (a + w c, a - w c) with
// w = 1 or i (the S of that coordinate applied first).  Backward, the inverse
// up to the factor 2: (A, C) -> (A + C, conj(w) (A - C)).
template <int L, bool TW>
__device__ __forceinline__ void bfly_fwd(double (&re)[kE], double (&im)[kE]) {
#pragma unroll
    for (int j = 0; j < kE; ++j)
        if (!((j >> L) & 1)) {
            const int k = j | (1 << L);
            const double ar = re[j], ai = im[j], cr = re[k], ci = im[k];
            if (TW) {
                re[j] = ar - ci;
                im[j] = ai + cr;
                re[k] = ar + ci;
                im[k] = ai - cr;
            } else {
                re[j] = ar + cr;
                im[j] = ai + ci;
                re[k] = ar - cr;
                im[k] = ai - ci;
            }
        }
}

// The same plain butterfly computed in place: the sum overwrites a, then
// the difference is the sum minus 2c (one FMA), so each result can take the
// register of the input it replaces.  Used where a stage runs under a branch:
// there the usual form leaves the sums in new registers that the join then
// moves back.  Its difference is rounded from the rounded sum, an error of
// the same size as the sum's own.
template <int L>
__device__ __forceinline__ void bfly_ip(double (&re)[kE], double (&im)[kE]) {
#pragma unroll
    for (int j = 0; j < kE; ++j)
        if (!((j >> L) & 1)) {
            const int k = j | (1 << L);
            re[j] = re[j] + re[k];
            im[j] = im[j] + im[k];
            re[k] = fma(-2.0, re[k], re[j]);
            im[k] = fma(-2.0, im[k], im[j]);
        }
}

template <int L, bool TW>
__device__ __forceinline__ void bfly_bwd(double (&re)[kE], double (&im)[kE]) {
#pragma unroll
    for (int j = 0; j < kE; ++j)
        if (!((j >> L) & 1)) {
            const int k = j | (1 << L);
            const double ar = re[j], ai = im[j], cr = re[k], ci = im[k];
            re[j] = ar + cr;
            im[j] = ai + ci;
            if (TW) {
                re[k] = ai - ci;
                im[k] = cr - ar;
            } else {
                re[k] = ar - cr;
                im[k] = ai - ci;
            }
        }
}

// Exchange register bit B with lane bit LB (4 or 5) inside the wave: for
// every register pair differing in bit B, a 2x2 transpose between the pair
// and the two lane halves, so that afterwards register bit B indexes the
// coordinate lane bit LB held and lane bit LB the one register bit B held.
template <int LB>
__device__ __forceinline__ void lane_swap(double &x, double &y) {
    const uint64_t ux = (uint64_t)__double_as_longlong(x), uy = (uint64_t)__double_as_longlong(y);
    const uint32_t xl = (uint32_t)ux, xh = (uint32_t)(ux >> 32);
    const uint32_t yl = (uint32_t)uy, yh = (uint32_t)(uy >> 32);
    uint32_t nxl, nyl, nxh, nyh;
    if (LB == 4) {
        const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        nxl = l[0];
        nyl = l[1];
        nxh = h[0];
        nyh = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        nxl = l[0];
        nyl = l[1];
        nxh = h[0];
        nyh = h[1];
    }
    x = __longlong_as_double((long long)(((uint64_t)nxh << 32) | nxl));
    y = __longlong_as_double((long long)(((uint64_t)nyh << 32) | nyl));
}

template <int B, int LB>
__device__ __forceinline__ void exch(double (&re)[kE], double (&im)[kE]) {
#pragma unroll
    for (int j = 0; j < kE; ++j)
        if (!((j >> B) & 1)) {
            lane_swap<LB>(re[j], re[j | (1 << B)]);
            lane_swap<LB>(im[j], im[j | (1 << B)]);
        }
}

__device__ __forceinline__ double2 to_c128(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 to_c128(double2 v) { return v; }
__device__ __forceinline__ void from_c128(float2 &o, double2 v) { o = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void from_c128(double2 &o, double2 v) { o = v; }

// One tile pass over tiles t0, t0 + stride, ... < t1 of the pass `pdp` (the
// whole pass when called with blockIdx.x, n_tiles, gridDim.x).  MODE 0
// evolves in place, MODE 1 adds this block's share of <psi|H_pass|psi> to
// acc[0], MODE 2 this wave's share of <psi|P_k|psi> for every term k of the
// pass to lane k mod 64's acc[k / 64].  OFF is the type of in-state byte offsets: uint32_t when the state is
// at most 4 GiB, else uint64_t.  GEN admits chunks of fewer than kLE span
// coordinates in rounds other than Lambda's; without it those rounds are
// straight-line code (four plain butterfly stages between one LDS read and
// one LDS write).
//
// Round 0 reads its amplitudes straight from HBM into registers (its lanes
// run over the lowest address bits) and its mirrored inverse round writes
// them straight back, so the tile crosses LDS only between rounds; a pass of
// a single round never touches LDS for amplitudes.
template <typename T, int MODE, typename OFF, bool GEN, typename PDP = const PassDev *>
__device__ __forceinline__ void tile_pass(T *__restrict__ state, PDP __restrict__ pdp,
                                          const uint8_t *__restrict__ ws, double tau, int64_t t0,
                                          int64_t t1, int64_t stride, double (&acc)[4]) {
    constexpr bool FULL = sizeof(T) == 16;
    // complex128 tiles and the general round code skip the register
    // prefetch of the next tile: it would not fit two waves per SIMD
    constexpr bool PF = MODE == 0 && sizeof(T) == 8;
    extern __shared__ double2 lds_dyn[];
    const auto &pd = *pdp;
    const int D = pd.D, TL = D - kLE, m = pd.m, nr = pd.nr;
    const uint32_t T_ = blockDim.x;
    const uint32_t tid = threadIdx.x;
    char *lbase = (char *)lds_dyn;
    const int nrounds = nr > 0 ? nr : 1;
    const TileLds L = tile_lds(D, (int)T_, nrounds, m);
    uint2 *thr = (uint2 *)(lbase + L.thr);
    double2 *trec = (double2 *)(lbase + L.trec);   // .x signed coefficient, .y bits: Lambda mask
    double2 *tsrc = (double2 *)(lbase + L.tsrc);   // .x coefficient, .y bits: tile Z mask
    uint32_t *s_rs = (uint32_t *)(lbase + L.rs);   // [4][kLE] byte offsets of register coordinates
    uint32_t *s_ws = s_rs + 4 * kLE;               // the same after the lane exchange
    int32_t *s_bk = (int32_t *)(lbase + L.bk);     // bucket bounds
    __syncthreads();  // a previous call of this block may still read the arrays
    int halv = 0;
    if (MODE == 0) {
        const double th = fabs(tau) * pd.coef_abs_sum;
        while (halv < 60 && ldexp(th, -halv) > 0.25) ++halv;
    }
    const uint32_t sw0 = pd.swz[0], sw1 = pd.swz[1], sw2 = pd.swz[2], sw3 = pd.swz[3];
    auto slot = [&](uint32_t t) {
        return t ^ ((uint32_t)(__popc(t & sw0) & 1) | ((uint32_t)(__popc(t & sw1) & 1) << 1) |
                    ((uint32_t)(__popc(t & sw2) & 1) << 2) | ((uint32_t)(__popc(t & sw3) & 1) << 3));
    };
    if (tid < 4 * kLE) {
        s_rs[tid] = slot(1u << pd.reg[tid / kLE][tid % kLE]) * 16u;
        s_ws[tid] = slot(1u << pd.regpost[tid / kLE][tid % kLE]) * 16u;
    }
    if (tid < 2 * kE + 1) s_bk[tid] = tid <= kE ? pd.bucket[tid] : 0;
    {
        const uint8_t *tb = ws + pd.term_off;
        const int64_t o2 = ((int64_t)m * 4 + 7) / 8 * 8;
        for (int k = tid; k < m; k += T_) {
            const uint32_t z = ((const uint32_t *)tb)[k];
            const uint64_t zt = ((const uint64_t *)(tb + o2))[k];
            const double cf = ((const double *)(tb + o2 + 8 * (int64_t)m))[k];
            trec[k] = make_double2(0.0, __longlong_as_double((long long)z));
            // (evolution: the coefficient times -tau, so that the bucket
            // sums are the phase angles themselves)
            // (term values: the sign (-1)^{r_k} i^{e_k} alone, without c_k)
            const double v = MODE == 0 ? -tau * cf
                             : MODE == 1 ? cf
                                         : ((const double *)(tb + o2 + 16 * (int64_t)m))[k];
            tsrc[k] = make_double2(v, __longlong_as_double((long long)zt));
        }
    }
    const double scale = pd.scale;

    // ---- per-thread constants (tile independent) ----
    // round 0: lane bit i is tile coordinate vector lanes[0][i] (physical
    // offset io_phys[i]); register slot l is coordinate reg[0][l] (offset
    // io_reg[l])
    // A staged pass moves the tile in pivot order instead: element j of
    // thread t is pivot pattern t + (j << TL), at LDS slot of tile
    // coordinate sum mr[i] over its pivot bits.
    const bool staged = pd.staged != 0;
    const int c = pd.c;
    OFF off_t = 0;
    OFF pv[kLE];
    uint32_t sl_t = 0, sv[kLE];
    if (!staged) {
        for (int i = 0; i < TL; ++i)
            if ((tid >> i) & 1) off_t ^= (OFF)pd.io_phys[i] * (OFF)sizeof(T);
#pragma unroll
        for (int b = 0; b < kLE; ++b) {
            pv[b] = (OFF)pd.io_reg[b] * (OFF)sizeof(T);
            sv[b] = 0;
        }
    } else {
        uint32_t tc_t = 0;
        for (int i = 0; i < TL; ++i)
            if ((tid >> i) & 1) {
                off_t ^= (OFF)(i < c ? ((uint64_t)1 << i) : pd.u_hi[i - c]) * (OFF)sizeof(T);
                tc_t ^= pd.mr[i];
            }
        sl_t = slot(tc_t) * 16u;
#pragma unroll
        for (int b = 0; b < kLE; ++b) {
            const int i = TL + b;
            pv[b] = (OFF)(i < c ? ((uint64_t)1 << i) : pd.u_hi[i - c]) * (OFF)sizeof(T);
            sv[b] = slot(pd.mr[i]) * 16u;
        }
    }
    // A direct pass whose low address bits (round 0's lanes 0..3) have
    // components d(t) along round 0's own coordinates: the thread's registers
    // sit at coordinates shifted by d(t), so the transform of round 0 comes
    // out as (-1)^{k.d(t)} times the true one at output coordinate k.  Its
    // outputs are written at k (lanes_post[0] without those components) and,
    // when round 0 is not Lambda's round, take the sign (-1)^{k.d(t)} after
    // the forward butterflies and again before the backward ones.  k covers
    // the 4 register slots after the exchange and the lane bits 4, 5, which
    // then hold register coordinates 2, 3.  Bit g of sgn0 is the sign of
    // register g; it is kept in the thread's round-0 read address, which a
    // direct pass never uses (round 0 reads HBM forward, its write layout
    // backward).
    // A CZ or S among round 0's register coordinates makes the shift also
    // move the outputs, by m0(t) = M d(t) (M: the CZ/S form on those
    // coordinates; added to the round's output layout and, in a single
    // round, to Lambda's sign coordinates), and adds the constant
    // (-1)^{Q(d)} (Q: the CZ pairs), folded into the sign.
    uint32_t sgn0 = 0, m0 = 0;
    if (pd.shift0 && !staged) {
        uint32_t d = 0;
        for (int i = 0; i < kLE && i < TL; ++i)
            if ((tid >> i) & 1) d ^= pd.lanes[0][i] ^ pd.lanes_post[0][i];
        const int nb0 = __popc(pd.bmask[0]);
        uint32_t regm = 0, qd = 0;
        for (int l = 0; l < nb0; ++l) regm |= 1u << pd.reg[0][l];
        for (int l = 0; l < nb0; ++l) {
            const int a = pd.reg[0][l];
            m0 |= (uint32_t)(__popc(pd.B[a] & regm & d) & 1) << a;
            const uint32_t higher = regm & ~((2u << a) - 1u);
            qd ^= (d >> a) & (uint32_t)__popc(pd.B[a] & higher & d);
        }
        uint32_t w = 0, kap = qd & 1u;
        for (int l = 0; l < kLE; ++l) w |= ((d >> pd.regpost[0][l]) & 1u) << l;
        for (int x = 0; x < pd.nx[0]; ++x) kap ^= (tid >> (kLE + x)) & (d >> pd.reg[0][2 + x]) & 1u;
        for (int g = 0; g < kE; ++g) sgn0 |= ((__popc(g & w) ^ kap) & 1u) << g;
    }
    const bool sh0 = pd.shift0 && !staged && nr >= 2;
    // thr[r] = (address the forward round reads, before the lane exchange;
    // address it writes, after the exchange, with the thread's output XOR)
    uint32_t sgnb = 0;  // tile coordinates for the signs of Lambda's terms
    for (int r = 0; r < nrounds; ++r) {
        uint32_t bt = 0, btp = 0;
        for (int i = 0; i < TL; ++i)
            if ((tid >> i) & 1) {
                bt ^= pd.lanes[r][i];
                btp ^= pd.lanes_post[r][i];
            }
        if (r == 0) btp ^= m0;
        uint32_t pm = 0;
        for (int l = 0; l < kLE + 2; ++l) {
            int a = -1;
            if (l < kLE) {
                if ((pd.bmask[r] >> l) & 1u) a = pd.reg[r][l];
            } else if (l - kLE < pd.nx[r]) {
                a = pd.xl[r][l - kLE];
            }
            if (a < 0) continue;
            const uint32_t bit = (__popc(pd.B[a] & pd.later[r] & bt) ^ (pd.dflag[r] >> l)) & 1u;
            pm |= bit << a;
        }
        const uint32_t rd = (r == 0 && sh0) ? sgn0 : slot(bt) * 16u;
        if (r == nrounds - 1) {
            sgnb = btp ^ pm;
            thr[r * T_ + tid] = make_uint2(rd, rd);
        } else {
            thr[r * T_ + tid] = make_uint2(rd, slot(btp ^ pm) * 16u);
        }
    }

    // Element address = tile base XOR in-tile offset (the lane and register
    // vectors may have bits at free positions, so the two are not added).
    // Offsets are in bytes from the state pointer.
    T pre[kE];
    const char *sbase = (const char *)state;
    // Tiles that differ only in free bits below the 128-byte line share every
    // line they touch (a pass with fewer than log2(128 / sizeof(T)) contiguous
    // low bits; 2^s partners).  Strided launches run partners at the same
    // time on one XCD: blocks are dealt to the 8 XCDs in turn (block b to XCD
    // b mod 8), and iteration k of block b (tile t0 + k * stride of the loop)
    // runs tile ((k * stride / 2^s + q * 8 + x) << s) | p with x = b mod 8,
    // j = b / 8, p = j mod 2^s, q = j / 2^s: the partners of a tile are the
    // same iteration of blocks b, b + 8, ..., so one fetch of a line from
    // memory serves all of them from that XCD's L2, and their partial-line
    // stores meet there.  Each iteration covers tiles k * stride ..
    // (k + 1) * stride - 1, a bijection when stride is a multiple of 8 * 2^s
    // dividing the tile count; otherwise a block runs the partners one after
    // the other (iteration k runs ((k >> s) * stride + b) * 2^s + (k mod 2^s),
    // a bijection when stride * 2^s divides the tile count).  The mapping
    // only changes the order of independent tiles.  Contiguous ranges (the
    // ensemble kernels) run partners in a row already.
    int sh = 0;
    bool xcd = false;
    if (stride > 1) {
        const int line_bits = sizeof(T) == 8 ? 4 : 3;
        while (sh < pd.n_free && pd.free_pos[sh] < line_bits) ++sh;
        if (t0 >= stride || t1 % stride != 0) sh = 0;
        xcd = sh && stride % (8 << sh) == 0;
        if (sh && !xcd && t1 % (stride << sh) != 0) sh = 0;
    }
    auto tile_off = [&](int64_t ti) {
        if (sh) {
            const int64_t k = (ti - t0) / stride;
            if (xcd) {
                const int64_t x = t0 & 7, j = t0 >> 3;
                const int64_t p = j & ((1 << sh) - 1), q = j >> sh;
                ti = ((k * (stride >> sh) + q * 8 + x) << sh) | p;
            } else {
                ti = (((k >> sh) * stride + t0) << sh) | (k & ((1 << sh) - 1));
            }
        }
        uint64_t xT = 0;
        for (int i = 0; i < pd.n_free; ++i)
            if ((ti >> i) & 1) xT |= (uint64_t)1 << pd.free_pos[i];
        return (OFF)xT * (OFF)sizeof(T);
    };
    // round 0's amplitudes of tile xb into pre[] (register index order)
    auto load_tile = [&](OFF xb) {
        OFF co = xb ^ off_t;
        asm volatile("" : "+v"(co));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) co ^= pv[__builtin_ctz(jj)];
            pre[jj ^ (jj >> 1)] = *(const T *)(sbase + co);
        }
    };
    auto signs = [&](OFF xb) {
        const uint64_t xT = (uint64_t)xb / sizeof(T);
        for (int k = tid; k < m; k += T_) {
            const double2 src = tsrc[k];
            const uint64_t zt = (uint64_t)__double_as_longlong(src.y);
            trec[k].x = (__popcll(zt & xT) & 1) ? -src.x : src.x;
        }
    };

    double re[kE], im[kE];
    auto read16 = [&](uint32_t cs, const uint32_t (&rs)[kLE]) {
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) cs ^= rs[__builtin_ctz(jj)];
            const double2 a = lds_ld(cs);
            re[jj ^ (jj >> 1)] = a.x;
            im[jj ^ (jj >> 1)] = a.y;
        }
    };
    auto write16 = [&](uint32_t cs, const uint32_t (&rs)[kLE]) {
        asm volatile("" : "+v"(cs));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) cs ^= rs[__builtin_ctz(jj)];
            lds_st(cs, make_double2(re[jj ^ (jj >> 1)], im[jj ^ (jj >> 1)]));
        }
    };
    auto from_pre = [&]() {
#pragma unroll
        for (int g = 0; g < kE; ++g) {
            const double2 a = to_c128(pre[g]);
            re[g] = a.x;
            im[g] = a.y;
        }
    };
    // without the prefetch, round 0's amplitudes go straight into re/im
    auto load_regs = [&](OFF xb) {
        OFF co = xb ^ off_t;
        asm volatile("" : "+v"(co));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) co ^= pv[__builtin_ctz(jj)];
            const double2 a = to_c128(*(const T *)(sbase + co));
            re[jj ^ (jj >> 1)] = a.x;
            im[jj ^ (jj >> 1)] = a.y;
        }
    };
    auto store16 = [&](OFF xb) {
        OFF co = xb ^ off_t;
        asm volatile("" : "+v"(co));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) co ^= pv[__builtin_ctz(jj)];
            const int g = jj ^ (jj >> 1);
            from_c128(*(T *)((char *)state + co), make_double2(re[g], im[g]));
        }
    };
    // staging of a staged pass (pivot order, Gray walk over the slots)
    auto scatter_pre = [&]() {
        uint32_t cs = sl_t;
        asm volatile("" : "+v"(cs));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) cs ^= sv[__builtin_ctz(jj)];
            lds_st(cs, to_c128(pre[jj ^ (jj >> 1)]));
        }
    };
    auto scatter_regs = [&]() {
        uint32_t cs = sl_t;
        asm volatile("" : "+v"(cs));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) cs ^= sv[__builtin_ctz(jj)];
            lds_st(cs, make_double2(re[jj ^ (jj >> 1)], im[jj ^ (jj >> 1)]));
        }
    };
    auto gather = [&](OFF xb) {
        uint32_t cs = sl_t;
        OFF co = xb ^ off_t;
        asm volatile("" : "+v"(cs), "+v"(co));
#pragma unroll
        for (int jj = 0; jj < kE; ++jj) {
            if (jj) {
                cs ^= sv[__builtin_ctz(jj)];
                co ^= pv[__builtin_ctz(jj)];
            }
            from_c128(*(T *)((char *)state + co), lds_ld(cs));
        }
    };
    // plain butterflies on register bits 1..nb-1 (they commute)
    auto plain_rest = [&](int nb) {
        if (nb > 1) bfly_ip<1>(re, im);
        if (nb > 2) bfly_ip<2>(re, im);
        if (nb > 3) bfly_ip<3>(re, im);
    };

    // The rounds of one tile.  Step 0 takes its input from pre[] and, with
    // PF, then refills pre[] with the next tile's round-0 amplitudes; the
    // last step stores to HBM.  Every step ends with a block barrier.
    // the sign (-1)^{k.d(t)} of round 0's outputs (see sgn0), flipped in
    // place in the high words
    auto apply_sign0 = [&](uint32_t sgn0) {
#pragma unroll
        for (int g = 0; g < kE; ++g) {
            const uint64_t mm = (uint64_t)((sgn0 << (31 - g)) & 0x80000000u) << 32;
            re[g] = __longlong_as_double((long long)((uint64_t)__double_as_longlong(re[g]) ^ mm));
            im[g] = __longlong_as_double((long long)((uint64_t)__double_as_longlong(im[g]) ^ mm));
        }
    };
    // the CZ between register slots of a round's chunk: a sign per register
    // pattern (bit g of czm), the same for every thread; in place on the
    // high words, before a forward round's butterflies and after a backward
    // round's
    auto apply_cz = [&](uint32_t czm) {
#pragma unroll
        for (int g = 0; g < kE; ++g) {
            const uint64_t mm = (uint64_t)(((czm >> g) & 1u) << 31) << 32;
            re[g] = __longlong_as_double((long long)((uint64_t)__double_as_longlong(re[g]) ^ mm));
            im[g] = __longlong_as_double((long long)((uint64_t)__double_as_longlong(im[g]) ^ mm));
        }
    };
    // exchange of register bits 2, 3 with lane bits 4, 5 (nx of them), and
    // butterflies on register bits 2, 3 (nx of them)
    auto xchg = [&](int nx) {
        if (nx >= 1) exch<2, 4>(re, im);
        if (nx == 2) exch<3, 5>(re, im);
    };
    auto stages_x = [&](int nx) {
        if (nx >= 1) bfly_ip<2>(re, im);
        if (nx == 2) bfly_ip<3>(re, im);
    };

    // The rounds of one tile.  A round other than Lambda's runs butterflies
    // on register bits 0..3, exchanges bits 2, 3 with lane bits 4, 5, and runs
    // butterflies on bits 2, 3 again: forward (from the layout before the
    // exchange) that transforms the register coordinates, then the exchanged
    // ones; backward (from the layout after it) the same sequence transforms
    // the exchanged coordinates first.  Butterflies on different coordinates
    // commute and carry no twiddle outside the Lambda round, so both
    // directions are the same code.  Step 0 of a direct pass finds its input
    // in re/im already and its last step leaves the results there.  Every
    // step ends with a block barrier.
    // One step of the tile's rounds (step `step` of `total`); true when
    // the expectation modes are done with the tile.
    auto one_step = [&](const int step, const int total) -> bool {
            const int r = step < nrounds ? step : 2 * nr - 2 - step;
            const bool lam = step == nrounds - 1;
            const bool fwd = step < nrounds - 1;
            const bool last = step == total - 1;
            const uint2 ab = thr[r * T_ + tid];
            const uint32_t ra = fwd || lam ? ab.x : ab.y;
            const uint32_t wa = fwd ? ab.y : ab.x;
            // uniform register offsets of the layouts read and written
            uint32_t rin[kLE], rout[kLE];
#pragma unroll
            for (int b = 0; b < kLE; ++b) {
                const uint32_t pre_off = s_rs[r * kLE + b], post_off = s_ws[r * kLE + b];
                rin[b] = fwd || lam ? pre_off : post_off;
                rout[b] = fwd ? post_off : pre_off;
            }
            const int nb = __popc(pd.bmask[r]);
            const int nx = pd.nx[r];
            const uint32_t czm = pd.czm[r];
            if (step > 0 || staged) read16(ra, rin);  // (step 0 of a direct pass: in re/im)
            if (!lam) {
                if (sh0 && last) apply_sign0(ab.x);
                if (fwd && czm) apply_cz(czm);
                bfly_fwd<0, false>(re, im);
                if (GEN) {
                    plain_rest(nb);
                    xchg(nx);
                    stages_x(nx);
                } else {
                    bfly_fwd<1, false>(re, im);
                    bfly_fwd<2, false>(re, im);
                    bfly_fwd<3, false>(re, im);
                    exch<2, 4>(re, im);
                    exch<3, 5>(re, im);
                    bfly_fwd<2, false>(re, im);
                    bfly_fwd<3, false>(re, im);
                }
                if (!fwd && czm) apply_cz(czm);
                if (sh0 && step == 0) apply_sign0(ab.x);
                if (!last || staged) write16(wa, rout);  // (else: results stay in re/im)
                __syncthreads();
                return false;
            }
            const bool tw = pd.iflag[r] & 1u;
            if (czm) apply_cz(czm);
            if (nb > 0) {
                if (tw) bfly_fwd<0, true>(re, im);
                else bfly_fwd<0, false>(re, im);
                plain_rest(nb);
                xchg(nx);
                stages_x(nx);
            }
            // phi over the kE register patterns: bucket sums of the signed
            // coefficients, then a kE-point Walsh-Hadamard of the sums
            double A[kE];
            int bk[kE + 1];
#pragma unroll
            for (int w = 0; w <= kE; ++w) bk[w] = s_bk[w];
#pragma unroll
            for (int w = 0; w < kE; ++w) {
                double sacc = 0.0;
                // the sign bit of the coefficient flipped by the parity of
                // the term's mask on the thread's coordinates
#pragma unroll 4
                for (int k = bk[w]; k < bk[w + 1]; ++k) {
                    const double2 rec = trec[k];
                    const uint32_t z = (uint32_t)__double_as_longlong(rec.y);
                    const uint64_t flip = (uint64_t)__popc(z & sgnb) << 63;
                    sacc += __longlong_as_double((long long)((uint64_t)__double_as_longlong(rec.x) ^ flip));
                }
                A[w] = sacc;
            }
#pragma unroll
            for (int b = 0; b < kLE; ++b)
#pragma unroll
                for (int j = 0; j < kE; ++j)
                    if (!((j >> b) & 1)) {
                        const double a0 = A[j], a1 = A[j | (1 << b)];
                        A[j] = a0 + a1;
                        A[j | (1 << b)] = a0 - a1;
                    }
            if (MODE == 1) {
#pragma unroll
                for (int j = 0; j < kE; ++j) acc[0] += (re[j] * re[j] + im[j] * im[j]) * A[j] * scale;
                __syncthreads();
                return true;
            }
            if (MODE == 2) {
                // term k of bucket w: its sign times sum_j |psi_j|^2
                // (-1)^{w.j} (a kE-point Walsh-Hadamard of the thread's
                // probabilities), summed over the wave; lane k mod 64 keeps
                // the running total
                double W[kE];
#pragma unroll
                for (int j = 0; j < kE; ++j) W[j] = (re[j] * re[j] + im[j] * im[j]) * scale;
#pragma unroll
                for (int b = 0; b < kLE; ++b)
#pragma unroll
                    for (int j = 0; j < kE; ++j)
                        if (!((j >> b) & 1)) {
                            const double a0 = W[j], a1 = W[j | (1 << b)];
                            W[j] = a0 + a1;
                            W[j | (1 << b)] = a0 - a1;
                        }
                const int lane = (int)(tid & 63u);
#pragma unroll
                for (int w = 0; w < kE; ++w) {
                    for (int k = bk[w]; k < bk[w + 1]; ++k) {
                        const double2 rec = trec[k];
                        const uint32_t z = (uint32_t)__double_as_longlong(rec.y);
                        const uint64_t flip = (uint64_t)__popc(z & sgnb) << 63;
                        double v = __longlong_as_double((long long)((uint64_t)__double_as_longlong(rec.x) ^ flip)) * W[w];
                        v = wave_sum_f64(v);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if ((k >> 6) == q && lane == (k & 63)) acc[q] += v;
                    }
                }
                __syncthreads();
                return true;
            }
            // (no double-angle steps is the common case: its own loop keeps
            // the halving loop out of the per-amplitude code)
            if (halv == 0) {
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    double cc, ss;
                    cis_scaled<FULL>(A[j], pd.kcos, pd.ksin, cc, ss);
                    const double ar = re[j], ai = im[j];
                    re[j] = fma(ar, cc, -ai * ss);
                    im[j] = fma(ar, ss, ai * cc);
                }
            } else {
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    double cc, ss;
                    cis<FULL>(A[j], halv, cc, ss);
                    cc *= scale;
                    ss *= scale;
                    const double ar = re[j], ai = im[j];
                    re[j] = fma(ar, cc, -ai * ss);
                    im[j] = fma(ar, ss, ai * cc);
                }
            }
            if (nb > 0) {
                stages_x(nx);
                xchg(nx);
                plain_rest(nb);
                if (tw) bfly_bwd<0, true>(re, im);
                else bfly_bwd<0, false>(re, im);
            }
            if (czm) apply_cz(czm);
            if (!last || staged) write16(wa, rout);  // (else: results stay in re/im)
            __syncthreads();
            return false;
    };
    // Step 0 is peeled off the loop: only it can take its input from
    // registers (a direct pass's round 0), every later step reads its input
    // from LDS, so the loop carries no register tile from one step to the
    // next.
    auto transform = [&](OFF xb) {
        const int total = nr > 0 ? 2 * nr - 1 : 1;
        if (!one_step(0, total))
            for (int step = 1; step < total; ++step)
                if (one_step(step, total)) break;
        // a direct pass's results: stored here without the prefetch, else at
        // the top of the next tile (see below)
        if (MODE == 0 && !staged && !PF) store16(xb);
    };

    __syncthreads();
    if (PF) {
        // Software pipeline: step 0 of tile t issues the loads of tile t +
        // stride right after consuming its own, so they overlap the rest of
        // tile t; the stores of tile t are issued after them (one counter
        // tracks loads and stores in issue order, so waiting for the next
        // tile's loads does not wait for these stores).
        // pre[] is converted into re/im (or, staged, scattered to LDS) before
        // the rounds start, and the next tile's loads go into it right away;
        // keeping that outside the round loop keeps pre[] one plain live range.
        // The results of a direct pass stay in re/im until the top of the next
        // tile and are stored right before its prefetched amplitudes are
        // consumed: one counter tracks loads and stores in issue order, and
        // these stores are younger than the loads waited for, so that wait
        // does not include them (in straight-line code the compiler counts
        // them exactly).
        if (t0 < t1) load_tile(tile_off(t0));
        bool have_prev = false;
        OFF xb_prev = 0;
        for (int64_t ti = t0; ti < t1; ti += stride) {
            const OFF xb = tile_off(ti);
            const int64_t tn = ti + stride;
            if (have_prev) store16(xb_prev);
            if (staged) scatter_pre();
            else from_pre();
            if (tn < t1) load_tile(tile_off(tn));
            signs(xb);
            __syncthreads();
            transform(xb);
            if (staged) {
                if (MODE == 0) gather(xb);
                __syncthreads();
            } else {
                have_prev = true;
                xb_prev = xb;
            }
        }
        if (have_prev) store16(xb_prev);
    } else {
        for (int64_t ti = t0; ti < t1; ti += stride) {
            const OFF xb = tile_off(ti);
            load_regs(xb);
            signs(xb);
            if (staged) scatter_regs();
            __syncthreads();
            transform(xb);
            if (staged) {
                if (MODE == 0) gather(xb);
                __syncthreads();
            }
        }
    }
}

// block sum in a fixed order: wave sums, then one value per wave through LDS
// (the slots after the tile-pass arrays)
__device__ __forceinline__ double block_sum_waves(double acc, double *red) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double s2 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s2 += red[w];
    return s2;
}

template <typename T, int MODE, typename OFF, bool GEN>
__global__ void __launch_bounds__(kMaxThreads)
k_tile(T *__restrict__ state, const PassDev *__restrict__ pdp, const uint8_t *__restrict__ ws,
       double tau, double *__restrict__ partial) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    tile_pass<T, MODE, OFF, GEN>(state, pdp, ws, tau, blockIdx.x, pdp->n_tiles, gridDim.x, acc);
    extern __shared__ double2 lds_dyn[];
    if (MODE == 1) {
        const int nrounds = pdp->nr > 0 ? pdp->nr : 1;
        double *red = (double *)((char *)lds_dyn + tile_lds(pdp->D, blockDim.x, nrounds, pdp->m).red);
        const double s2 = block_sum_waves(acc[0], red);
        if (threadIdx.x == 0) partial[blockIdx.x] += s2;
    }
    if (MODE == 2) {
        // per-wave totals of the pass's terms through the (now free) tile
        // area of LDS (2^(D-10) waves x kMaxPassTerms doubles = 2^(D+1)
        // bytes of its 2^(D+4)), then the block's total of term k into
        // partial[block * kMaxPassTerms + k]
        double *red = (double *)lds_dyn;
        const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63u);
        const int nw = (int)(blockDim.x >> 6), m = pdp->m;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wave * kMaxPassTerms + q * 64 + lane] = acc[q];
        __syncthreads();
        for (int k = (int)threadIdx.x; k < m; k += (int)blockDim.x) {
            double s2 = 0.0;
            for (int w = 0; w < nw; ++w) s2 += red[w * kMaxPassTerms + k];
            partial[(int64_t)blockIdx.x * kMaxPassTerms + k] = s2;
        }
    }
}

// Ensemble level launch: segment i is one pass of one instance (its tiles are
// items first_item .. first_item + n_tiles - 1 of a flat list); every block
// takes a contiguous share of the items, so it changes instance rarely.
template <typename P>
__device__ __forceinline__ P *uniform_ptr(P *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}

struct MultiSeg {
    void *state;
    const PassDev *pd;
    const uint8_t *ws;
    double tau;
    int64_t first_item;
    int64_t n_tiles;
};

template <typename T, bool GEN>
__global__ void __launch_bounds__(kMaxThreads)
k_tile_multi(const MultiSeg *__restrict__ segs, int nseg, int64_t total) {
    const int64_t lo = (total * (int64_t)blockIdx.x) / gridDim.x;
    const int64_t hi = (total * (int64_t)(blockIdx.x + 1)) / gridDim.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < nseg; ++i) {
        const MultiSeg sg = segs[i];
        const int64_t a = sg.first_item, b = sg.first_item + sg.n_tiles;
        const int64_t s0 = a > lo ? a : lo, s1 = b < hi ? b : hi;
        if (s0 >= s1) continue;
        // the record is read from a pointer held in memory; it is read-only
        // while kernels run, so it is addressed as constant memory with a
        // wave-uniform address: its fields then come in through scalar
        // loads, as from k_tile's kernel argument
        typedef const __attribute__((address_space(4))) PassDev *ConstRec;
        tile_pass<T, 0, uint32_t, GEN, ConstRec>((T *)sg.state, (ConstRec)uniform_ptr(sg.pd), sg.ws,
                                                 sg.tau, s0 - a, s1 - a, 1, acc);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_norm2(const T *__restrict__ a, int64_t dim, double *__restrict__ partial) {
    __shared__ double red[kBlock];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 v = ld_amp(a, i);
        acc += v.x * v.x + v.y * v.y;
    }
    double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_inner(const T *__restrict__ a, const T *__restrict__ b, int64_t dim,
        double *__restrict__ partial) {
    __shared__ double red[kBlock];
    double re = 0.0, im = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 u = ld_amp(a, i), v = ld_amp(b, i);
        re += u.x * v.x + u.y * v.y;
        im += u.x * v.y - u.y * v.x;
    }
    double s1 = block_sum(re, red);
    double s2 = block_sum(im, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s1;
        partial[2 * blockIdx.x + 1] = s2;
    }
}

// per-term totals of MODE 2: out[k] = sum over blocks b < count of
// partial[b * kMaxPassTerms + k] in a fixed order.  A block takes 64 terms
// (one per lane, so that a wave reads 64 neighbouring values of one block's
// row); wave q of the 4 adds rows q, q + 4, ..., and the four wave sums are
// added in wave order.
constexpr int kTermFinalThreads = 256;
__global__ void __launch_bounds__(kTermFinalThreads)
k_term_final(const double *__restrict__ partial, int count, int m, double *__restrict__ out) {
    __shared__ double red[kTermFinalThreads];
    const int lane = (int)(threadIdx.x & 63u), q = (int)(threadIdx.x >> 6);
    const int k = (int)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (k < m)
        for (int b = q; b < count; b += kTermFinalThreads / 64) s += partial[(int64_t)b * kMaxPassTerms + k];
    red[threadIdx.x] = s;
    __syncthreads();
    if (q == 0 && k < m) out[k] = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
}

// final sum of `count` interleaved groups of `width` (1 or 2) partials in a
// fixed order: thread t adds partials t, t + kFinalThreads, ... in turn, then
// a binary tree of the same shape on every call combines the threads
constexpr int kFinalThreads = 256;
__global__ void __launch_bounds__(kFinalThreads)
k_final(const double *__restrict__ partial, int count, int width, double *__restrict__ out) {
    __shared__ double red[2][kFinalThreads];
    const int t = threadIdx.x;
    for (int w = 0; w < width; ++w) {
        double s = 0.0;
        for (int i = t; i < count; i += kFinalThreads) s += partial[(int64_t)i * width + w];
        red[w][t] = s;
    }
    __syncthreads();
    for (int h = kFinalThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int w = 0; w < width; ++w) red[w][t] += red[w][t + h];
        __syncthreads();
    }
    if (t < width) out[t] = red[t][0];
}

__global__ void k_fill(double *__restrict__ p, int count, double v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
constexpr int kPartialSlots = 2048;  // per-block partial sums in the scratch

static sd_status hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess)
        return fail(SD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return SD_OK;
}

static int g_num_cu = 0;
static bool g_generic = false;   // SD_GENERIC_KERNEL=1 routes every pass to k_pass
static std::once_flag g_once;
static sd_status g_init_status = SD_OK;

template <typename K>
static void set_lds(K kernel, int bytes) {
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// The tile kernels address LDS by absolute byte offsets with the tile at 0:
// they must not have static LDS (it would be placed before the dynamic part).
template <typename K>
static bool no_static_lds(K kernel) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, (const void *)kernel) != hipSuccess) return false;
    return a.sharedSizeBytes == 0;
}

static void init_device_props() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) g_num_cu = prop.multiProcessorCount;
    if (const char *e = std::getenv("SD_GENERIC_KERNEL")) g_generic = std::atoi(e) != 0;
    const int lds_generic = (1 << kMaxTileLog2) * 16;
    set_lds(k_pass<float2, 0>, lds_generic);
    set_lds(k_pass<float2, 1>, lds_generic);
    set_lds(k_pass<double2, 0>, lds_generic);
    set_lds(k_pass<double2, 1>, lds_generic);
    set_lds(k_pass<float2, 2>, lds_generic);
    set_lds(k_pass<double2, 2>, lds_generic);
    const int lds = (int)kTileLdsMax;
    bool ok = true;
    auto prep = [&](auto kernel) {
        set_lds(kernel, lds);
        ok = ok && no_static_lds(kernel);
    };
    prep(k_tile<float2, 0, uint32_t, false>);
    prep(k_tile<float2, 0, uint32_t, true>);
    prep(k_tile<double2, 0, uint32_t, false>);
    prep(k_tile<double2, 0, uint32_t, true>);
    prep(k_tile<float2, 0, uint64_t, false>);
    prep(k_tile<float2, 0, uint64_t, true>);
    prep(k_tile<double2, 0, uint64_t, false>);
    prep(k_tile<double2, 0, uint64_t, true>);
    prep(k_tile<float2, 1, uint32_t, true>);
    prep(k_tile<float2, 2, uint32_t, true>);
    prep(k_tile<double2, 2, uint32_t, true>);
    prep(k_tile<float2, 2, uint64_t, true>);
    prep(k_tile<double2, 2, uint64_t, true>);
    prep(k_tile<double2, 1, uint32_t, true>);
    prep(k_tile<float2, 1, uint64_t, true>);
    prep(k_tile<double2, 1, uint64_t, true>);
    prep(k_tile_multi<float2, false>);
    prep(k_tile_multi<float2, true>);
    prep(k_tile_multi<double2, false>);
    prep(k_tile_multi<double2, true>);
    if (!ok) g_init_status = fail(SD_ERR_INTERNAL, "tile kernels were built with static LDS");
}

// Resident blocks of k_tile per CU: the kernel needs up to 256 VGPRs per
// lane, i.e. two waves per SIMD, eight per CU; a tile of 2^D amplitudes has
// 2^(D-4) threads.  (The LDS of that many tiles fits in 160 KB.)
static int blocks_per_cu(int D) {
    const int waves = std::max(1, (1 << (D - kLE)) / 64);
    return std::max(1, 8 / waves);
}

static int grid_for(int64_t tiles) {
    std::call_once(g_once, init_device_props);
    int cap = std::max(1, g_num_cu) * 2;
    return (int)std::min<int64_t>(tiles, cap);
}

template <typename T, int MODE>
static sd_status launch_pass(const sd_plan_t *p, sd_dtype dt, int i, void *state, double tau,
                             hipStream_t s) {
    const PassHost &ph = p->prog[dt].passes[i];
    const uint8_t *ws = (const uint8_t *)p->ws;
    const PassDev *pd = (const PassDev *)(ws + p->ws_off_prog[dt] + (int64_t)i * sizeof(PassDev));
    double *partial = (double *)(ws + p->ws_off_scratch);
    const int64_t tiles = (int64_t)1 << (p->n - ph.D);
    const int grid_evolve = grid_for(tiles);  // also runs the one-time LDS attribute setup
    if (g_init_status != SD_OK) return fail(g_init_status, "device initialisation failed");
    const int grid = MODE == 1 ? (int)std::min<int64_t>(tiles, kPartialSlots / 2) : grid_evolve;
    if (ph.D > kMaxTileLog2 || (int)ph.terms.size() > kMaxPassTerms)
        return fail(SD_ERR_INTERNAL, "pass exceeds the on-chip tile limits");
    const size_t lds = (size_t)16 << ph.D;
    static_assert(kLE == kRegBits, "register round width mismatch");
    if (ph.D >= kTileMinD && !g_generic) {
        const int threads = 1 << (ph.D - kLE);
        // tiles of 2^13 fill one CU's LDS: one block per CU, next tile
        // prefetched into registers; smaller tiles run two or more blocks per CU
        const int per_cu = blocks_per_cu(ph.D);
        const size_t lds_tile = tile_lds(ph.D, threads, std::max(ph.nr, 1), (int)ph.terms.size()).total;
        const int g2 = MODE == 1 ? grid
                                 : (int)std::min<int64_t>(tiles, (int64_t)std::max(1, g_num_cu) * per_cu);
        // byte offsets inside the state fit 32 bits up to 4 GiB
        const bool narrow = ((uint64_t)sizeof(T) << p->n) <= ((uint64_t)1 << 32);
        // the expectation (MODE 1) always takes the general round code
        const bool gen = MODE == 1 || !ph.full_rounds;
        if (narrow && gen)
            hipLaunchKernelGGL((k_tile<T, MODE, uint32_t, true>), dim3(g2), dim3(threads), lds_tile, s,
                               (T *)state, pd, ws, tau, partial);
        else if (narrow)
            hipLaunchKernelGGL((k_tile<T, 0, uint32_t, false>), dim3(g2), dim3(threads), lds_tile, s,
                               (T *)state, pd, ws, tau, partial);
        else if (gen)
            hipLaunchKernelGGL((k_tile<T, MODE, uint64_t, true>), dim3(g2), dim3(threads), lds_tile, s,
                               (T *)state, pd, ws, tau, partial);
        else
            hipLaunchKernelGGL((k_tile<T, 0, uint64_t, false>), dim3(g2), dim3(threads), lds_tile, s,
                               (T *)state, pd, ws, tau, partial);
        return hip_check(hipGetLastError(), "k_tile launch");
    }
    hipLaunchKernelGGL((k_pass<T, MODE>), dim3(grid), dim3(kBlock), lds, s, (T *)state, pd, ws,
                       tau, partial);
    return hip_check(hipGetLastError(), "k_pass launch");
}

// Group applications of one step as (group, fraction of dt): order 1 the
// groups in order; order 2 the symmetric (Strang) sequence; order 4 Suzuki's
// fractal S2(p) S2(p) S2(1 - 4p) S2(p) S2(p), p = 1 / (4 - 4^(1/3)), with the
// second-order sequences not merged at their boundaries.
static std::vector<std::pair<int, double>> step_schedule(int K, int order) {
    std::vector<std::pair<int, double>> seq;
    if (order == 4) {
        const double p = 1.0 / (4.0 - std::cbrt(4.0));
        for (double w : {p, p, 1.0 - 4.0 * p, p, p})
            for (auto &gf : step_schedule(K, 2)) seq.push_back({gf.first, gf.second * w});
    } else if (order == 1 || K == 1) {
        for (int g = 0; g < K; ++g) seq.push_back({g, 1.0});
    } else {
        for (int g = 0; g < K - 1; ++g) seq.push_back({g, 0.5});
        seq.push_back({K - 1, 1.0});
        for (int g = K - 2; g >= 0; --g) seq.push_back({g, 0.5});
    }
    return seq;
}

// The group applications of `steps` steps, merged where one group follows
// itself: G_g(a) G_g(b) = G_g(a + b) exactly (a group is one exponential),
// and each merge saves a pass over the state per sub-group (and, complex64,
// one rounding of every amplitude).  Inside a step that joins the halves at
// the boundaries of the second-order steps of order 4; across steps it joins
// the last application of a step with the first of the next one when they
// are the same group (order 2: G_0(dt/2) G_0(dt/2) = G_0(dt)).  The calls of
// `steps` steps then run
//   prologue, core x (steps - 1), epilogue
// with core the step from its second application on, ending in the joined
// one.  Without a join across steps the prologue is empty and core and
// epilogue are the (inside-merged) step.  A result is that of `steps` whole
// steps; only the grouping of the applications differs.
struct CallSchedule {
    std::vector<std::pair<int, double>> pro, core, epi;
};

static CallSchedule call_schedule(int K, int order) {
    std::vector<std::pair<int, double>> m;
    for (auto &gf : step_schedule(K, order)) {
        if (!m.empty() && m.back().first == gf.first)
            m.back().second += gf.second;
        else
            m.push_back(gf);
    }
    CallSchedule cs;
    if (m.size() >= 2 && m.front().first == m.back().first) {
        cs.pro.push_back(m.front());
        cs.core.assign(m.begin() + 1, m.end() - 1);
        cs.core.push_back({m.back().first, m.back().second + m.front().second});
        cs.epi.assign(m.begin() + 1, m.end());
    } else {
        cs.core = m;
        cs.epi = m;
    }
    return cs;
}

}  // namespace sd

using namespace sd;

extern "C" sd_status sd_bind_workspace(sd_plan_t *p, void *dev_ptr, size_t bytes, void *stream) {
    if (!p || !dev_ptr) return fail(SD_ERR_ARG, "sd_bind_workspace: null argument");
    if ((int64_t)bytes < p->ws_needed)
        return fail(SD_ERR_WORKSPACE, "workspace of " + std::to_string(bytes) + " bytes < required " +
                                          std::to_string(p->ws_needed));
    if (((uintptr_t)dev_ptr) & 255) return fail(SD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    for (int d = 0; d < 2; ++d) {
        std::vector<uint8_t> buf;
        pack_program(p->prog[d], p->n, p->ws_off_prog[d], buf);
        if (!buf.empty()) {
            sd_status st = hip_check(hipMemcpyAsync((uint8_t *)dev_ptr + p->ws_off_prog[d], buf.data(),
                                                    buf.size(), hipMemcpyHostToDevice, s),
                                     "workspace upload");
            if (st != SD_OK) return st;
            // buf is pageable: the copy is staged before hipMemcpyAsync returns
            st = hip_check(hipStreamSynchronize(s), "workspace upload sync");
            if (st != SD_OK) return st;
        }
    }
    if (!p->layer_data.empty()) {
        sd_status st = hip_check(hipMemcpyAsync((uint8_t *)dev_ptr + p->ws_off_layers, p->layer_data.data(),
                                                p->layer_data.size() * sizeof(uint64_t), hipMemcpyHostToDevice,
                                                s),
                                 "layer table upload");
        if (st == SD_OK) st = hip_check(hipStreamSynchronize(s), "layer table upload sync");
        if (st != SD_OK) return st;
    }
    p->ws = dev_ptr;
    p->ws_bytes = bytes;
    p->bound = true;
    ++p->bind_epoch;
    return SD_OK;
}

extern "C" sd_status sd_evolve(const sd_plan_t *p, void *state, sd_dtype dtype, double dt,
                               int64_t steps, int32_t order, void *stream) {
    if (!p || !state) return fail(SD_ERR_ARG, "sd_evolve: null argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_evolve: bad dtype");
    if (order != 1 && order != 2 && order != 4)
        return fail(SD_ERR_ARG, "sd_evolve: order must be 1, 2 or 4");
    if (steps < 0) return fail(SD_ERR_ARG, "sd_evolve: steps < 0");
    if (!std::isfinite(dt)) return fail(SD_ERR_ARG, "sd_evolve: non-finite dt");
    if (!p->bound) return fail(SD_ERR_WORKSPACE, "sd_evolve: no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    const Program &P = p->prog[dtype];
    const int K = (int)p->groups.size();
    if (K == 0 || steps == 0) return SD_OK;
    const CallSchedule cs = call_schedule(K, order);
    auto run = [&](const std::vector<std::pair<int, double>> &seq) -> sd_status {
        for (auto &gf : seq) {
            const double tau = dt * gf.second;
            if (p->mode != SD_MODE_TILES) {
                sd_status r = run_group_reference(p, state, dtype, gf.first, tau, s);
                if (r != SD_OK) return r;
                continue;
            }
            for (int i = P.group_first[gf.first]; i < P.group_first[gf.first + 1]; ++i) {
                sd_status r = dtype == SD_C64 ? launch_pass<float2, 0>(p, dtype, i, state, tau, s)
                                              : launch_pass<double2, 0>(p, dtype, i, state, tau, s);
                if (r != SD_OK) return r;
            }
        }
        return SD_OK;
    };
    sd_status r = run(cs.pro);
    for (int64_t st = 1; st < steps && r == SD_OK; ++st) r = run(cs.core);
    if (r == SD_OK) r = run(cs.epi);
    return r;
}

extern "C" sd_status sd_expectation(const sd_plan_t *p, const void *state, sd_dtype dtype,
                                    double *energy, void *stream) {
    if (!p || !state || !energy) return fail(SD_ERR_ARG, "sd_expectation: null argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_expectation: bad dtype");
    if (!p->bound) return fail(SD_ERR_WORKSPACE, "sd_expectation: no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    double *partial = (double *)((uint8_t *)p->ws + p->ws_off_scratch);
    double *out = partial + kPartialSlots;
    hipLaunchKernelGGL(k_fill, dim3(8), dim3(256), 0, s, partial, kPartialSlots, 0.0);
    sd_status r = hip_check(hipGetLastError(), "fill");
    if (r != SD_OK) return r;
    const Program &P = p->prog[dtype];
    int maxgrid = 1;
    for (int i = 0; i < (int)P.passes.size(); ++i) {
        r = dtype == SD_C64 ? launch_pass<float2, 1>(p, dtype, i, (void *)state, 0.0, s)
                            : launch_pass<double2, 1>(p, dtype, i, (void *)state, 0.0, s);
        if (r != SD_OK) return r;
        maxgrid = std::max<int>(maxgrid, (int)std::min<int64_t>((int64_t)1 << (p->n - P.passes[i].D),
                                                                 kPartialSlots / 2));
    }
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kFinalThreads), 0, s, partial, maxgrid, 1, out);
    r = hip_check(hipGetLastError(), "final reduce");
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(energy, out, sizeof(double), hipMemcpyDeviceToHost, s), "copy energy");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_expectation sync");
}

extern "C" sd_status sd_term_expectations(const sd_plan_t *p, const void *state, sd_dtype dtype,
                                          double *out, void *stream) {
    if (!p || !state || !out) return fail(SD_ERR_ARG, "sd_term_expectations: null argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_term_expectations: bad dtype");
    if (!p->bound) return fail(SD_ERR_WORKSPACE, "sd_term_expectations: no workspace bound");
    std::call_once(g_once, init_device_props);
    if (g_init_status != SD_OK) return fail(g_init_status, "device initialisation failed");
    hipStream_t s = (hipStream_t)stream;
    const uint8_t *ws = (const uint8_t *)p->ws;
    double *partial = (double *)(ws + p->ws_off_terms);
    double *res = partial + (int64_t)kTermGrid * kMaxPassTerms;
    const Program &P = p->prog[dtype];
    int64_t off = 0;
    for (int i = 0; i < (int)P.passes.size(); ++i) {
        const PassHost &ph = P.passes[i];
        const int m = (int)ph.terms.size();
        if (m == 0) continue;
        if (ph.D > kMaxTileLog2 || m > kMaxPassTerms)
            return fail(SD_ERR_INTERNAL, "pass exceeds the on-chip tile limits");
        const PassDev *pd = (const PassDev *)(ws + p->ws_off_prog[dtype] + (int64_t)i * sizeof(PassDev));
        int grid = (int)std::min<int64_t>((int64_t)1 << (p->n - ph.D), kTermGrid);
        if (ph.D >= kTileMinD && !g_generic) {
            // as many blocks as fit the CUs at once (several per CU for
            // tiles below 2^13)
            grid = std::min(grid, std::max(1, g_num_cu) * blocks_per_cu(ph.D));
            // the tile kernel's forward rounds, then per-term sums in the
            // Lambda round (the general round code, as for the expectation)
            const int threads = 1 << (ph.D - kLE);
            const size_t lds_tile = tile_lds(ph.D, threads, std::max(ph.nr, 1), m).total;
            const bool narrow = ((uint64_t)(dtype == SD_C64 ? sizeof(float2) : sizeof(double2)) << p->n) <=
                                ((uint64_t)1 << 32);
            void *st = const_cast<void *>(state);
            if (dtype == SD_C64 && narrow)
                hipLaunchKernelGGL((k_tile<float2, 2, uint32_t, true>), dim3(grid), dim3(threads), lds_tile, s,
                                   (float2 *)st, pd, ws, 0.0, partial);
            else if (dtype == SD_C64)
                hipLaunchKernelGGL((k_tile<float2, 2, uint64_t, true>), dim3(grid), dim3(threads), lds_tile, s,
                                   (float2 *)st, pd, ws, 0.0, partial);
            else if (narrow)
                hipLaunchKernelGGL((k_tile<double2, 2, uint32_t, true>), dim3(grid), dim3(threads), lds_tile, s,
                                   (double2 *)st, pd, ws, 0.0, partial);
            else
                hipLaunchKernelGGL((k_tile<double2, 2, uint64_t, true>), dim3(grid), dim3(threads), lds_tile, s,
                                   (double2 *)st, pd, ws, 0.0, partial);
        } else {
            const size_t lds = (size_t)16 << ph.D;
            if (dtype == SD_C64)
                hipLaunchKernelGGL((k_pass<float2, 2>), dim3(grid), dim3(kBlock), lds, s, (float2 *)state, pd,
                                   ws, 0.0, partial);
            else
                hipLaunchKernelGGL((k_pass<double2, 2>), dim3(grid), dim3(kBlock), lds, s, (double2 *)state,
                                   pd, ws, 0.0, partial);
        }
        sd_status r = hip_check(hipGetLastError(), "term expectation pass launch");
        if (r != SD_OK) return r;
        hipLaunchKernelGGL(k_term_final, dim3((m + 63) / 64), dim3(kTermFinalThreads), 0, s, partial, grid, m,
                           res + off);
        r = hip_check(hipGetLastError(), "term reduce");
        if (r != SD_OK) return r;
        off += m;
    }
    std::vector<double> host((size_t)off);
    if (off) {
        sd_status r = hip_check(hipMemcpyAsync(host.data(), res, (size_t)off * sizeof(double),
                                               hipMemcpyDeviceToHost, s), "copy term values");
        if (r != SD_OK) return r;
    }
    sd_status r = hip_check(hipStreamSynchronize(s), "sd_term_expectations sync");
    if (r != SD_OK) return r;
    for (size_t k = 0; k < p->terms.size(); ++k) out[k] = 0.0;
    off = 0;
    for (const PassHost &ph : P.passes)
        for (size_t j = 0; j < ph.terms.size(); ++j) out[ph.terms[j]] = host[(size_t)off++];
    return SD_OK;
}

// Per-block partial sums of the stand-alone reductions: up to kPartialSlots
// blocks, two values each (sd_inner), then the two final values.
constexpr int64_t kReductionScratchBytes = (int64_t)(2 * kPartialSlots + 64) * (int64_t)sizeof(double);

static sd_status check_scratch(void *scratch, size_t bytes, const char *who) {
    if (!scratch) return fail(SD_ERR_ARG, std::string(who) + ": null scratch");
    if ((int64_t)bytes < kReductionScratchBytes)
        return fail(SD_ERR_WORKSPACE, std::string(who) + ": scratch of " + std::to_string(bytes) +
                                          " bytes < required " + std::to_string(kReductionScratchBytes));
    if (((uintptr_t)scratch) & 7) return fail(SD_ERR_WORKSPACE, std::string(who) + ": scratch not 8-byte aligned");
    return SD_OK;
}

extern "C" int64_t sd_reduction_scratch_bytes(void) { return kReductionScratchBytes; }

namespace sd {
// norm or inner product over 2^n amplitudes into buf[2 * kPartialSlots ...]
// (width 1: norm of a; width 2: re, im of <a|b>), fixed summation order
static sd_status launch_reduction(const void *a, const void *b, sd_dtype dtype, int32_t n, double *buf,
                                  hipStream_t s) {
    const int64_t dim = (int64_t)1 << n;
    const int grid = (int)std::min<int64_t>(kPartialSlots, (dim + kBlock - 1) / kBlock);
    if (!b) {
        if (dtype == SD_C64)
            hipLaunchKernelGGL(k_norm2<float2>, dim3(grid), dim3(kBlock), 0, s, (const float2 *)a, dim, buf);
        else
            hipLaunchKernelGGL(k_norm2<double2>, dim3(grid), dim3(kBlock), 0, s, (const double2 *)a, dim, buf);
    } else if (dtype == SD_C64) {
        hipLaunchKernelGGL(k_inner<float2>, dim3(grid), dim3(kBlock), 0, s, (const float2 *)a,
                           (const float2 *)b, dim, buf);
    } else {
        hipLaunchKernelGGL(k_inner<double2>, dim3(grid), dim3(kBlock), 0, s, (const double2 *)a,
                           (const double2 *)b, dim, buf);
    }
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kFinalThreads), 0, s, buf, grid, b ? 2 : 1,
                       buf + 2 * kPartialSlots);
    return hip_check(hipGetLastError(), b ? "inner launch" : "norm2 launch");
}
}  // namespace sd

extern "C" sd_status sd_norm2(const void *state, sd_dtype dtype, int32_t n, double *out, void *scratch,
                              size_t scratch_bytes, void *stream) {
    if (!state || !out) return fail(SD_ERR_ARG, "sd_norm2: null argument");
    if (n < 0 || n > 40) return fail(SD_ERR_RANGE, "sd_norm2: n_qubits out of range");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_norm2: bad dtype");
    sd_status r = check_scratch(scratch, scratch_bytes, "sd_norm2");
    if (r != SD_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    double *buf = (double *)scratch;
    r = launch_reduction(state, nullptr, dtype, n, buf, s);
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(out, buf + 2 * kPartialSlots, sizeof(double), hipMemcpyDeviceToHost, s),
                  "copy norm");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_norm2 sync");
}

extern "C" sd_status sd_inner(const void *a, const void *b, sd_dtype dtype, int32_t n, double *out,
                              void *scratch, size_t scratch_bytes, void *stream) {
    if (!a || !b || !out) return fail(SD_ERR_ARG, "sd_inner: null argument");
    if (n < 0 || n > 40) return fail(SD_ERR_RANGE, "sd_inner: n_qubits out of range");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_inner: bad dtype");
    sd_status r = check_scratch(scratch, scratch_bytes, "sd_inner");
    if (r != SD_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    double *buf = (double *)scratch;
    r = launch_reduction(a, b, dtype, n, buf, s);
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(out, buf + 2 * kPartialSlots, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, s),
                  "copy inner");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_inner sync");
}

// ---------------------------------------------------------------------------
// sd_inner_noalloc: sd_inner with its per-block partial sums in a file-scope
// device array instead of caller scratch.  Each GPU holds its own copy of
// the array; its device address is looked up once per device (on the first
// call with that device current) and kept.  Calls on one GPU share the
// array, so calls that overlap on one GPU (other streams, other threads)
// race; the partials are written before they are read, nothing needs
// clearing.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocSlots = (int)(kReductionScratchBytes / (int64_t)sizeof(double));
static __device__ __align__(256) double scratch[kNoAllocSlots];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kNoAllocDevices] = {};  // by device ordinal; null = not looked up yet

sd_status noalloc_scratch(double **out) {
    int dev = -1;
    sd_status r = hip_check(hipGetDevice(&dev), "sd_inner_noalloc: hipGetDevice");
    if (r != SD_OK) return r;
    if (dev < 0 || dev >= kNoAllocDevices) return fail(SD_ERR_RANGE, "sd_inner_noalloc: device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        r = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                      "sd_inner_noalloc: hipGetSymbolAddress(scratch)");
        if (r != SD_OK) return r;
        if (!ptr) return fail(SD_ERR_HIP, "sd_inner_noalloc: null address for the static scratch");
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return SD_OK;
}
}  // namespace

extern "C" sd_status sd_inner_noalloc(const void *a, const void *b, sd_dtype dtype, int32_t n,
                                      double *out, void *stream) {
    if (!a || !b || !out) return fail(SD_ERR_ARG, "sd_inner_noalloc: null argument");
    if (n < 0 || n > 40)
        return fail(SD_ERR_RANGE, "sd_inner_noalloc: n_qubits " + std::to_string(n) +
                                      " outside 0..40");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_inner_noalloc: bad dtype");
    double *buf = nullptr;
    sd_status r = noalloc_scratch(&buf);
    if (r != SD_OK) return r;
    static_assert(2 * kPartialSlots + 2 <= kNoAllocSlots, "static scratch too small");
    hipStream_t s = (hipStream_t)stream;
    r = launch_reduction(a, b, dtype, n, buf, s);
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(out, buf + 2 * kPartialSlots, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, s),
                  "sd_inner_noalloc: copy result");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_inner_noalloc sync");
}

extern "C" sd_status sd_sync(void *stream) {
    sd_status r = hip_check(hipStreamSynchronize((hipStream_t)stream), "sd_sync");
    if (r != SD_OK) return r;
    return hip_check(hipGetLastError(), "sd_sync (async error)");
}

namespace sd {
// the options of candidate i of an autotuning run
static sd_plan_options autotune_options(const sd_plan_options &opt, sd_dtype dtype, int cand) {
    sd_plan_options o = opt;
    if (dtype == SD_C64) o.tile_log2_c64 = cand;
    else o.tile_log2_c128 = cand;
    o.small_state_tiles = 0;  // (each candidate at its own size)
    if ((dtype == SD_C64 ? o.coalesce_log2_c64 : o.coalesce_log2_c128) >= cand) {
        // (the coalescing default must stay below the tile)
        if (dtype == SD_C64) o.coalesce_log2_c64 = std::min(4, cand - 1);
        else o.coalesce_log2_c128 = std::min(3, cand - 1);
    }
    return o;
}

static sd_status autotune_check(const sd_hamiltonian *h, sd_dtype dtype, const int32_t *candidates,
                                int32_t n_candidates) {
    if (!h || !candidates || n_candidates < 1) return fail(SD_ERR_ARG, "sd_autotune: bad argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_autotune: bad dtype");
    for (int i = 0; i < n_candidates; ++i)
        if (candidates[i] < kMinTileLog2 || candidates[i] > kMaxTileLog2)
            return fail(SD_ERR_RANGE, "sd_autotune: candidate tile size out of range");
    return SD_OK;
}
}  // namespace sd

extern "C" sd_status sd_autotune_workspace_bytes(const sd_hamiltonian *h, const sd_plan_options *base,
                                                 sd_dtype dtype, const int32_t *candidates,
                                                 int32_t n_candidates, int64_t *bytes) {
    if (!bytes) return fail(SD_ERR_ARG, "sd_autotune_workspace_bytes: null argument");
    sd_status r = autotune_check(h, dtype, candidates, n_candidates);
    if (r != SD_OK) return r;
    sd_plan_options opt;
    sd_plan_options_default(&opt);
    if (base) opt = *base;
    int64_t most = 0;
    for (int i = 0; i < n_candidates; ++i) {
        const sd_plan_options o = autotune_options(opt, dtype, candidates[i]);
        sd_plan_t *p = nullptr;
        r = sd_plan(h, &o, &p);
        if (r != SD_OK) return r;
        most = std::max<int64_t>(most, p->ws_needed);
        sd_plan_destroy(p);
    }
    *bytes = most;
    return SD_OK;
}

extern "C" sd_status sd_autotune_tiles(const sd_hamiltonian *h, const sd_plan_options *base,
                                       sd_dtype dtype, void *state, double dt, int32_t order,
                                       int32_t steps, const int32_t *candidates, int32_t n_candidates,
                                       void *workspace, size_t workspace_bytes,
                                       sd_plan_options *best, double *seconds, void *stream) {
    if (!state || !best || steps < 1 || !workspace)
        return fail(SD_ERR_ARG, "sd_autotune_tiles: bad argument");
    sd_status r = autotune_check(h, dtype, candidates, n_candidates);
    if (r != SD_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    sd_plan_options opt;
    sd_plan_options_default(&opt);
    if (base) opt = *base;
    double best_t = -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    r = hip_check(hipEventCreate(&e0), "event");
    if (r == SD_OK) r = hip_check(hipEventCreate(&e1), "event");
    for (int i = 0; i < n_candidates && r == SD_OK; ++i) {
        const sd_plan_options o = autotune_options(opt, dtype, candidates[i]);
        sd_plan_t *p = nullptr;
        r = sd_plan(h, &o, &p);
        if (r != SD_OK) break;
        // (a previous candidate's kernels may still read the workspace the
        // new programs are uploaded into: sd_bind_workspace orders the upload
        // on the same stream)
        r = sd_bind_workspace(p, workspace, workspace_bytes, stream);
        if (r == SD_OK) r = sd_evolve(p, state, dtype, dt, 1, order, stream);
        if (r == SD_OK) r = hip_check(hipEventRecord(e0, s), "event record");
        if (r == SD_OK) r = sd_evolve(p, state, dtype, dt, steps, order, stream);
        if (r == SD_OK) r = hip_check(hipEventRecord(e1, s), "event record");
        if (r == SD_OK) r = hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        if (r == SD_OK) r = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
        sd_plan_destroy(p);
        if (r != SD_OK) break;
        const double t = (double)ms / 1e3 / steps;
        if (seconds) seconds[i] = t;
        if (best_t < 0 || t < best_t) {
            best_t = t;
            *best = o;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    return r;
}

// ---------------------------------------------------------------------------
// ensemble
// ---------------------------------------------------------------------------
// Instances are independent; within an instance the passes of a step are
// sequential.  Level l of a part of a call (see call_schedule: prologue,
// core step, epilogue) holds pass l of that part's pass sequence of every
// instance that has one; a level is one k_tile_multi launch over all its
// instances' tiles (grouped by tile size), so a part costs as many launches
// as the longest instance sequence, whatever the number of instances.  Each
// part's launches are captured once as a HIP graph on an internal stream
// and replayed: a call of S steps replays the prologue once, the core S - 1
// times and the epilogue once, exactly as sd_evolve runs each instance.
constexpr int kParts = 3;  // prologue, core, epilogue

struct sd_ensemble {
    std::vector<const sd_plan_t *> plans;
    sd_dtype dtype = SD_C64;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t ws_needed = 0;
    int64_t part_bytes = 0;  // segment table bytes of one part
    int max_levels = 0;
    // graph cache
    hipStream_t cstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph[kParts] = {};
    hipGraphExec_t exec[kParts] = {};
    bool cached = false;
    double g_dt = 0;
    int g_order = 0;
    std::vector<void *> g_states;
    std::vector<const void *> g_plan_ws;  // each plan's workspace when the graphs were built
    std::vector<int> g_small;   // instances run by single-instance pass launches (in the same graphs)
    void drop_graphs() {
        for (int q = 0; q < kParts; ++q) {
            if (exec[q]) (void)hipGraphExecDestroy(exec[q]);
            if (graph[q]) (void)hipGraphDestroy(graph[q]);
            exec[q] = nullptr;
            graph[q] = nullptr;
        }
        cached = false;
    }
    ~sd_ensemble() {
        drop_graphs();
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (cstream) (void)hipStreamDestroy(cstream);
    }
};

namespace {
// group applications of one part (0 prologue, 1 core, 2 epilogue) of a call
const std::vector<std::pair<int, double>> &part_of(const CallSchedule &cs, int q) {
    return q == 0 ? cs.pro : q == 1 ? cs.core : cs.epi;
}

// pass indices of one part of a call of an instance, with the fraction of dt
// of each
std::vector<std::pair<int, double>> part_passes(const sd_plan_t *p, sd_dtype dt, int order, int q) {
    std::vector<std::pair<int, double>> out;
    const Program &P = p->prog[dt];
    const CallSchedule cs = call_schedule((int)p->groups.size(), order);
    for (auto &gf : part_of(cs, q))
        for (int i = P.group_first[gf.first]; i < P.group_first[gf.first + 1]; ++i)
            out.push_back({i, gf.second});
    return out;
}
}  // namespace

extern "C" sd_status sd_ensemble_create(const sd_plan_t *const *plans, int32_t count, sd_dtype dtype,
                                        sd_ensemble **out) {
    if (!plans || !out || count <= 0) return fail(SD_ERR_ARG, "sd_ensemble_create: bad argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_ensemble_create: bad dtype");
    *out = nullptr;
    sd_ensemble *e = new sd_ensemble();
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) {
            delete e;
            return fail(SD_ERR_ARG, "sd_ensemble_create: null plan");
        }
        e->plans.push_back(plans[i]);
        // (segment tables for the longest part of any order, so that one
        // workspace serves every order)
        for (int order : {1, 2, 4})
            for (int q = 0; q < kParts; ++q)
                e->max_levels = std::max<int>(e->max_levels, (int)part_passes(plans[i], dtype, order, q).size());
    }
    e->dtype = dtype;
    e->part_bytes = ((int64_t)e->max_levels * count * (int64_t)sizeof(MultiSeg) + 255) / 256 * 256;
    e->ws_needed = kParts * e->part_bytes;
    *out = e;
    return SD_OK;
}

extern "C" sd_status sd_ensemble_workspace_bytes(const sd_ensemble *e, int64_t *bytes) {
    if (!e || !bytes) return fail(SD_ERR_ARG, "sd_ensemble_workspace_bytes: null argument");
    *bytes = std::max<int64_t>(e->ws_needed, 256);
    return SD_OK;
}

extern "C" sd_status sd_ensemble_bind_workspace(sd_ensemble *e, void *dev_ptr, size_t bytes,
                                                void *stream) {
    (void)stream;
    if (!e || !dev_ptr) return fail(SD_ERR_ARG, "sd_ensemble_bind_workspace: null argument");
    if ((int64_t)bytes < e->ws_needed) return fail(SD_ERR_WORKSPACE, "ensemble workspace too small");
    if (((uintptr_t)dev_ptr) & 255) return fail(SD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    e->ws = dev_ptr;
    e->ws_bytes = bytes;
    e->drop_graphs();
    return SD_OK;
}

namespace {
struct LevelLaunch {
    int64_t off, nseg, total;
    int D;
    bool gen;       // some segment needs the general round code
    uint32_t lds;   // largest LDS layout of its segments
};

// instances that run through the single-instance pass launches: any tile
// below the multi-instance kernel's minimum, or a state above 4 GiB (the
// multi-instance kernel uses 32-bit in-state offsets)
std::vector<int> small_instances(const sd_ensemble *e) {
    std::vector<int> small;
    const size_t amp = e->dtype == SD_C64 ? sizeof(float2) : sizeof(double2);
    for (int i = 0; i < (int)e->plans.size(); ++i) {
        bool is_small = ((uint64_t)amp << e->plans[i]->n) > ((uint64_t)1 << 32);
        for (const PassHost &ph : e->plans[i]->prog[e->dtype].passes) is_small = is_small || ph.D < kTileMinD;
        if (is_small) small.push_back(i);
    }
    return small;
}

// Build and upload the level tables of part q of a call into the part's
// region of the workspace.
sd_status build_levels(sd_ensemble *e, void *const *states, double dt, int order, int q,
                       const std::vector<int> &small, std::vector<LevelLaunch> *launches) {
    const int n_inst = (int)e->plans.size();
    std::vector<std::vector<std::pair<int, double>>> seq(n_inst);
    std::vector<char> is_small(n_inst, 0);
    for (int i : small) is_small[i] = 1;
    int levels = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (is_small[i]) continue;
        seq[i] = part_passes(e->plans[i], e->dtype, order, q);
        levels = std::max<int>(levels, (int)seq[i].size());
    }
    std::vector<MultiSeg> host;
    launches->clear();
    const int64_t base = (int64_t)q * e->part_bytes;
    for (int l = 0; l < levels; ++l) {
        for (int D = kTileMinD; D <= kMaxTileLog2; ++D) {
            LevelLaunch L{base + (int64_t)(host.size() * sizeof(MultiSeg)), 0, 0, D, false, 0};
            for (int i = 0; i < n_inst; ++i) {
                if (is_small[i] || l >= (int)seq[i].size()) continue;
                const sd_plan_t *p = e->plans[i];
                const PassHost &ph = p->prog[e->dtype].passes[seq[i][l].first];
                if (ph.D != D) continue;
                if (!ph.full_rounds) L.gen = true;
                L.lds = std::max(L.lds, tile_lds(D, 1 << (D - kLE), std::max(ph.nr, 1),
                                                 (int)ph.terms.size()).total);
                MultiSeg sg;
                sg.state = states[i];
                sg.ws = (const uint8_t *)p->ws;
                sg.pd = (const PassDev *)((const uint8_t *)p->ws + p->ws_off_prog[e->dtype] +
                                          (int64_t)seq[i][l].first * sizeof(PassDev));
                sg.tau = dt * seq[i][l].second;
                sg.first_item = L.total;
                sg.n_tiles = (int64_t)1 << (p->n - ph.D);
                L.total += sg.n_tiles;
                host.push_back(sg);
                ++L.nseg;
            }
            if (L.nseg) launches->push_back(L);
        }
    }
    if ((int64_t)(host.size() * sizeof(MultiSeg)) > e->part_bytes ||
        base + e->part_bytes > (int64_t)e->ws_bytes)
        return fail(SD_ERR_WORKSPACE, "ensemble workspace too small for the segment tables");
    if (host.empty()) return SD_OK;
    return hip_check(hipMemcpy((char *)e->ws + base, host.data(), host.size() * sizeof(MultiSeg),
                               hipMemcpyHostToDevice),
                     "ensemble segment upload");
}

template <typename T>
sd_status launch_levels(sd_ensemble *e, const std::vector<LevelLaunch> &launches, hipStream_t s) {
    std::call_once(g_once, init_device_props);
    if (g_init_status != SD_OK) return fail(g_init_status, "device initialisation failed");
    for (auto &L : launches) {
        const MultiSeg *dsegs = (const MultiSeg *)((const char *)e->ws + L.off);
        const int threads = 1 << (L.D - kLE);
        const int per_cu = blocks_per_cu(L.D);
        const int grid = (int)std::min<int64_t>(L.total, (int64_t)std::max(1, g_num_cu) * per_cu);
        const size_t lds = L.lds;
        if (L.gen)
            hipLaunchKernelGGL((k_tile_multi<T, true>), dim3(grid), dim3(threads), lds, s, dsegs,
                               (int)L.nseg, L.total);
        else
            hipLaunchKernelGGL((k_tile_multi<T, false>), dim3(grid), dim3(threads), lds, s, dsegs,
                               (int)L.nseg, L.total);
        sd_status r = hip_check(hipGetLastError(), "k_tile_multi launch");
        if (r != SD_OK) return r;
    }
    return SD_OK;
}

// the single-instance pass launches of part q for one small instance
sd_status run_small(sd_ensemble *e, int i, void *state, double dt, int order, int q, hipStream_t s) {
    for (auto &pf : part_passes(e->plans[i], e->dtype, order, q)) {
        sd_status r = e->dtype == SD_C64 ? launch_pass<float2, 0>(e->plans[i], e->dtype, pf.first, state,
                                                                  dt * pf.second, s)
                                         : launch_pass<double2, 0>(e->plans[i], e->dtype, pf.first, state,
                                                                   dt * pf.second, s);
        if (r != SD_OK) return r;
    }
    return SD_OK;
}
}  // namespace

extern "C" sd_status sd_ensemble_evolve(sd_ensemble *e, void *const *states, double dt, int64_t steps,
                                        int32_t order, void *stream) {
    if (!e || !states) return fail(SD_ERR_ARG, "sd_ensemble_evolve: null argument");
    if (order != 1 && order != 2 && order != 4)
        return fail(SD_ERR_ARG, "sd_ensemble_evolve: order must be 1, 2 or 4");
    if (steps < 0 || !std::isfinite(dt)) return fail(SD_ERR_ARG, "sd_ensemble_evolve: bad steps/dt");
    if (!e->ws) return fail(SD_ERR_WORKSPACE, "sd_ensemble_evolve: no workspace bound");
    for (size_t i = 0; i < e->plans.size(); ++i) {
        if (!states[i]) return fail(SD_ERR_ARG, "sd_ensemble_evolve: null state");
        if (!e->plans[i]->bound) return fail(SD_ERR_WORKSPACE, "sd_ensemble_evolve: plan without workspace");
    }
    if (steps == 0) return SD_OK;
    hipStream_t user = (hipStream_t)stream;
    sd_status r;
    if (!e->cstream) {
        r = hip_check(hipStreamCreateWithFlags(&e->cstream, hipStreamNonBlocking), "ensemble stream");
        if (r != SD_OK) return r;
        r = hip_check(hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming), "ensemble event");
        if (r != SD_OK) return r;
        r = hip_check(hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming), "ensemble event");
        if (r != SD_OK) return r;
    }
    std::vector<void *> st(states, states + e->plans.size());
    // The captured parts hold every plan's workspace addresses (its pass
    // records and term tables): a plan rebound to other memory since then
    // invalidates them, like new state pointers or another dt or order.
    std::vector<const void *> pws(e->plans.size());
    for (size_t i = 0; i < e->plans.size(); ++i) pws[i] = e->plans[i]->ws;
    if (!(e->cached && e->g_dt == dt && e->g_order == order && e->g_states == st && e->g_plan_ws == pws)) {
        e->drop_graphs();
        // no earlier replay may still read the segment tables being replaced
        r = hip_check(hipStreamSynchronize(e->cstream), "ensemble stream sync");
        if (r != SD_OK) return r;
        e->g_small = small_instances(e);
        for (int q = 0; q < kParts; ++q) {
            std::vector<LevelLaunch> launches;
            r = build_levels(e, states, dt, order, q, e->g_small, &launches);
            if (r != SD_OK) return r;
            bool small_work = false;
            for (int i : e->g_small) small_work = small_work || !part_passes(e->plans[i], e->dtype, order, q).empty();
            if (launches.empty() && !small_work) continue;
            // one graph per part: the level launches, then the pass launches
            // of the instances outside them
            r = hip_check(hipStreamBeginCapture(e->cstream, hipStreamCaptureModeThreadLocal), "begin capture");
            if (r != SD_OK) return r;
            r = e->dtype == SD_C64 ? launch_levels<float2>(e, launches, e->cstream)
                                   : launch_levels<double2>(e, launches, e->cstream);
            for (size_t k = 0; k < e->g_small.size() && r == SD_OK; ++k)
                r = run_small(e, e->g_small[k], states[e->g_small[k]], dt, order, q, e->cstream);
            hipGraph_t g = nullptr;
            sd_status r2 = hip_check(hipStreamEndCapture(e->cstream, &g), "end capture");
            if (r != SD_OK) {
                if (g) (void)hipGraphDestroy(g);
                return r;
            }
            if (r2 != SD_OK) return r2;
            e->graph[q] = g;
            r = hip_check(hipGraphInstantiate(&e->exec[q], e->graph[q], nullptr, nullptr, 0), "graph instantiate");
            if (r != SD_OK) return r;
        }
        e->cached = true;
        e->g_dt = dt;
        e->g_order = order;
        e->g_states = st;
        e->g_plan_ws = pws;
    }
    r = hip_check(hipEventRecord(e->ev_in, user), "event record");
    if (r != SD_OK) return r;
    r = hip_check(hipStreamWaitEvent(e->cstream, e->ev_in, 0), "stream wait");
    if (r != SD_OK) return r;
    // prologue, core x (steps - 1), epilogue
    auto part = [&](int q) -> sd_status {
        if (!e->exec[q]) return SD_OK;
        return hip_check(hipGraphLaunch(e->exec[q], e->cstream), "graph launch");
    };
    r = part(0);
    for (int64_t k = 1; k < steps && r == SD_OK; ++k) r = part(1);
    if (r == SD_OK) r = part(2);
    if (r != SD_OK) return r;
    r = hip_check(hipEventRecord(e->ev_out, e->cstream), "event record");
    if (r != SD_OK) return r;
    return hip_check(hipStreamWaitEvent(user, e->ev_out, 0), "stream wait");
}

extern "C" void sd_ensemble_destroy(sd_ensemble *e) { delete e; }
