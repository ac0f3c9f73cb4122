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
        for (int j = p.c; j < p.D; ++j) d.u_hi[j - p.c] = p.u[j];
        for (int j = 0; j < p.D; ++j) d.mr[j] = p.mr[j];
        for (int j = 0; j < p.rho; ++j) d.B[j] = p.B[j];
        int f = 0;
        for (int q = 0; q < n; ++q)
            if ((p.free_mask >> q) & 1) d.free_pos[f++] = (uint8_t)q;
        d.nr = p.nr;
        d.lam_round = p.lam_round;
        for (int r = 0; r < 4; ++r) {
            for (int b = 0; b < 5; ++b) d.reg[r][b] = p.reg[r][b];
            d.bmask[r] = p.bmask[r];
        }
        for (int w = 0; w < 33; ++w) d.bucket[w] = p.bucket.empty() ? 0 : p.bucket[w];
        d.coef_abs_sum = p.coef_abs_sum;
        std::memcpy(buf.data() + i * sizeof(PassDev), &d, sizeof(d));
        uint8_t *t = buf.data() + toff;
        const int m = d.m;
        std::memcpy(t, p.zeta.data(), 4 * (size_t)m);
        int64_t o2 = ((int64_t)m * 4 + 7) / 8 * 8;
        std::memcpy(t + o2, p.ztile.data(), 8 * (size_t)m);
        std::memcpy(t + o2 + 8 * m, p.coef.data(), 8 * (size_t)m);
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

__device__ __forceinline__ int quad_form(const uint32_t *B, int rho, uint32_t y) {
    int q = 0;
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
    const uint32_t rmask = (rho >= 32) ? ~0u : ((1u << rho) - 1);
    const uint64_t cmask = ((uint64_t)1 << c) - 1;
    const double scale = pd.scale;
    double acc = 0.0;

    for (int64_t ti = blockIdx.x; ti < pd.n_tiles; ti += gridDim.x) {
        uint64_t xT = 0;
        for (int i = 0; i < pd.n_free; ++i)
            if ((ti >> i) & 1) xT |= (uint64_t)1 << pd.free_pos[i];
        for (int k = threadIdx.x; k < m; k += blockDim.x) {
            const double v = coef[k];
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
                tile[t] = mul_ipow(tile[t], quad_form(pd.B, rho, (uint32_t)t & rmask));
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
                    tile[t] = mul_ipow(tile[t], -quad_form(pd.B, rho, (uint32_t)t & rmask));
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
        } else {
            for (int64_t t = threadIdx.x; t < size; t += blockDim.x) {
                double phi = 0.0;
                for (int k = 0; k < m; ++k)
                    phi += (__popc(zs[k] & (uint32_t)t) & 1) ? -cks[k] : cks[k];
                const double2 a = tile[t];
                acc += (a.x * a.x + a.y * a.y) * phi * scale;
            }
        }
        __syncthreads();
    }
    if (MODE == 1) {
        double s = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] += s;
    }
}

// ---------------------------------------------------------------------------
// k_tile: register-round tile pass (tiles of 2^D amplitudes, D >= kTileMinD)
// ---------------------------------------------------------------------------
// A block of 2^(D-5) threads owns one tile at a time; every thread holds 32
// amplitudes in FP64 registers.  In the round of chunk r the 32 amplitudes of
// a thread differ in the 5 tile coordinates reg[r] and share the others
// (taken from the thread index), so the butterflies of those coordinates run
// in registers; between rounds the tile is exchanged through LDS.  The LDS
// slot of tile coordinate t is t ^ fold(t >> 3), fold = XOR of its 3-bit
// groups: whenever the three lowest thread-index bits address three adjacent
// coordinates, the 8 lanes of a 128-byte LDS phase land in distinct banks.
constexpr int kE = 32;
constexpr int kTileMinD = 10;

__device__ __forceinline__ uint32_t lds_slot(uint32_t t) {
    uint32_t h = t >> 3;
    h ^= (h >> 3) ^ (h >> 6) ^ (h >> 9);
    return t ^ (h & 7u);
}

// e^{i theta} in FP64: Taylor polynomials of cos and sin at theta / 2^halv
// (|theta / 2^halv| <= 1/4, truncation < 1e-17), then halv double-angle steps.
__device__ __forceinline__ void cis(double th, int halv, double &c, double &s) {
    const double x = ldexp(th, -halv);
    const double x2 = x * x;
    double pc = 1.0 / 479001600.0;
    pc = fma(pc, x2, -1.0 / 3628800.0);
    pc = fma(pc, x2, 1.0 / 40320.0);
    pc = fma(pc, x2, -1.0 / 720.0);
    pc = fma(pc, x2, 1.0 / 24.0);
    pc = fma(pc, x2, -0.5);
    c = fma(pc, x2, 1.0);
    double ps = 1.0 / 6227020800.0;
    ps = fma(ps, x2, -1.0 / 39916800.0);
    ps = fma(ps, x2, 1.0 / 362880.0);
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

// a * i^e, e in 0..3
__device__ __forceinline__ double2 rot_ipow(double2 a, uint32_t e) {
    double2 r = (e & 1u) ? make_double2(-a.y, a.x) : a;
    return (e & 2u) ? make_double2(-r.x, -r.y) : r;
}

__device__ __forceinline__ void bfly_bit(double2 (&v)[kE], int b) {
#pragma unroll
    for (int j = 0; j < kE; ++j)
        if (!((j >> b) & 1)) {
            const double2 a = v[j], c = v[j | (1 << b)];
            v[j] = make_double2(a.x + c.x, a.y + c.y);
            v[j | (1 << b)] = make_double2(a.x - c.x, a.y - c.y);
        }
}

__device__ __forceinline__ void bfly(double2 (&v)[kE], uint32_t bm) {
    if (bm & 1u) bfly_bit(v, 0);
    if (bm & 2u) bfly_bit(v, 1);
    if (bm & 4u) bfly_bit(v, 2);
    if (bm & 8u) bfly_bit(v, 3);
    if (bm & 16u) bfly_bit(v, 4);
}

template <typename T, int MODE, bool PREFETCH>
__global__ void __launch_bounds__(256)
k_tile(T *__restrict__ state, const PassDev *__restrict__ pdp, const uint8_t *__restrict__ ws,
       double tau, int halv, double *__restrict__ partial) {
    extern __shared__ double2 lds[];
    __shared__ double cks[kMaxPassTerms];
    __shared__ double red[256];
    const PassDev &pd = *pdp;
    const int D = pd.D, TL = D - 5, c = pd.c, m = pd.m, nr = pd.nr, rho = pd.rho;
    const int L = pd.lam_round;
    const uint32_t tid = threadIdx.x;
    const uint8_t *tb = ws + pd.term_off;
    const uint32_t *zeta = (const uint32_t *)tb;
    const int64_t o2 = ((int64_t)m * 4 + 7) / 8 * 8;
    const uint64_t *ztile = (const uint64_t *)(tb + o2);
    const double *coef = (const double *)(tb + o2 + 8 * (int64_t)m);
    const uint32_t rmask = (rho >= 32) ? ~0u : ((1u << rho) - 1);
    const double scale = pd.scale;

    // ---- per-thread constants (tile independent) ----
    // scatter/gather: element j of thread t is pivot pattern t + (j << TL)
    auto pivot_vec = [&](int i) -> uint64_t { return i < c ? ((uint64_t)1 << i) : pd.u_hi[i - c]; };
    uint64_t off_t = 0;
    uint32_t tc_t = 0;
    for (int i = 0; i < TL; ++i)
        if ((tid >> i) & 1) {
            off_t ^= pivot_vec(i);
            tc_t ^= pd.mr[i];
        }
    const uint32_t sl_t = lds_slot(tc_t);
    uint64_t pvh[5];
    uint32_t slh[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        pvh[b] = pivot_vec(TL + b);
        slh[b] = lds_slot(pd.mr[TL + b]);
    }
    // rounds: thread-index bits fill the tile coordinates outside reg[r], lowest first
    const int nrounds = nr > 0 ? nr : 1;
    uint32_t base_t[4] = {0, 0, 0, 0}, base_sl[4] = {0, 0, 0, 0}, rs[4][5] = {};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r >= nrounds) break;
        uint32_t regm = 0;
        for (int b = 0; b < 5; ++b) regm |= 1u << pd.reg[r][b];
        uint32_t bt = 0;
        int i = 0;
        for (int q = 0; q < D; ++q)
            if (!((regm >> q) & 1)) {
                bt |= ((tid >> i) & 1u) << q;
                ++i;
            }
        base_t[r] = bt;
        base_sl[r] = lds_slot(bt);
        for (int b = 0; b < 5; ++b) rs[r][b] = lds_slot(1u << pd.reg[r][b]);
    }
    // CZ/S phase exponents i^{q(y)} of this thread's 32 amplitudes in chunk 0
    uint64_t qe = 0;
    if (nr > 0) {
        for (int j = 0; j < kE; ++j) {
            uint32_t t = base_t[0];
            for (int b = 0; b < 5; ++b)
                if ((j >> b) & 1) t ^= 1u << pd.reg[0][b];
            const uint32_t y = t & rmask;
            uint32_t q = 0;
            for (int i2 = 0; i2 < rho; ++i2)
                if ((y >> i2) & 1) q += __popc(pd.B[i2] & y);
            qe |= (uint64_t)(q & 3u) << (2 * j);
        }
    }

    double acc = 0.0;
    T pre[kE];
    auto load_tile = [&](int64_t ti, uint64_t &xT_out) {
        uint64_t xT = 0;
        for (int i = 0; i < pd.n_free; ++i)
            if ((ti >> i) & 1) xT |= (uint64_t)1 << pd.free_pos[i];
        xT_out = xT;
        uint64_t co = xT ^ off_t;
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            if (j) co ^= pvh[__builtin_ctz(j)];
            pre[j] = state[co];
        }
    };
    auto to_d2 = [](T a) -> double2 { return make_double2((double)a.x, (double)a.y); };

    int64_t ti = blockIdx.x;
    uint64_t xT_cur = 0, xT_next = 0;
    if (PREFETCH && ti < pd.n_tiles) load_tile(ti, xT_cur);
    for (; ti < pd.n_tiles; ti += gridDim.x) {
        if (!PREFETCH) load_tile(ti, xT_cur);
        // scatter the prefetched tile into LDS
        {
            uint32_t cs = sl_t;
            asm volatile("" : "+v"(cs));
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                if (j) cs ^= slh[__builtin_ctz(j)];
                lds[cs] = to_d2(pre[j]);
            }
        }
        for (int k = tid; k < m; k += blockDim.x) {
            const double v = coef[k];
            cks[k] = (__popcll(ztile[k] & xT_cur) & 1) ? -v : v;
        }
        const int64_t tn = ti + gridDim.x;
        if (PREFETCH && tn < pd.n_tiles) load_tile(tn, xT_next);
        __syncthreads();

        double2 v[kE];
        // the asm barriers keep the loop-invariant address chains from being
        // hoisted out of the tile loop (they would stay live in registers)
        auto rd = [&](int r) {
            uint32_t cs = base_sl[r];
            asm volatile("" : "+v"(cs));
#pragma unroll
            for (int jj = 0; jj < kE; ++jj) {
                if (jj) cs ^= rs[r][__builtin_ctz(jj)];
                v[jj ^ (jj >> 1)] = lds[cs];
            }
        };
        auto wr = [&](int r) {
            uint32_t cs = base_sl[r];
            asm volatile("" : "+v"(cs));
#pragma unroll
            for (int jj = 0; jj < kE; ++jj) {
                if (jj) cs ^= rs[r][__builtin_ctz(jj)];
                lds[cs] = v[jj ^ (jj >> 1)];
            }
        };
        auto lam = [&](int r) {
            // phi over the 32 register patterns: bucketed coefficients, then a
            // 32-point Walsh-Hadamard of the bucket sums
            double A[kE];
            const uint32_t bb = base_t[r];
#pragma unroll
            for (int w = 0; w < kE; ++w) {
                double sacc = 0.0;
                for (int k = pd.bucket[w]; k < pd.bucket[w + 1]; ++k) {
                    const double ck = cks[k];
                    sacc += (__popc(zeta[k] & bb) & 1) ? -ck : ck;
                }
                A[w] = sacc;
            }
#pragma unroll
            for (int b = 0; b < 5; ++b)
#pragma unroll
                for (int j = 0; j < kE; ++j)
                    if (!((j >> b) & 1)) {
                        const double a0 = A[j], a1 = A[j | (1 << b)];
                        A[j] = a0 + a1;
                        A[j | (1 << b)] = a0 - a1;
                    }
            if (MODE == 0) {
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    double cc, ss;
                    cis(-tau * A[j], halv, cc, ss);
                    cc *= scale;
                    ss *= scale;
                    const double2 a = v[j];
                    v[j] = make_double2(fma(a.x, cc, -a.y * ss), fma(a.x, ss, a.y * cc));
                }
            } else {
#pragma unroll
                for (int j = 0; j < kE; ++j) acc += (v[j].x * v[j].x + v[j].y * v[j].y) * A[j] * scale;
            }
        };

        if (nr == 0) {
            rd(0);
            lam(0);
            if (MODE == 0) wr(0);
            __syncthreads();
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (r >= nr) break;
                rd(r);
                if (r == 0) {
#pragma unroll
                    for (int j = 0; j < kE; ++j) v[j] = rot_ipow(v[j], (uint32_t)(qe >> (2 * j)) & 3u);
                }
                bfly(v, pd.bmask[r]);
                if (r == nr - 1) {
                    lam(r);
                    if (MODE == 0) {
                        bfly(v, pd.bmask[r]);
                        if (r == 0) {
#pragma unroll
                            for (int j = 0; j < kE; ++j)
                                v[j] = rot_ipow(v[j], (4u - ((uint32_t)(qe >> (2 * j)) & 3u)) & 3u);
                        }
                    }
                }
                if (MODE == 0 || r < nr - 1) wr(r);
                __syncthreads();
            }
            if (MODE == 0) {
#pragma unroll
                for (int r = 2; r >= 0; --r) {
                    if (r > nr - 2) continue;
                    rd(r);
                    bfly(v, pd.bmask[r]);
                    if (r == 0) {
#pragma unroll
                        for (int j = 0; j < kE; ++j)
                            v[j] = rot_ipow(v[j], (4u - ((uint32_t)(qe >> (2 * j)) & 3u)) & 3u);
                    }
                    wr(r);
                    __syncthreads();
                }
            }
        }
        if (MODE == 0) {
            // gather back to HBM
            uint32_t cs = sl_t;
            asm volatile("" : "+v"(cs));
            uint64_t co = xT_cur ^ off_t;
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                if (j) {
                    cs ^= slh[__builtin_ctz(j)];
                    co ^= pvh[__builtin_ctz(j)];
                }
                st_amp(state, (int64_t)co, lds[cs]);
            }
            __syncthreads();
        }
        if (PREFETCH) xT_cur = xT_next;
    }
    if (MODE == 1) {
        double s2 = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] += s2;
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

// fixed-order final sum of `count` interleaved groups of `width` partials
__global__ void k_final(const double *__restrict__ partial, int count, int width,
                        double *__restrict__ out) {
    if (threadIdx.x < width) {
        double s = 0.0;
        for (int i = 0; i < count; ++i) s += partial[i * width + threadIdx.x];
        out[threadIdx.x] = s;
    }
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
static bool g_prefetch = true;   // SD_PREFETCH=0 disables the register prefetch
static bool g_generic = false;   // SD_GENERIC_KERNEL=1 routes every pass to k_pass
static std::once_flag g_once;

static void init_device_props() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) g_num_cu = prop.multiProcessorCount;
    if (const char *e = std::getenv("SD_PREFETCH")) g_prefetch = std::atoi(e) != 0;
    if (const char *e = std::getenv("SD_GENERIC_KERNEL")) g_generic = std::atoi(e) != 0;
    const int lds = (1 << kMaxTileLog2) * 16;
    hipFuncSetAttribute((const void *)k_pass<float2, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_pass<float2, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_pass<double2, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_pass<double2, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_tile<float2, 0, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_tile<float2, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_tile<double2, 0, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_tile<double2, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_tile<float2, 0, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipFuncSetAttribute((const void *)k_tile<double2, 0, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
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
    const int grid = MODE == 1 ? (int)std::min<int64_t>(tiles, kPartialSlots / 2) : grid_evolve;
    if (ph.D > kMaxTileLog2 || (int)ph.terms.size() > kMaxPassTerms)
        return fail(SD_ERR_INTERNAL, "pass exceeds the on-chip tile limits");
    const size_t lds = (size_t)16 << ph.D;
    if (ph.D >= kTileMinD && !g_generic) {
        int halv = 0;
        const double th = std::fabs(tau) * ph.coef_abs_sum;
        while (halv < 60 && std::ldexp(th, -halv) > 0.25) ++halv;
        const int threads = 1 << (ph.D - 5);
        // tiles of 2^13 fill one CU's LDS: one block per CU, next tile
        // prefetched into registers; smaller tiles run two or more blocks per CU
        const bool pf = MODE == 0 && ph.D >= 13 && g_prefetch;
        const int per_cu = ph.D >= 13 ? 1 : 2;
        const int g2 = MODE == 1 ? grid
                                 : (int)std::min<int64_t>(tiles, (int64_t)std::max(1, g_num_cu) * per_cu);
        if (pf)
            hipLaunchKernelGGL((k_tile<T, MODE, true>), dim3(g2), dim3(threads), lds, s, (T *)state,
                               pd, ws, tau, halv, partial);
        else
            hipLaunchKernelGGL((k_tile<T, MODE, false>), dim3(g2), dim3(threads), lds, s, (T *)state,
                               pd, ws, tau, halv, partial);
        return hip_check(hipGetLastError(), "k_tile launch");
    }
    hipLaunchKernelGGL((k_pass<T, MODE>), dim3(grid), dim3(kBlock), lds, s, (T *)state, pd, ws,
                       tau, partial);
    return hip_check(hipGetLastError(), "k_pass launch");
}

static std::vector<std::pair<int, double>> step_schedule(int K, int order) {
    std::vector<std::pair<int, double>> seq;
    if (order == 1 || K == 1) {
        for (int g = 0; g < K; ++g) seq.push_back({g, 1.0});
    } else {
        for (int g = 0; g < K - 1; ++g) seq.push_back({g, 0.5});
        seq.push_back({K - 1, 1.0});
        for (int g = K - 2; g >= 0; --g) seq.push_back({g, 0.5});
    }
    return seq;
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
    p->ws = dev_ptr;
    p->ws_bytes = bytes;
    p->bound = true;
    return SD_OK;
}

extern "C" sd_status sd_evolve(const sd_plan_t *p, void *state, sd_dtype dtype, double dt,
                               int64_t steps, int32_t order, void *stream) {
    if (!p || !state) return fail(SD_ERR_ARG, "sd_evolve: null argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_evolve: bad dtype");
    if (order != 1 && order != 2) return fail(SD_ERR_ARG, "sd_evolve: order must be 1 or 2");
    if (steps < 0) return fail(SD_ERR_ARG, "sd_evolve: steps < 0");
    if (!std::isfinite(dt)) return fail(SD_ERR_ARG, "sd_evolve: non-finite dt");
    if (!p->bound) return fail(SD_ERR_WORKSPACE, "sd_evolve: no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    const Program &P = p->prog[dtype];
    const int K = (int)p->groups.size();
    if (K == 0 || steps == 0) return SD_OK;
    auto seq = step_schedule(K, order);
    for (int64_t st = 0; st < steps; ++st)
        for (auto &gf : seq) {
            const double tau = dt * gf.second;
            for (int i = P.group_first[gf.first]; i < P.group_first[gf.first + 1]; ++i) {
                sd_status r = dtype == SD_C64 ? launch_pass<float2, 0>(p, dtype, i, state, tau, s)
                                              : launch_pass<double2, 0>(p, dtype, i, state, tau, s);
                if (r != SD_OK) return r;
            }
        }
    return SD_OK;
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
    hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, partial, maxgrid, 1, out);
    r = hip_check(hipGetLastError(), "final reduce");
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(energy, out, sizeof(double), hipMemcpyDeviceToHost, s), "copy energy");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_expectation sync");
}

namespace {
// small per-thread scratch for the stand-alone reductions
struct RedScratch {
    double *buf = nullptr;
    int dev = -1;
};
thread_local RedScratch g_red;

sd_status red_scratch(double **out) {
    int dev = 0;
    sd_status r = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (r != SD_OK) return r;
    if (!g_red.buf || g_red.dev != dev) {
        r = hip_check(hipMalloc((void **)&g_red.buf, (kPartialSlots * 2 + 64) * sizeof(double)),
                      "reduction scratch");
        if (r != SD_OK) return r;
        g_red.dev = dev;
    }
    *out = g_red.buf;
    return SD_OK;
}
}  // namespace

extern "C" sd_status sd_norm2(const void *state, sd_dtype dtype, int32_t n, double *out,
                              void *stream) {
    if (!state || !out) return fail(SD_ERR_ARG, "sd_norm2: null argument");
    if (n < 0 || n > 40) return fail(SD_ERR_RANGE, "sd_norm2: n_qubits out of range");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_norm2: bad dtype");
    hipStream_t s = (hipStream_t)stream;
    double *buf = nullptr;
    sd_status r = red_scratch(&buf);
    if (r != SD_OK) return r;
    const int64_t dim = (int64_t)1 << n;
    const int grid = (int)std::min<int64_t>(kPartialSlots, (dim + kBlock - 1) / kBlock);
    if (dtype == SD_C64)
        hipLaunchKernelGGL(k_norm2<float2>, dim3(grid), dim3(kBlock), 0, s, (const float2 *)state, dim, buf);
    else
        hipLaunchKernelGGL(k_norm2<double2>, dim3(grid), dim3(kBlock), 0, s, (const double2 *)state, dim, buf);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, buf, grid, 1, buf + 2 * kPartialSlots);
    r = hip_check(hipGetLastError(), "norm2 launch");
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(out, buf + 2 * kPartialSlots, sizeof(double), hipMemcpyDeviceToHost, s),
                  "copy norm");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_norm2 sync");
}

extern "C" sd_status sd_inner(const void *a, const void *b, sd_dtype dtype, int32_t n, double *out,
                              void *stream) {
    if (!a || !b || !out) return fail(SD_ERR_ARG, "sd_inner: null argument");
    if (n < 0 || n > 40) return fail(SD_ERR_RANGE, "sd_inner: n_qubits out of range");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_inner: bad dtype");
    hipStream_t s = (hipStream_t)stream;
    double *buf = nullptr;
    sd_status r = red_scratch(&buf);
    if (r != SD_OK) return r;
    const int64_t dim = (int64_t)1 << n;
    const int grid = (int)std::min<int64_t>(kPartialSlots, (dim + kBlock - 1) / kBlock);
    if (dtype == SD_C64)
        hipLaunchKernelGGL(k_inner<float2>, dim3(grid), dim3(kBlock), 0, s, (const float2 *)a,
                           (const float2 *)b, dim, buf);
    else
        hipLaunchKernelGGL(k_inner<double2>, dim3(grid), dim3(kBlock), 0, s, (const double2 *)a,
                           (const double2 *)b, dim, buf);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, buf, grid, 2, buf + 2 * kPartialSlots);
    r = hip_check(hipGetLastError(), "inner launch");
    if (r != SD_OK) return r;
    r = hip_check(hipMemcpyAsync(out, buf + 2 * kPartialSlots, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, s),
                  "copy inner");
    if (r != SD_OK) return r;
    return hip_check(hipStreamSynchronize(s), "sd_inner sync");
}

extern "C" sd_status sd_sync(void *stream) {
    sd_status r = hip_check(hipStreamSynchronize((hipStream_t)stream), "sd_sync");
    if (r != SD_OK) return r;
    return hip_check(hipGetLastError(), "sd_sync (async error)");
}

// ---------------------------------------------------------------------------
// ensemble
// ---------------------------------------------------------------------------
struct sd_ensemble {
    std::vector<const sd_plan_t *> plans;
    sd_dtype dtype = SD_C64;
};

extern "C" sd_status sd_ensemble_create(const sd_plan_t *const *plans, int32_t count, sd_dtype dtype,
                                        sd_ensemble **out) {
    if (!plans || !out || count <= 0) return fail(SD_ERR_ARG, "sd_ensemble_create: bad argument");
    if (dtype != SD_C64 && dtype != SD_C128) return fail(SD_ERR_ARG, "sd_ensemble_create: bad dtype");
    sd_ensemble *e = new sd_ensemble();
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) {
            delete e;
            return fail(SD_ERR_ARG, "sd_ensemble_create: null plan");
        }
        e->plans.push_back(plans[i]);
    }
    e->dtype = dtype;
    *out = e;
    return SD_OK;
}

extern "C" sd_status sd_ensemble_workspace_bytes(const sd_ensemble *e, int64_t *bytes) {
    if (!e || !bytes) return fail(SD_ERR_ARG, "sd_ensemble_workspace_bytes: null argument");
    *bytes = 256;
    return SD_OK;
}

extern "C" sd_status sd_ensemble_bind_workspace(sd_ensemble *e, void *dev_ptr, size_t bytes,
                                                void *stream) {
    (void)stream;
    if (!e || !dev_ptr || bytes < 256) return fail(SD_ERR_WORKSPACE, "sd_ensemble_bind_workspace");
    return SD_OK;
}

extern "C" sd_status sd_ensemble_evolve(sd_ensemble *e, void *const *states, double dt, int64_t steps,
                                        int32_t order, void *stream) {
    if (!e || !states) return fail(SD_ERR_ARG, "sd_ensemble_evolve: null argument");
    for (int64_t st = 0; st < steps; ++st)
        for (size_t i = 0; i < e->plans.size(); ++i) {
            sd_status r = sd_evolve(e->plans[i], states[i], e->dtype, dt, 1, order, stream);
            if (r != SD_OK) return r;
        }
    return SD_OK;
}

extern "C" void sd_ensemble_destroy(sd_ensemble *e) { delete e; }
