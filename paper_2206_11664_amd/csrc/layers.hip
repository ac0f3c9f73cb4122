// Reference execution modes on the device: the paper's circuit layer by layer
// and term-by-term Pauli rotations.  Every kernel is one HBM pass over the
// state (grid-stride, FP64 arithmetic, complex64 rounded once per pass).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "sd_internal.h"

namespace sd {

namespace {

__device__ __forceinline__ double2 ld2(const float2 *p, int64_t i) {
    float2 v = p[i];
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 ld2(const double2 *p, int64_t i) { return p[i]; }
__device__ __forceinline__ void st2(float2 *p, int64_t i, double2 v) {
    p[i] = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ void st2(double2 *p, int64_t i, double2 v) { p[i] = v; }

__device__ __forceinline__ uint64_t insert0(uint64_t i, int q) {
    const uint64_t low = ((uint64_t)1 << q) - 1;
    return ((i & ~low) << 1) | (i & low);
}

// H on qubit q, unnormalised butterfly (a + b, a - b)
template <typename T>
__global__ void k_layer_h(T *__restrict__ s, int64_t half, int q) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < half;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = insert0((uint64_t)i, q), y = x | ((uint64_t)1 << q);
        const double2 a = ld2(s, (int64_t)x), b = ld2(s, (int64_t)y);
        st2(s, (int64_t)x, make_double2(a.x + b.x, a.y + b.y));
        st2(s, (int64_t)y, make_double2(a.x - b.x, a.y - b.y));
    }
}

// CNOT fan-out: control c, target mask t; swap amp[x] <-> amp[x ^ t] for x_c = 1
template <typename T>
__global__ void k_layer_cnot(T *__restrict__ s, int64_t quarter, int c, uint64_t t) {
    const int tl = __builtin_ctzll(t);
    const int lo = c < tl ? c : tl, hi = c < tl ? tl : c;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < quarter;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = insert0(insert0((uint64_t)i, lo), hi) | ((uint64_t)1 << c);
        const uint64_t y = x ^ t;
        const double2 a = ld2(s, (int64_t)x), b = ld2(s, (int64_t)y);
        st2(s, (int64_t)x, b);
        st2(s, (int64_t)y, a);
    }
}

// diagonal: i^{s_sign popcount(x & smask)} (-1)^{sum_pairs x_a popcount(x & m)}
//           exp(-i tau sum_k c_k (-1)^{popcount(x & z_k)}) * scale
template <typename T>
__global__ void k_layer_diag(T *__restrict__ s, int64_t dim, int s_sign, uint64_t smask,
                             const uint64_t *__restrict__ cz, int ncz, const uint64_t *__restrict__ lam,
                             int nlam, double tau, double scale) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = (uint64_t)i;
        int e = s_sign * __popcll(x & smask);
        for (int k = 0; k < ncz; ++k)
            if ((x >> cz[2 * k]) & 1) e += 2 * __popcll(x & cz[2 * k + 1]);
        double2 a = ld2(s, i);
        e &= 3;
        if (e & 1) a = make_double2(-a.y, a.x);
        if (e & 2) a = make_double2(-a.x, -a.y);
        if (nlam) {
            double phi = 0.0;
            for (int k = 0; k < nlam; ++k) {
                const double ck = __longlong_as_double((long long)lam[2 * k + 1]);
                phi += (__popcll(x & lam[2 * k]) & 1) ? -ck : ck;
            }
            double sn, cs;
            sincos(-tau * phi, &sn, &cs);
            a = make_double2((a.x * cs - a.y * sn) * scale, (a.x * sn + a.y * cs) * scale);
        }
        st2(s, i, a);
    }
}

// exp(-i theta P), P|x> = i^{ny} (-1)^{popcount(x & z)} |x ^ xm>
template <typename T>
__global__ void k_rotation(T *__restrict__ s, int64_t half, int64_t dim, uint64_t xm, uint64_t zm,
                           int ny, double c, double sn) {
    const int hb = xm ? 63 - __builtin_clzll(xm) : 0;
    // i^{ny} as (re, im)
    const double ir = (ny & 1) ? 0.0 : ((ny & 2) ? -1.0 : 1.0);
    const double ii = (ny & 1) ? ((ny & 2) ? -1.0 : 1.0) : 0.0;
    if (!xm) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
             i += (int64_t)gridDim.x * blockDim.x) {
            const double sg = (__popcll((uint64_t)i & zm) & 1) ? -1.0 : 1.0;
            // (c - i s sg) a
            const double2 a = ld2(s, i);
            st2(s, i, make_double2(c * a.x + sn * sg * a.y, c * a.y - sn * sg * a.x));
        }
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < half;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = insert0((uint64_t)i, hb), y = x ^ xm;
        const double2 a = ld2(s, (int64_t)x), b = ld2(s, (int64_t)y);
        // (P psi)[x] = i^ny (-1)^{z.y} b ; (P psi)[y] = i^ny (-1)^{z.x} a
        const double sy = (__popcll(y & zm) & 1) ? -1.0 : 1.0;
        const double sx = (__popcll(x & zm) & 1) ? -1.0 : 1.0;
        const double pxr = sy * (ir * b.x - ii * b.y), pxi = sy * (ir * b.y + ii * b.x);
        const double pyr = sx * (ir * a.x - ii * a.y), pyi = sx * (ir * a.y + ii * a.x);
        // new = c * amp - i s * P amp
        st2(s, (int64_t)x, make_double2(c * a.x + sn * pxi, c * a.y - sn * pxr));
        st2(s, (int64_t)y, make_double2(c * b.x + sn * pyi, c * b.y - sn * pyr));
    }
}

int grid_1d(int64_t work) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 8192));
}

sd_status hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(SD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return SD_OK;
}

template <typename T>
sd_status run_layers_t(const sd_plan_s *p, T *state, int g, double tau, hipStream_t st) {
    const int n = p->n;
    const int64_t dim = (int64_t)1 << n;
    const uint64_t *base = (const uint64_t *)((const uint8_t *)p->ws + p->ws_off_layers);
    for (const LayerOp &op : p->layers[g]) {
        if (op.kind == LayerOp::H) {
            hipLaunchKernelGGL(k_layer_h<T>, dim3(grid_1d(dim / 2)), dim3(256), 0, st, state, dim / 2, op.a);
        } else if (op.kind == LayerOp::CNOT_FAN) {
            hipLaunchKernelGGL(k_layer_cnot<T>, dim3(grid_1d(dim / 4)), dim3(256), 0, st, state, dim / 4,
                               op.a, op.mask);
        } else {
            hipLaunchKernelGGL(k_layer_diag<T>, dim3(grid_1d(dim)), dim3(256), 0, st, state, dim, op.s_sign,
                               op.smask, base + op.cz_off, (int)op.cz_n, base + op.lam_off, (int)op.lam_n,
                               tau, op.scale);
        }
        sd_status r = hip_ok(hipGetLastError(), "layer kernel launch");
        if (r != SD_OK) return r;
    }
    return SD_OK;
}

template <typename T>
sd_status run_terms_t(const sd_plan_s *p, T *state, int g, double tau, hipStream_t st) {
    const int64_t dim = (int64_t)1 << p->n;
    for (int64_t k : p->groups[g]) {
        const Term &t = p->terms[k];
        const double th = t.c * tau;
        hipLaunchKernelGGL(k_rotation<T>, dim3(grid_1d(t.x ? dim / 2 : dim)), dim3(256), 0, st, state,
                           dim / 2, dim, t.x, t.z, __builtin_popcountll(t.x & t.z) & 3, std::cos(th),
                           std::sin(th));
        sd_status r = hip_ok(hipGetLastError(), "rotation kernel launch");
        if (r != SD_OK) return r;
    }
    return SD_OK;
}

}  // namespace

// one application of group g at angle tau, in the plan's reference mode
sd_status run_group_reference(const sd_plan_s *p, void *state, sd_dtype dtype, int g, double tau,
                              hipStream_t st) {
    if (p->n < 2) return fail(SD_ERR_RANGE, "reference modes need at least 2 qubits");
    if (p->mode == SD_MODE_PAPER_LAYERS)
        return dtype == SD_C64 ? run_layers_t(p, (float2 *)state, g, tau, st)
                               : run_layers_t(p, (double2 *)state, g, tau, st);
    return dtype == SD_C64 ? run_terms_t(p, (float2 *)state, g, tau, st)
                           : run_terms_t(p, (double2 *)state, g, tau, st);
}

}  // namespace sd
