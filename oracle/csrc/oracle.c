/*
 * CPU oracle kernels -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 loops over the state vector.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * this library; the product path never does.  Shares no code with the GPU
 * library.
 *
 * State layout: 2^n complex128 amplitudes stored as interleaved (re, im)
 * doubles; qubit q is bit q of the index (paper, Sec. "Quantum States and
 * Quantum Gates": basis |b_n ... b_1> with qubit 1 the least significant bit).
 *
 * A Hermitian Pauli string is given by (xmask, zmask): qubit q carries
 *   X if x_q=1,z_q=0;  Z if x_q=0,z_q=1;  Y if x_q=1,z_q=1.
 * Its action on a basis state follows from the single-qubit matrices of the
 * paper's Eq. for sigma_1..sigma_3:
 *   X|b> = |b^1>,   Y|b> = i(-1)^b |b^1>,   Z|b> = (-1)^b |b>
 * hence  P|x> = i^{#Y} (-1)^{popcount(x & zmask)} |x ^ xmask>.
 *
 * The rotation e^{-i theta P} = cos(theta) I - i sin(theta) P holds for any
 * Pauli P because P^2 = I; it is the per-term factor of the first-order
 * Trotter product (Sec. "Classical Simulation of Quantum Dynamics", Eq.
 * trotter_decomp).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static int parity64(uint64_t v) { return __builtin_popcountll(v) & 1; }

/* i^k for k mod 4 */
static cplx ipow(int k) {
    switch (k & 3) {
        case 0: return 1.0;
        case 1: return I;
        case 2: return -1.0;
        default: return -I;
    }
}

/* (P psi)[y] = i^{ny} (-1)^{popcount((y^xmask) & zmask)} psi[y ^ xmask] */
static inline cplx pauli_coef(uint64_t src, uint64_t zmask, cplx iy) {
    return parity64(src & zmask) ? -iy : iy;
}

/* psi <- exp(-i theta P) psi, in place. */
void or_pauli_rotate(int32_t n, double *psi_ri, uint64_t xmask, uint64_t zmask,
                     double theta) {
    const int64_t dim = (int64_t)1 << n;
    cplx *psi = (cplx *)psi_ri;
    const int ny = __builtin_popcountll(xmask & zmask);
    const cplx iy = ipow(ny);
    const double c = cos(theta), s = sin(theta);
    if (xmask == 0) {
        /* diagonal: P|x> = i^{ny}(-1)^{..}|x>, ny = 0 here */
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < dim; ++x) {
            cplx p = pauli_coef((uint64_t)x, zmask, iy);
            psi[x] = c * psi[x] - I * s * p * psi[x];
        }
        return;
    }
    /* pairs {x, x^xmask}: visit each pair once from the member whose highest
       set bit of xmask is 0 */
    const uint64_t hb = (uint64_t)1 << (63 - __builtin_clzll(xmask));
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; ++x) {
        if ((uint64_t)x & hb) continue;
        const int64_t y = (int64_t)((uint64_t)x ^ xmask);
        const cplx a = psi[x], b = psi[y];
        /* (P psi)[x] = coef(src=y) * psi[y]; (P psi)[y] = coef(src=x) * psi[x] */
        const cplx pa = pauli_coef((uint64_t)y, zmask, iy) * b;
        const cplx pb = pauli_coef((uint64_t)x, zmask, iy) * a;
        psi[x] = c * a - I * s * pa;
        psi[y] = c * b - I * s * pb;
    }
}

/* Apply a list of rotations in order: psi <- prod_k exp(-i theta_k P_k) psi
   with the first listed term acting first. */
void or_apply_rotations(int32_t n, double *psi_ri, int64_t count,
                        const uint64_t *xmask, const uint64_t *zmask,
                        const double *theta) {
    for (int64_t k = 0; k < count; ++k)
        or_pauli_rotate(n, psi_ri, xmask[k], zmask[k], theta[k]);
}

/* <psi| P |psi>  (real for Hermitian P); returned as (re, im) in out[2]. */
void or_pauli_expect(int32_t n, const double *psi_ri, uint64_t xmask,
                     uint64_t zmask, double *out) {
    const int64_t dim = (int64_t)1 << n;
    const cplx *psi = (const cplx *)psi_ri;
    const int ny = __builtin_popcountll(xmask & zmask);
    const cplx iy = ipow(ny);
    double re = 0.0, im = 0.0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (int64_t x = 0; x < dim; ++x) {
        const uint64_t src = (uint64_t)x;
        const int64_t y = (int64_t)(src ^ xmask);
        /* <y| P |x> psi[x] contributes conj(psi[y]) coef psi[x] */
        cplx v = conj(psi[y]) * pauli_coef(src, zmask, iy) * psi[x];
        re += creal(v);
        im += cimag(v);
    }
    out[0] = re;
    out[1] = im;
}

/* sum_x conj(a[x]) b[x] */
void or_inner(int32_t n, const double *a_ri, const double *b_ri, double *out) {
    const int64_t dim = (int64_t)1 << n;
    const cplx *a = (const cplx *)a_ri, *b = (const cplx *)b_ri;
    double re = 0.0, im = 0.0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (int64_t x = 0; x < dim; ++x) {
        cplx v = conj(a[x]) * b[x];
        re += creal(v);
        im += cimag(v);
    }
    out[0] = re;
    out[1] = im;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
