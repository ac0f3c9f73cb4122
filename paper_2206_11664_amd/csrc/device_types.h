// Device-side record of one tile pass (packed into the caller's workspace).
#pragma once
#include <cstdint>

namespace sd {

constexpr int kMaxD = 16;            // tile dims a record can describe
constexpr int kMaxPassTerms = 256;   // Lambda terms per pass (LDS budget)
constexpr int kTermGrid = 2048;      // blocks of a per-term expectation pass (at most)

struct alignas(256) PassDev {
    int32_t n;          // qubits
    int32_t D;          // tile dims (log2 of amplitudes per tile)
    int32_t rho;        // Hadamard (X-span) dims, tile coordinates 0..rho-1
    int32_t c;          // contiguous low address bits (pivots 0..c-1)
    int32_t m;          // Lambda terms
    int32_t n_free;     // n - D
    int64_t n_tiles;    // 2^(n-D)
    int64_t term_off;   // byte offset of the term arrays from the workspace base
    double scale;       // 2^-rho
    double kcos[7];     // 2^-rho times the Taylor coefficients of cos in x^2 (constant first)
    double ksin[7];     // 2^-rho times those of sin(x)/x
    uint64_t u_hi[kMaxD];   // physical vectors of tile pivots c..D-1
    uint32_t mr[kMaxD];     // tile coordinates of each pivot vector
    uint32_t B[kMaxD];      // CZ/S quadratic form rows (rho used)
    uint32_t zq;            // span coordinates with an extra Z in the CZ/S layer
    int32_t free_pos[64];   // physical bit of each tile-index bit (32-bit words:
                            // uniform reads of them stay scalar loads)
    // register-round schedule (k_tile), one entry per chunk
    int32_t nr;             // chunks of span coordinates (0 when rho = 0)
    int32_t lam_round;      // chunk whose round applies Lambda
    int32_t reg[4][4];      // tile coordinates in register slots per chunk
    int32_t regpost[4][4];  // register coordinates after the lane exchange
    int32_t xl[4][2];       // chunk coordinates on lane bits 4, 5
    int32_t nx[4];          // how many of them are exchanged (0..2)
    uint32_t bmask[4];      // register slots that get butterflies (low bits)
    uint32_t iflag[4];      // slots whose coordinate carries an S (i twiddle)
    uint32_t dflag[4];      // chunk slots (0..3 registers, 4..5 lanes) with a Z
    uint32_t later[4];      // span coordinates of the chunks after this one
    int32_t bucket[33];     // term offsets by Lambda pattern on regpost[lam_round]
    double coef_abs_sum;    // sum |coef| of the pass
    uint32_t lanes[4][kMaxD];       // tile coordinates of lane bits per round
    uint32_t lanes_post[4][kMaxD];  // the same after the lane exchange
    uint64_t io_phys[kMaxD];        // physical offsets of round 0's lane bits
    uint64_t io_reg[4];             // physical offsets of round 0's register slots
    uint32_t swz[4];                // LDS slot of t: t ^ sum_j parity(t & swz[j]) << j
    int32_t staged;                 // round 0 reads the tile from LDS, staged in
                                    // pivot order (u_hi, mr), not from HBM
    uint32_t czm[4];                // round r: bit g = sign of register pattern g
                                    // (CZ between the chunk's register slots)
    int32_t shift0;                 // round 0's lanes 0..3 (lanes) have components
                                    // along its own coordinates, which its LDS
                                    // layout (lanes_post) drops: the outputs of
                                    // a round 0 before Lambda's take a sign
};

// term arrays at term_off: uint32 zeta[m]; (pad to 8) uint64 ztile[m]; double coef[m];
// double usign[m] (coef without the Hamiltonian coefficient: +-1)
inline int64_t term_bytes(int m) {
    int64_t a = ((int64_t)m * 4 + 7) / 8 * 8;
    return a + (int64_t)m * 24;
}

}  // namespace sd
