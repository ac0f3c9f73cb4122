// Internal types of the sd library (host side).  Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sd.h"

namespace sd {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
sd_status fail(sd_status s, const std::string &msg);  // sets sd_last_error

// ---------------------------------------------------------------------------
// GF(2) helpers on 64-bit rows
// ---------------------------------------------------------------------------
inline int popc(uint64_t v) { return __builtin_popcountll(v); }
inline int parity(uint64_t v) { return __builtin_popcountll(v) & 1; }
inline int ctz(uint64_t v) { return __builtin_ctzll(v); }

// Incremental echelon basis: every stored vector has a 1 at its pivot and 0
// at every other stored pivot.  comb[i] records which inserted generators
// (by insertion index, up to 64) XOR to vec[i].
struct Echelon {
    std::vector<uint64_t> vec, comb;
    std::vector<int> piv;
    int inserted = 0;
    bool high_pivot = false;  // pivot = highest (else lowest) set bit of the remainder
    // Reduce v against the basis; returns the remainder, and the combination
    // of basis vectors used in *used (as generator combination).
    uint64_t reduce(uint64_t v, uint64_t *used = nullptr) const;
    // Insert; returns true if v was independent.
    bool insert(uint64_t v);
    bool contains(uint64_t v) const { return reduce(v) == 0; }
    int dim() const { return (int)vec.size(); }
};

int gf2_rank(std::vector<uint64_t> rows);

// ---------------------------------------------------------------------------
// Hamiltonian
// ---------------------------------------------------------------------------
struct Term {
    uint64_t x, z;  // symplectic masks; Hermitian Pauli = i^{|x&z|} X^x Z^z
    double c;
    int64_t src;    // input index of first occurrence
};

}  // namespace sd

struct sd_hamiltonian {
    int32_t n = 0;
    std::vector<sd::Term> terms;
    // flat views for sd_hamiltonian_terms
    std::vector<uint64_t> xs, zs;
    std::vector<double> cs;
    std::vector<int64_t> srcs;
};

namespace sd {

// ---------------------------------------------------------------------------
// Clifford synthesis on the binary tableau (paper steps (i)-(iv))
// ---------------------------------------------------------------------------
struct Gate {
    int32_t kind, a, b;  // SD_GATE_*, qubits (b = -1 for one-qubit gates)
};

// A row of the tableau [X | Z | r] (Eq. binary_tableau), qubit q = bit q.
struct Row {
    uint64_t x, z;
    int r;
};

// Conjugation rules U P U^dagger of the tableau (Sec. "Tableau Representation",
// gate table).  CNOT uses z_c ^= z_t: the printed z-rule of the CNOT row
// disagrees with the two-qubit table, and the standard rule agrees with it.
void apply_gate(Row &row, const Gate &g);

struct SynthOptions {
    bool skip_rule = true;     // {I,Z}/{I,X} qubit pre-pass
    bool step_i = true;        // run step (i), maximise X-block rank with H
};

struct SynthResult {
    bool ok = false;
    std::string error;
    std::vector<Gate> gates;            // application order
    std::vector<int64_t> independent;   // indices into the input list
    std::vector<uint64_t> zmask;        // per input term
    std::vector<int8_t> sign;           // per input term
    int n_h_first = 0, n_h_last = 0, n_cnot_controls = 0, n_diag = 0;
};

// Appendix algorithm: linearly independent rows over the columns
// x_{act[0..]} then z_{act[0..]}; returns indices into `rows`, final order.
std::vector<int64_t> independent_rows(const std::vector<Row> &rows,
                                      const std::vector<int> &act);

// Steps (i)-(iv) for one commuting set of n-qubit Paulis.
SynthResult synthesize(int n, const std::vector<Row> &terms, const SynthOptions &opt);

// ---------------------------------------------------------------------------
// Device tile programs
// ---------------------------------------------------------------------------
constexpr int kMaxTileLog2 = 13;   // on-chip tile limit (LDS, FP64 staging)
constexpr int kMinTileLog2 = 6;
constexpr int kRegBits = 4;        // tile coordinates held in registers per round
constexpr int kTileMinLog2Fast = 10;   // smallest tile of the register-round kernel
constexpr int kLatencyTilesLog2 = 8;   // below 2^8 tiles a pass leaves CUs idle (256 CUs)
constexpr int kXBits = 2;          // coordinates exchanged with lane bits 4, 5
constexpr int kChunkBits = kRegBits + kXBits;   // span coordinates per round

struct PassHost {
    int32_t group = -1;
    std::vector<int64_t> terms;     // merged-term ids
    int rho = 0, D = 0, c = 0;      // active dims, tile dims, coalescing pivots
    std::vector<uint64_t> basis;    // b_0..b_{D-1}: X-span basis, then spectators
    uint64_t free_mask = 0;         // non-pivot bit positions
    std::vector<uint64_t> u;        // echelon vectors sorted by pivot (D)
    std::vector<int> upiv;          // their pivots (ascending, first c = 0..c-1)
    std::vector<uint32_t> mr;       // column i = tile coords of u[i] (D-bit)
    std::vector<uint32_t> B;        // rho rows of the CZ/S form (bit j of B[i])
    uint32_t zq = 0;                // span coordinates with an extra Z: the layer
                                    // is i^{q(y)} (-1)^{popcount(y & zq)}
    std::vector<uint32_t> zeta;     // per term, D-bit mask of Lambda
    std::vector<uint64_t> ztile;    // per term, physical z for the tile sign
    std::vector<double> coef;       // per term, c_k (-1)^{r_k} i^{e_k}
    std::vector<double> usign;      // per term, (-1)^{r_k} i^{e_k} (+-1): coef without c_k
    double coef_abs_sum = 0;        // sum |c_k| (bounds the phase angle)
    // register-round schedule of the on-chip Walsh-Hadamard (see device.hip)
    int nr = 0;                     // chunks of <= kChunkBits span coordinates
    std::vector<int> chunk;         // span coordinates per chunk (contiguous)
    uint8_t reg[4][8] = {};         // tile coordinates in register slots 0..3
    uint8_t xl[4][2] = {};          // chunk coordinates on lane bits 4, 5
    int nx[4] = {};                 // how many of them are exchanged with
                                    // register bits 2, 3 (0..2)
    uint8_t regpost[4][4] = {};     // register coordinates after the exchange
    uint32_t bmask[4] = {};         // register slots that get butterflies (low bits)
    uint32_t iflag[4] = {};         // register slots whose coordinate has an S
    uint32_t dflag[4] = {};         // chunk slots (0..3 registers, 4..5 lanes) with a Z
    uint32_t later[4] = {};         // span coordinates of the chunks after r
    uint32_t czm[4] = {};           // bit g: sign of register pattern g from the
                                    // CZ between register slots of chunk r
    int lam_round = 0;              // chunk whose round applies Lambda
    bool full_rounds = true;        // every chunk before lam_round is full
    // lane bit i of a thread is tile coordinate vector lanes[r][i] in round r
    // before the exchange, lanes_post[r][i] after it; round 0 moves the tile
    // between HBM and registers directly
    std::vector<uint32_t> lanes[4], lanes_post[4];
    std::vector<uint64_t> io_phys;  // physical offsets of round 0's lane vectors
    uint64_t io_reg[4] = {};        // physical offsets of round 0's register slots
    int io_k = 0;                   // leading lanes on the lowest address bits
    bool staged = false;            // tile moves HBM <-> LDS in pivot order instead
    bool shift0 = false;            // round 0's lanes have components along its own
                                    // coordinates (lanes_post[0] drops them; the
                                    // kernel corrects the signs)
    uint32_t swz[4] = {};           // LDS swizzle: slot(t) = t ^ sum_j parity(t & swz[j]) << j
    std::vector<int32_t> bucket;    // 33 offsets: terms sorted by their Lambda
                                    // pattern on the registers of lam_round
};

// One HBM pass of the layer-by-layer (paper) execution of a group
// application, in application order.
struct LayerOp {
    enum Kind { H = 0, CNOT_FAN = 1, DIAG = 2 } kind;
    int a = -1;             // H: qubit; CNOT_FAN: control
    uint64_t mask = 0;      // CNOT_FAN: target mask
    // DIAG: multiply by i^{s_sign * popcount(x & smask)} (-1)^{sum_pairs x_a popcount(x & m)}
    //       exp(-i tau_frac * dt * sum_k c_k (-1)^{popcount(x & z_k)}) * scale
    int s_sign = 0;
    uint64_t smask = 0;
    int64_t cz_off = 0, cz_n = 0;      // pairs (a, mask) as 2 words each in layer_data
    int64_t lam_off = 0, lam_n = 0;    // (zmask, coef bits) as 2 words each
    double scale = 1.0;
};

struct Program {
    int D_max = 13, c = 4;
    std::vector<PassHost> passes;        // group order, sub-groups in order
    std::vector<int32_t> group_first;    // first pass of group g (K+1 entries)
};

// shrink: give each pass the smallest tile (down to 2^10) that holds it, so
// that small passes run several blocks per CU (complex64 runs faster so;
// complex128 keeps D_max).  c: contiguous low address bits of every tile;
// c_min < c lets a group's passes take down to c_min (at most two fewer)
// where the cost model finds that cheaper (fewer passes).
sd_status compile_program(int n, const std::vector<Term> &terms,
                          const std::vector<std::vector<int64_t>> &groups,
                          int D_max, int c, int c_min, Program *out, bool shrink);

// bytes of the packed device records of a program (device.hip)
int64_t pack_size(const Program &P);

}  // namespace sd

struct sd_plan_s {
    int32_t n = 0;
    std::vector<sd::Term> terms;
    std::vector<std::vector<int64_t>> groups;
    std::vector<sd::SynthResult> circuits;      // paper circuit per group
    std::vector<std::vector<int32_t>> gate_flat; // for export
    sd::Program prog[2];                        // [SD_C64], [SD_C128]
    int64_t paper_model_passes = 0;
    double plan_seconds = 0;
    // device side
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t ws_needed = 0;
    int64_t ws_off_prog[2] = {0, 0};   // byte offsets of packed pass tables
    int64_t ws_off_scratch = 0;        // reduction scratch
    int64_t ws_off_terms = 0;          // per-term expectations: partials, then results
    bool bound = false;
    uint64_t bind_epoch = 0;           // incremented by every sd_bind_workspace
    // layer-by-layer and term-by-term execution
    int32_t mode = SD_MODE_TILES;
    std::vector<std::vector<sd::LayerOp>> layers;   // per group, one application
    std::vector<uint64_t> layer_data;               // packed CZ pairs and Lambda terms
    int64_t ws_off_layers = 0;
};

namespace sd {
void build_layers(sd_plan_s &p);
// one application of group g in the plan's layer or term-by-term mode (layers.hip)
sd_status run_group_reference(const sd_plan_s *p, void *state, sd_dtype dtype, int g, double tau,
                              struct ihipStream_t *stream);
}
