/*
 * sd.h -- C ABI of the simultaneous-diagonalisation Trotter engine (gfx950).
 *
 * Method: Kawase & Fujii, "Fast classical simulation of Hamiltonian dynamics
 * by simultaneous diagonalization using Clifford transformation with parallel
 * computation" (arXiv:2206.11664).  A Hamiltonian H = sum_j c_j P_j (real c_j,
 * P_j in {I,X,Y,Z}^n; Sec. "Classical Simulation of Quantum Dynamics") is
 * partitioned into mutually commuting groups (Sec. "Partitioning Hamiltonian
 * Terms"); each group is diagonalised by a Clifford circuit found on the
 * binary tableau (Sec. "Partial Diagonalization of Hamiltonian", the
 * algorithms for steps (i)-(iv) and the appendix algorithm for independent
 * terms) and evolved as C^dagger exp(-i dt Lambda) C (Eq. trotter_simul_diag).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: every call returns sd_status; nothing throws across the ABI.
 *   sd_last_error() returns a thread-local message describing the last
 *   failure on the calling thread.
 * - Qubits: qubit q (0-based) is bit q of the amplitude index (the paper's
 *   basis |b_n...b_1> with qubit 1 least significant).  A dense Pauli string
 *   has character i acting on qubit i.  1 <= n_qubits <= 63.
 * - State: 2^n contiguous amplitudes, interleaved (re, im): float pairs for
 *   SD_C64, double pairs for SD_C128 (the layouts of torch.complex64 and
 *   torch.complex128).  The state is caller-owned device memory and is
 *   updated in place.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  Device work is enqueued asynchronously unless stated otherwise.
 * - Handles: distinct handles may be used from distinct threads at once; one
 *   handle must not be used by two threads at once.  Plans are immutable
 *   after sd_plan, except for the workspace binding.
 */
#ifndef SD_H
#define SD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SD_OK = 0,
    SD_ERR_ARG = 1,        /* null pointer, bad size, bad enum value          */
    SD_ERR_PARSE = 2,      /* malformed Pauli string                          */
    SD_ERR_RANGE = 3,      /* qubit index / qubit count / value out of range  */
    SD_ERR_WORKSPACE = 4,  /* no workspace bound, or workspace too small      */
    SD_ERR_HIP = 5,        /* a HIP runtime call or kernel launch failed      */
    SD_ERR_INTERNAL = 6,   /* planner self-check failed (e.g. a term not
                              diagonalised by its group's Clifford)          */
    SD_ERR_STATE = 7       /* object in the wrong state (e.g. destroyed)      */
} sd_status;

typedef enum {
    SD_C64 = 0,   /* complex64 amplitudes; phase angle, phase factor and
                     butterflies evaluated in FP64, rounded once per pass     */
    SD_C128 = 1   /* complex128 amplitudes, FP64 throughout                   */
} sd_dtype;

typedef struct sd_hamiltonian sd_hamiltonian;
typedef struct sd_plan_s sd_plan_t;
typedef struct sd_ensemble sd_ensemble;

/* --------------------------------------------------------------------------
 * Hamiltonian: H = sum_j c_j P_j (Sec. "Classical Simulation of Quantum
 * Dynamics").  Exact duplicate strings are merged by summing their
 * coefficients at the first occurrence; identity terms and zero coefficients
 * are kept.  Inputs are copied; the caller may free them after the call.
 * -------------------------------------------------------------------------- */

/* paulis[j]: dense "XIZY..." (length n, character i = qubit i) or sparse
   "X0 Y3 Z7" (letter + 0-based qubit, each qubit at most once).
   Errors: SD_ERR_ARG (null pointers, n_terms < 0), SD_ERR_RANGE (n outside
   1..63, qubit >= n), SD_ERR_PARSE (other characters, repeated qubit, wrong
   dense length), SD_ERR_ARG for a non-finite coefficient. */
sd_status sd_hamiltonian_create(int32_t n_qubits, int64_t n_terms,
                                const char *const *paulis, const double *coeffs,
                                sd_hamiltonian **out);

/* Symplectic form (Sec. "Tableau Representation"): bit q of xmask/zmask is
   x_q/z_q; (1,0)=X, (0,1)=Z, (1,1)=Y.  Bits at q >= n are SD_ERR_RANGE. */
sd_status sd_hamiltonian_create_masks(int32_t n_qubits, int64_t n_terms,
                                      const uint64_t *xmask, const uint64_t *zmask,
                                      const double *coeffs, sd_hamiltonian **out);

/* Merged terms (read-only views valid until sd_hamiltonian_destroy).
   source[j] is the input index of the first occurrence of merged term j. */
sd_status sd_hamiltonian_terms(const sd_hamiltonian *h, int32_t *n_qubits,
                               int64_t *n_terms, const uint64_t **xmask,
                               const uint64_t **zmask, const double **coeffs,
                               const int64_t **source);

void sd_hamiltonian_destroy(sd_hamiltonian *h);

/* --------------------------------------------------------------------------
 * Planning (host only, no device work).
 * -------------------------------------------------------------------------- */
typedef struct {
    /* Apply the skip rule before steps (ii)/(iii): qubits carrying only
       {I,Z} in a group are left alone and qubits carrying only {I,X} get a
       Hadamard (end of Sec. "Partial Diagonalization of Hamiltonian").
       Default 1. Affects the exported paper circuit only. */
    int32_t skip_rule;
    /* Largest tile (amplitudes staged on chip per work-group) as log2, per
       dtype.  Range 6..13; the default (sd_plan_options_default) is 13 for
       both, and values outside the range are SD_ERR_RANGE.  complex64
       passes take the smallest tile of at least 2^10 that holds them, up to
       this size; sd_autotune_tiles measures which maximum runs fastest.
       Callers start from sd_plan_options_default and change fields: a
       zero-filled struct is not the default. */
    int32_t tile_log2_c64;
    int32_t tile_log2_c128;
    /* Low qubits every tile must contain so that global accesses are whole
       runs of 2^c amplitudes.  Range 0..6 and below the tile size; 0 means
       no such qubits (not the default).  Default 4 for c64 (128 B runs) and
       3 for c128 (128 B). */
    int32_t coalesce_log2_c64;
    int32_t coalesce_log2_c128;
    /* Execution mode of sd_evolve (sd_expectation always uses the tiles):
       SD_MODE_TILES (default): one fused tile pass per commuting sub-group;
       SD_MODE_PAPER_LAYERS: the paper's circuit layer by layer, one HBM pass
         per H gate, per CNOT control (its fan-out applied at once), for all
         S+CZ, and for Lambda (Sec. "Implementations");
       SD_MODE_TERMWISE: one Pauli-rotation pass per term (Eq. trotter_decomp,
         the paper's baseline), in the same group order. */
    int32_t mode;
    /* complex64: the fewest contiguous low bits a group's passes may fall
       back to (at most two below coalesce_log2_c64) where that needs fewer
       passes and the planner's cost model finds it cheaper: each fewer
       pass is one fewer HBM round trip and one fewer complex64 rounding of
       every amplitude.  Default 2 (32-byte runs); a value of at least
       coalesce_log2_c64 keeps every pass at that width; negative values
       are SD_ERR_RANGE. */
    int32_t coalesce_min_log2_c64;
    /* complex64: 1 (default) gives each pass the smallest tile (at least
       2^10) that holds its sub-group, so that small passes run several
       blocks per CU, and splits each group for tiles one or two
       coordinates smaller where that needs no more passes; 0 keeps every
       pass at min(tile_log2_c64, n_qubits) (one tile size for the whole
       plan, as complex128 always has). */
    int32_t tile_shrink_c64;
    /* 1 (default): a state of fewer than 256 tiles of the size above (too
       few to occupy the 256 CUs; each pass then waits on the latency of one
       tile) takes, per dtype, the smallest tile of at least 2^10 that needs
       no more passes, so that a pass spreads over more CUs.  0 keeps the
       size above (ensembles, whose instances share the GPU, may prefer
       it). */
    int32_t small_state_tiles;
} sd_plan_options;

enum { SD_MODE_TILES = 0, SD_MODE_PAPER_LAYERS = 1, SD_MODE_TERMWISE = 2 };

/* Fill `opt` with the defaults. */
void sd_plan_options_default(sd_plan_options *opt);

/* Partition the merged terms into commuting groups by first fit in term
   order (greedy colouring of the anticommutation graph), synthesise each
   group's diagonalising Clifford (paper steps (i)-(iv)), verify that every
   term of every group becomes a signed Z-string, and compile the device
   tile programs.  opt may be NULL (defaults).  The plan keeps no reference
   to h.  Errors: SD_ERR_ARG, SD_ERR_INTERNAL (self-check failed). */
sd_status sd_plan(const sd_hamiltonian *h, const sd_plan_options *opt,
                  sd_plan_t **out);

typedef struct {
    int32_t n_qubits;
    int64_t n_terms;            /* merged terms                               */
    int32_t n_groups;           /* commuting groups (K)                       */
    int64_t max_group_terms;
    int32_t passes_c64;         /* device passes per first-order step         */
    int32_t passes_c128;
    int64_t paper_model_passes; /* passes per first-order step in the paper's
                                   cost model: one per H gate, one per CNOT
                                   control, one for S+CZ, one for Lambda,
                                   doubled for C and C^dagger except Lambda  */
    int64_t workspace_bytes;    /* device bytes sd_bind_workspace needs       */
    double plan_seconds;
} sd_plan_info;

sd_status sd_plan_info_get(const sd_plan_t *p, sd_plan_info *info);

/* Gate kinds of an exported circuit. */
enum { SD_GATE_H = 0, SD_GATE_S = 1, SD_GATE_CNOT = 2, SD_GATE_CZ = 3 };

typedef struct {
    int32_t n_terms;
    const int64_t *term_ids;   /* merged-term indices, group order            */
    const uint64_t *zmask;     /* C P_k C^dagger = (-1)^sign[k] Z^{zmask[k]}  */
    const int8_t *sign;        /* 0 or 1                                      */
    int32_t n_gates;
    const int32_t *gates;      /* n_gates triples (kind, a, b), application
                                  order (first acts first); b = -1 for 1q     */
    int32_t n_independent;     /* terms returned by the independent-set step  */
    const int64_t *independent;/* their merged-term indices, tableau order    */
} sd_group_view;

/* Group g's terms and its Clifford as the paper's algorithm builds it.
   Views stay valid until sd_plan_destroy. */
sd_status sd_plan_export_group(const sd_plan_t *p, int32_t g, sd_group_view *v);

typedef struct {
    int32_t group;       /* owning commuting group                            */
    int32_t n_terms;
    const int64_t *term_ids;
    int32_t rho;         /* dimension of the terms' X span (Hadamard dims)    */
    int32_t tile_log2;   /* D: rho plus spectator low qubits                  */
    const uint64_t *basis;     /* D physical vectors: rho X-span basis vectors,
                                  then the spectator unit vectors             */
    int32_t coalesce_log2;     /* c: address bits 0..c-1 are tile pivots      */
    uint64_t free_mask;        /* address bits enumerated by the tile index   */
    const uint64_t *pivot_vec; /* D vectors, one per tile pivot (ascending
                                  pivot bit); address = base ^ sum pi_i vec_i */
    const uint32_t *pivot_coord; /* D masks: tile coordinates of pivot_vec[i] */
    const uint32_t *cz_s;      /* rho rows of the CZ/S layer: bit j of row i
                                  set for CZ(i,j), bit i for S(i)             */
    const uint32_t *zeta;      /* per term: Lambda Z-mask in tile coordinates  */
    const uint64_t *ztile;     /* per term: physical Z part for the tile sign  */
    const double *coef;        /* per term: signed coefficient                */
    uint32_t z_sign;           /* span coordinates with an extra Z in the CZ/S
                                  layer: it multiplies tile coordinate y by
                                  i^{q(y)} (-1)^{popcount(y & z_sign)}, q(y) =
                                  sum_i y_i popcount(cz_s[i] & y)             */
} sd_pass_view;

/* Device pass list for one dtype, in application order for group order 1. */
sd_status sd_plan_pass_count(const sd_plan_t *p, sd_dtype dt, int32_t *count);
sd_status sd_plan_export_pass(const sd_plan_t *p, sd_dtype dt, int32_t i,
                              sd_pass_view *v);

/* Register-round schedule of one tile pass.  The on-chip Walsh-Hadamard of
   the rho span coordinates runs in rounds; a thread holds 16 amplitudes.
   Round r transforms chunk r: its first coordinates sit in register slots
   0..3 (reg[r]; only the low popcount(bmask[r]) slots are transformed, the
   others carry filler coordinates), the next nx[r] on lane bits 4 and 5
   (xl[r]); after the register butterflies register bits 2, 3 are exchanged
   with lane bits 4, 5, leaving register coordinates regpost[r].  Lane bit i
   of a thread is tile coordinate vector lanes[r][i] before the exchange and
   lanes_post[r][i] after it; round 0 moves amplitudes between HBM and
   registers directly, and its first io_coalesced lanes are the lowest
   address bits.  iflag/dflag mark chunk slots (0..3 registers, 4..5 lanes)
   whose coordinate carries an S / a Z of the CZ/S layer; later[r] is the
   mask of span coordinates of the chunks after r.  Lambda is applied in the
   round of lam_round; terms (in the pass view's order) are grouped by their
   Lambda pattern on that round's registers after the exchange: pattern w owns
   terms bucket[w] .. bucket[w+1]-1.  On-chip slot of tile coordinate t:
   t ^ sum_j parity(t & swz[j]) << j.  Views stay valid until sd_plan_destroy.
   Errors: SD_ERR_ARG, SD_ERR_RANGE (pass index). */
typedef struct {
    int32_t n_rounds;          /* chunks (0 when rho = 0: one Lambda round)    */
    int32_t lam_round;
    int32_t reg[4][4];
    int32_t regpost[4][4];
    int32_t xl[4][2];
    int32_t nx[4];
    uint32_t bmask[4];
    uint32_t iflag[4];
    uint32_t dflag[4];
    uint32_t later[4];
    const int32_t *bucket;     /* 17 offsets                                    */
    int32_t n_lanes;           /* D - 4                                         */
    int32_t io_coalesced;
    const uint32_t *lanes[4];
    const uint32_t *lanes_post[4];
    uint32_t swz[4];
    int32_t staged;            /* 1: the tile moves between HBM and LDS in pivot
                                  order (pivot_vec / pivot_coord of the pass
                                  view) and round 0 reads it from LDS; used when
                                  the lowest address bits cannot be round 0's
                                  leading lanes                                */
    uint32_t czmask[4];        /* round r: bit g = 1 if register pattern g takes
                                  a sign from the CZ between the chunk's register
                                  slots (before a forward round's butterflies,
                                  after a backward round's)                    */
    int32_t shift0;            /* 1: round 0's leading lanes (the low address
                                  bits) have components along round 0's own
                                  coordinates; lanes_post[0] holds them without
                                  those components (the layout round 0 writes
                                  to LDS), and the outputs of round 0, when it
                                  is not Lambda's round, carry the sign
                                  (-1)^{k.d}: k the output coordinates, d the
                                  dropped components of the thread's lanes    */
} sd_round_view;
sd_status sd_plan_export_rounds(const sd_plan_t *p, sd_dtype dt, int32_t i,
                                sd_round_view *v);

void sd_plan_destroy(sd_plan_t *p);

/* --------------------------------------------------------------------------
 * Device execution.
 * -------------------------------------------------------------------------- */

/* Bind caller-allocated device memory (>= workspace_bytes, 256-byte aligned)
   to the plan and upload the tile programs into it on `stream`.  The memory
   must stay allocated while the plan is used on the device.  Rebinding is
   allowed.  Errors: SD_ERR_WORKSPACE (too small / misaligned), SD_ERR_HIP. */
sd_status sd_bind_workspace(sd_plan_t *p, void *dev_ptr, size_t bytes, void *stream);

/* state <- (prod over the step schedule of C_g^dagger exp(-i tau Lambda_g) C_g)^steps
   state, Eq. trotter_simul_diag, with tau = dt (order 1: groups 0..K-1), the
   symmetric sequence dt/2 (0..K-2), dt (K-1), dt/2 (K-2..0) for order 2, or
   for order 4 Suzuki's fractal of five order-2 sequences at p dt, p dt,
   (1-4p) dt, p dt, p dt with p = 1/(4 - 4^(1/3)) (boundaries not merged).
   Asynchronous on `stream`.  state: device pointer to 2^n amplitudes of
   `dtype`.  Errors: SD_ERR_ARG (order not 1/2/4, steps < 0, non-finite dt),
   SD_ERR_WORKSPACE (no workspace), SD_ERR_HIP. */
sd_status sd_evolve(const sd_plan_t *p, void *state, sd_dtype dtype, double dt,
                    int64_t steps, int32_t order, void *stream);

/* energy = <psi|H|psi> / 1 (not normalised by <psi|psi>), evaluated per
   group through its diagonal form (the grouped-expectation use of the
   partition, Sec. "Partitioning Hamiltonian Terms"), accumulated in FP64.
   Synchronises `stream`; energy is a host pointer. */
sd_status sd_expectation(const sd_plan_t *p, const void *state, sd_dtype dtype,
                         double *energy, void *stream);

/* out[k] = <psi|P_k|psi> (not normalised) for every merged term k of the
   plan's Hamiltonian (the order of sd_hamiltonian_terms): the grouped
   measurement of Sec. "Partitioning Hamiltonian Terms" -- one transform per
   (sub-)group, C_g psi, gives every term of the group at once through its
   diagonal form, here all of them from one pass per tile program.  Any
   observable that is a linear combination of the terms then follows on the
   host, e.g. at every step of a time series; observables outside H get a
   plan of their own.  FP64 accumulation, fixed summation order.  state:
   device pointer to 2^n amplitudes of `dtype`; out: host array of
   sd_plan_info.n_terms doubles.  Synchronises `stream`.  Errors: SD_ERR_ARG,
   SD_ERR_WORKSPACE (no workspace), SD_ERR_HIP. */
sd_status sd_term_expectations(const sd_plan_t *p, const void *state, sd_dtype dtype,
                               double *out, void *stream);

/* Autotuning of the tile size (the on-chip block of 2^D amplitudes a
   work-group transforms) for one Hamiltonian on this GPU.  For each of the
   n_candidates maximum tile sizes (log2, 6..13) a plan with the options
   `base` (NULL: defaults) and that size for `dtype` is built and bound to the
   caller's `workspace`, one step is run as warm-up and `steps` Trotter steps
   (dt, order) are timed with HIP events on `stream`.  workspace: caller-owned
   device memory, 256-byte aligned, of at least the bytes that
   sd_autotune_workspace_bytes reports for the same h, base, dtype and
   candidates (the largest plan workspace among the candidates); the library
   allocates no device memory.  state: device pointer to 2^n amplitudes of
   `dtype`, used as scratch (its contents are evolved).  best: the options of
   the fastest candidate (base with the winning size for `dtype` and
   small_state_tiles 0: every candidate runs at its own size); seconds:
   host array of n_candidates per-step times, or NULL.  Synchronises
   `stream`.  Errors: SD_ERR_ARG, SD_ERR_RANGE (candidate out of range),
   SD_ERR_WORKSPACE (workspace too small or misaligned), SD_ERR_HIP, and
   those of sd_plan. */
sd_status sd_autotune_workspace_bytes(const sd_hamiltonian *h, const sd_plan_options *base,
                                      sd_dtype dtype, const int32_t *candidates,
                                      int32_t n_candidates, int64_t *bytes);
sd_status sd_autotune_tiles(const sd_hamiltonian *h, const sd_plan_options *base,
                            sd_dtype dtype, void *state, double dt, int32_t order,
                            int32_t steps, const int32_t *candidates, int32_t n_candidates,
                            void *workspace, size_t workspace_bytes,
                            sd_plan_options *best, double *seconds, void *stream);

/* FP64 reductions over 2^n amplitudes (device inputs, host outputs;
   synchronise `stream`).  sd_norm2: sum |a_x|^2.  sd_inner: sum conj(a_x) b_x
   written to out[0] (re), out[1] (im).  Per-block partial sums go to the
   caller's `scratch`: device memory of at least
   sd_reduction_scratch_bytes() bytes, 8-byte aligned, not used by other
   work while the call runs; its contents are overwritten.  The partial sums
   are combined in a fixed order, so equal inputs give bit-identical results.
   Errors: SD_ERR_ARG (null pointers, bad dtype), SD_ERR_RANGE (n_qubits
   outside 0..40), SD_ERR_WORKSPACE (scratch too small or misaligned),
   SD_ERR_HIP. */
int64_t sd_reduction_scratch_bytes(void);
sd_status sd_norm2(const void *state, sd_dtype dtype, int32_t n_qubits,
                   double *out, void *scratch, size_t scratch_bytes, void *stream);
sd_status sd_inner(const void *a, const void *b, sd_dtype dtype, int32_t n_qubits,
                   double *out, void *scratch, size_t scratch_bytes, void *stream);

/* sd_inner for callers that cannot allocate device memory at all (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same kernels and the same fixed summation order as sd_inner (equal
   inputs give bit-identical results), with the per-block partial sums in a
   library-owned static device array of 33,280 bytes instead of caller
   scratch.  Every GPU the library runs on holds one such array until the
   process ends; calls on one GPU share it, so calls that overlap on one GPU
   (other streams or threads) race and must be serialised by the caller.
   The call allocates nothing.  a, b: device arrays of 2^n_qubits amplitudes
   of `dtype`; out: host, out[0] = re, out[1] = im of sum conj(a_x) b_x;
   synchronises `stream`.  Errors: SD_ERR_ARG (null pointers, bad dtype),
   SD_ERR_RANGE (n_qubits outside 0..40, or a device ordinal above 63),
   SD_ERR_HIP. */
sd_status sd_inner_noalloc(const void *a, const void *b, sd_dtype dtype, int32_t n_qubits,
                           double *out, void *stream);

/* Ensemble of independent instances (uneven sizes allowed), evolved together.
   plans: `count` plans, each with a bound workspace; states: host array of
   `count` device pointers.  One launch per pass level (and tile size) per
   step over the tiles of every instance; instances with tiles below 2^10
   or states above 4 GiB take their own pass launches after those.  A step
   is captured once as one HIP graph and replayed (a call: prologue, core
   step x (steps - 1), epilogue, where group applications joined across
   steps differ).
   sd_ensemble_workspace_bytes: the device bytes for the per-level segment
   tables, enough for every order (1, 2, 4); the caller allocates them
   (256-byte aligned) and binds them with sd_ensemble_bind_workspace before
   sd_ensemble_evolve (SD_ERR_WORKSPACE otherwise).  The ensemble keeps
   pointers to the plans, which must outlive it; a plan may be rebound to
   another workspace between calls (the next sd_ensemble_evolve rebuilds
   its step tables, as it does for other state pointers, dt or order). */
sd_status sd_ensemble_create(const sd_plan_t *const *plans, int32_t count,
                             sd_dtype dtype, sd_ensemble **out);
sd_status sd_ensemble_workspace_bytes(const sd_ensemble *e, int64_t *bytes);
sd_status sd_ensemble_bind_workspace(sd_ensemble *e, void *dev_ptr, size_t bytes,
                                     void *stream);
sd_status sd_ensemble_evolve(sd_ensemble *e, void *const *states, double dt,
                             int64_t steps, int32_t order, void *stream);
void sd_ensemble_destroy(sd_ensemble *e);

/* Wait for `stream` and report any asynchronous HIP error as SD_ERR_HIP. */
sd_status sd_sync(void *stream);

const char *sd_status_string(sd_status s);
const char *sd_last_error(void);
const char *sd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SD_H */
