/*
 * qsim355 -- full-state quantum circuit simulation on one AMD Instinct MI355X.
 *
 * C ABI.  Every function returns a sim_status (SIM_OK == 0) unless stated;
 * no C++ exception crosses this boundary.  A context is not thread-safe;
 * distinct contexts may be used from distinct threads.
 *
 * Semantics (paper Sec. 2.1-2.2, Eq. (1)): an N-qubit state holds 2^N complex
 * amplitudes a_i, i in [0, 2^N); qubit j is bit j of i.  A k-qubit gate on
 * the ordered qubit list q[0..k-1] multiplies, for every assignment of the
 * other bits, the 2^k amplitudes it touches by its 2^k x 2^k matrix, where
 * bit t of the matrix row/column index is bit q[t] of i (an ascending list
 * reproduces the two-qubit layout of Sec. 2.2).  sim_run starts from
 * |0...0> and applies the circuit in input order (gate-by-gate definition,
 * Alg. 1); every optimisation the library applies (merge booster Sec. 4.4,
 * diagonal detector Sec. 4.5, cache-blocked stages Alg. 2, gate fusion,
 * qubit reordering Sec. 2.3) yields that same state up to rounding.
 *
 * All indices, amplitudes and probabilities at this boundary are in logical
 * qubit order; internal qubit remapping is undone by the library.
 *
 * Memory: the state vector lives in a caller-owned device buffer (e.g. a
 * torch tensor) passed in sim_options and must outlive the context.  The
 * context owns its plan and the small device tables it uploads.  Host output
 * buffers are caller-owned.
 */
#ifndef QSIM355_H
#define QSIM355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_ctx sim_ctx;
typedef struct sim_plan sim_plan;

typedef enum {
    SIM_OK = 0,
    SIM_E_INVAL = 1,       /* bad argument: qubit >= N, duplicate qubits, k > 6,
                              NULL data for MATRIX/DIAG, non-unitary MATRIX
                              (error > 1e-10), non-unit DIAG entry, NULL pointer */
    SIM_E_NOMEM = 2,       /* a device or host buffer is too small / allocation failed */
    SIM_E_DEVICE = 3,      /* a HIP runtime error; text from sim_last_error */
    SIM_E_STATE = 4,       /* call out of order (e.g. outputs before sim_run) */
    SIM_E_UNSUPPORTED = 5  /* valid request outside what the library implements */
} sim_status;

typedef enum { SIM_C128 = 0, SIM_C64 = 1 } sim_dtype;

/* Gate kinds.  Matrices of the named gates are the textbook ones:
 *   H, X, Y, Z, S = diag(1, i), T = diag(1, e^{i pi/4}),
 *   SX = (1/2)[[1+i, 1-i], [1-i, 1+i]],
 *   RX/RY/RZ(theta) = exp(-i theta P / 2) for P = X, Y, Z,
 *   CZ = diag(1, 1, 1, -1), CPHASE(theta) = diag(1, 1, 1, e^{i theta}),
 *   RZZ(theta) = exp(-i theta Z(x)Z / 2),
 *   CNOT: q[0] control, q[1] target; SWAP exchanges q[0] and q[1]. */
typedef enum {
    SIM_G_MATRIX = 0,  /* data: 2^k x 2^k complex, row-major, interleaved (re, im) FP64 */
    SIM_G_DIAG = 1,    /* data: 2^k complex diagonal, interleaved (re, im) FP64 */
    SIM_G_H, SIM_G_X, SIM_G_Y, SIM_G_Z, SIM_G_S, SIM_G_T, SIM_G_SX,
    SIM_G_RX, SIM_G_RY, SIM_G_RZ,
    SIM_G_CZ, SIM_G_CNOT, SIM_G_CPHASE, SIM_G_RZZ, SIM_G_SWAP,
    SIM_G_NKINDS
} sim_gate_kind;

typedef struct {
    uint32_t kind;      /* sim_gate_kind */
    uint32_t nq;        /* number of qubits k (1..6); must equal the kind's arity */
    uint32_t q[6];      /* ordered qubit list; bit t of the matrix index <-> q[t] */
    double theta;       /* angle of RX/RY/RZ/CPHASE/RZZ, ignored otherwise */
    const double *data; /* MATRIX/DIAG payload (host memory, read during the call) */
} sim_gate;

/* Optimisation passes (bit flags for sim_options.opt). */
enum {
    SIM_OPT_DIAG = 1u << 0,    /* diagonal detector (Sec. 4.5, Alg. 8) */
    SIM_OPT_FUSE = 1u << 1,    /* cost-based gate fusion up to F qubits */
    SIM_OPT_STAGES = 1u << 2,  /* cache blocking: chunk-resident stages (Alg. 2, Alg. 5) */
    SIM_OPT_BOOST = 1u << 3,   /* merge booster (Sec. 4.4, Alg. 6-7) */
    SIM_OPT_REMAP = 1u << 4,   /* qubit reordering (Sec. 2.3): permutation passes between
                                  stages (needs STAGES), and SWAP gates (an exact 0/1 exchange
                                  matrix) become relabellings that move no data */
    SIM_OPT_QUAD = 1u << 5,    /* with FUSE: the one- and two-qubit diagonals a register phase
                                  collects become one quadratic-phase operator (phase
                                  c + sum a_q x_q + sum b_qp x_q x_p) when that costs less than
                                  their diagonal tables; not used with host-memory
                                  offload */
    SIM_OPT_ALL = 0x3Fu
};

typedef struct {
    uint32_t opt;          /* SIM_OPT_* flags; 0 = gate by gate (Alg. 1) */
    uint32_t C;            /* chunk qubits of a stage: 0 = default (12 for C128, 13 for C64);
                              otherwise 10..13 (C128) or 11..14 (C64), else sim_create
                              returns SIM_E_INVAL */
    uint32_t F;            /* max qubits of a fused dense gate (0 = default 5) */
    uint32_t D;            /* max qubits of a fused diagonal (0 = default 10) */
    uint32_t B;            /* booster division parameter (0 = default 4) */
    uint32_t force_fuse_k; /* >0: fusion-only plans fuse greedily to this many qubits
                              regardless of cost (exercises the MFMA path) */
    uint32_t L;            /* lowest physical qubits every stage keeps local, 1..6 (0 = default:
                              one 128-byte cache line per contiguous run, 3 for C128, 4 for C64) */
    uint32_t reserved;     /* 0 */
    void *dev_state;           /* device buffer, >= 2^N * 16 B (C128) or 8 B (C64) */
    uint64_t dev_state_bytes;
    void *stream;              /* hipStream_t the context launches on (NULL = default) */
    /* Host-memory offload (states larger than the device memory given to the
     * library; the related-work direction of Sec. 2.5 with the cache-blocked
     * stages of Alg. 2 run window by window).  NULL: the state lives in
     * dev_state.  Otherwise host_state holds the 2^N amplitudes (pinned host
     * memory from hipHostMalloc, caller-owned, >= 2^N * 16 B or 8 B), and
     * dev_state is only a work area of two windows: the largest W with
     * 2 * 2^W amplitudes <= dev_state_bytes (W <= N - 1) sets the window.
     * Each offload pass fixes S = N - W outer qubits (a contiguous range of
     * bit positions that the pass's gates only read as controls or diagonal
     * indices), copies the 2^S windows through the device in turn, runs the
     * pass's stages on each and copies it back, with the copies overlapping
     * the compute on two extra streams.  Needs SIM_OPT_STAGES; the booster
     * and qubit reordering are not used in this mode.  Outputs:
     * sim_amplitudes, sim_probabilities and sim_stats; the other output and
     * measurement calls return SIM_E_UNSUPPORTED. */
    void *host_state;
    uint64_t host_state_bytes;
} sim_options;

typedef struct {
    uint64_t n_gates;          /* gates of the loaded circuit */
    uint64_t n_ops;            /* ops of the executed plan */
    uint64_t full_passes;      /* read+write passes over the full state */
    uint64_t write_passes;     /* write-only passes (init, tensor product not formed on load) */
    uint64_t read_passes;      /* read-only passes (reductions) of the last output call */
    uint64_t n_stages;         /* cache-blocked stage ops */
    uint64_t n_dense;          /* full-pass dense ops */
    uint64_t n_diag;           /* full-pass diagonal ops */
    uint64_t n_kron;           /* tensor products */
    uint64_t n_perm;           /* qubit permutations */
    uint64_t n_subruns;        /* ops run on booster sub-states */
    double plan_ms;            /* host optimiser time of the last sim_load_circuit */
    double run_ms;             /* device time of the last sim_run (HIP events) */
    double algorithmic_bytes;  /* bytes the plan moves over the full state (a tensor product
                                  formed by the next stage's chunk loads counts neither its
                                  write nor that stage's read) */
    double flops;              /* floating-point operations of the plan (estimate) */
    double est_ms;             /* device time of the plan predicted by the optimiser's cost model */
    uint64_t offload_passes;   /* host-memory offload: passes that stream the whole state through
                                  the device (0 when the state is device-resident) */
    uint64_t window_qubits;    /* host-memory offload: qubits W of a device window */
    double pcie_bytes;         /* host-memory offload: bytes copied between host and device per run */
} sim_run_stats;

/* Create a context for an n_qubits state of the given dtype (the N-qubit
 * state of Sec. 2.1: 2^N complex amplitudes, qubit j = bit j of the index).
 * opts->dev_state must hold 2^n amplitudes (SIM_E_NOMEM otherwise).
 * n_qubits: 1..36 (35 qubits in complex64 fill 256 GiB of HBM; larger
 * states need host-memory offload).  *out receives the context (caller
 * frees with sim_destroy). */
sim_status sim_create(uint32_t n_qubits, sim_dtype dtype, const sim_options *opts, sim_ctx **out);

/* Validate and deep-copy the circuit (gates as defined in Sec. 2.2), then
 * build the execution plan with the context's options: the optimiser of
 * Sec. 4 (gate block search of Sec. 4.2 with limits C and F, merge booster
 * Sec. 4.4, diagonal detector Sec. 4.5) choosing among the simulation
 * schemes of Sec. 2.4.  Host only; no device work except uploading tables.
 * On error the previously loaded circuit stays in place. */
sim_status sim_load_circuit(sim_ctx *ctx, const sim_gate *gates, uint64_t n_gates);

/* Initialise |0...0>, execute the plan on the context's stream and wait
 * for completion (Alg. 5 adaptive simulation). */
sim_status sim_run(sim_ctx *ctx);

/* As sim_run, without waiting: the work is enqueued on the stream; the
 * state may be read only after the stream has been synchronised. */
sim_status sim_run_async(sim_ctx *ctx);

/* Copy amplitudes to host (the simulation result of Sec. 2.4: all amplitudes
 * of the final state): out[2*i], out[2*i+1] = re, im of amplitude
 * idx[i] (logical index).  idx == NULL copies all 2^N amplitudes (n must then
 * be 2^N).  Synchronises the stream.  Requires a completed sim_run. */
sim_status sim_amplitudes(sim_ctx *ctx, const uint64_t *idx, uint64_t n, double *out);

/* Marginal probabilities over the qubit list (the paper's measurement
 * background in Sec. 2, an unnumbered subsection between Sec. 2.3 and
 * Sec. 2.4: the probability of an outcome is the squared norm of the
 * amplitudes the projector keeps):
 * out[y] = sum over i whose bit qubits[t] equals bit t of y of |a_i|^2,
 * accumulated in FP64 in a fixed order (deterministic).  nq = 0 gives the
 * norm in out[0].  nq <= 16.  out holds 2^nq doubles (host). */
sim_status sim_probabilities(sim_ctx *ctx, const uint32_t *qubits, uint32_t nq, double *out);

/* sim_probabilities for callers that cannot allocate device memory (code
 * that must not call hipMalloc: under HIP graph capture, in tight serving
 * loops, in harnesses that forbid it).  Same arguments, validation, kernels
 * and results (bitwise) as sim_probabilities, but every intermediate lives in
 * a static device array of 24 MiB per GPU (held until the process ends)
 * instead of context-owned buffers: the call allocates nothing.  A request
 * whose partial sums would exceed that array fails with SIM_E_UNSUPPORTED
 * (not reachable for nq <= 16 at any supported N).  All contexts on one GPU
 * share the array, so calls that overlap on one GPU (from several threads or
 * streams) race; calls in sequence are safe (every value is written before
 * it is read).  The device is that of the context's creation; out is host
 * memory of 2^nq doubles; the call synchronises the context's stream. */
sim_status sim_probabilities_noalloc(sim_ctx *ctx, const uint32_t *qubits, uint32_t nq, double *out);

/* <a|b> = sum_i conj(a_i) b_i between the states of two contexts with the
 * same N (any dtypes), accumulated in FP64 in a fixed order. out[0..1] =
 * (re, im).  Both contexts must have run; launched on a's stream. */
sim_status sim_inner(sim_ctx *a, sim_ctx *b, double *out);

sim_status sim_stats(const sim_ctx *ctx, sim_run_stats *out);

/* ---- measurement (the projective model of the paper's measurement
 * background, Sec. 2: M_i^j keeps the amplitudes whose qubit j is i, and
 * <psi|M_i^j|psi> is the probability of outcome i) ----------------------------
 * All require a completed run, act on the state the last run produced, take
 * qubits and indices in logical order, and synchronise the stream.  Random
 * numbers are inputs: u values are uniforms in [0, 1) the caller draws
 * (SIM_E_INVAL for any other value). */

/* Measure qubit `qubit`: with p0 = sum over i with bit qubit = 0 of |a_i|^2
 * and p1 likewise (FP64, fixed order), the outcome is 0 if u < p0 / (p0 + p1)
 * and 1 otherwise.  The state collapses in place: amplitudes of the other
 * outcome become 0 and the kept ones are divided by sqrt(p_outcome), one
 * pass.  *outcome (may be NULL) receives the outcome, *prob (may be NULL)
 * its probability p_outcome / (p0 + p1). */
sim_status sim_measure(sim_ctx *ctx, uint32_t qubit, double u, uint32_t *outcome, double *prob);

/* Draw n_shots basis states by inverting the cumulative distribution in
 * logical index order: out[s] = the smallest x whose cumulative mass
 * sum_{y <= x} |a_y|^2 exceeds u[s] * T, T the total mass.  The result
 * always has nonzero probability.  Cumulative sums are FP64 in a fixed order
 * (a marginal over the top logical qubits, then in-block prefix sums), so
 * for a u within rounding of a boundary the index next to it may come out.
 * The state is not changed.  n_shots <= 2^31; u and out are host arrays of
 * n_shots entries. */
sim_status sim_sample(sim_ctx *ctx, const double *u, uint64_t n_shots, uint64_t *out);

/* Expectation values of Z strings: out[k] = <psi| Z_S |psi> =
 * sum_x |a_x|^2 (-1)^popcount(x & masks[k]), masks[k] a bit mask of logical
 * qubits (mask 0 gives the squared norm).  One FP64 pass over the state per
 * 16 masks; deterministic. */
sim_status sim_expect_z(sim_ctx *ctx, const uint64_t *masks, uint32_t n_masks, double *out);

/* Expectation value of a real diagonal observable on nq <= 16 qubits:
 * *out = sum_y P(y) f[y], P the marginal of sim_probabilities over `qubits`
 * (bit t of y <-> qubits[t]); f holds 2^nq doubles. */
sim_status sim_expect_diagonal(sim_ctx *ctx, const uint32_t *qubits, uint32_t nq, const double *f, double *out);

/* Per-op device timing: when enabled, sim_run records a pair of HIP events on
 * the context's stream around every kernel launch of the plan. */
sim_status sim_set_profiling(sim_ctx *ctx, uint32_t enable);

typedef struct {
    uint32_t kind;      /* sim_op_kind of the plan op */
    uint32_t buffer;    /* 0 = full state */
    double ms;          /* device time between the op's events (0 if not timed) */
    double flops;       /* floating-point operations of the op (plan accounting) */
    double bytes;       /* algorithmic HBM bytes of the op (plan accounting) */
} sim_op_timing;

/* Timings of the last profiled run, one entry per plan op (waits for the
 * stream).  cap = room in out; *n receives the number of plan ops. */
sim_status sim_op_timings(sim_ctx *ctx, sim_op_timing *out, uint64_t cap, uint64_t *n);

/* Device memory the context itself holds, in bytes, beside the caller-owned
 * state: booster sub-states, operator tables, stage programs, small-circuit
 * descriptors and reduction scratch (admission control of the serving loop
 * counts it with the state).  Grows with sim_load_circuit and with output
 * calls that need scratch; released by sim_destroy. */
sim_status sim_device_bytes(const sim_ctx *ctx, uint64_t *out);

/* Text of the last error on this context (static storage; never NULL). */
const char *sim_last_error(const sim_ctx *ctx);

sim_status sim_destroy(sim_ctx *ctx);

/* ---- batched runs (serving) -------------------------------------------------
 * Run several loaded contexts of one dtype on `stream` (NULL: the first
 * context's stream) with fewer, fuller launches than one sim_run each:
 *  - small states (N <= 13 for C128, N <= 14 for C64): ONE launch per 128
 *    contexts, one workgroup per circuit keeping the whole state in LDS
 *    (applies the whole gate list from |0...0> and writes the final state);
 *  - every other resident state: its plan's ops run in order on `stream`,
 *    and the full-state cache-blocked stages (Alg. 2) of all waiting states
 *    with the same chunk size go out together, up to 64 states per launch,
 *    one workgroup per chunk; each chunk is computed exactly as by the
 *    state's own stage launch, so results are bitwise those of sim_run.
 * Contexts must be distinct and loaded (SIM_E_STATE otherwise) and share the
 * dtype (SIM_E_INVAL); host-memory offload contexts are SIM_E_UNSUPPORTED.
 * Does not wait: synchronise `stream` before reading the states.  Small
 * states equal those of sim_run up to rounding order. */
sim_status sim_run_batch(sim_ctx *const *ctxs, uint32_t n_ctx, void *stream);

/* ---- host-only planning (no device needed) --------------------------------
 * Build the plan the library would execute for this circuit, for inspection
 * and for checking the optimiser on a machine without a GPU.  The plan is
 * independent of any context; free it with sim_plan_destroy. */
typedef enum {
    SIM_OP_INIT = 0,     /* buffer := |0...0> */
    SIM_OP_KRON = 1,     /* buffer := src_hi (x) src_lo (tensor product, Alg. 5) */
    SIM_OP_DENSE = 2,    /* full-pass dense gate on `qubits` (matrix in payload) */
    SIM_OP_DIAG = 3,     /* full-pass diagonal on `qubits` (table in payload) */
    SIM_OP_STAGE = 4,    /* cache-blocked stage: gates applied chunk by chunk */
    SIM_OP_PERM = 5,     /* qubit permutation: physical bit p -> perm[p] */
    SIM_OP_WINDOW = 6    /* host-memory offload pass: the next `nq` ops run on every window
                            of 2^W amplitudes whose outer qubits (bit positions
                            qubits[0] .. qubits[0] + qubits[1] - 1) are fixed; the ops' qubits
                            are physical bits of the full state; qubits[2] = 1 when the
                            windows start as |0...0> instead of being read */
} sim_op_kind;

typedef struct {
    uint32_t kind;          /* sim_op_kind */
    uint32_t buffer;        /* 0 = the full state, >0 = booster sub-state */
    uint32_t buffer_qubits; /* qubits of that buffer */
    uint32_t src_lo, src_hi;/* KRON sources (buffer ids); lo supplies the low bits */
    uint32_t nq;            /* qubits of a DENSE/DIAG op, gates of a STAGE */
    uint32_t qubits[32];    /* DENSE/DIAG: physical qubits (bit t <-> qubits[t]);
                               PERM: destination bit of each source bit;
                               STAGE: physical local qubits (first `local_qubits`) */
    uint32_t local_qubits;  /* STAGE: C */
    uint32_t n_phases;      /* STAGE: register phases */
    uint64_t payload_len;   /* complex entries in the payload (matrix / table) */
    uint64_t first_gate;    /* STAGE: index of its first gate in sim_plan_stage_gate */
} sim_plan_op;

/* A gate as executed inside a stage or a sub-state run, after fusion:
 * a dense or diagonal operator on `nq` physical qubits of its buffer. */
typedef struct {
    uint32_t diagonal;      /* 1: payload is a 2^nq diagonal; 0: 2^nq x 2^nq matrix;
                               2 (stage-kernel operators only): a quadratic phase
                               e^{i phi(x)}, nq = 0, payload = (code, angle) pairs as
                               (re, im): code -1 the constant, 64 q + q the linear term
                               of qubit q, 64 q + p (q < p) the pair term */
    uint32_t nq;
    uint32_t qubits[16];
    uint64_t payload_len;
    uint32_t n_register;    /* stage-kernel operators: how many of the qubits the
                               kernel holds in registers; the others select a
                               block of the operator (0 in stage gate lists) */
    uint32_t reserved;
} sim_plan_gate;

sim_status sim_plan_build(uint32_t n_qubits, sim_dtype dtype, const sim_options *opts,
                          const sim_gate *gates, uint64_t n_gates, sim_plan **out);
uint64_t sim_plan_num_ops(const sim_plan *plan);
/* payload: NULL or room for payload_len complex values (2*payload_len doubles) */
sim_status sim_plan_get_op(const sim_plan *plan, uint64_t i, sim_plan_op *op, double *payload);
/* gates of a STAGE op in execution order: i in [0, op.nq) */
sim_status sim_plan_stage_gate(const sim_plan *plan, uint64_t op_index, uint64_t i,
                               sim_plan_gate *g, double *payload);
/* The i-th operator the stage kernel applies for STAGE op `op_index`, after
 * register phasing and fusion (all phases flattened, in execution order), as a
 * dense (2^nq x 2^nq, block diagonal in its selector qubits) or diagonal
 * operator on physical qubits.  Returns SIM_E_INVAL past the last one. */
sim_status sim_plan_stage_kernel_op(const sim_plan *plan, uint64_t op_index, uint64_t i,
                                    sim_plan_gate *g, double *payload);
/* final logical -> physical map of the full state: phys[q] = bit position */
sim_status sim_plan_layout(const sim_plan *plan, uint32_t *phys);
sim_status sim_plan_stats(const sim_plan *plan, sim_run_stats *out);
/* Diagnostics of the optimiser passes: number of gates each pass visited. */
sim_status sim_plan_counters(const sim_plan *plan, uint64_t *dd_visits, uint64_t *booster_gates,
                             uint64_t *booster_groups);
sim_status sim_plan_destroy(sim_plan *plan);

/* Plain device-to-device copy of `bytes` (a multiple of 16) on `stream`: the
 * achievable-HBM-bandwidth reference the benchmark reports next to the peak.
 * Device pointers; does not synchronise. */
sim_status sim_device_copy(void *dst, const void *src, uint64_t bytes, void *stream);

/* Library version string. */
const char *sim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QSIM355_H */
