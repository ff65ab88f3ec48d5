/*
 * qsim.h -- C-ABI of libqsim, an MI355X (gfx950) engine for expectation
 * values of variational quantum circuits and their gradients.
 *
 * What is computed follows the paper (Patti, Kossaifi, Yelin, Anandkumar,
 * "TensorLy-Quantum: Quantum Machine Learning with Tensor Methods"):
 *   - Sec. 1: quantum expectation values define the objective of variational
 *     (QML) algorithms, optimised by classical gradient descent;
 *   - Sec. 2: circuits are built from pre-defined or custom gates acting on
 *     states; operators are kept in factorized form;
 *   - Sec. 3: the forward value <H> and the full gradient d<H>/dtheta for a
 *     transverse-field Ising Hamiltonian; a dense operator matrix is never
 *     formed (its memory grows as 4^n);
 *   - Sec. 4: "causality-simplified contraction" (future work there) is the
 *     light-cone mode here.
 *
 * Conventions (readings of points the paper leaves open):
 *   - qubit q is bit q of an amplitude index (little-endian);
 *   - RX/RY/RZ(t) = exp(-i t P / 2) with P = X/Y/Z;
 *   - CZ = diag(1,1,1,-1) on (q0, q1); CNOT has control q0 and target q1;
 *   - U1 is a fixed caller-given 2x2 unitary (row-major complex128, 8 doubles
 *     re,im interleaved); a matrix with an entry of U^dagger U - I above 1e-8 in
 *     magnitude is rejected with QSIM_EINVAL;
 *   - H = sum_t coeff[t] * P_t with real coefficients and Pauli strings P_t
 *     on distinct qubits; the empty string is the identity.
 *
 * Status codes: every call returns QSIM_OK (0) or a negative QSIM_E* code and
 * never throws across the ABI.  A context records the text of its last error
 * (qsim_last_error).  NaN parameters propagate to the results; they are not
 * rejected.
 *
 * Memory: every array passed in is owned by the caller and only read during
 * the call (qsim_submit deep-copies its request).  Results are written to
 * caller-owned host buffers.  Objects returned through out-pointers
 * (contexts, states) are owned by the library until the matching destroy or
 * finalize call.
 *
 * Streams: "stream" arguments are hipStream_t values (NULL = the context's
 * own stream).  Calls that return host results synchronize that stream.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSIM_OK 0
#define QSIM_PENDING 1      /* qsim_poll: result not ready yet (not an error) */
#define QSIM_EINVAL (-1)    /* bad argument: qubit, duplicate qubit, kind, Pauli, n, batch */
#define QSIM_ENOMEM (-2)    /* device or host allocation failed */
#define QSIM_ETOOBIG (-3)   /* footprint above the budget, or a light cone above the cap */
#define QSIM_EAGAIN (-4)    /* serving queue full: retry later */
#define QSIM_ENOTFOUND (-5) /* unknown or already-consumed ticket */
#define QSIM_EDEVICE (-6)   /* HIP runtime error (text in qsim_last_error) */
#define QSIM_ECANCELED (-7) /* request was cancelled */
#define QSIM_ESHUTDOWN (-8) /* context shut down with the request pending */

enum { QSIM_RX = 0, QSIM_RY = 1, QSIM_RZ = 2, QSIM_CZ = 3, QSIM_CNOT = 4, QSIM_U1 = 5 };
enum { QSIM_C64 = 0, QSIM_C128 = 1 };
/* LIGHTCONE: every term on its canonical cone.  LIGHTCONE_FACTORED: for Z-string
 * terms, trailing diagonal gates (which commute with the term) are dropped and
 * the term splits into factors whose remaining cones are disjoint (the
 * expectation of a product over disjoint cones on |0...0> is the product of
 * expectations); factors are shared between terms.  Both are exact. */
enum { QSIM_MODE_AUTO = 0, QSIM_MODE_DENSE = 1, QSIM_MODE_LIGHTCONE = 2, QSIM_MODE_LIGHTCONE_FACTORED = 3 };

/* One gate.  Rotations take theta[param] when param >= 0, else 'angle'.
 * Two-qubit gates use q0 and q1 (distinct); others use q0 only.  'mat' is read
 * for U1 only.  Layout (32 bytes): kind@0, q0@4, q1@8, param@12, angle@16, mat@24. */
typedef struct {
    uint8_t kind;
    uint8_t pad[3];
    int32_t q0, q1;
    int32_t param;
    double angle;
    const double* mat;
} qsim_gate;

/* A circuit: gates applied in array order to |0...0> on n_qubits qubits. */
typedef struct {
    int32_t n_qubits;
    int32_t n_gates;
    int32_t n_params;
    int32_t pad;
    const qsim_gate* gates;
} qsim_circuit;

/* H = sum_t coeff[t] * prod_{k in [term_off[t], term_off[t+1])} paulis[k] on qubits[k];
 * paulis are the bytes 'X', 'Y', 'Z'. */
typedef struct {
    int32_t n_terms;
    int32_t pad;
    const double* coeff;
    const int32_t* term_off;
    const int32_t* qubits;
    const uint8_t* paulis;
} qsim_hamiltonian;

/* Context options, fixed for the context's lifetime; zero fields take the
 * defaults (an environment variable of the same meaning, where one exists,
 * replaces a default: QSIM_FWD_M, QSIM_FWD_R, QSIM_FWD_CLOW, QSIM_DUAL_CLOW). */
typedef struct {
    int32_t device;             /* HIP device ordinal; -1 = host-only context (plans, simulated serving) */
    int32_t max_queue;          /* serving: queued + in-flight requests (default 4096) */
    int32_t cone_cap;           /* light cones above this many qubits are ETOOBIG (default 20) */
    int32_t max_inflight;       /* serving: scheduler steps in flight on the device, 1..8 (default 3) */
    uint64_t hbm_budget_bytes;  /* serving: bytes of state memory in flight (default 64 GiB) */
    int32_t tile_qubits;        /* complex64 forward passes: tiles of 2^m amplitudes, m in 12..14 (default 13) */
    int32_t register_bits;      /* complex64 forward passes: 2^r amplitudes per thread, r in 3..5 (default 4) */
    int32_t coalesce_bits;      /* forward passes: lowest index bits local in every pass, 3..6 (default 4) */
    int32_t dual_coalesce_bits; /* adjoint (two-state) passes: the same, 3..6 (default 6) */
    int32_t disable;            /* QSIM_OFF_* bits, each switching one optimisation off (default 0) */
    int32_t reserved[3];
} qsim_options;

#define QSIM_OFF_FACTORED 1   /* rotations on a stage's register bits as one factored op */
#define QSIM_OFF_ABSORB 2     /* runs of CNOTs applied as stage exit permutations */
#define QSIM_OFF_ENTRY 4      /* a permute-only first stage folded into the loads */
#define QSIM_OFF_EXIT 8       /* a pass's last CNOT run folded into the store addresses */
#define QSIM_OFF_PRODUCT 16   /* leading single-qubit gates folded into a product start state */
#define QSIM_OFF_PREFETCH 32  /* register prefetch of the next tile */
#define QSIM_OFF_IO_REGS 64   /* load/store stages may hold the always-local low bits in registers */
#define QSIM_OFF_BATCH_PROBES 128  /* adjoint: inverse phases as one table, gradient probes in groups */
#define QSIM_OFF_RELABEL 256  /* forward plans whose final state is not kept: the qubits held in the
                                 coalesced low index bits may change from pass to pass */
#define QSIM_OFF_EARLY_TERMS 512  /* terms with X/Y factors measured in the gate passes once every gate
                                     they do not commute with has been applied */

typedef struct qsim_ctx qsim_ctx;
typedef struct qsim_state qsim_state;

/* Create a context on opt->device (opt may be NULL: device 0, defaults).  Owns a
 * HIP stream, device workspaces and the plan cache; *out is NULL on failure.
 * QSIM_EDEVICE when the device does not exist.  Every evaluation of the paper's
 * objective (Sec. 1: expectation values of circuits, Sec. 3: values and
 * gradients) goes through a context. */
int qsim_init(qsim_ctx** out, const qsim_options* opt);
/* Stop the serving loop (pending tickets end with QSIM_ESHUTDOWN), free everything. */
void qsim_finalize(qsim_ctx* ctx);
/* Static text for a status code. */
const char* qsim_strerror(int code);
/* Text of the context's most recent error ("" if none).  Valid until the next call on ctx. */
const char* qsim_last_error(qsim_ctx* ctx);

/* ---- stateful interface (Sec. 2: gates acting on states) --------------------------- */

/* A batch of 'batch' states of n_qubits each, set to |0...0>.  dtype: QSIM_C64 or
 * QSIM_C128.  dev_buf NULL = library-owned memory, else a caller device buffer of
 * batch * 2^n * (8 or 16) bytes that must outlive the state (borrowed).  Layout:
 * state b, amplitude x at element b*2^n + x, (re, im) interleaved. */
int qsim_create_state(qsim_ctx* ctx, int n_qubits, int batch, int dtype, void* dev_buf, void* stream,
                      qsim_state** out);
int qsim_destroy_state(qsim_state* st);
/* Append gates to the state's queue.  params: float64 [batch * n_params] (row b for
 * state b); host memory, or device memory when params_on_device != 0 (read in the
 * order of the state's stream; the coefficients are then built on the device and
 * the values never reach the host).  May be NULL when no gate has param >= 0.
 * Queued gates are planned and applied at the next qsim_expect or qsim_state_to_host. */
int qsim_apply_layer(qsim_state* st, const qsim_gate* gates, int n_gates, const double* params, int n_params,
                     int params_on_device);
/* out[b] = <psi_b|H|psi_b> (float64, host, [batch]); flushes queued gates. */
int qsim_expect(qsim_state* st, const qsim_hamiltonian* H, double* out);
/* Copy the states to host memory (batch * 2^n complex of the state's dtype); flushes. */
int qsim_state_to_host(qsim_state* st, void* host);
/* Device pointer of the amplitudes (layout as in qsim_create_state); flushes first. */
int qsim_state_device_ptr(qsim_state* st, void** ptr);

/* Reduced density matrices of the batch's states (Sec. 2: partial trace as a
 * contraction of the state with its conjugate over the traced modes; the paper's
 * n=20 example keeps 14 or 10 qubits): rho_b[i][j] = sum_k psi_b(i, k) conj(psi_b(j, k)),
 * where bit a of i and j is qubit qubits[a] (any order, distinct) and k runs over the
 * other qubits.  m = number of kept qubits, 1 <= m <= min(n, 15).  rho: [batch][2^m][2^m]
 * complex of the state's dtype, row-major; a device buffer if rho_on_device, else host
 * memory (the library stages through device memory).  Computed on the matrix cores in
 * the state's precision (fp32 / fp64 accumulation); rho is exactly Hermitian (each
 * off-diagonal pair is written from one value).  Flushes queued gates; returns when
 * rho is complete.  QSIM_EINVAL on bad qubits or m. */
int qsim_reduced_density(qsim_state* st, const int32_t* qubits, int m, void* rho, int rho_on_device);

/* A dense five-qubit gate (Sec. 2: custom gates acting on states; here a
 * 32 x 32 unitary such as several layers on five qubits contracted into one
 * tensor) applied to qubits 0..4 of every state: amplitude x = 32 h + j becomes
 * sum_i u[j][i] psi[32 h + i], u row-major complex128 (2048 doubles, host; j
 * and i little-endian over qubits 0..4), rounded once to fp32.  method 0: fp32
 * matrix cores (the block in real form, 256 flops per amplitude; batch *
 * 2^(n-5) must be a multiple of 32); method 1: vector ALUs.  Measurement call:
 * the engine's own passes factor single-qubit rotations instead of forming
 * dense blocks.  Flushes queued gates; *ms (optional) = kernel time.
 * QSIM_EINVAL unless the states are complex64 of at least 5 qubits. */
int qsim_apply_block5(qsim_state* st, const double* u, int method, double* ms);

/* ---- one-call evaluation (Sec. 3: forward value) ----------------------------------- */

/* out[b] = <psi(theta_b)|H|psi(theta_b)> for b < batch, theta_b = params + b*n_params
 * (float64; host memory, or device memory when params_on_device != 0, in which
 * case the gate coefficients are built on the device and the parameters are never
 * copied to the host).  mode: dense state vector, per-term light cones, factored light
 * cones, or AUTO (factored light cones when n > 30, else dense).  If keep != NULL
 * (dense mode only), the final states are returned in *keep for qsim_expect_grad. */
int qsim_expect_circuit(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch,
                        int params_on_device, const qsim_hamiltonian* H, int mode, int dtype, void* stream,
                        double* out, qsim_state** keep);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): qsim_expect_circuit in
 * dense mode, with the final states kept, that calls no hipMalloc, hipFree or
 * other allocating routine.  out[b] = <psi(theta_b)|H|psi(theta_b)> (float64,
 * host, [batch]); params and params_on_device as in qsim_expect_circuit.  state:
 * caller device buffer of state_bytes >= batch * 2^n * (8 or 16) bytes (layout as
 * in qsim_create_state); the passes work in it and it holds the final states
 * psi(theta_b) on return (the same values, bit for bit, as the state that
 * qsim_expect_circuit returns in *keep).  Plan descriptors, coefficient rows,
 * partial sums and the results live in a fixed 64 MiB device array that the
 * library holds on each GPU it runs on until the process ends; a call needs
 * about batch * (measurement passes) * 2^(n - 13) * 8 bytes of it for partial
 * sums (n = 30, batch 1: 2 MiB) and returns QSIM_ETOOBIG, allocating nothing,
 * when the whole need exceeds 64 MiB.  Plans are built on the host and kept per
 * circuit structure in the context's host memory.  Every call on one GPU (any
 * context, any thread) uses that GPU's single array and overwrites what the
 * last call left there: calls that overlap in time on one GPU race and give
 * wrong results (calls on one context are serialised).  Returns when out is
 * written.  QSIM_EINVAL for a short or NULL state buffer and for the errors of
 * qsim_expect_circuit. */
int qsim_expect_circuit_noalloc(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch,
                                int params_on_device, const qsim_hamiltonian* H, int dtype, void* state,
                                uint64_t state_bytes, void* stream, double* out);

/* Per-term values (Sec. 1 and Sec. 3: <H> = sum_t coeff[t] <P_t>):
 * out[b * n_terms + t] = <psi(theta_b)|P_t|psi(theta_b)> without the coefficient (1
 * for identity terms), float64, host, [batch][n_terms].  params and params_on_device
 * as in qsim_expect_circuit.  mode: QSIM_MODE_DENSE (the final states once, then one
 * read-only measurement pass per term), QSIM_MODE_LIGHTCONE (each term on its
 * canonical cone), QSIM_MODE_LIGHTCONE_FACTORED (Z-strings as products of disjoint
 * pruned factors), or AUTO (factored cones when n > 30, else dense).  Errors as for
 * qsim_expect_circuit. */
int qsim_expect_terms(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                      const qsim_hamiltonian* H, int mode, int dtype, void* stream, double* out);

/* ---- gradient (Sec. 3: full gradient; here by the adjoint method) ------------------ */

/* E[b] = <H> and grad[b*n_params + j] = d<H>/dtheta_j (float64, host) for b < batch;
 * E may be NULL.  params and params_on_device as in qsim_expect_circuit.  saved: final
 * states from qsim_expect_circuit(keep) with the same circuit/params, or NULL to run
 * the forward pass first.  A saved state is consumed (its amplitudes are overwritten
 * by the backward sweep) but must still be destroyed by the caller. */
int qsim_expect_grad(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                     const qsim_hamiltonian* H, int dtype, void* stream, qsim_state* saved, double* E,
                     double* grad);

/* E[b] = <H> and grad[b*n_params + j] = d<H>/dtheta_j (float64, host) for b < batch,
 * with every term evaluated on light cones instead of the full state (Sec. 3's
 * forward value and full gradient; Sec. 4's causality-based contraction), so n may
 * be in the hundreds.  mode: QSIM_MODE_LIGHTCONE (each term on its canonical cone)
 * or QSIM_MODE_LIGHTCONE_FACTORED / QSIM_MODE_AUTO (Z-string terms split into
 * disjoint pruned factors, shared across terms).  Inside each cone the gradient is
 * taken by the adjoint method; per-cone parameter gradients are weighted by
 * d<H>/d<cone> and summed per parameter on the device in a fixed order.  params and
 * params_on_device as in qsim_expect_circuit; E and grad are host buffers owned by
 * the caller; E may be NULL.  Errors as for qsim_expect_circuit; QSIM_ETOOBIG when a
 * cone exceeds the context's cone_cap. */
int qsim_expect_grad_cones(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch,
                           int params_on_device, const qsim_hamiltonian* H, int mode, int dtype, void* stream,
                           double* E, double* grad);

/* ---- light cones (Sec. 4: causality-simplified contraction) ------------------------- */

/* Canonical light-cone qubit sets, ascending, term by term: set t is
 * qubits[off[t] .. off[t+1]).  Start from the term's qubits, walk the gates
 * backwards, add both qubits of every two-qubit gate touching the set.  Host only
 * (no device use, ctx not needed).  cap = capacity of 'qubits'; QSIM_ETOOBIG if short. */
int qsim_lightcone_sets(const qsim_circuit* c, const qsim_hamiltonian* H, int32_t* off, int32_t* qubits,
                        int cap);

/* Plan summary for a dense evaluation on the host (no device use): passes,
 * stages and ops of the plan that an expectation with default options runs
 * (final state not kept).  info[0] = passes, info[1] =
 * stages, info[2] = device ops, info[3] = measurement passes.  If 'order' is not
 * NULL it receives, for every gate of c in execution order, (pass, stage, op,
 * gate index) quadruples of int32 (op: the op's index within its stage; -1 for a
 * CNOT folded into the loads); cap_entries bounds the number of quadruples (the
 * buffer holds 4 * cap_entries int32), and QSIM_ETOOBIG is returned, writing
 * nothing, when the plan has more. */
int qsim_plan_dense(const qsim_circuit* c, const qsim_hamiltonian* H, int dtype, int64_t* info, int32_t* order,
                    int cap_entries);

/* Passes that qsim_expect_circuit launches for (c, H) in dense mode on ctx (with
 * keep != 0: the variant that stores the final state), as 8 int32 per pass:
 * flags (as in qsim_timing_get), number of stages, index of the storing stage
 * within the pass (-1: none), 1 if the loads go through an entry permutation,
 * 1 if the stores go through an exit permutation, measurement column (-1: none),
 * gradient probes, tile qubits m.  Plans come from ctx's cache (a host-only
 * context, device -1, works without a GPU).  rec holds cap records; QSIM_ETOOBIG
 * with *count = the number needed when cap is short. */
int qsim_plan_passes(qsim_ctx* ctx, const qsim_circuit* c, const qsim_hamiltonian* H, int dtype, int keep,
                     int32_t* rec, int cap, int* count);

/* Stage trace of the same plan (diagnostic for host tests; no device use): what
 * every stage applies, in order, on index bits (the qubit held at an index bit
 * may change between passes).  One record of 8 int64 per entry:
 *   {kind, q, q2, src_begin, src_count, ph, fmask, zmask}
 * kind 0: single-qubit gate on index bit q, the product of the circuit gates
 * srcs[src_begin .. src_begin + src_count) applied in that order; 1: CNOT, q
 * target, q2 control; 2: CZ on q, q2; 3: Pauli term measured here, i^ph times
 * the product over index bits of X (fmask only), Y (both) or Z (zmask only),
 * weight coef[i]; 4: a stage ends (its permutation has been applied); 5: a
 * circuit gate srcs[src_begin] folded into the start state (these come first).
 * cap bounds the records, cap_srcs the source indices; QSIM_ETOOBIG (with
 * *count and *n_srcs set to the sizes needed) when either is too small.  The
 * identity part of H is not recorded. */
int qsim_plan_trace(qsim_ctx* ctx, const qsim_circuit* c, const qsim_hamiltonian* H, int dtype, int keep,
                    int64_t* rec, double* coef, int cap, int32_t* srcs, int cap_srcs, int* count, int* n_srcs);

/* Coefficient rows (diagnostic for tests): the scalars that the dense passes of
 * the gate plan of c read, for batch parameter rows, built on the host
 * (params_on_device = 0) or by the device kernel from a device parameter buffer
 * (1), copied raw into out (host memory, rows of 8 scalars per coefficient slot;
 * float for QSIM_C64, double for QSIM_C128; entries 68 and 69 of a factored
 * block are 32-bit words).  Both builders follow one fp64 definition, so the two
 * results are expected to agree bit for bit.  *bytes = size of the rows;
 * QSIM_ETOOBIG when cap is smaller. */
int qsim_coef_rows(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                   int dtype, void* out, uint64_t cap, uint64_t* bytes);

/* ---- measurement ------------------------------------------------------------------ */

/* Per-launch timing of the synchronous calls' pass kernels on ctx: with on != 0,
 * every pass launch that follows is bracketed by HIP events recorded on the
 * stream it runs on; on == 0 stops recording.  Enabling clears old records. */
int qsim_timing_enable(qsim_ctx* ctx, int on);
/* Copy up to cap records of launches finished so far: ms[i] = kernel time in
 * milliseconds, bytes[i] = algorithmic HBM bytes of that launch (each amplitude
 * read and/or written once, per the pass's flags), flops[i] = algorithmic
 * floating-point operations (16 per amplitude per general 2x2 gate, 8 per real
 * rotation, 6 per phase, 0 per CNOT/CZ, plus measurement terms), flags[i] = the
 * pass flags (bit 1 generate |0...0>, 2 load psi, 4 store psi, 8 load lambda,
 * 16 store lambda, 64 measure, 128 gradient), kind[i] = 0 dense pass, 1
 * light-cone batch, 2 reduced density matrix (bytes = state read once plus rho
 * written once; flops = 4 N (N + 1) K per state for N = 2^m, K = 2^(n-m): the
 * Hermitian product's lower triangle at 8 real flops per complex multiply-add),
 * 3 dense five-qubit block (16 bytes and 256 flops per amplitude).
 * Any output pointer may be NULL.  *count = records copied. */
int qsim_timing_get(qsim_ctx* ctx, double* ms, double* bytes, double* flops, int32_t* flags, int32_t* kind, int cap,
                    int* count);

/* Reference stream: copy 'bytes' (multiple of 16) between two device buffers
 * with a plain vectorised copy kernel, 'reps' times on ctx's stream; *ms = mean
 * kernel time (HIP events).  Gives the achievable HBM rate next to which the
 * pass kernels are reported, and calibrates HBM byte counters. */
int qsim_copy_probe(qsim_ctx* ctx, uint64_t bytes, int reps, double* ms);

/* ---- serving (continuous batching) -----------------------------------------------
 *
 * The paper offers the library as an efficient backend for quantum machine
 * learning (Sec. 1; Sec. 4 names faster backends as the direction of further
 * work), where many objective evaluations (Sec. 1: expectation values, with
 * their gradients for the classical optimiser) are requested at once.  These
 * calls accept such requests from any thread and share the device between
 * them: requests are admitted in arrival order while their device memory
 * (states, (1 + want_grad) * 2^n * 8 bytes, plus plan descriptors, coefficients,
 * partial sums and results) fits the context's hbm_budget_bytes; every running
 * request advances one pass per scheduler step
 * in multi-request launches; results do not depend on what else is running. */

typedef struct {
    const qsim_circuit* circuit;
    const double* params;      /* host float64 [n_params] */
    const qsim_hamiltonian* H;
    int32_t want_grad;
    int32_t pad;
} qsim_request;

typedef struct {
    uint64_t submitted, completed, rejected, cancelled, failed;
    uint64_t steps, launches, inflight_bytes, peak_inflight_bytes;
    uint64_t queued, running;
    uint64_t pool_outstanding_bytes;  /* device blocks handed out to admitted requests now */
    uint64_t accounting_violations;   /* admissions after which those blocks exceeded inflight_bytes (0) */
} qsim_server_stats;

/* Enqueue a request (deep copy of the circuit, H and parameters; complex64 dense
 * evaluation, with the adjoint gradient when want_grad).  *ticket identifies it.
 * EAGAIN when the queue is full, ETOOBIG when the request alone exceeds the memory
 * budget, EINVAL for an invalid circuit or H.  Thread-safe. */
int qsim_submit(qsim_ctx* ctx, const qsim_request* req, uint64_t* ticket);
/* QSIM_PENDING while running; QSIM_OK once done: E[0] and, if the request asked
 * for it, grad[n_params] are written and the ticket is consumed.  A failed or
 * cancelled request returns its error code and is consumed.  Thread-safe. */
int qsim_poll(qsim_ctx* ctx, uint64_t ticket, double* E, double* grad);
/* qsim_poll that also writes times[0..2] (if times != NULL): the qsim_clock()
 * seconds at which the request was submitted, admitted to the device and
 * completed.  Thread-safe. */
int qsim_poll_timed(qsim_ctx* ctx, uint64_t ticket, double* E, double* grad, double* times);
/* Monotonic clock in seconds used for the serving timestamps. */
double qsim_clock(void);
/* Cancel a queued or running request; its next qsim_poll returns QSIM_ECANCELED.
 * ENOTFOUND for an unknown or consumed ticket.  Thread-safe. */
int qsim_cancel(qsim_ctx* ctx, uint64_t ticket);
/* Counters of the serving loop since the context was created (requests by
 * outcome, scheduler steps and launches, device bytes in flight now and at
 * peak, requests queued and running now).  A request's footprint is every
 * device block it holds while admitted (states, plan descriptors,
 * coefficients, partial sums, results), computed from its plans at submit.
 * Thread-safe. */
int qsim_server_stats_get(qsim_ctx* ctx, qsim_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* QSIM_H */
