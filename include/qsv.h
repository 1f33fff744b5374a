/*
 * qsv.h -- C ABI of libqsv.so, an MI355X (gfx950) state-vector simulator core.
 *
 * The library applies circuits of k <= 5-qubit unitaries to a 2^n complex amplitude
 * vector (the paper's problem statement: a gate sequence U_m ... U_1 applied to
 * |0...0>, Section 3 and Eq. 5 / Eq. 10), after fusing the gate sequence on the host
 * with the DAG fusion of Section 5.2 (Algorithm 2), and evaluates norm, probability
 * and Pauli-expectation reductions over the vector.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - Qubit t is bit t of the amplitude index (qubit 0 = least significant bit), as in
 *   Eq. 2 and Eq. 3.  A state is 2^n contiguous complex numbers, real and imaginary
 *   parts interleaved: complex64 (QSV_C64, 8 bytes) or complex128 (QSV_C128, 16 bytes).
 * - A k-target matrix is row-major 2^k x 2^k complex128 given as 2*4^k doubles
 *   (re, im interleaved); bit j of its row/column index belongs to targets[j].
 * - Pointers named host_* or documented as host memory are CPU memory; the state
 *   buffer and `out` buffers flagged as device memory are GPU memory.  The caller
 *   owns every array it passes; the library copies what it needs before returning.
 * - Every call returns a qsv_status; on failure nothing is modified (the state is
 *   left untouched) and qsv_last_error() describes the failure.  No exception
 *   crosses the ABI.
 * - Device work is enqueued on the state's stream (a hipStream_t given at
 *   qsv_alloc; NULL = the default stream).  qsv_apply_* return before the device
 *   finishes; calls that return host results synchronise that stream.  Calls on one
 *   state must not overlap from several host threads.
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QSV_OK = 0,
    QSV_E_ARG = 1,          /* invalid argument (targets, sizes, names, null pointers) */
    QSV_E_OOM = 2,          /* device memory exhausted; nothing was allocated */
    QSV_E_DEVICE = 3,       /* a HIP runtime call failed */
    QSV_E_UNSUPPORTED = 4   /* valid request outside what this build supports */
} qsv_status;

typedef enum { QSV_C64 = 0, QSV_C128 = 1, QSV_AUTO = 2 } qsv_dtype;   /* AUTO: serving only */

typedef struct qsv_state_s* qsv_state;   /* opaque */
typedef struct qsv_plan_s* qsv_plan;     /* opaque */

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* qsv_last_error(void);

/* Library version string. */
const char* qsv_version(void);

/* ------------------------------------------------------------------ states */

/* State-vector allocation and initialisation to |0...0> (Eq. 1 with alpha_0 = 1).
 * n_qubits in [1, 34].  buf == NULL: the library allocates 2^n * elem bytes of device
 * memory on the current HIP device and owns it.  buf != NULL: the library adopts the
 * caller's device buffer (e.g. a torch tensor's data_ptr) of buf_bytes >= 2^n * elem
 * bytes, 16-byte aligned, and never frees it.  stream: hipStream_t used for all device
 * work on this state (NULL = default stream).  Errors: QSV_E_ARG (n out of range,
 * buffer too small or misaligned, out == NULL), QSV_E_OOM (allocation failed),
 * QSV_E_DEVICE. */
qsv_status qsv_alloc(int n_qubits, qsv_dtype dtype, void* buf, size_t buf_bytes,
                     void* stream, qsv_state* out);

/* Releases the state, its workspace and (if library-owned) its buffer after the
 * state's stream has drained.  NULL is accepted. */
qsv_status qsv_free(qsv_state s);

/* Re-initialises the state to |0...0> (asynchronous). */
qsv_status qsv_reset(qsv_state s);

/* Queries: qubit count, dtype, device pointer of the amplitudes. */
qsv_status qsv_info(qsv_state s, int* n_qubits, qsv_dtype* dtype, void** device_ptr);

/* Copies the amplitudes to host memory host_out (2^n elements of the state's dtype);
 * synchronises the stream. */
qsv_status qsv_get_state(qsv_state s, void* host_out);

/* Overwrites the amplitudes from host memory host_in (2^n elements of the state's
 * dtype); synchronises the stream.  Used for checkpoint/restore and tests. */
qsv_status qsv_set_state(qsv_state s, const void* host_in);

/* ------------------------------------------------------------------ gates */

/* One gate of a circuit (Section 3: a unitary, a tuple of targets).  k in [1, 5],
 * targets distinct and < n.  mat: host pointer to 2*4^k doubles (dense) or, when
 * diag != 0, to 2*2^k doubles holding only the diagonal. */
typedef struct {
    int k;
    int targets[5];
    int diag;
    const double* mat;
} qsv_gate;

/* Canonical gate set of Eq. 4 (Section 3): "I","X","Y","Z","H","S","SDG","T","TDG",
 * "RX","RY","RZ" (params[0] = theta, R_P(theta) = exp(-i theta P / 2)), "U3"
 * (params = theta, phi, lambda; OpenQASM 2 convention), "CNOT" (local bit 0 = control),
 * "CZ", "SWAP", "TOFFOLI" (local bits 0, 1 = controls).  Writes k and 2*4^k doubles
 * into mat_out (capacity 2*64 doubles suffices).  QSV_E_ARG for an unknown name. */
qsv_status qsv_gate_matrix(const char* name, const double* params, int* k, double* mat_out);

/* ------------------------------------------------------------------ plans */

/* Planner options.  Zero-initialise and set what you need; 0 selects the default. */
typedef struct {
    int fuse;            /* 0: no fusion, one gate per HBM pass (the plain path);
                            1: DAG fusion (Algorithm 2) + multi-gate passes (default);
                            2: no fusion, but consecutive gates share HBM passes */
    int kmax;            /* fusion width q_max^fuse in [1, 5]; default 5 */
    int cost_aware;      /* 1 (default): only fuse when the fused op costs no more
                            arithmetic than its parts (Eq. 13 trade-off); -1: pure
                            Algorithm 2 (fuse whenever the width allows) */
    int tile_qubits;     /* log2 amplitudes per on-chip tile, 0 = default */
    int low_qubits;      /* contiguous low qubits kept in every tile, 0 = default */
    double pass_budget;  /* per-pass arithmetic budget (FMA per amplitude: a dense op
                            4 * 2^k, halved on complex64 matrix cores, times 3/4 for a
                            4-qubit matrix-core op), 0 = default, < 0 = unlimited.  A pass
                            also ends where its next matrix-core op's operand would not
                            fit the pass's LDS operand block */
    int matrix_cores;    /* dense ops on >= this many (and at most 4) targets run on matrix
                            cores (MFMA; FP32 for complex64, FP64 for complex128) when their
                            operand block fits the pass's LDS budget: 0 = default (3),
                            -1 = never, 3 or 4 otherwise */
    int commute;         /* fuse = 1 only.  1 (default): commutation-aware DAG -- ops that
                            are diagonal on every qubit they share are left unordered, so
                            fusion may merge them across one another and a pass may take
                            such an op ahead of deferred ones; -1: the per-qubit DAG of
                            Section 5.1 exactly */
    double op_cost;      /* on-chip cost of one op beyond its arithmetic, in FMA per
                            amplitude (its LDS round trip and barrier), charged by the
                            cost-aware fusion (Eq. 13 trade-off) and by the pass budget;
                            0 = default, > 0 otherwise */
} qsv_plan_opts;

typedef struct {
    size_t gates_in;       /* gates given */
    size_t fused_out;      /* fused gates after DAG fusion */
    size_t passes;         /* HBM passes (kernel launches) per application */
    size_t dense_ops, diag_ops, perm_ops;
    size_t mfma_ops;       /* dense ops run on matrix cores (FP32 MFMA for complex64,
                              FP64 MFMA for complex128) */
    double fma_per_amp;    /* complex-arithmetic cost summed over all passes */
    double hbm_bytes;      /* algorithmic HBM bytes per application = passes * 2 * 2^n * elem */
    double mfma_fma_per_amp;  /* the part of fma_per_amp done by the matrix-core ops */
} qsv_plan_stats;

/* Fuses the gate list with Algorithm 2 (Section 5.2; Eq. 9 products in FP64; a fused
 * gate is kept diagonal or as a generalised permutation when it is one) and
 * schedules the fused gates into HBM passes.  Host-only: touches no device.  The
 * plan is specific to (n_qubits, dtype).  opts may be NULL.  Errors: QSV_E_ARG. */
qsv_status qsv_plan_create(int n_qubits, qsv_dtype dtype, const qsv_gate* gates,
                           size_t n_gates, const qsv_plan_opts* opts, qsv_plan* out);
qsv_status qsv_plan_free(qsv_plan p);
qsv_status qsv_plan_get_stats(qsv_plan p, qsv_plan_stats* st);

/* Re-fills plan p with new matrices for the same circuit shape (n_gates equal to the
 * plan's gate count; gate by gate the same k and targets), keeping its fusion and its
 * passes: each fused matrix becomes the Eq. 9 product of its members' new matrices, in
 * the plan's order.  For circuits whose structure is fixed while parameters change
 * (variational loops): planning is done once, refreshing costs a few matrix products
 * per fused gate.  It is exact only while the plan's structure holds for the new
 * matrices, which is checked: a fused gate kept diagonal or as a permutation must still
 * be one, and every fused gate must stay diagonal on the qubits the planner treated it
 * as diagonal on (the commutations it used).  A plan made from parameters with special
 * values (angles of 0 or pi, where rotations become diagonal, permutations or the
 * identity) can fail that check for general values: make the plan from generic ones.
 * Host-only, unless the plan's tables are already on a device: then the device is
 * synchronised and the stale tables freed (the next application uploads the new ones).
 * Errors: QSV_E_ARG (null or invalid gate, shape differs), QSV_E_UNSUPPORTED (the
 * structure does not hold, or the plan dropped a fused product as the identity: make
 * a new plan); on error the plan is unchanged. */
qsv_status qsv_plan_refresh(qsv_plan p, const qsv_gate* gates, size_t n_gates);

/* Fused gate i (in application order): k, sorted targets, diag flag and the dense
 * 2^k x 2^k FP64 matrix (2*4^k doubles; mat may be NULL).  For host-side checking. */
qsv_status qsv_plan_fused_gate(qsv_plan p, size_t i, int* k, int targets[5], int* diag,
                               double* mat);

/* Pass i: number of ops and the physical qubits held in its tile. */
qsv_status qsv_plan_pass_info(qsv_plan p, size_t i, int* n_ops, int* n_active,
                              int active[40]);

/* Pass i, in application order: the indices (into the fused-gate list) of its ops, in
 * the order the pass applies them.  fused_idx must hold n_ops ints. */
qsv_status qsv_plan_pass_ops(qsv_plan p, size_t i, int* fused_idx);

/* Re-enacts the plan's passes on the host, in FP64, with the exact tile placement and
 * op tables the pass kernel consumes.  state: host array of 2^n complex128 (2^(n+1)
 * doubles), updated in place.  A checking aid for host-only tests; slow. */
qsv_status qsv_plan_emulate(qsv_plan p, double* state);

/* Enqueues the plan's passes on the state's stream (Eq. 10: the fused product applied
 * in order).  The plan must match the state's n and dtype.  The plan may be freed
 * only after the stream has finished with it (qsv_sync). */
qsv_status qsv_plan_apply(qsv_state s, qsv_plan p);

/* Enqueues only passes [first, first+count) of the plan (for timing single passes). */
qsv_status qsv_plan_apply_range(qsv_state s, qsv_plan p, size_t first, size_t count);

/* Sets the state to passes [0, count) of the plan applied to |0...0> (Eq. 1), whatever
 * the buffer held: the first pass builds the |0...0> tiles on chip instead of reading
 * them, so the initialisation costs no HBM traffic of its own.  count = the plan's pass
 * count applies the whole circuit; count == 0 only resets the state.  QSV_E_ARG when
 * count exceeds the pass count or the plan does not match the state.  Asynchronous,
 * like qsv_plan_apply. */
qsv_status qsv_plan_apply_zero(qsv_state s, qsv_plan p, size_t count);

/* One call = plan + apply + release: the gate sequence applied in order to the state
 * (Section 3 and Eq. 10), fused by Algorithm 2 (Section 5.2) under `opts` (NULL = the
 * defaults of qsv_plan_create), then scheduled into HBM passes.  stats (may be NULL)
 * receives the plan's counts: gates in, fused gates out, passes, algorithmic HBM bytes.
 * Synchronises the stream before returning.  Errors: as qsv_plan_create, plus
 * QSV_E_DEVICE. */
qsv_status qsv_apply_fused(qsv_state s, const qsv_gate* gates, size_t n_gates,
                           const qsv_plan_opts* opts, qsv_plan_stats* stats);

/* Waits for all work enqueued on the state's stream. */
qsv_status qsv_sync(qsv_state s);

/* ------------------------------------------------------------------ reductions */

/* sum_k |alpha_k|^2 (Eq. 1 normalisation), accumulated in FP64 per thread, combined
 * with Neumaier's compensated sum in a fixed order (deterministic).  Synchronous. */
qsv_status qsv_norm(qsv_state s, double* out);

/* For callers that cannot allocate (code under stream or graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): qsv_norm on a raw device state, allocating
 * nothing -- no device, pinned or host allocation, no library routine that allocates.
 * amps: device pointer to 2^n_qubits amplitudes of `dtype`, 16-byte aligned (e.g. a torch
 * tensor's data_ptr or the pointer qsv_info returns); n_qubits in [1, 34].  out_dev: device pointer to
 * one double that receives sum_k |alpha_k|^2, bit-identical to qsv_norm's result.  The
 * workgroup partials live in a fixed 16 KiB device array per GPU (its device address is
 * looked up on the first call on each device and kept); every call on one device shares
 * it, so calls that overlap on one device race -- order them on one stream.  Asynchronous
 * on `stream` (hipStream_t, NULL = default stream): nothing is synchronised.  Errors:
 * QSV_E_ARG (null or misaligned pointer, n_qubits out of range, bad dtype), QSV_E_DEVICE. */
qsv_status qsv_norm_noalloc(const void* amps, int n_qubits, qsv_dtype dtype, double* out_dev, void* stream);

/* One Pauli-sum term: coeff * prod_j sigma_{paulis[j]}(qubits[j]), paulis in "IXYZ",
 * n Pauli factors on distinct qubits.  qubits/paulis are host arrays. */
typedef struct {
    double coeff;
    int n;
    const int* qubits;
    const char* paulis;
} qsv_pauli_term;

/* <psi|P_t|psi> for every term (Hermitian Pauli strings, real result), evaluated in
 * as few read passes over the state as the terms allow, FP64 accumulation with a
 * compensated, fixed-order combination.  Expectation values are one of the core
 * operations of a state-vector library (Section 2.2); the definition used is the
 * textbook one: with x the bit mask of the term's X and Y qubits, z that of its Z and Y
 * qubits and n_Y its number of Y factors (Y = i X Z),
 *     <psi|P|psi> = sum_k conj(alpha_{k xor x}) * i^{n_Y} * (-1)^{popcount(k and z)} * alpha_k.  per_term (host, n_terms doubles) receives
 * coeff_t * <P_t>; sum (host) receives their compensated sum.  Either may be NULL.
 * Synchronous.  Errors: QSV_E_ARG for bad qubits or letters. */
qsv_status qsv_expval_pauli(qsv_state s, const qsv_pauli_term* terms, size_t n_terms,
                            double* per_term, double* sum);

/* Outcome probabilities (Eq. 1 and Eq. 18).  m == n and qubits == NULL or (0..n-1):
 * the full distribution |alpha_k|^2, written in the state's real precision (float
 * for C64, double for C128).  Otherwise the marginal over `qubits` (m distinct
 * qubits, output index bit j <-> qubits[j]) written as 2^m doubles accumulated in
 * FP64.  out is device memory when out_on_device != 0, else host memory (then the
 * call synchronises).  Errors: QSV_E_ARG. */
qsv_status qsv_probs(qsv_state s, const int* qubits, int m, void* out, int out_on_device);

/* Measurement sampling in the computational basis (the backend's third operation,
 * Section 4; Born probabilities of Eq. 1).  Measures `qubits` (m distinct qubits, bit j
 * of an outcome <-> qubits[j]; NULL = all n in order) once per uniform: shot i's outcome
 * is the smallest k with uniforms[i] * P < p_0 + ... + p_k, where p is the distribution
 * over the measured qubits accumulated in FP64 and P its total (an unnormalised state is
 * sampled from its normalised distribution); an outcome of probability zero is never
 * returned.  The caller supplies the random numbers (host array of `shots` values in
 * [0, 1)), so results are reproducible.  out: host array of `shots` outcomes.  The
 * partial sums are taken in a fixed order, so the call is deterministic; where u * P
 * falls within rounding of a boundary between two outcomes either may be returned.
 * Synchronous.  Errors: QSV_E_ARG (bad qubits, a uniform outside [0, 1), null
 * pointers), QSV_E_UNSUPPORTED (a marginal or reordered distribution over more than 26
 * qubits), QSV_E_OOM. */
qsv_status qsv_sample(qsv_state s, const int* qubits, int m, const double* uniforms, long long shots,
                      long long* out);

/* ------------------------------------------------------------------ density matrices */

/* A mixed state of n qubits (the noise study of Table 8) is held in an ordinary state of
 * 2n qubits as vec(rho), entry rho[row, col] at index row + 2^n col; qsv_alloc(2n, ...)
 * and qsv_reset give rho = |0...0><0...0|.  Then U rho U^dagger = (conj(U) (x) U) vec(rho):
 * a gate U on targets T acts as U on T and conj(U) on T + n, and a channel with Kraus
 * operators K_a acts as sum_a conj(K_a) (x) K_a on (T, T + n) -- ordinary (non-unitary)
 * matrices for the same planner and kernels. */
typedef struct {
    int kind;            /* 0: unitary gate on k <= 5 targets (mat as in qsv_gate, not diagonal);
                            1: depolarizing channel on k = 1 or 2 targets: each of the 4^k - 1
                               non-identity Pauli strings with probability p / (4^k - 1);
                            2: amplitude damping on k = 1 target with decay probability p */
    int k;
    int targets[5];      /* system qubits, < n */
    const double* mat;   /* kind 0 only */
    double p;            /* kinds 1, 2: in [0, 1] */
} qsv_dm_op;

/* Applies the ops in order to the density matrix held in s (s has 2n qubits), fused and
 * scheduled like qsv_apply_fused (opts may be NULL).  Synchronous.  Errors: QSV_E_ARG
 * (odd qubit count, bad op), QSV_E_OOM, QSV_E_DEVICE. */
qsv_status qsv_dm_apply(qsv_state s, const qsv_dm_op* ops, size_t n_ops, const qsv_plan_opts* opts);

/* Outcome probabilities of measuring `qubits` (m distinct system qubits; bit j of the
 * outcome <-> qubits[j]; NULL = all n in order) on the density matrix: the marginal of
 * its diagonal, FP64, written to host `out` (2^m doubles).  Synchronous. */
qsv_status qsv_dm_probs(qsv_state s, const int* qubits, int m, double* out);

/* Tr(rho P_t) for Pauli terms on the system qubits (FP64 per thread, compensated
 * combination); per_term (host) receives coeff_t Tr(rho P_t), sum their total; either may
 * be NULL.  Synchronous. */
qsv_status qsv_dm_expval_pauli(qsv_state s, const qsv_pauli_term* terms, size_t n_terms, double* per_term,
                               double* sum);

/* ------------------------------------------------------------------ gradients */

/* One op of a parameterised circuit.  kind 0: fixed gate (k, targets, mat as in
 * qsv_gate with diag = 0).  kind 1/2/3: RX/RY/RZ(params[b*P + param]) on targets[0]
 * (R_P(theta) = exp(-i theta P / 2), Eq. 4). */
typedef struct {
    int kind;
    int k;
    int targets[5];
    const double* mat;
    int param;
} qsv_op;

/* Energies E_b = <psi_b|H|psi_b>, psi_b = U(theta_b)|0...0>, and their gradients
 * dE_b/dtheta_j by the adjoint method (one forward sweep, one reverse sweep that
 * uncomputes the state and the co-state layer by layer).  params: host, B x P
 * row-major doubles.  energy: host, B doubles; grad: host, B x P doubles (entries of
 * parameters no op uses are 0).  Runs on `stream` (hipStream_t, NULL = default) and, for
 * B > 1, on a second stream of its own that first waits for the work already queued on
 * `stream` (consecutive parameter vectors alternate between the two, each with its own
 * pair of state buffers); returns when both are done.  Temporary device memory: four
 * states of n_qubits (two when B = 1 or when the second pair does not fit).  Errors:
 * QSV_E_ARG, QSV_E_OOM, QSV_E_DEVICE. */
qsv_status qsv_adjoint_grad(int n_qubits, qsv_dtype dtype, const qsv_op* ops, size_t n_ops,
                            const double* params, int B, int P,
                            const qsv_pauli_term* H, size_t n_terms,
                            double* energy, double* grad, void* stream);

/* ------------------------------------------------------------------ serving */

/* Continuous-batching server.  Requests are planned on host threads, admitted FIFO while
 * a slot is free and their HBM footprint fits (state 2^n * elem + the plan's resident
 * matrices and tables + reduction workspace: the memory model of Eq. 14, against the
 * device's free memory minus a reserve at creation: Eq. 15), and advanced together: each
 * step moves every running request by its next pass(es) in one batched launch per dtype
 * (replayed from a hipGraph), then reduces the requests that finished.  Each finished
 * request yields its norm and per-qubit <Z_i>. */
typedef struct qsv_server_s* qsv_server;

typedef struct {
    size_t capacity_bytes;  /* 0: free device memory at creation minus reserve_bytes */
    size_t reserve_bytes;   /* M_reserve of Eq. 15; 0 = 1 GiB */
    int max_slots;          /* requests running at once; 0 = 64, at most 256 */
    int passes_per_step;    /* passes each running request advances per step; 0 = 1 */
    int grid;               /* workgroups of the persistent batched launch; 0 = 2048 */
    int use_graph;          /* 1: capture the step's launches once and replay them */
    int planner_threads;    /* host planning threads; 0 = 4 */
    int keep_states;        /* 1: finished states stay on the device until qsv_server_release */
    int dry_run;            /* 1: no device work at all (admission and scheduling only) */
    double eps_tol;         /* QSV_AUTO requests: complex64 when Eq. 12 holds for this
                               tolerance (qsv_precision_select); 0 = its default */
    double norm_guard;      /* QSV_AUTO requests run in complex64 are run again in
                               complex128 when |norm - 1| exceeds this; 0 = no guard */
} qsv_server_opts;

typedef struct {
    long long id;
    int n, dtype, status;   /* status: QSV_OK, QSV_E_ARG (bad circuit), QSV_E_OOM (never fits) */
    double norm;
    double zexp[34];        /* <Z_i>, i < n */
    double t_submit, t_admit, t_finish;   /* seconds on the server's clock */
    long long passes, fused;
    int requested;          /* the dtype asked for (QSV_AUTO possible); dtype is the one used */
    int promoted;           /* 1: first run in complex64, repeated in complex128 by the guard */
} qsv_result;

typedef struct {
    long long submitted, admitted, finished, rejected, steps, graph_replays, tiles, admission_waits;
    long long peak_running, peak_used_bytes, capacity_bytes, used_bytes, running, pending;
    long long auto_c64, auto_c128, promoted;   /* QSV_AUTO requests: precision chosen, rerun */
} qsv_server_stats;

/* stream: hipStream_t for all of the server's device work (NULL: the server creates
 * its own stream; graph capture needs a non-default stream).  Errors: QSV_E_DEVICE,
 * QSV_E_OOM. */
qsv_status qsv_server_create(const qsv_server_opts* opts, void* stream, qsv_server* out);
qsv_status qsv_server_free(qsv_server s);

/* Adaptive precision (Section 5.4): the rounding bound of Eq. 11 for complex64,
 * g * 2^n * 1.19e-7 (g gate applications on 2^n amplitudes), against eps_tol (Eq. 12):
 * complex64 when it holds, else complex128.  eps_tol <= 0 selects the default
 * 49.5 * 2^20 * 1.19e-7 (about 6.18): the paper's 20-qubit circuits of fewer than 50 gates
 * then run in complex64 and deeper ones in complex128 (Section 8.4). */
qsv_status qsv_precision_select(int n_qubits, size_t n_gates, double eps_tol, qsv_dtype* out);

/* Queues a request (gates copied; planning starts on a host thread).  dtype QSV_AUTO
 * selects the precision by qsv_precision_select with the server's eps_tol.  popts may
 * be NULL (defaults).  *id receives the request id.  Errors: QSV_E_ARG. */
qsv_status qsv_server_submit(qsv_server s, int n_qubits, qsv_dtype dtype, const qsv_gate* gates,
                             size_t n_gates, const qsv_plan_opts* popts, long long* id);

/* Admission + one step (blocking until the step's device work is done). */
qsv_status qsv_server_step(qsv_server s, int* n_running, int* n_pending);

/* Pops up to max finished results into out (host); *count receives how many. */
qsv_status qsv_server_results(qsv_server s, qsv_result* out, int max, int* count);

qsv_status qsv_server_get_stats(qsv_server s, qsv_server_stats* st);

/* keep_states only: copy a finished request's final state to host memory (2^n elements
 * of its dtype), and release it. */
qsv_status qsv_server_get_state(qsv_server s, long long id, void* host_out);
qsv_status qsv_server_release(qsv_server s, long long id);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H */
