/*
 * qsim.h - C ABI of the MI355X (gfx950) state-vector gate engine, libqsim.so.
 *
 * The engine applies a sequence of quantum gates to the state of n qubits, a vector of 2^n complex
 * amplitudes a(x_{n-1} ... x_0), following De Raedt et al., "Massive Parallel Quantum Computer
 * Simulator": the state and its normalisation (Sec. II.A, Eqs. STAT2 and STAT1), the elementary
 * gates (Sec. II.B-II.D) and their in-place update rules (Sec. III.A, Eqs. NUM2-NUM8).
 *
 * Conventions shared by every call
 *   - Qubit q is bit q of the amplitude index; qubit 0 is the least significant bit (Sec. II.A).
 *   - Device layout: amplitude i is stored interleaved as (re, im) at element i of a contiguous
 *     array: 16 bytes per amplitude for QSIM_C128 (two doubles), 8 bytes for QSIM_C64 (two floats).
 *   - 2x2 matrices cross the ABI as 8 host doubles, row-major complex (re, im) pairs:
 *     U = {u00r, u00i, u01r, u01i, u10r, u10i, u11r, u11i}; the update is a' = U a on every pair
 *     (a(..0_t..), a(..1_t..)) (the common form of Eqs. NUM2-NUM8). Matrices are copied before the
 *     call returns; complex64 states round them to FP32 at launch. Unitarity is not checked.
 *   - Control masks: bit q set = qubit q is a control; the gate acts only on indices whose control
 *     bits are all 1 (Eqs. NUM6-NUM8). A mask must not contain the target and must be < 2^n.
 *   - Every apply call is asynchronous on the state's HIP stream; calls that return host data
 *     (norm, probabilities to host, marginals, download, renormalize) synchronise that stream.
 *   - Return codes: QSIM_OK (0) or a negative QSIM_E* code; nothing is launched when an argument is
 *     rejected. qsim_last_error() returns the calling thread's message for the last failure.
 *   - Thread safety: one thread per state (or external locking). Different states may be used
 *     from different threads.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsim_state qsim_state; /* opaque: device buffer + stream + small reduction buffer */
typedef struct qsim_plan qsim_plan;   /* opaque: a circuit lowered to kernel launches */

typedef enum { QSIM_C64 = 0, QSIM_C128 = 1 } qsim_dtype;

enum {
    QSIM_OK = 0,
    QSIM_EINVAL = -1,      /* bad argument (range, null pointer, size mismatch, duplicate qubit) */
    QSIM_ENOMEM = -2,      /* device allocation failed or the state does not fit */
    QSIM_EDEVICE = -3,     /* a HIP runtime error; text in qsim_last_error() */
    QSIM_EUNSUPPORTED = -4 /* valid request that the library does not support */
};

#define QSIM_MAX_QUBITS 40 /* index arithmetic limit; memory is the practical limit (34 c64 / 33 c128) */

/* Thread-local text of the last error (never NULL; "" when none). */
const char *qsim_last_error(void);
/* Library version string. */
const char *qsim_version(void);

/* ---------------------------------------------------------------------------------------------
 * State vectors (Sec. II.A, Eq. STAT2; memory 2^n amplitudes, Sec. III.A)
 * ------------------------------------------------------------------------------------------- */

/* Allocate a state of n qubits (1 <= n <= QSIM_MAX_QUBITS) on the current HIP device and set it to
 * |0...0>. The library owns the buffer (freed by qsim_free). stream: a hipStream_t, or NULL for the
 * null stream. Errors: EINVAL (n, dtype, out), ENOMEM (allocation), EDEVICE. */
int qsim_alloc(int n, int dtype, void *stream, qsim_state **out);

/* Wrap an existing device buffer of 2^n amplitudes (borrowed: not freed by qsim_free; it must stay
 * alive as long as the state). The contents are left as they are. The buffer must be 16-byte
 * aligned. Errors: EINVAL. */
int qsim_wrap(void *dev_ptr, int n, int dtype, void *stream, qsim_state **out);

/* Release the state (and its buffer if the library owns it). NULL is accepted. */
int qsim_free(qsim_state *s);

/* Device pointer of the amplitudes, qubit count and dtype of a state. */
void *qsim_data(qsim_state *s);
int qsim_num_qubits(const qsim_state *s);
int qsim_get_dtype(const qsim_state *s);

/* Change the HIP stream the state's work is issued on. */
int qsim_set_stream(qsim_state *s, void *stream);

/* Set the state to the basis state |x> (a_x = 1, all others 0). EINVAL if x >= 2^n. */
int qsim_set_basis(qsim_state *s, uint64_t x);

/* Copy 2^n amplitudes (bytes must equal 2^n * amplitude size) from host memory into the state /
 * from the state into host memory. Synchronous. EINVAL on a size mismatch or NULL pointer. */
int qsim_upload(qsim_state *s, const void *host, size_t bytes);
int qsim_download(qsim_state *s, void *host, size_t bytes);

/* Wait for all work issued on the state's stream. */
int qsim_sync(qsim_state *s);

/* ---------------------------------------------------------------------------------------------
 * Elementary gates (Sec. II.B-II.D; update rules Sec. III.A)
 * ------------------------------------------------------------------------------------------- */

/* Single-qubit gate U on `target` (Eqs. NUM2-NUM5 are the cases H, X, Y and R(phi)). Touches 2^n
 * amplitudes; a diagonal U with u00 = 1 touches only the 2^(n-1) amplitudes with bit target = 1
 * (Eq. NUM5); U = [[0,1],[1,0]] is carried out as a swap with no arithmetic. EINVAL: target out of
 * range, U NULL. */
int qsim_apply_1q(qsim_state *s, int target, const double U[8]);

/* Controlled single-qubit gate: U on `target` for the indices whose bits in control_mask are all 1
 * (CNOT Eq. NUM6, controlled V Eq. NUM7, Toffoli Eq. NUM8 with two control bits; any number of
 * controls). Touches 2^(n-|C|) amplitudes; permutation matrices are exact swaps (bit-exact).
 * EINVAL: target out of range, mask >= 2^n or containing the target, U NULL. */
int qsim_apply_ctrl(qsim_state *s, uint64_t control_mask, int target, const double U[8]);

/* Phase shift R(theta) = diag(1, e^{i theta}) on `target`, controlled by control_mask (Eq. NUM5,
 * Eq. COMM5). The phase factor cos(theta) + i sin(theta) is evaluated in FP64 on the device
 * (rounded to FP32 only when applied to a complex64 state). Touches 2^(n-1-|C|) amplitudes. */
int qsim_apply_phase(qsim_state *s, uint64_t control_mask, int target, double theta);

/* Quantum swap of qubits q0 != q1 (controlled by control_mask): exchanges a(..1_q0..0_q1..) with
 * a(..0_q0..1_q1..); no arithmetic. Not the paper's data-distribution SWAP command (App. A). */
int qsim_apply_swap(qsim_state *s, uint64_t control_mask, int q0, int q1);

/* Dense k-qubit gate (1 <= k <= 5, k <= n) on the distinct, possibly unsorted qubits[0..k-1]:
 * U is 2^k x 2^k complex128, row-major interleaved (re, im), 2^(2k+1) host doubles; matrix index
 * bit s <-> qubits[s]. For every base index b with zero bits at the k qubits, the 2^k amplitudes
 * v_r = a(b + sum_s bit_s(r) 2^qubits[s]) are replaced by U v (a generalisation of Eqs. NUM2-NUM8
 * to k qubits). k >= 4 runs as a dense block contraction on the matrix cores (FP64 MFMA for
 * complex128, FP32 MFMA with FP32 accumulation for complex64); k <= 3 on the vector ALUs.
 * EINVAL: k out of range, qubit out of range or repeated, NULL pointers. */
int qsim_apply_fused(qsim_state *s, int k, const int *qubits, const double *U);

/* The conditional operation of Shor's period finding (Sec. V, the step from Eq. Shor1 to Eq. Shor2):
 * with x = the value of qubits x_first .. x_first+x_qubits-1 and z = the value of qubits
 * f_first .. f_first+f_qubits-1 of a basis state, |x>|z> -> |x>|z XOR (y^x mod G)>. On a state whose
 * f-register is |0> this writes f(x) = y^x mod G into it. The map is a permutation of basis states
 * (its own inverse); amplitudes are moved without arithmetic, so the result is bit-exact. The powers
 * come from two tables of at most 2^15 residues each, built on the device in the state's scratch
 * buffer (y^xl and y^(xh 2^h) for the low and high halves of x); nothing is allocated and the call is
 * asynchronous on the state's stream like the other gates.
 * EINVAL: registers overlap or leave the state, x_qubits outside 1..30, f_qubits outside 1..32,
 * G < 2, G > 2^f_qubits or G >= 2^32. EDEVICE from the launch. */
int qsim_apply_modexp(qsim_state *s, int x_first, int x_qubits, int f_first, int f_qubits, uint64_t y, uint64_t G);

/* ---------------------------------------------------------------------------------------------
 * Reductions and normalisation (Eq. STAT1; probabilities Sec. II.A; <Q_i> Eq. Shor7)
 * All accumulate in FP64 for both dtypes.
 * ------------------------------------------------------------------------------------------- */

/* *out = sum_i |a_i|^2. Deterministic order (fixed grid, tree reductions). Synchronises. */
int qsim_norm(qsim_state *s, double *out);

/* out[i] = |a_i|^2 in FP64 for i < 2^n. out_is_device != 0: out is a device pointer to 2^n
 * doubles (asynchronous); otherwise a host pointer (synchronises). */
int qsim_probs(qsim_state *s, double *out, int out_is_device);

/* Expectation values of the qubit occupation operators, out[q] = sum_k |a_k|^2 bit_q(k) for
 * q < n (Eq. Shor7), FP64, host pointer to n doubles. Synchronises. */
int qsim_marginals(qsim_state *s, double *out);

/* Rescale the state to unit norm (Eq. STAT1): a <- a / sqrt(sum |a|^2), the norm and the factor
 * computed in FP64 on the device. norm_before (may be NULL) receives the norm before rescaling.
 * EINVAL if the norm is 0. Synchronises. */
int qsim_renormalize(qsim_state *s, double *norm_before);

/* Allocation-free form of qsim_renormalize, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. It takes the amplitudes of a
 * state as a raw device buffer (dev_amps: 2^n amplitudes of the given dtype, 16-byte aligned; 1 <= n
 * <= QSIM_MAX_QUBITS) and rescales them to unit norm in place with the kernels and reduction grid of
 * qsim_renormalize (same results, bit for bit). The FP64 norm before the rescale is written to
 * dev_norm_before (a device pointer to one double, may be NULL). A state of norm 0 is left unchanged
 * (its norm, 0, is still reported). The norm partials (at most 4096) and the norm live in a static
 * device array of 32.8 KB, one per device, held until the process ends: the call allocates nothing,
 * never synchronises and is asynchronous on hip_stream (NULL: the null stream). Calls that overlap on
 * one device share that array and race: serialise them (one stream, or events). Nothing has to be
 * cleared between calls. EINVAL on a NULL or misaligned buffer, n or dtype out of range; EDEVICE if a
 * launch fails. */
int qsim_renormalize_noalloc(void *dev_amps, int n, int dtype, void *hip_stream, double *dev_norm_before);

/* Draw `shots` basis states with probability |a_x|^2 (Sec. V: sampling of the final state).
 * uniforms: host array of `shots` doubles in [0, 1) supplied by the caller; out: host array of
 * `shots` indices. Inverse-CDF sampling over the FP64 cumulative probabilities. Synchronises. */
int qsim_sample(qsim_state *s, int64_t shots, const double *uniforms, uint64_t *out);

/* ---------------------------------------------------------------------------------------------
 * Circuits: a gate list lowered once to kernel launches, then executed on any state of that size
 * ------------------------------------------------------------------------------------------- */

typedef enum {
    QSIM_OP_MATRIX = 0, /* explicit 2x2 in u[] */
    QSIM_OP_H,          /* Eq. Hadamard */
    QSIM_OP_X,          /* Pauli sigma_x (with controls: CNOT Eq. CNOT2, Toffoli Eq. Toffoli) */
    QSIM_OP_Y,          /* Pauli sigma_y */
    QSIM_OP_Z,          /* Pauli sigma_z (with a control: CZ) */
    QSIM_OP_S,          /* diag(1, i) */
    QSIM_OP_SDG,        /* diag(1, -i) */
    QSIM_OP_T,          /* diag(1, e^{i pi/4}) */
    QSIM_OP_TDG,        /* diag(1, e^{-i pi/4}) */
    QSIM_OP_RX90,       /* the paper's X = exp(i pi S^x/2), Eq. Xoperation */
    QSIM_OP_RX90DG,     /* its inverse */
    QSIM_OP_RY90,       /* the paper's Y = exp(i pi S^y/2), Eq. Yoperation */
    QSIM_OP_RY90DG,     /* its inverse */
    QSIM_OP_PHASE,      /* R(theta) = diag(1, e^{i theta}), Eq. singlephase (controlled: Eq. COMM5) */
    QSIM_OP_RZ,         /* diag(e^{-i theta/2}, e^{+i theta/2}) */
    QSIM_OP_V,          /* V(theta) of Eq. COMM4 (controlled: Eq. NUM7) */
    QSIM_OP_SWAP,       /* quantum swap of target and target2 */
    QSIM_OP_RK,         /* R(2 pi / 2^k) = diag(1, e^{2 pi i / 2^k}) with k = target2 (0..63), the phase shift
                           of the Fourier transform and the register adders (Fig. gates, Sec. V); the
                           angle is formed from k in FP64 by the library (on the device for plain and
                           staged plans and batches, on the host where gates are fused into matrices) */
    QSIM_OP_RKDG,       /* R(-2 pi / 2^k), the inverse of QSIM_OP_RK */
    QSIM_OP_RENORM,     /* renormalisation point (plans only; target 0, no controls): the state is rescaled
                           by 1/sqrt(sum |a_i|^2) so that Eq. STAT1 holds again, the sum formed in FP64
                           (a state whose sum is 0 is left as it is). A staged plan folds it into its
                           passes: the pass before the point sums |a|^2 of what it stores, the pass after
                           it multiplies what it loads; where no pass follows (the point ends the plan)
                           or none precedes, it runs as a sweep of its own. The squared norms found are
                           read back with qsim_plan_get_norms */
    QSIM_OP_COUNT_
} qsim_op;

typedef struct qsim_gate {
    int32_t op;        /* qsim_op */
    int32_t target;    /* target qubit (QSIM_OP_SWAP: first qubit) */
    int32_t target2;   /* QSIM_OP_SWAP: second qubit; QSIM_OP_RK / QSIM_OP_RKDG: k; ignored otherwise */
    int32_t reserved;  /* must be 0 */
    uint64_t controls; /* control mask */
    double theta;      /* angle of QSIM_OP_PHASE, QSIM_OP_RZ, QSIM_OP_V */
    double u[8];       /* QSIM_OP_MATRIX entries, row-major (re, im) */
} qsim_gate;           /* 96 bytes */

typedef enum {
    QSIM_PLAN_PLAIN = 0,  /* one in-place sweep per gate (Sec. III.A) */
    QSIM_PLAN_FUSED = 1,  /* greedy fusion of consecutive gates into dense k-qubit gates */
    QSIM_PLAN_STAGED = 2, /* LDS-resident blocks: several gates per read/write of the state */
    QSIM_PLAN_AUTO = 3    /* pick the fastest of the above from the tuning table */
} qsim_plan_method;

typedef struct qsim_plan_opts {
    int32_t method;     /* qsim_plan_method */
    int32_t fuse_k;     /* QSIM_PLAN_FUSED: largest fused width, 1..5 (0 = 5) */
    int32_t lds_qubits; /* QSIM_PLAN_STAGED: qubits resident per LDS block (0 = default) */
    int32_t use_graph;  /* nonzero: record the launch sequence in a HIP graph on the first execute
                           and replay it afterwards (per state) */
    int32_t lds_regs;   /* QSIM_PLAN_STAGED: log2 of the amplitudes each thread holds in registers
                           (0 = default; 3..5 allowed); the thread count is 2^(lds_qubits - lds_regs) */
} qsim_plan_opts;

typedef struct qsim_plan_info {
    int64_t gates;          /* gates of the original circuit */
    int64_t launches;       /* launches per execute (a renormalisation step that is not folded into a
                               staged pass counts as one: QSIM_KERNEL_RENORM) */
    int64_t passes;         /* launches that read and write the whole state */
    double alg_bytes;       /* algorithmic HBM bytes per execute (per state) */
    double alg_flops;       /* algorithmic flops per execute: 8 * 2^(n+k) per fused k-qubit block;
                               for gates applied one by one (plain and staged plans, unfused gates
                               of fused plans) 14 flops per touched amplitude for a dense 2x2, 6 for
                               a phase factor, 0 for permutations and exact sign changes */
    int32_t method;         /* method actually used */
    int32_t fuse_k;         /* fused width used (QSIM_PLAN_FUSED) */
    int32_t lds_qubits;     /* resident qubits used (QSIM_PLAN_STAGED) */
    int32_t lds_regs;       /* log2 amplitudes per thread used (QSIM_PLAN_STAGED) */
    double issued_flops;    /* vector flops the kernels issue per execute (a multiply 1, a multiply-add
                               2), QSIM_PLAN_STAGED only (0 otherwise): below alg_flops where the plan
                               applies a 2x2 with a real first column (20 flops per pair) or merges
                               gates into two-qubit blocks (120 flops per four amplitudes) */
    int64_t renorms;        /* renormalisation points (QSIM_OP_RENORM) in the gate list */
} qsim_plan_info;

/* Lower `ngates` gates for states of n qubits and the given dtype. The gate list is copied.
 * EINVAL on a malformed gate (qubit range, mask, op code) or options. */
int qsim_plan_create(int n, int dtype, const qsim_gate *gates, int64_t ngates, const qsim_plan_opts *opts,
                     qsim_plan **out);
int qsim_plan_get_info(const qsim_plan *p, qsim_plan_info *info);
/* The FP64 squared norms sum |a_i|^2 (Eq. STAT1) that the plan's latest execution found at its first
 * `count` renormalisation points, in gate-list order, each taken just before its rescaling; 0 before
 * the first execution. Waits for that execution's stream. Executions of one plan on different
 * streams share these values (and a plan's buffer of per-block partial sums): they must not overlap.
 * EINVAL if count < 0 or count > info.renorms, or if host_out is NULL with count > 0. */
int qsim_plan_get_norms(const qsim_plan *p, double *host_out, int64_t count);
/* Apply the plan to the state (asynchronous on its stream). EINVAL if n or dtype differ. */
int qsim_plan_execute(qsim_plan *p, qsim_state *s);
/* Run the plan's circuit from |0...0> (the state's previous contents are ignored): the same result as
 * qsim_set_basis(s, 0) followed by qsim_plan_execute, but a staged plan generates the initial state
 * inside its first pass (no separate write of the state and no read of it). Never through a graph.
 * Asynchronous on the state's stream. EINVAL as qsim_plan_execute. */
int qsim_plan_execute_from_zero(qsim_plan *p, qsim_state *s);
int qsim_plan_free(qsim_plan *p);

/* Autotuner: lower the circuit with every candidate method and parameter set (plain if
 * include_plain; fused with k = 2..5; staged with the compiled resident-qubit / per-thread-register
 * variants of the dtype), execute each `reps` times on `scratch` (a state of the same n and dtype
 * whose contents are overwritten), and return the options of the fastest in *best and its mean
 * time per execute in *best_ms. Candidates are timed in increasing order of their HBM lower bound
 * (algorithmic bytes at 8 TB/s); one whose bound is not below the best time so far is not run. The
 * per-candidate results (opts, ms; ms < 0 if the candidate is not available or was not run) are
 * written to tried_opts / tried_ms (arrays of max_tried entries, may be NULL); *ntried receives
 * the number of candidates. Timing uses HIP events on the scratch state's stream. EINVAL on bad
 * arguments; EUNSUPPORTED if no candidate could run. */
int qsim_plan_tune(int n, int dtype, const qsim_gate *gates, int64_t ngates, qsim_state *scratch, int reps,
                   int include_plain, qsim_plan_opts *best, double *best_ms, qsim_plan_opts *tried_opts, double *tried_ms,
                   int max_tried, int *ntried);

/* Kernel classes reported by qsim_plan_execute_timed. */
enum {
    QSIM_KERNEL_GENERAL = 0,    /* 2x2 pair sweep (Eqs. NUM2-NUM4, NUM7) */
    QSIM_KERNEL_PHASE = 1,      /* phase on the |1> amplitudes (Eq. NUM5, Eq. COMM5) */
    QSIM_KERNEL_DIAG = 2,       /* diagonal 2x2 on every amplitude */
    QSIM_KERNEL_SWAP = 3,       /* permutation (Eqs. NUM6, NUM8, quantum swap) */
    QSIM_KERNEL_FUSED_VALU = 4, /* dense k <= 3 gate on the vector ALUs */
    QSIM_KERNEL_FUSED_MFMA = 5, /* dense k = 4, 5 gate on the matrix cores */
    QSIM_KERNEL_STAGED = 6,     /* LDS-resident multi-gate pass */
    QSIM_KERNEL_RENORM = 7      /* renormalisation sweep(s) outside a staged pass (Eq. STAT1) */
};

/* Kernel forms of an LDS-staged pass, reported by qsim_plan_launches. */
enum {
    QSIM_STAGED_FULL = 0, /* block in an LDS buffer of its full size */
    QSIM_STAGED_HALF = 1, /* every LDS round trip in two halves through a buffer of half the block */
    QSIM_STAGED_WAVE = 2  /* half buffer, every half a set of whole wavefronts */
};

/* The launches of a plan without running it (host only): kind[i] receives the QSIM_KERNEL_* class of
 * launch i and variant[i] its form: the fused width for fused gates, the QSIM_STAGED_* form for
 * staged passes, 0 otherwise. Each array needs info.launches entries and may be NULL. */
int qsim_plan_launches(const qsim_plan *p, int32_t *kind, int32_t *variant);

/* Execute like qsim_plan_execute (never through a graph), or like qsim_plan_execute_from_zero if
 * from_zero is nonzero, with a pair of HIP events recorded on the state's stream around every launch,
 * then synchronise. launch_ms[i] receives the duration of launch i and kind[i] its QSIM_KERNEL_* class,
 * fused_k[i] the fused width (0 if none); each array needs info.launches entries and may be NULL (a
 * plain or fused plan run from zero writes |0...0> first, outside the timed launches). */
int qsim_plan_execute_timed(qsim_plan *p, qsim_state *s, int from_zero, double *launch_ms, int32_t *kind,
                            int32_t *fused_k);

/* ---------------------------------------------------------------------------------------------
 * Batches of independent small circuits in one persistent launch
 * ------------------------------------------------------------------------------------------- */

typedef struct qsim_batch qsim_batch; /* opaque */

typedef struct qsim_batch_stats {
    double launch_ms;       /* wall time of the launch, HIP events */
    int64_t circuits;
    int64_t gates;
} qsim_batch_stats;

/* Build a batch of `count` circuits for one dtype: circuit c has nqubits[c] qubits (1..26) and the
 * gates gates[offsets[c] .. offsets[c+1]-1] (offsets has count + 1 entries, offsets[0] = 0); every
 * circuit starts from |0...0>. Each circuit is scheduled into LDS-staged passes (opts: lds_qubits,
 * lds_regs as for QSIM_PLAN_STAGED; use_graph records the run's launch sequence in a HIP graph on the
 * first run, which needs a non-NULL stream; opts may be NULL). A circuit whose state holds at least 8
 * LDS blocks is split: each of its passes runs as chunks of 4 blocks that any workgroup may take, pass
 * p in launch step p; smaller circuits run whole on one workgroup in step 0. The gate tables, the
 * work lists and the state pool are placed in device memory owned by the batch. EINVAL on malformed
 * input (a renormalisation point included), ENOMEM if the pool does not fit. */
int qsim_batch_create(int count, const int *nqubits, const int64_t *offsets, const qsim_gate *gates, int dtype,
                      const qsim_plan_opts *opts, void *stream, qsim_batch **out);
/* Run every circuit of the batch from |0...0>: one short launch that clears the stamps, then per
 * launch step one persistent kernel per kernel form (wave-split, half-buffer or full-buffer LDS
 * passes), workgroups walking the step's items in a fixed cyclic order (whole circuits first,
 * largest first). stats may be NULL. Per-circuit device timestamps (first start of its first pass ->
 * last end of its last pass) are kept for qsim_batch_latencies. Synchronises. */
int qsim_batch_run(qsim_batch *b, qsim_batch_stats *stats);
/* Per-circuit latencies of the last run in microseconds (host array of count doubles). */
int qsim_batch_latencies(qsim_batch *b, double *out_us);

typedef struct qsim_batch_info {
    int64_t circuits;       /* circuits in the batch */
    int64_t gates;          /* gates over all circuits */
    int64_t split_circuits; /* circuits whose passes are split over workgroups */
    int64_t steps;          /* launch steps (the most passes of a split circuit, at least 1) */
    int64_t launches;       /* kernel launches per run */
    int32_t lds_qubits;     /* resident qubits per LDS block */
    int32_t lds_regs;       /* log2 amplitudes per thread */
} qsim_batch_info;
/* Shape of a batch's schedule (host only). */
int qsim_batch_get_info(const qsim_batch *b, qsim_batch_info *info);
/* Copy circuit c's final state (2^nqubits[c] amplitudes) to host memory. */
int qsim_batch_download(qsim_batch *b, int c, void *host, size_t bytes);
int qsim_batch_free(qsim_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* QSIM_H */
