/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector simulator core.
 *
 * The library applies quantum gates to a state vector of 2^N complex
 * amplitudes held in GPU memory (QueenV2, arXiv 2409.14697, Sec. II-A):
 *
 *   |phi> = sum_{i in [0, 2^N)} a_i |i>                          (Eq. 1)
 *
 * stored as one contiguous array of interleaved (re, im) pairs, complex64
 * (two float32) or complex128 (two float64).  Qubit q is bit q (weight 2^q)
 * of the index i.
 *
 * A one-qubit gate G on qubit q maps every pair of amplitudes whose indices
 * differ only in bit q to G times that pair (Eq. 2).  A k-qubit gate is a
 * 2^k x 2^k matrix applied the same way to every group of 2^k amplitudes that
 * differ only in its k bits; the local row order is the one of Eq. 3:
 * for qubits (q[0], q[1]) the rows are 0_{q0}0_{q1}, 0_{q0}1_{q1},
 * 1_{q0}0_{q1}, 1_{q0}1_{q1}, i.e. q[0] is the most significant bit of the
 * local index.  The CNOT of Eq. 3 is {SV_G_CNOT, q = {control, target}}.
 *
 * Conventions shared by every entry point
 *  - Return value: SV_OK (0) or a negative sv_status.  On error nothing has
 *    been enqueued and the state is unchanged; sv_last_error() returns a
 *    message for the calling thread.
 *  - Validation happens on the host before anything is enqueued.  Device
 *    faults of earlier asynchronous work surface as SV_ERR_DEVICE at the next
 *    call that checks (at the latest at sv_sync).
 *  - Host inputs (gates, matrices, qubit lists, options) are owned by the
 *    caller and only read during the call; the library keeps its own copies.
 *  - Device work is enqueued on the state's HIP stream and is asynchronous
 *    with respect to the host; outputs written to device memory are valid
 *    once the stream reaches that point.
 *  - A state handle is not thread-safe.  Different handles may be used from
 *    different threads.  Plans are immutable once built and may be shared.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SV_OK = 0,
  SV_ERR_ARG = -1,         /* null pointer, bad size, bad enum, bad option   */
  SV_ERR_QUBIT = -2,       /* qubit index out of range or repeated           */
  SV_ERR_NOMEM = -3,       /* device or host allocation failed               */
  SV_ERR_DEVICE = -4,      /* HIP runtime / device error                     */
  SV_ERR_UNSUPPORTED = -5  /* valid request the library does not implement   */
} sv_status;

typedef enum { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

/* Gate kinds.  Parameterised kinds read sv_gate.theta (radians).  Matrices of
 * the named gates are the textbook ones, built on the host in FP64:
 *   H = [[1,1],[1,-1]]/sqrt2, X, Y, Z (Pauli), S = diag(1,i),
 *   T = diag(1, e^{i pi/4}), RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2),
 *   RZ(t) = exp(-i t Z/2) = diag(e^{-it/2}, e^{it/2}), P(t) = diag(1, e^{it}),
 *   CNOT = Eq. 3 with q = {control, target}, CZ = diag(1,1,1,-1),
 *   SWAP = exchange of |01> and |10>, CPHASE(t) = diag(1,1,1,e^{it}),
 *   RZZ(t) = exp(-i t Z(x)Z/2).
 * SV_G_MATRIX carries an explicit 2^nq x 2^nq unitary (Sec. III-B: gates the
 * library has no name for are supplied as a unitary it supports). */
typedef enum {
  SV_G_MATRIX = 0,
  SV_G_H = 1, SV_G_X = 2, SV_G_Y = 3, SV_G_Z = 4, SV_G_S = 5, SV_G_T = 6,
  SV_G_RX = 7, SV_G_RY = 8, SV_G_RZ = 9, SV_G_P = 10,
  SV_G_CNOT = 11, SV_G_CZ = 12, SV_G_SWAP = 13, SV_G_CPHASE = 14, SV_G_RZZ = 15
} sv_gate_kind;

#define SV_MAX_GATE_QUBITS 6   /* largest dense gate (64 x 64)              */
#define SV_MAX_QUBITS 34       /* 2^34 complex64 = 128 GiB                    */

/* One gate.  Caller-owned; read only during the call.
 *   kind  : sv_gate_kind
 *   nq    : number of qubits (must match the kind; 1..6 for SV_G_MATRIX)
 *   q     : qubit indices, q[0] = most significant bit of the local index
 *   theta : angle for RX/RY/RZ/P/CPHASE/RZZ, ignored otherwise
 *   m     : SV_G_MATRIX only: 2^nq x 2^nq complex matrix, row-major,
 *           interleaved (re, im) FP64, host memory; NULL for named kinds.
 * The library does not check unitarity. */
typedef struct {
  int32_t kind;
  int32_t nq;
  int32_t q[SV_MAX_GATE_QUBITS];
  double theta;
  const double *m;
} sv_gate;

typedef struct sv_state sv_state;  /* opaque: one state vector on one GPU    */
typedef struct sv_plan sv_plan;    /* opaque: host-only executable schedule   */

/* Execution strategy of a plan. */
typedef enum {
  SV_MODE_AUTO = 0,   /* cost model picks the cheapest of a tile-pass plan,
                         a matrix-pass plan and a one-sweep-per-fused-op
                         plan                                              */
  SV_MODE_SWEEP = 1,  /* one full-state sweep per (fused) op                */
  SV_MODE_PASS = 2,   /* LDS in-cache passes that apply many ops per sweep  */
  SV_MODE_MATRIX = 3  /* fused dense ops (Sec. II-B gate fusion) grouped by
                         locality: each group runs in one in-cache pass
                         (Sec. II-B, III-B) as matrix-core products on the
                         tiles; ops that gain nothing grouped run as sweeps */
} sv_mode;

/* Planner / executor options.  Pass NULL for the defaults that
 * sv_default_opts() fills in. */
typedef struct {
  int32_t max_fuse_qubits;  /* general gate fusion width (Sec. II-B, III-A
                               tier 5); 0 or 1 disables dense fusion; <= 6.
                               default 5                                      */
  int32_t lds_qubits;       /* local qubits per in-cache tile, 5..12 (complex128)
                               or 5..13 (complex64); 0 = auto (the maximum)   */
  int32_t pinned_low_bits;  /* low index bits always inside a tile (memory
                               coalescing); 0 = auto                          */
  int32_t reorder;          /* 1 = let passes move qubits (Sec. II-B qubit
                               reordering), restoring logical order at the end;
                               default 1                                      */
  int32_t fp32_mfma;        /* complex64 states: dense fused ops of >= 4
                               qubits run as FP32 MFMA contractions; default 1 */
  int32_t renorm_interval;  /* complex64 states: rescale to unit norm (FP64
                               norm) every R dense ops; 0 = never; default 0   */
  int32_t mode;             /* sv_mode; default SV_MODE_AUTO                   */
  int32_t max_pass_ops;     /* tile passes: at most this many ops per pass, so
                               that passes of many states in one launch take
                               similar times; 0 = no limit; default 0          */
} sv_opts;

/* Fill *o with the defaults.  Never fails for non-null o. */
sv_status sv_default_opts(sv_opts *o);

#define SV_NO_INIT 1u  /* sv_create flag: keep the buffer's current contents */

/* Create a state vector |phi> = sum_i a_i |i> of 2^n_qubits amplitudes
 * (Eq. 1 and the state of Sec. II-A: one complex amplitude per basis state,
 * qubit q = index bit q), n_qubits in 1..SV_MAX_QUBITS, of type dt.
 *   dev_ptr    : NULL -> the library allocates 2^n elements on the current
 *                HIP device and frees them in sv_destroy; otherwise borrowed
 *                device memory of at least 2^n elements, 256-byte aligned,
 *                that the caller keeps alive until sv_destroy.
 *   hip_stream : hipStream_t used for all work on this state (NULL = the
 *                null stream).
 *   flags      : 0 -> initialise to |0...0>; SV_NO_INIT -> leave contents.
 * Errors: SV_ERR_ARG (n, dt, out, alignment), SV_ERR_NOMEM, SV_ERR_DEVICE. */
sv_status sv_create(int n_qubits, sv_dtype dt, void *dev_ptr, void *hip_stream,
                    unsigned flags, sv_state **out);

/* Destroy a state; frees only memory the library allocated.  When it frees
 * device memory (an owned state buffer, reduction scratch, upload buffers) it
 * first waits for the state's stream; a state on a borrowed buffer that never
 * needed scratch returns at once, and the caller orders the reuse of its
 * buffer after the work it queued.  NULL is accepted. */
sv_status sv_destroy(sv_state *s);

/* Query n, dtype and device pointer (any output may be NULL). */
sv_status sv_state_info(const sv_state *s, int *n_qubits, sv_dtype *dt, void **dev_ptr);

/* Change the stream later work is enqueued on (no synchronisation is done). */
sv_status sv_set_stream(sv_state *s, void *hip_stream);

/* Set the state to the basis state |index> (index < 2^n).  Async. */
sv_status sv_init_basis(sv_state *s, uint64_t index);

/* Apply one gate by one sweep over the state (Eq. 2 / Eq. 3; the
 * gate-by-gate scheme).  Async.  Errors: SV_ERR_ARG, SV_ERR_QUBIT. */
sv_status sv_apply_gate(sv_state *s, const sv_gate *g);

/* Plan a gate list for an n_qubits state of type dt (host only, no device
 * needed): general gate fusion up to o->max_fuse_qubits (Sec. II-B, III-A),
 * grouping of ops into in-cache passes (Sec. II-B, III-B) and qubit
 * reordering with a logical<->physical map (Sec. II-B, III-A).  The plan
 * applies exactly the product of the gates; only rounding differs. */
sv_status sv_fuse(int n_qubits, sv_dtype dt, const sv_gate *g, size_t n_gates,
                  const sv_opts *o, sv_plan **out);

/* Plan introspection: number of fused ops (Sec. II-B gate fusion) and of
 * state sweeps (passes: in-cache tile passes of Sec. III-B count one each). */
sv_status sv_plan_info(const sv_plan *p, size_t *n_ops, size_t *n_passes);

/* Export fused op `op` (0-based, in execution order) in logical qubits, as
 * the generic gate that general gate fusion produces (Sec. II-B "Gate
 * Fusion", Sec. III-A tier 5: the product of the fused gates' matrices):
 *   *nq, q[0..nq-1] (q[0] = MSB of the local index), the 2^nq x 2^nq matrix
 *   into m (row-major interleaved FP64; caller buffer of 2*64*64 doubles) and
 *   the pass it runs in (-1: a SWAP realised by relabeling qubits, no data
 *   moves).  Replaying all ops in order reproduces the circuit. */
sv_status sv_plan_export(const sv_plan *p, size_t op, int32_t *nq, int32_t q[SV_MAX_GATE_QUBITS],
                         double *m, int32_t *pass);

/* Describe pass `pass`: kind (0 = sweep kernel, 1 = LDS in-cache tile pass,
 * 2 = dense fused kernel, 3 = permutation, 4 = matrix pass), number of ops,
 * the number of local qubits of its tile (0 for sweeps) and of stages (LDS
 * round trips of the tile; one per op in a matrix pass; 0 for sweeps).
 * Outputs may be NULL. */
sv_status sv_plan_pass_info(const sv_plan *p, size_t pass, int32_t *kind, int32_t *n_ops,
                            int32_t *n_local, int32_t *n_stages);

/* Algorithmic arithmetic of pass `pass`, in real flops per amplitude of the
 * state: the sum over its ops of 8 * 2^k for a dense k-qubit op (one complex
 * multiply-add per matrix entry), 6 for a diagonal op (one complex multiply)
 * and 0 for a permutation.  Errors: SV_ERR_ARG. */
sv_status sv_plan_pass_flops(const sv_plan *p, size_t pass, double *flops_per_amp);

/* The same for every pass at once: flops_per_amp[i] for each pass i (host
 * memory of `count` doubles, count >= the plan's number of passes; entries
 * beyond it are not written).  Errors: SV_ERR_ARG. */
sv_status sv_plan_flops(const sv_plan *p, double *flops_per_amp, size_t count);

/* Kernel ops of tile pass `pass` after register staging: *n_ops ops in
 * total (per register stage: one per single-qubit gate of its tensor-product
 * layer, one for a dense two-qubit gate, one for its register-index factor
 * table, one per lane item and one per permutation gate), *n_ladders of them
 * fixed-point phase functions: a phase ladder (the
 * phases of a run of diagonal gates that fall on the amplitudes whose
 * register qubit is 1) or a quadratic phase over the bits outside the
 * registers (the rest of such a run), each applied as one op with a
 * fixed-point angle sum (Sec. III-A: gate grouping inside a tile and the
 * fusion of diagonal gates).  Both 0 for passes that are not tile passes.
 * Outputs may be NULL.
 * Errors: SV_ERR_ARG. */
sv_status sv_plan_pass_ops(const sv_plan *p, size_t pass, int32_t *n_ops, int32_t *n_ladders);

sv_status sv_plan_destroy(sv_plan *p);

/* Execute a plan built for this state's n and dtype: the gate-by-gate
 * result of Eq. 2 / Eq. 3 for every gate of the planned circuit, reached
 * through fused ops, in-cache tile passes and qubit reordering (Sec. II-B,
 * Sec. III-A/B).  Async.  The state is in logical qubit order again when the
 * plan's last pass completes.  Errors: SV_ERR_ARG (null, or a plan built for
 * another n or dtype), SV_ERR_NOMEM (upload buffer), SV_ERR_DEVICE. */
sv_status sv_apply_plan(sv_state *s, const sv_plan *p);

/* Apply a gate list (a circuit, Sec. II-B / Sec. III: simulation applies its
 * gates in order by Eq. 2 / Eq. 3) to the state: sv_fuse + sv_apply_plan +
 * sv_plan_destroy with options o (NULL = defaults).  Async.  Errors: those of
 * sv_fuse (nothing enqueued) and of sv_apply_plan. */
sv_status sv_apply_circuit(sv_state *s, const sv_gate *g, size_t n_gates, const sv_opts *o);

/* Physically reorder qubits (Sec. II-B qubit reordering / in-memory
 * swapping): the amplitude at index i moves to the index whose bit dest[q]
 * equals bit q of i.  dest is a permutation of 0..n-1 (n entries).  Runs as
 * in-cache permutation passes (bitwise exact; a few full read+write sweeps
 * of the state at most).  Async.  Errors: SV_ERR_ARG (null), SV_ERR_QUBIT
 * (entry out of range or repeated; the state is untouched), SV_ERR_NOMEM,
 * SV_ERR_DEVICE. */
sv_status sv_permute_qubits(sv_state *s, const int32_t *dest);

/* Marginal probabilities over m qubits (0 <= m <= n, distinct), from the
 * probability |a_i|^2 of basis state |i> (Eq. 1) and the normalisation
 * sum_i |a_i|^2 = 1 of Sec. II-A:
 *   out_dev[b] = sum of |a_i|^2 over all i whose bit qubits[r] equals bit
 *   (m-1-r) of b, i.e. qubits[0] is the most significant bit of b.
 * m = 0 gives out_dev[0] = sum |a_i|^2 (the squared norm).  Accumulated in
 * FP64 for both dtypes; deterministic (fixed reduction order).
 * out_dev: device memory for 2^m doubles.  Async. */
sv_status sv_measure_probs(sv_state *s, const int32_t *qubits, int m, double *out_dev);

/* sv_measure_probs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same marginal, bitwise, with its reduction partials in a
 * static device array of the library (8 MiB per GPU, held until the process
 * ends) instead of the state's lazily allocated scratch.  Calls no hipMalloc
 * or hipFree; the first call on a GPU resolves the array's address there.
 * Every call on one GPU shares that array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and may return wrong
 * values; order them.  Same arguments, ownership and errors as
 * sv_measure_probs, plus SV_ERR_UNSUPPORTED if a reduction ever needed more
 * than the array holds (the reduction's geometry keeps every marginal
 * within it). */
sv_status sv_measure_probs_noalloc(sv_state *s, const int32_t *qubits, int m, double *out_dev);

/* Multiply every amplitude by the real factor `scale` (e.g. 1/||psi|| in
 * FP64).  Async. */
sv_status sv_scale(sv_state *s, double scale);

/* Wait for all work on the state's stream; reports device errors. */
sv_status sv_sync(sv_state *s);

/* Message for the last failure on the calling thread ("" if none). */
const char *sv_last_error(void);

/* ---- Serving: device-resident programs and batched passes ---------------
 * A request loop keeps many states resident and advances all of them with one
 * step per pass (continuous batching): one kernel launch runs the next
 * in-cache tile pass of every active state, so requests admitted later join
 * the next launch and their work overlaps with older ones on the device;
 * a state whose next pass is a matrix, dense or sweep pass runs it as a
 * launch of its own in the same step. */
typedef struct sv_program sv_program;  /* the passes of one plan, in device memory */
typedef struct sv_batcher sv_batcher;  /* launches one pass of many states at once        */

/* Device bytes a program of plan p occupies (for a caller-owned buffer).
 * Errors: SV_ERR_ARG, SV_ERR_UNSUPPORTED (a pass the packer cannot encode:
 * an internal planner failure, not expected for plans sv_fuse returns). */
sv_status sv_program_bytes(const sv_plan *p, size_t *bytes);

/* Upload the program of plan p (any mode: tile, permutation, matrix, dense
 * and sweep passes), stream-ordered on hip_stream (NULL = null stream).  A
 * program does not renormalise: the plan's renorm_interval is not applied
 * to complex64 states run through a batcher.
 *   dev_buf : NULL -> the library allocates the device copy and frees it in
 *             sv_program_destroy; otherwise caller device memory of at least
 *             sv_program_bytes(p) bytes, 256-byte aligned, kept alive while
 *             work that uses the program may run.
 * The program keeps its own host copy; the plan may be destroyed at once.
 * Errors: SV_ERR_ARG, SV_ERR_UNSUPPORTED (as sv_program_bytes), SV_ERR_NOMEM,
 * SV_ERR_DEVICE. */
sv_status sv_program_create(const sv_plan *p, void *dev_buf, size_t buf_bytes, void *hip_stream,
                            sv_program **out);

/* Qubits, dtype and number of passes of a program (outputs may be NULL). */
sv_status sv_program_info(const sv_program *prog, int32_t *n_qubits, sv_dtype *dt, int32_t *n_passes);

/* Free a program.  When the library owns its device copy it first waits for
 * the upload stream; with a caller buffer it waits only for the program's
 * own upload (so that its host copy may be freed) and the caller orders the
 * reuse of the buffer after the work that reads it.  NULL is accepted. */
sv_status sv_program_destroy(sv_program *prog);

/* A batcher owns its stream and small descriptor buffers. */
sv_status sv_batcher_create(void *hip_stream, sv_batcher **out);

/* One step: for every i < count, run pass pass_index[i] of programs[i] on
 * states[i] -- the tile and permutation passes of all items in one launch,
 * each matrix, dense or sweep pass in a launch of its own.  All states and programs must share one dtype; states[i] must
 * have programs[i]'s qubit count; a state may appear at most once.  Work is
 * enqueued on the batcher's stream: the caller orders it against other work
 * on the states (e.g. by creating the states on the same stream).  A state's
 * result depends only on its own program -- bitwise the same in any batch.
 * Errors: SV_ERR_ARG (count, null entries, mismatched n/dtype, pass index out
 * of range; checked before anything is enqueued), SV_ERR_NOMEM, SV_ERR_DEVICE
 * (the passes of some items may already be enqueued). */
sv_status sv_batcher_run(sv_batcher *b, int count, sv_state *const *states, const sv_program *const *programs,
                         const int32_t *pass_index);

/* Marginal probabilities of one state as sv_measure_probs defines them, but
 * enqueued on the batcher's stream with reduction scratch the batcher owns,
 * so that serving loops allocate nothing per request.  out_dev: device
 * memory for 2^m doubles.  Errors: SV_ERR_ARG, SV_ERR_QUBIT, SV_ERR_NOMEM,
 * SV_ERR_DEVICE. */
sv_status sv_batcher_probs(sv_batcher *b, const sv_state *s, const int32_t *qubits, int m, double *out_dev);

/* Free a batcher (waits for its stream).  NULL is accepted. */
sv_status sv_batcher_destroy(sv_batcher *b);

/* Library version string. */
const char *sv_version(void);

/* Which kernel sv_apply_gate would launch for gate g on an n-qubit state of
 * type dt (host only; no device needed).  Writes a NUL-terminated identifier
 * into buf (at most len bytes), e.g. "group/c128/SWAP/z2v2" (touched-subset
 * group sweep), "lane/c64/K2/INTRA-REG/z1" (lane-exchange sweep) or
 * "dense/c128/k5".  For attributing measured kernel time to gates.
 * Errors: SV_ERR_ARG, SV_ERR_QUBIT (as sv_apply_gate). */
sv_status sv_gate_kernel(int n_qubits, sv_dtype dt, const sv_gate *g, char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* SV_H */
