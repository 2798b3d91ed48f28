/*
 * qs.h -- C ABI of libqs: a fused, LDS-blocked state-vector simulator hot
 * path for AMD MI355X (gfx950).
 *
 * The method is the cache-aware state-vector simulation of arXiv 2406.14084
 * ("Queen"): gates are grouped into gate blocks whose qubits fit in an
 * on-chip chunk (Sec. IV, Eq. 5-7, Alg. 1-2), qubit-reorder swaps bring the
 * qubits a block needs into its chunk (Sec. II-B Eq. 4, Sec. V-B Alg. 4), and
 * every chunk is staged on chip once per block while all of the block's gates
 * are applied to it (Sec. V-A, Alg. 3).
 *
 * Conventions used by every entry point:
 *   - State: 2^n amplitudes a_i (Eq. 1), interleaved (re, im), complex128
 *     (16 B) or complex64 (8 B).  Qubit q is bit q of the index (q0 = LSB).
 *   - A k-qubit gate on targets t[0..k-1] is a 2^k x 2^k complex128 matrix,
 *     row-major, interleaved (re, im); bit (k-1-j) of the local row/column
 *     index is the bit of qubit t[j] (t[0] is the most significant, as in
 *     Eq. 3 where the first listed qubit is CNOT's control).
 *   - Memory: the caller (PyTorch) owns the state vector and any output
 *     buffer.  The library never frees them.  Plans and handles are owned
 *     by the library and freed with qs_plan_free / qs_destroy.
 *   - Errors: every call returns a qs_status; on failure nothing is written
 *     to outputs and qs_last_error() gives a message (thread-local).  No call
 *     throws or aborts across the ABI.
 *   - Asynchrony: device work is queued on the stream given to qs_attach;
 *     calls that return host values synchronise that stream.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define QS_API __attribute__((visibility("default")))
#else
#define QS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { QS_C128 = 0, QS_C64 = 1 } qs_dtype;

typedef enum {
    QS_OK = 0,
    QS_EINVAL = -1,        /* bad argument: target out of range or repeated, k outside 1..5, n outside 1..34, size mismatch */
    QS_ENOMEM = -2,        /* host or device allocation failed */
    QS_EHIP = -3,          /* a HIP runtime call failed; qs_last_error() has its text */
    QS_EUNSUPPORTED = -4,  /* valid request this build does not implement */
    QS_ESTATE = -5         /* handle not attached, or plan and state disagree on n or dtype */
} qs_status;

typedef struct qs_state qs_state;
typedef struct qs_plan qs_plan;
typedef struct qs_costmodel qs_costmodel;

/* A circuit: an ordered gate list (the paper's raw circuit, one gate per
 * line, Sec. VI / artifact "[Gate type] [Target qubits] [ID]"), with an
 * explicit matrix per gate.
 *   k[g]            number of qubits of gate g, 1..5
 *   targets[5*g+j]  qubit t[j] of gate g (j < k[g]; other slots ignored)
 *   matrices        the gates' matrices back to back: gate g's 2^k x 2^k
 *                   complex128 matrix (2 * 4^k doubles) follows gate g-1's. */
typedef struct {
    int n;
    int ngates;
    const int *k;
    const int *targets;
    const double *matrices;
} qs_circuit;

/* Planner options (the paper's optimizer arguments: cache size C, fusion
 * size F and the on/off switches of its artifact command line). */
typedef struct {
    int chunk_qubits;     /* C: qubits per on-chip chunk; 0 = default for the dtype (12 for complex128, 13 for complex64) */
    int low_qubits;       /* L: lowest physical qubits always in the chunk (contiguous 2^L-amplitude runs); 0 = default (4) */
    int enable_swaps;     /* 1: reorder qubits between blocks (folded into block write-back, or standalone swap passes) */
    int enable_fusion;    /* 1: fuse gates inside a block into <= kmax-qubit unitaries / merged diagonals */
    int planner;          /* 0 = heuristic (fixed geometry C, r, L); 1 = learned: candidate plans over C, r, L and the
                             fusion width ranked by the cost model's predicted time, the heuristic kept unless a
                             candidate is predicted >= 2 % faster; 2 = gate-by-gate (no blocking); 3 = the same
                             candidates ranked by the number of passes (the paper's objective, Eq. 7) */
    const qs_costmodel *cost_model;  /* required when planner == 1, else NULL */
    qs_dtype dtype;       /* precision the plan will run at (matrices are rounded once, after FP64 composition) */
    int reg_qubits;       /* r: register-resident qubits per thread (4 or 5); 0 = default */
    int no_mfma;          /* complex64: 1 keeps dense ops of 4-5 qubits on vector FMA instead of matrix cores */
    int no_split;         /* 1 keeps single-qubit gates whole; 0 (default, with fusion on) applies each unitary
                             single-qubit gate as diag * real rotation * diag: the rotation runs as three in-place
                             shears (3 FMAs per amplitude instead of 8), the diagonals merge with their neighbours */
} qs_plan_opts;

/* One Pauli string times a real coefficient.  Per qubit q the letter is
 * (bit q of xmask, bit q of zmask): (0,0)=I, (1,0)=X, (0,1)=Z, (1,1)=Y.
 * Requires n <= 64. */
typedef struct {
    uint64_t xmask;
    uint64_t zmask;
    double coeff;
} qs_pauli;

/* Summary of a plan (algorithmic figures, independent of timing). */
typedef struct {
    int n;
    int dtype;
    int gates;            /* gates in the input circuit */
    int blocks;           /* gate blocks = HBM passes that apply gates */
    int swap_passes;      /* HBM passes that only permute qubits */
    int ops;              /* fused ops over all blocks */
    int ops_dense[6];     /* dense ops by qubit count (index 1..5) */
    int ops_diag;         /* diagonal ops (merged diagonals) */
    int phases;           /* register phases over all blocks (LDS exchanges) */
    int chunk_qubits;
    int low_qubits;
    int reg_qubits;
    double flops_per_amp; /* sum over ops of algorithmic flops per amplitude (dense k: 8*2^k, diagonal: 6, rotation: 6) */
    double hbm_bytes;     /* (blocks + swap_passes) * 2 * 2^n * bytes per amplitude */
    double plan_seconds;  /* host time spent in qs_fuse */
    int planner;          /* planner that produced the plan: 0 heuristic, 1 learned, 2 gate by gate, 3 pass count */
    int candidates;       /* plans compared (1 unless the learned planner ran) */
    double predicted_ms;  /* learned planner: predicted time of the chosen plan, else -1 */
    double predicted_heuristic_ms; /* learned planner: predicted time of the heuristic plan, else -1 */
    int ops_mfma;         /* dense ops (counted in ops_dense too) that run on matrix cores */
    int ops_rot;          /* single-qubit real rotations applied as shears (one per bit of each rotation op) */
    int ops_perm;         /* permutation ops (X, CX, CCX, SWAP on register bits): data movement, no arithmetic */
} qs_plan_stats;

/* ---- state handles ------------------------------------------------------ */

/* Create a handle for an n-qubit state of the given dtype (1 <= n <= 34).
 * The handle owns no state memory until qs_attach.  Paper: Sec. III (2^N
 * amplitudes; here one device holds all of them). */
QS_API qs_status qs_create(int n, qs_dtype dtype, qs_state **out);

/* Bind caller-owned device memory of exactly 2^n amplitudes (bytes =
 * 2^n * 16 or 2^n * 8, 256-byte aligned) and a hipStream_t (NULL = default
 * stream) to the handle.  The memory stays the caller's.
 * workspace / ws_bytes: caller-owned device scratch on the same device, at
 * least qs_workspace_size() bytes, 256-byte aligned; the library keeps gate
 * matrices of 4-5 qubits, swap programs and reduction partials there, in
 * stream order, and never frees it.  workspace = NULL makes the handle
 * allocate its own scratch of that size (freed by qs_destroy).
 * QS_EINVAL for a size or alignment mismatch or a pointer that is not
 * device memory. */
QS_API qs_status qs_attach(qs_state *st, void *amps_dev, size_t bytes, void *hip_stream, void *workspace,
                           size_t ws_bytes);

/* Bytes of device workspace a handle for (n, dtype) needs (qs_attach).
 * Host only. */
QS_API qs_status qs_workspace_size(int n, qs_dtype dtype, size_t *bytes);

/* Free the handle (not the attached memory). */
QS_API qs_status qs_destroy(qs_state *st);

/* |0...0>: a_0 = 1, all others 0 (Alg. 3 input).  Async. */
QS_API qs_status qs_init_zero(qs_state *st);

/* |i>: a_i = 1, all others 0.  Async. */
QS_API qs_status qs_init_basis(qs_state *st, uint64_t index);

/* ---- gate-by-gate path -------------------------------------------------- */

/* Apply one k-qubit gate (1 <= k <= 5) with one full pass over the state
 * (Eq. 2, Eq. 3; the gate-by-gate scheme the paper compares against).
 * targets: host array of k distinct qubits; matrix: host, 2 * 4^k doubles,
 * copied before return.  Async. */
QS_API qs_status qs_apply_gate(qs_state *st, int k, const int *targets, const double *matrix);

/* How qs_apply_gate runs a gate (host only, no state needed): qubits on
 * which the matrix acts as the identity unless the qubit is 1 are controls
 * (*ctrl_mask, qubit numbers as bits) and the pass visits only amplitudes
 * with every control set; on the *active remaining targets the matrix is
 * *kind = 0 dense, 1 diagonal (only entries different from 1 are applied:
 * CZ and CP touch a quarter of the state), 2 a permutation with phases (only
 * rows that move or change are written; with unit phases no arithmetic: CX
 * and SWAP move half the state).  Paper: Sec. VI-D (gates that touch less of
 * the state, or do no floating-point work, run faster), Eq. 2 / Eq. 3. */
QS_API qs_status qs_gate_class(int k, const int *targets, const double *matrix, int *kind, uint64_t *ctrl_mask,
                               int *active);

/* In-memory swap of qubit sets (Eq. 4, Alg. 4): exchange index bits a[j] and
 * b[j] for j < s (all 2s qubits distinct, s <= 8).  One pass.  Async. */
QS_API qs_status qs_swap_qubits(qs_state *st, int s, const int *a, const int *b);

/* ---- planner and blocked path ------------------------------------------- */

/* Plan a circuit (host only; copies everything it reads): classify gates,
 * find gate blocks at chunk size C with qubit-reorder swaps (Alg. 1-2),
 * fuse gates inside each block into ops of at most kmax qubits (1..5)
 * composed in FP64 (Alg. 2 level 3), and schedule each block's ops into
 * register phases.  opts may be NULL (defaults).  The plan does not depend
 * on any state handle; *out is freed with qs_plan_free. */
QS_API qs_status qs_fuse(const qs_circuit *circ, int kmax, const qs_plan_opts *opts, qs_plan **out);

/* Run a plan on a state (Alg. 3): for each step, one blocked pass or one
 * swap pass over HBM.  The state is left in canonical qubit order.  The
 * plan keeps its device tables (program words, matrices) per device: the
 * first call on a device allocates them and uploads them with
 * hipMemcpyAsync on the state's stream (later calls from other streams wait
 * for that upload through an event); the upload is guarded by a per-plan
 * lock, so one plan may be applied from several threads.  The plan must
 * outlive the queued work that uses it.  Async. */
QS_API qs_status qs_apply_plan(qs_state *st, qs_plan *plan);

/* Same as qs_apply_plan, but records a hipEvent on the bound stream before
 * and after every step and returns each step's device time in ms (ms_out:
 * host array of at least the plan's step count).  *kinds_out (optional)
 * gets 1 for a gate block, 0 for a swap pass.  Synchronises the stream. */
QS_API qs_status qs_apply_plan_timed(qs_state *st, qs_plan *plan, float *ms_out, int *kinds_out, int cap);

/* Release a plan and its device tables. */
QS_API qs_status qs_plan_free(qs_plan *plan);

/* Text form of the plan in the spirit of the paper's optimized-circuit file:
 * per step a count line then the step's lines ("SWAP ...", "BLOCK ...",
 * "PHASE ...", "U<k> ..."/"D<k> ..." with physical local targets and source
 * gate ids).  Writes at most len bytes including the NUL; *needed gets the
 * full size.  Host only. */
QS_API qs_status qs_plan_dump(const qs_plan *plan, char *buf, size_t len, size_t *needed);

/* Fill *out with the plan's summary.  Host only. */
QS_API qs_status qs_plan_get_stats(const qs_plan *plan, qs_plan_stats *out);

/* Detailed per-block structure for tests and for the cost model:
 * for block b (0-based in step order, swap passes excluded),
 * phys[0..C-1] = physical qubits of the chunk, gate_ids = the original gate
 * indices the block applies (in execution order).  Returns QS_EINVAL when b
 * is out of range.  *ngids gets the count; at most cap ids are written. */
QS_API qs_status qs_plan_block(const qs_plan *plan, int b, int *phys, int *gate_ids, int cap, int *ngids);

/* Logical->physical qubit map in force before each step (perm[q] = physical
 * position of logical qubit q), for step s of the plan's nsteps (swap and
 * block steps counted together); s == nsteps gives the final map (identity).
 * *nsteps may be NULL. */
QS_API qs_status qs_plan_layout(const qs_plan *plan, int s, int *perm, int *nsteps);

/* The encoded device program of a plan, for host-side inspection (tests
 * replay it on the CPU to check every index the blocked kernel forms).
 * words: int32 program of all steps back to back (*nwords of them, at most
 * cap written); offsets: start word of each step (*nsteps, at most
 * cap_steps written).  *r and *C receive the register and chunk widths the
 * program was encoded for.  Host only. */
QS_API qs_status qs_plan_program(const qs_plan *plan, int32_t *words, size_t cap, size_t *nwords,
                                 int64_t *offsets, int cap_steps, int *nsteps, int *r, int *C,
                                 double *mats, size_t cap_mats, size_t *nmats);

/* ---- readout ------------------------------------------------------------- */

/* p_i = |a_i|^2 for all i, FP64, into caller device memory out_dev (2^n
 * doubles).  Paper: Sec. II-A Eq. 1 (the squared magnitude of amplitude
 * a_i is the probability of basis state i).  Async. */
QS_API qs_status qs_probs(qs_state *st, double *out_dev);

/* sum_t coeff_t <psi|P_t|psi> over nterms Pauli strings (FP64 accumulation),
 * written to *out_host.  Paper: Sec. II-A Eq. 1 (a measurement outcome i has
 * probability |a_i|^2; a Pauli string is diagonal, up to the bit flips of
 * its X/Y letters, in that basis: <P> = sum_i conj(a_{i^x}) ph(i) a_i with
 * ph(i) = i^{#Y} (-1)^{popcount(i & zmask)}).  Uses the workspace for the
 * terms and per-workgroup partial sums; the partials are added on the host
 * in a fixed order.  Synchronises the stream. */
QS_API qs_status qs_expect(qs_state *st, int nterms, const qs_pauli *terms, double *out_host);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * value as qs_expect, but the terms and the per-workgroup partial sums go to
 * a fixed array inside the library (about 1 MiB per GPU, held until the
 * process ends) instead of the handle's workspace, and the partials are
 * summed on the device in the same fixed order.  At most 64 terms per call
 * (QS_EINVAL beyond).  Calls no hipMalloc/hipFree.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other threads,
 * other streams) race.  Synchronises the stream. */
QS_API qs_status qs_expect_noalloc(qs_state *st, int nterms, const qs_pauli *terms, double *out_host);

/* Copy amplitudes [first, first + count) of the state (2^n of them,
 * interleaved re/im at the state's precision, 16 or 8 bytes each) to host
 * memory host_out, in canonical qubit order.  Paper: Alg. 3's output, the
 * simulated amplitudes of the state vector.  QS_EINVAL when the range
 * leaves the state.  Synchronises the stream. */
QS_API qs_status qs_get_amplitudes(qs_state *st, uint64_t first, uint64_t count, void *host_out);

/* ---- batched QAOA (many small uneven circuits in one launch) ------------- */

/* Descriptor of one MaxCut QAOA instance: n qubits (2..20), nedges edges
 * (u, v) at edges[2*e], p layers with angles gammas[l], betas[l].  Circuit:
 * |+>^n, then per layer a_z *= exp(-i gamma C(z)) (C = cut size) and RX(2 beta)
 * on every qubit; output <C> in FP64. */
typedef struct {
    int n;
    int nedges;
    int p;
    const int *edges;
    const double *gammas;
    const double *betas;
} qs_qaoa_instance;

typedef struct qs_batch qs_batch;

/* Pack count instances into device tables and a task queue.  An instance of
 * at most CB qubits runs whole in one workgroup's LDS; a larger one keeps its
 * state (and one byte per amplitude of cached cut values) in a workspace and
 * is split into chunk tasks of 2^CB amplitudes, two passes per layer.  CB is
 * 13 for complex64 and 12 for complex128 until qs_batch_autotune picks
 * between that and one less (the workspace covers both).  dtype: QS_C64 (complex64 state, FP64 reductions) or
 * QS_C128.  hip_stream: stream for all work.  workspace / ws_bytes:
 * caller-owned device memory of at least qs_batch_qaoa_workspace_size()
 * bytes (256-byte aligned) for those states, or NULL to let the batch
 * allocate it.  The small tables (descriptors, tasks, edges, phases,
 * counters) are allocated by the batch and freed by qs_batch_free.
 * Launch shape defaults to 256 threads, 2 workgroups per CU and 8 chunks per
 * task until qs_batch_autotune picks one.  Paper: QAOA is one of the
 * benchmark circuits of Sec. VI-A (Table II); batching is this library's
 * addition. */
QS_API qs_status qs_batch_qaoa_create(int count, const qs_qaoa_instance *inst, qs_dtype dtype,
                               void *hip_stream, void *workspace, size_t ws_bytes, qs_batch **out);

/* Workspace bytes qs_batch_qaoa_create needs for these instances (0 when
 * every instance fits one workgroup's LDS).  Host only. */
QS_API qs_status qs_batch_qaoa_workspace_size(int count, const qs_qaoa_instance *inst, qs_dtype dtype,
                                              size_t *bytes);

/* Run every instance in one persistent launch; out_dev: count doubles of
 * <C> in device memory (caller-owned).  use_graph = 1 replays a captured
 * hipGraph of the launch (captured on first use).  Async. */
QS_API qs_status qs_batch_qaoa_run(qs_batch *b, double *out_dev, int use_graph);

/* Reference schedule: one launch per instance, in sequence (same kernels,
 * same results), for comparison.  Async. */
QS_API qs_status qs_batch_qaoa_run_sequential(qs_batch *b, double *out_dev);

QS_API qs_status qs_batch_free(qs_batch *b);

/* Nonzero *err if a pass of a large instance gave up waiting for its
 * previous pass (a bounded spin in the persistent kernel; its results are
 * then invalid).  Synchronises the stream. */
QS_API qs_status qs_batch_error(qs_batch *b, int *err);

/* Choose the launch shape (threads 256/512 x workgroups per CU, 5 shapes),
 * the number of chunks per task of the large instances (2, 8, 32 or 128) and
 * the LDS chunk size CB (12 or 13 qubits for complex64, 11 or 12 for
 * complex128) by timing all 40 combinations on the device for this batch;
 * *chosen gets shape + 5 * (grouping + 4 * chunk size index), and the choice
 * stays in force for later runs of this batch (a captured graph is
 * re-captured).  Synchronises. */
QS_API qs_status qs_batch_autotune(qs_batch *b, int *chosen, double *best_ms);

/* Pin the configuration instead of tuning it: choice in 0..39, numbered as
 * qs_batch_autotune's *chosen (shape + 5 * (grouping + 4 * chunk size index)).
 * Host only; QS_EINVAL outside that range.  A captured graph is re-captured on
 * the next graph run. */
QS_API qs_status qs_batch_set_choice(qs_batch *b, int choice);

/* ---- learned cost model (48 -> 128 -> 128 -> 1, FP32) --------------------- */
/* The paper's planner minimises the number of passes over the state (Sec. IV,
 * Eq. 7); the learned planner (qs_fuse with planner = 1) scores candidate
 * plans by a predicted time per pass instead.  The network itself has no
 * counterpart in the paper: 48 features per pass (qs_plan_block_features) ->
 * 128 -> 128 -> 1, ReLU, FP32, trained by MSE on ln(picoseconds per
 * amplitude) with Adam, all in the library's own kernels. */

#define QS_COST_FEATURES 48

/* Create a model with He-uniform weights from the given seed, on the device
 * (allocates parameters, Adam moments and a minibatch workspace). */
QS_API qs_status qs_costmodel_create(uint64_t seed, void *hip_stream, qs_costmodel **out);
QS_API qs_status qs_costmodel_free(qs_costmodel *m);

/* Copy the parameters (FP32, order W1[128x48], b1[128], W2[128x128], b2[128],
 * W3[1x128], b3[1], row-major) out to host / in from host; 22913 floats. */
QS_API qs_status qs_costmodel_get_params(const qs_costmodel *m, float *host_out);
QS_API qs_status qs_costmodel_set_params(qs_costmodel *m, const float *host_in);

/* One training step on a minibatch of B rows (B <= 1024): X_dev (B x 48 FP32,
 * device), y_dev (B FP32 targets, device): forward, MSE loss, backward
 * (gradients kept on device), Adam update (lr, beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8).  *loss_host gets the minibatch loss before the update if not
 * NULL (then the call synchronises). */
QS_API qs_status qs_costmodel_train_step(qs_costmodel *m, const float *X_dev, const float *y_dev, int B,
                                  float lr, float *loss_host);

/* Forward only: y_dev[b] = model(X_dev[b]) for B rows (device pointers), in
 * chunks of 1024 rows through the model's own activation workspace: calls on
 * one model (predict, train_step, or qs_fuse with planner 1) must not overlap.
 * Async on the model's stream. */
QS_API qs_status qs_costmodel_predict(const qs_costmodel *m, const float *X_dev, float *y_dev, int B);

/* Gradients of the last train step (same layout as the parameters). */
QS_API qs_status qs_costmodel_get_grads(const qs_costmodel *m, float *host_out);

/* Features of every block of a plan (B x 48 FP32, host), for training and
 * for the learned planner; *nblocks gets B (at most cap rows written). */
QS_API qs_status qs_plan_block_features(const qs_plan *plan, float *host_out, int cap, int *nblocks);

/* ---- misc ---------------------------------------------------------------- */

/* Message of the last failed call on this thread ("" if none). */
QS_API const char *qs_last_error(void);

/* Library version string. */
QS_API const char *qs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
