/*
 * qvpu.h - C interface of the qvpu library: batched state-vector execution of parameterised quantum
 * circuits on one AMD MI355X (gfx950), with weighted Pauli-sum expectations and gradients.
 *
 * The operation follows the paper's problem statement (Section 3.2 and Section 4.1): a caller submits a
 * collection of circuits, every circuit is executed from |0...0>, and the result consolidated for each
 * circuit is the expectation value <0|U(theta)^dagger P_t U(theta)|0> of each Pauli string P_t of an
 * observable H = sum_t c_t P_t, plus the weighted sum E = sum_t c_t <P_t> (Eq. 1). Results are returned
 * in the caller's circuit and term order, exactly as if the circuits had run one after another
 * (Section 3.2). Gradients dE/dtheta are produced by the parameter-shift rule the paper uses
 * (Section 4.1, Section 4.2) or by the adjoint method (one forward and one reverse sweep).
 *
 * One process drives one GPU; the whole batch is that GPU's share of the paper's array of virtual QPUs.
 *
 * Conventions
 *   - qubit q is bit q of the amplitude index (qubit 0 is the least significant bit);
 *   - RX/RY/RZ(a) = exp(-i a sigma / 2) with sigma = X/Y/Z; H, X, Y, Z, S = diag(1, i),
 *     T = diag(1, e^{i pi/4}) as in any textbook; CNOT(control q0, target q1); CZ(q0, q1);
 *   - a Pauli string is a pair of masks (xmask, zmask): X where only x is set, Z where only z is set,
 *     Y where both are set; its phase convention is P|b> = i^{popcount(x&z)} (-1)^{popcount(b&z)} |b^x>;
 *   - states are never renormalised; expectations are <psi|P|psi>.
 *
 * Precision
 *   QV_C64:  complex64 amplitudes, FP32 gate arithmetic; expectation reductions and the norm are
 *            accumulated in FP64; the adjoint inner products are summed over a thread's 16 amplitudes in
 *            FP32 and across threads, tiles and circuits in FP64.
 *   QV_C128: complex128 amplitudes, FP64 everywhere.
 *
 * Errors
 *   Every function returns a qv_status. A failing call leaves every object unchanged; qv_last_error()
 *   returns a message describing the most recent failure on the calling thread. Device faults surface
 *   as QV_E_DEVICE at the next call that synchronises. Nothing throws across this interface.
 *
 * Ownership and streams
 *   Input arrays belong to the caller and are copied during the call. Output arrays are allocated by the
 *   caller, either in host memory or in device memory of the context's device (flag *_on_device).
 *   All device work of a context is ordered on the context's stream (the caller's HIP stream; NULL is the
 *   device's default stream). Calls that write host outputs return after the
 *   results are in place; calls that write device outputs return once the work is enqueued.
 *   A context and its batches must be used from one thread at a time.
 */
#ifndef QVPU_H
#define QVPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QV_OK = 0,
    QV_E_INVALID = -1,     /* malformed argument (bad qubit, NULL pointer, non-finite angle, ...) */
    QV_E_OOM = -2,         /* device memory for states would exceed what the device can hold */
    QV_E_DEVICE = -3,      /* a HIP runtime error, with hipGetErrorString in the message */
    QV_E_UNSUPPORTED = -4, /* valid request the library does not implement */
    QV_E_STATE = -5        /* call out of order (e.g. gradient of a batch without parameters) */
} qv_status;

typedef enum { QV_C64 = 0, QV_C128 = 1 } qv_precision;

typedef enum { QV_ADJOINT = 0, QV_PARAM_SHIFT = 1 } qv_grad_method;

typedef enum {
    QV_H = 0, QV_X = 1, QV_Y = 2, QV_Z = 3, QV_S = 4, QV_T = 5,
    QV_RX = 6, QV_RY = 7, QV_RZ = 8, QV_CNOT = 9, QV_CZ = 10
} qv_gate_kind;

/* One gate, 24 bytes. One-qubit gates act on q0 (q1 ignored). CNOT: control q0, target q1. CZ: q0, q1.
 * For RX/RY/RZ, param >= 0 makes the angle theta[param] of the circuit's parameter vector (trainable);
 * param = -1 makes it the fixed value `angle`. Other kinds ignore param and angle (param must be -1). */
typedef struct {
    int32_t kind;
    int32_t q0;
    int32_t q1;
    int32_t param;
    double angle;
} qv_gate;

typedef struct {
    int64_t passes;            /* tile passes executed by the last call (forward + reverse) */
    int64_t launches;          /* kernel launches recorded for the last call */
    int64_t algorithmic_bytes; /* state bytes read + written by the last call's passes and reductions */
    double kernel_ms;          /* device time of the last call, from HIP events on the context stream */
    double norm_err_max;       /* max |<psi|psi> - 1| over the batch after the last forward call */
    int32_t tile_qubits;       /* tile size of the batch's plans (after autotuning) */
    int32_t contig_qubits;     /* qubits 0..contig_qubits-1 are in every tile */
    int32_t passes_per_circuit_max; /* longest plan */
    int32_t fuse_min_run;           /* fused blocks: shortest run of gates made into one block (0: none) */
} qv_stats;

/* Kernels named in launch records. */
typedef enum {
    QV_K_INIT = 0,          /* psi = |0...0> */
    QV_K_TILE = 1,          /* LDS tile pass, forward */
    QV_K_TILE_ADJ = 2,      /* LDS tile pass, adjoint reverse sweep (psi and lambda) */
    QV_K_STRIDE = 3,        /* one gate straight from global memory, forward */
    QV_K_STRIDE_ADJ = 4,    /* one gate straight from global memory, adjoint */
    QV_K_EXPECT = 5,        /* Pauli-string expectation partial sums */
    QV_K_FINALIZE = 6,      /* term values and energies from partial sums */
    QV_K_LAMBDA = 7,        /* adjoint seed lambda = w H psi */
    QV_K_GRAD_REDUCE = 8,   /* adjoint gradient from partial sums */
    QV_K_SHIFT_COMBINE = 9, /* parameter-shift gradient from shifted energies */
    QV_K_RTILE = 10,        /* register-tiled LDS pass, forward */
    QV_K_RTILE_ADJ = 11,    /* register-tiled LDS pass, adjoint reverse sweep */
    QV_K_MATRICES = 12,     /* 2x2 matrices of every gate at the current parameters */
    QV_K_RTILE_PERSIST = 13,     /* all forward register-tiled passes in one persistent launch */
    QV_K_RTILE_ADJ_PERSIST = 14, /* all adjoint register-tiled passes in one persistent launch */
    QV_K_FUSE = 15,              /* fused 4-qubit block matrices (products of their gates) */
    QV_K_PROBS = 16,             /* output distributions |psi|^2; with a target, divergence partials and weights */
    QV_K_DIAG_SEED = 17,         /* adjoint seed lambda = u diag(w) psi of the divergence weights */
    QV_K_DIAG_EXPECT = 18,       /* <psi|diag(w)|psi> partial sums (parameter-shift variants) */
    QV_K_SEGMENT_SUM = 19,       /* per-circuit sums of partials in a fixed order */
    QV_K_SAMPLE = 20,            /* shots from the output distributions and their bit-string counts */
    QV_K_RTILE_GEN = 21,         /* register-tiled pass, forward, kernel generated for the pass */
    QV_K_RTILE_ADJ_GEN = 22,     /* register-tiled pass, adjoint, kernel generated for the pass */
    QV_K_RTILE_LAM = 23          /* register-tiled pass, adjoint, tiles where psi is zero: lambda alone */
} qv_kernel_id;

/* One kernel launch of the last call, timed with a HIP event pair on the context's stream. bytes is the
 * algorithmic state traffic of the launch: for a gate pass 2 * (state bytes) per circuit (read + write),
 * 4 * for an adjoint pass (psi and lambda), one state read per term group for expectations. */
typedef struct {
    int32_t kernel;  /* qv_kernel_id */
    int32_t level;   /* pass level within the call, -1 for other kernels */
    int64_t bytes;   /* algorithmic state bytes the launch reads and writes */
    double ms;       /* duration between HIP events recorded around the launch on the context stream */
    double flops;    /* algorithmic flops of gate passes (per amplitude: 14 for H/RX/RY, 6 for S/T/RZ, 0 for
                        X/Y/Z/CNOT/CZ; adjoint: twice that plus 4 per trainable gate); 0 for other kernels */
} qv_launch_rec;

typedef struct qv_ctx_s *qv_ctx;
typedef struct qv_batch_s *qv_batch;

/* Creates a context on HIP device `device`. hip_stream is the hipStream_t all work is ordered on (NULL:
 * the device's default stream). options_json is NULL or a flat JSON object; recognised keys:
 *   "n-virtual-qpus" : int >= 1   how many circuits may be in flight at once (default: all); results do
 *                                 not depend on it (the paper's option of the same name, Section 3.2);
 *   "engine"         : "tiled" (default: LDS tile passes whose gates run on register-resident segments),
 *                      "lds" (LDS tile passes, one gate at a time in LDS) or "stride" (one global-memory
 *                      pass per gate);
 *   "tile_qubits"    : int 6..14 or "auto" (default "auto": the autotuner's choice);
 *   "launch"         : "levels" (one launch per pass level, default) or "persistent" (all levels of a
 *                      sweep in one launch: resident workgroups take tiles from a queue in level order and
 *                      wait until their circuit's earlier passes are complete; a wait that runs out makes
 *                      every later item skip its work and the call return QV_E_DEVICE). Sweeps whose passes
 *                      are not all register-tiled, or whose tiles do not fit one persistent workgroup's
 *                      LDS, run one launch per level;
 *   "persist_chunk"  : 0..64, consecutive queue items a persistent workgroup claims at once (default 0:
 *                      4 forward, 8 reverse, fewer when the sweep has few items); where consecutive
 *                      items are tiles of one circuit's pass, each prefetches the next;
 *   "wait_ms"        : 0..600000, longest dependency wait of a persistent launch (default 4000);
 *   "wait_extra"     : int >= 0 (default 0), added to every dependency count of a persistent launch so that
 *                      those waits cannot be met: for testing the time-out path only;
 *   "fusion"         : "off" (default), "on" (runs of >= 6 gates), a minimum run length, or "auto"
 *                      (the autotuner times runs of >= 4, 6, 8 and no fused blocks; 8 until it has run):
 *                      within a register segment, consecutive gates acting only on its 4 register qubits
 *                      are multiplied into one 16x16 block (complex64: applied on MFMA in forward passes);
 *   "fold_cnots"     : "on" (default) or "off": runs of CNOTs at either end of a register segment
 *                      permute the tile's amplitudes, so they are folded into the segment's LDS load and
 *                      store addresses instead of running as ops (same results, no arithmetic);
 *   "specialize"     : "off" (default), "adjoint", "on" or "auto": every register-tiled level whose
 *                      circuits all run one plan pass runs a kernel generated for that pass (its ops as
 *                      straight-line code, compiled with hipRTC on the first call that needs it, by
 *                      QV_GEN_THREADS threads, default one per host CPU up to 16; code
 *                      objects are kept in the directory named by QV_GEN_CACHE, default
 *                      $HOME/.cache/qvpu_gen), in reverse (adjoint) sweeps only, in both directions, or
 *                      ("auto") in the levels of either direction where it measured faster: the first call
 *                      that runs sweeps of a direction times two of them with each kind of kernel. A
 *                      generated forward pass applies a fused block's gates one by one. Same results as the
 *                      general kernels, up to floating-point contraction; QV_E_DEVICE if the compilation
 *                      fails;
 *   "adjoint_inner"  : "f32" (default) or "f64" (needs "specialize" "adjoint", "on" or "auto"): in complex64
 *                      adjoint sweeps a thread's Im <lambda| G |psi> products are summed in FP32 before the
 *                      FP64 wave, tile and circuit sums ("f32"), or every product of two FP32 amplitude
 *                      components is formed exactly in FP64 and summed in FP64 from there ("f64");
 *   "autotune"       : "off", "cached" (default: reuse a choice stored by an earlier search) or
 *                      "search" (on the first forward call, time one forward pass for each candidate tile
 *                      size, contiguous-run length and, under "fusion": "auto", fused-block minimum run,
 *                      and keep the fastest; stored as tile qubits, contiguous qubits, block width (4) and
 *                      minimum run in the text file named by QV_TUNE_CACHE, default
 *                      $HOME/.cache/qvpu_tune.txt). "tile_qubits" or "contig_qubits" given explicitly
 *                      take those out of the search;
 *   "graph"          : true (default) to capture each call's launches in a hipGraph and replay it;
 *   "contig_qubits"  : 1..6: qubits 0..k-1 are in every tile, so tiles move in runs of 2^k amplitudes
 *                      (default 4 for complex64, 3 for complex128: 128-byte runs);
 *   "launch_events"  : true to time every launch with a HIP event pair (only with "graph": false);
 *                      the records of the last call are read with qv_batch_launch_log. */
qv_status qv_ctx_create(int32_t device, void *hip_stream, const char *options_json, qv_ctx *out);

/* Points the context at another hipStream_t (NULL: the device's default stream). */
qv_status qv_ctx_set_stream(qv_ctx ctx, void *hip_stream);

/* Releases the caller's context. Batches created on it keep it alive: the context is freed when it has
 * been destroyed and its last batch too, so batches and their context may be destroyed in either order. */
qv_status qv_ctx_destroy(qv_ctx ctx);

/* Submits a batch of circuits and its observable (Section 3.2: a vector of circuits executed on one
 * buffer; Section 4.1: a Hamiltonian given as a weighted sum of Pauli strings).
 *   n_circuits          B >= 1
 *   n_qubits[B]         1 <= n <= 34
 *   gate_offsets[B+1]   circuit b owns gates[gate_offsets[b] .. gate_offsets[b+1]), offsets monotone, [0] = 0
 *   n_params[B]         parameters of each circuit; every gate param must be < n_params[b]
 *   params_shared       nonzero: all circuits read one vector theta[n_params[0]] (all n_params equal);
 *                       zero: circuit b reads its own slice, concatenated in circuit order
 *   term_offsets        obs_shared nonzero: [2], every circuit uses terms [term_offsets[0], term_offsets[1]);
 *                       obs_shared zero: [B+1], circuit b uses terms [term_offsets[b], term_offsets[b+1])
 *   xmask, zmask, coeff one entry per term; masks must be < 2^n of the circuits that use them
 *   precision           QV_C64 or QV_C128
 * On success *out receives the batch. Nothing is executed until qv_batch_expectations or
 * qv_batch_gradient is called. Returns QV_E_OOM when the states (and, for gradients, one extra state
 * per circuit) cannot fit on the device. */
qv_status qv_batch_create(qv_ctx ctx, int32_t n_circuits, const int32_t *n_qubits, const int64_t *gate_offsets,
                          const qv_gate *gates, const int32_t *n_params, int32_t params_shared,
                          const int64_t *term_offsets, const uint64_t *xmask, const uint64_t *zmask,
                          const double *coeff, int32_t obs_shared, qv_precision precision, qv_batch *out);

/* Runs every check qv_batch_create performs, without a context or a device. Returns the status and sets
 * the message qv_batch_create would set. */
qv_status qv_validate_batch(int32_t n_circuits, const int32_t *n_qubits, const int64_t *gate_offsets,
                            const qv_gate *gates, const int32_t *n_params, int32_t params_shared,
                            const int64_t *term_offsets, const uint64_t *xmask, const uint64_t *zmask,
                            const double *coeff, int32_t obs_shared, qv_precision precision);

/* Sets the parameter vector (Section 4.1 and Section 4.2: each iteration of the variational loop runs the
 * same circuits again with new angles): n_params[0] doubles when shared, else sum of n_params. theta is a
 * host pointer, or a device pointer when theta_on_device is nonzero. Host values are checked to be finite. */
qv_status qv_batch_set_params(qv_batch batch, const double *theta, int32_t theta_on_device);

/* Executes every circuit from |0...0> (Section 3.2: the whole circuit vector on one buffer) and writes
 * energies[B] (E_b = sum_t c_t <P_t>, Eq. 1) and, when
 * term_values is not NULL, the expectation of every term in term order: for a shared observable
 * B*T values, circuit-major; otherwise sum_b T_b values in the order of the term arrays.
 * The final states stay on the device for a following adjoint gradient. */
qv_status qv_batch_expectations(qv_batch batch, double *energies, double *term_values, int32_t out_on_device);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same computation and outputs as qv_batch_expectations, with no
 * hipMalloc, hipFree or other allocating call. The expectation partial sums live in a static device array
 * of the library (8 MiB, at most 2^20 partial sums, held by every device the library runs on until the
 * process ends); a batch needing more (about 2^20 / ceil(2^n / 2^14) x-mask groups of up to 8 terms per
 * n-qubit circuit) gets QV_E_INVALID and nothing runs. Every call on one device shares that array, so
 * calls that overlap on one device (several streams or threads) race; calls in one stream do not. The
 * work is launched eagerly on the context's stream (no graph), and the batch must already have its launch
 * configuration: a batch whose autotuner has still to choose tiles (context option "autotune" "search",
 * or a stored choice that differs) gets QV_E_STATE until one qv_batch_expectations call has run. Outputs
 * as for qv_batch_expectations (host outputs synchronise). */
qv_status qv_batch_expectations_static(qv_batch batch, double *energies, double *term_values, int32_t out_on_device);

/* Gradient of L = sum_b w_b E_b with w = upstream[B] (NULL: all ones). grad receives n_params[0] values
 * when parameters are shared (summed over circuits), else sum n_params values (circuit b's own slice).
 * QV_ADJOINT runs the forward pass, seeds lambda_b = w_b H psi_b and sweeps the gates backwards,
 * accumulating Im <lambda|G_k|psi> for every trainable gate exp(-i a G_k / 2) in FP64.
 * QV_PARAM_SHIFT evaluates, for every trainable gate occurrence, the circuit with that angle moved by
 * +pi/2 and -pi/2 and adds w_b (E+ - E-)/2 (the rule the paper applies in Section 4.1 and 4.2); a
 * parameter that drives several gates receives the sum over its gates. When energies is not NULL the
 * forward energies are written too. upstream, grad and energies are device pointers when on_device. */
qv_status qv_batch_gradient(qv_batch batch, qv_grad_method method, const double *upstream, double *grad,
                            double *energies, int32_t on_device);

/* Output distributions (Section 4.2: running a circuit yields a probability for each of the 2^n bit
 * strings): executes every circuit from |0...0> and writes P_b(x) = |<x|U_b|0>|^2 in FP64 for every
 * circuit b and bit string x (x read as an amplitude index, qubit q = bit q). probs holds
 * sum_b 2^{n_b} doubles, circuit b's distribution starting at sum_{b' < b} 2^{n_b'}; caller-owned, a
 * device pointer when out_on_device. The final states stay on the device. */
qv_status qv_batch_probabilities(qv_batch batch, double *probs, int32_t out_on_device);

/* Jensen-Shannon divergence of Eq. 3 (the data-driven circuit-learning loss of Section 4.2) between a
 * target distribution P_b and each circuit's output distribution Q_b,
 *     JS_b = 1/2 sum_x [ P_b(x) log(P_b(x)/M(x)) + Q_b(x) log(Q_b(x)/M(x)) ],  M = (P_b + Q_b)/2,
 * natural logarithm, 0 log 0 = 0, and the gradient of L = sum_b u_b JS_b with u = upstream[B] (NULL:
 * all ones). target has the layout of qv_batch_probabilities' output; host targets are checked to be
 * finite and non-negative (device targets are the caller's responsibility; they are not renormalised).
 * dJS_b/dQ_b(x) = log(Q_b(x)/M(x))/2 (weight 0 where Q_b(x) = 0) turns the gradient into that of the
 * diagonal observable diag(u_b dJS_b/dQ_b) at fixed weights: QV_ADJOINT seeds lambda_b with it and sweeps
 * the gates backwards; QV_PARAM_SHIFT evaluates that observable on the +-pi/2 variants of every trainable
 * gate. js[B] (may be NULL) receives the divergences; grad as in qv_batch_gradient, or NULL for the
 * divergences alone (one forward pass; method is then ignored, and the final states stay for a following
 * QV_ADJOINT call, which does not repeat the forward pass). target, upstream, js and grad are device
 * pointers when on_device. Buffers of sum_b 2^{n_b} doubles (target copy, weights)
 * are allocated on first use and kept with the batch. */
qv_status qv_batch_js_gradient(qv_batch batch, qv_grad_method method, const double *target, const double *upstream,
                               double *js, double *grad, int32_t on_device);

/* Shots and bit-string counts (Section 3.1: a circuit's execution result is the table of observed bit
 * strings and how often each occurred; Section 4.2: the circuit-learning application consumes these
 * counts). Runs the forward pass at the current parameters, forms each circuit's output distribution
 * Q_b(x) = |psi_b[x]|^2 (FP64, as qv_batch_probabilities) and its running sum C_b(x) = Q_b(0) + ... + Q_b(x)
 * in bit-string order (FP64, fixed summation order: blocks of 4096 bit strings summed left to right, then
 * block offsets), and draws `shots` shots per circuit by inverse transform sampling: shot j of circuit b
 * takes u = uniforms[b * shots + j] and is the first x with C_b(x) > u * C_b(2^{n_b} - 1). The uniforms
 * are the caller's (any generator; host values must lie in [0, 1), device values outside it are clamped
 * into it), so a draw is reproducible and can be checked against another implementation of the same rule.
 * Outputs, each a device pointer when on_device, else host:
 *   samples[B * shots]        (may be NULL) the bit string of every shot, in uniform order;
 *   bitstrings, counts[B * shots] circuit b's distinct drawn bit strings in increasing order, from index
 *                             b * shots on, and how many shots drew each (entries past n_distinct[b] are
 *                             unspecified);
 *   n_distinct[B]             how many distinct bit strings circuit b drew.
 * bitstrings, counts and n_distinct are all given or all NULL; samples or they must be given.
 * 1 <= shots <= 2^31 - 1. Buffers (the running sums, a 32-bit count per amplitude, the shot arrays) are
 * allocated on first use and kept with the batch. QV_E_INVALID for bad arguments (nothing runs). */
qv_status qv_batch_sample(qv_batch batch, int64_t shots, const double *uniforms, int64_t *samples,
                          uint64_t *bitstrings, int64_t *counts, int64_t *n_distinct, int32_t on_device);

/* Copies the final state of circuit b after the last forward pass (the state-vector simulation behind
 * every result of Section 4): 2^n complex numbers, interleaved (re, im), float for QV_C64 and double for
 * QV_C128. */
qv_status qv_batch_state(qv_batch batch, int32_t circuit, void *out, int32_t out_on_device);

/* Counts and timing of the last call (passes, launches, algorithmic bytes, device time: the quantities
 * behind a timing like those of Section 4), the norm check and the batch's tuned plan parameters, written
 * to *out. QV_E_INVALID when batch or out is NULL. */
qv_status qv_batch_stats(qv_batch batch, qv_stats *out);

/* Launch records of the qv_batch_expectations / qv_batch_gradient calls made since the records were
 * last read, for a context created with "launch_events": true and "graph": false. Writes the number of
 * pending records to *n_records and at most max_records of them to out (waiting for their work to
 * finish); when every pending record fits in out they are consumed, otherwise they stay pending (call
 * with max_records = 0 to query the count). */
qv_status qv_batch_launch_log(qv_batch batch, qv_launch_rec *out, int32_t max_records, int32_t *n_records);

/* Waits for the batch's work on its context's stream, frees its device memory and graphs, and drops its
 * reference to the context. */
qv_status qv_batch_destroy(qv_batch batch);

/* Message of the last failure on the calling thread ("" if none); valid until the next call. */
const char *qv_last_error(void);

/* One pass of a circuit's execution plan (see qv_plan_circuit). */
typedef struct {
    uint64_t local_mask;  /* qubits held in the pass's tile */
    int32_t qubits;       /* tile size: popcount(local_mask) */
    int32_t n_ops;        /* gates the pass applies */
    int32_t n_trainable;  /* of them trainable */
    int32_t n_segments;   /* register segments (0: gates run one at a time in LDS or from HBM) */
    int32_t first_gate;   /* circuit index of the pass's first gate in execution order */
    int32_t contiguous_low; /* qubits 0..contiguous_low-1 are all local (length of contiguous runs) */
    int32_t n_fused;      /* fused blocks among the pass's gates */
    int32_t n_folded;     /* CNOTs folded into register-segment LDS addressing ("tiled" engine) */
    uint64_t zero_mask;   /* qubits outside the tile that no earlier pass touches (bits below n_qubits):
                             still |0>, so tiles with one of them at 1 hold zeros through the pass */
} qv_pass_info;

/* Plans one circuit without a device, as qv_batch_create would for a batch with the given engine
 * (0 "tiled", 1 "lds", 2 "stride"), tile size (0: the default) and fusion minimum run length (0: no
 * fused blocks; only the "tiled" engine fuses): each pass is one read and one write
 * of the state. Writes the pass count to *n_passes and the first max_passes passes to out; when order
 * is not NULL it receives the n_gates gate indices in execution order (passes in turn, each pass's
 * gates in the order the kernel applies them). Host only; for inspecting and testing the planner. */
qv_status qv_plan_circuit(int32_t n_qubits, int64_t n_gates, const qv_gate *gates, int32_t tile_qubits,
                          qv_precision precision, int32_t engine, int32_t fuse_min, int32_t max_passes,
                          qv_pass_info *out, int32_t *n_passes, int32_t *order);

/* Library version string. */
const char *qv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QVPU_H */
