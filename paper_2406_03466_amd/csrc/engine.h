// Device-side data layout shared by the host planner (qvpu_api.cpp) and the HIP kernels (kernels.hip).
//
// A batch holds B circuits. Each circuit's state is a contiguous array of 2^n interleaved (re, im)
// amplitudes inside one pool, qubit q being bit q of the index. Circuits that share a gate structure
// share one plan: a list of passes. A pass gathers a tile of 2^t amplitudes (the t "local" qubits vary,
// the other n - t qubits are fixed per tile) into LDS, applies a run of gates whose qubits are all local,
// and writes the tile back. All passes at the same position of their circuits' plans form a level;
// one kernel launch runs a level for every circuit.
#pragma once
#include <stdint.h>

#include "qvpu.h"

namespace qv {

constexpr int kMaxTileQubits = 14;   // 2^14 complex64 = 128 KiB of LDS
constexpr int kBlock = 256;          // threads per workgroup for every kernel
constexpr int kMaxGroupTerms = 8;    // Pauli terms evaluated together by one expectation item
constexpr int kExpChunkLog2 = 14;    // amplitude pairs per expectation workgroup (16384; 4096 measured 15-17 % slower)
constexpr int kStrideGroupsPerBlock = 1024;
// Non-temporal hints for data that cannot stay in the L2 and last-level caches (4 MB per XCD, 256 MB)
// until it is read again. A stride level makes one pass over every state of the batch, so its accesses
// stream when the batch's states total kStreamBatchBytes; an expectation reads one state once per x-mask
// group, so its reads stream when the largest state has kStreamStateBytes. Smaller data is re-read from
// the caches and keeps the default policy.
constexpr int64_t kStreamBatchBytes = (int64_t)256 << 20;
constexpr int64_t kStreamStateBytes = (int64_t)64 << 20;
constexpr int kRtileThreads = 512;  // register-tiled passes: workgroup size
constexpr int kRegBitsC64 = 4;       // 16 complex64 amplitudes per thread (2^13-amplitude tiles)
constexpr int kRegBitsC128 = 3;      // 8 complex128 amplitudes per thread (2^12-amplitude tiles)

enum OpFlags : uint8_t { OP_TRAIN = 1 };

// Register-segment op codes, stored in DevOp::flags above the OP_TRAIN bit: one code per gate class and
// register bit(s), so a tile kernel picks an op's code path with one switch.
enum OpCode : int {
    OC_NONE = 0,        // not in a register segment (op-by-op LDS passes, stride passes)
    OC_RY = 1,          // + register bit k (1..4): [[c, -s], [s, c]]
    OC_DIAG = 5,        // + register bit k (5..8): RZ, Z, S, T on a register qubit
    OC_DIAG_T = 9,      // RZ, Z, S, T on a thread qubit
    OC_GEN = 10,        // + register bit k (10..13): H, X, Y, RX (dense 2x2)
    OC_CNOT_RR = 14,    // + 4 * control bit + target bit (14..29): a register permutation
    OC_CNOT_TR = 30,    // + target bit (30..33): control on a thread qubit
    OC_CZ = 34,
    OC_FUSED = 35,      // fused-block marker
};
constexpr int kOpCodeShift = 1;

// One gate inside a pass, with its qubits translated to tile-local bit positions.
struct DevOp {
    int32_t gate;        // gate index within its circuit (angle and parameter are read per circuit)
    uint8_t kind;        // qv_gate_kind
    uint8_t p0, p1;      // local positions of q0 / q1
    uint8_t flags;       // OP_TRAIN when the gate's angle is a trainable parameter
    int32_t train_slot;  // position among the pass's trainable gates (adjoint partial sums), else -1
    int8_t k0, k1;       // register-tiled passes: register bit holding p0 / p1, -1 when it is a thread bit
    int16_t pad;
};
static_assert(sizeof(DevOp) == 16, "DevOp layout");

// Register-tiled passes run their ops in segments. Within a segment every thread holds 2^RB amplitudes of
// the LDS tile in registers: register bit k is local position rpos[k], thread bit m is local position
// tpos[m]. Every op of a segment that mixes amplitude pairs has its target among rpos, so it runs without
// leaving registers; diagonal ops and CNOT controls may sit on thread bits.
struct DevSeg {
    int32_t op_begin;
    int32_t n_ops;
    int8_t rpos[8];
    int8_t tpos[16];
    // CNOT runs folded into the segment's LDS addressing, in program order; entry k (byte k) is the local
    // control position | target position << 4, unused entries 0xFF. `lead` runs before the segment's ops,
    // `trail` after them.
    uint64_t lead;
    uint64_t trail;
    int8_t n_lead, n_trail;
    int8_t pad[2];
    // images of the register bits (1 << rpos[k]) under the inverse of the leading run (rimg_lead) and under
    // the trailing run (rimg_trail)
    uint16_t rimg_lead[4], rimg_trail[4];
    int32_t pad2;
};

struct DevPass {
    uint64_t local_mask;  // qubits of the tile
    int32_t t;            // number of local qubits
    int32_t op_begin;     // into the op array
    int32_t n_ops;
    int32_t n_train;      // trainable ops in the pass
    int32_t stride;       // 1: stride pass (one gate straight from global memory), 0: LDS tile pass
    int32_t pad;          // lowc: local positions 0..lowc-1 are qubits 0..lowc-1
    int32_t seg_begin;    // register-tiled passes: segments [seg_begin, seg_begin + n_seg)
    int32_t n_seg;        // 0: the pass runs op by op in LDS
    int8_t lq[16];        // local position -> qubit, ascending
    // A circuit's first pass, undone last by the adjoint, needs no work below its first trainable op: the
    // reverse sweep stops there. first_train: index (in the op array) of that op; adj_last_nseg: segments,
    // counted from the pass's end, that hold it or later ops (0: the pass has no trainable op).
    int32_t first_train;
    int32_t adj_last_nseg;
    // Qubits outside the tile that no earlier pass of the circuit touches: they are still |0>, so a tile with
    // one of them at 1 holds zeros throughout the pass.
    uint64_t zero_mask;
};

struct DevCirc {
    int64_t state_off;    // amplitude offset of this circuit's state in the pool
    int64_t gate_off;     // offset of its gate records
    int64_t param_base;   // offset of its parameters in theta
    int32_t n;            // qubits
    int32_t shift_gate;   // parameter-shift variant: index of the gate whose angle is moved, -1 none
    double shift;         // the move (+pi/2 or -pi/2)
    int32_t base_circ;    // the batch circuit this entry evaluates (variants point at their base)
    int32_t pad;
    int64_t op_base;      // first op of the circuit's plan; matrix of op o is mats[mat_off + o - op_base]
    int64_t mat_off;      // this circuit's range of the per-op matrix table
    int64_t fused_off;    // this circuit's first fused block in the fused-matrix table
    int64_t fused_ops;    // offset of its plan's fused-block marker list
};

constexpr int kFusedKind = 100;      // op kind of a fused-block marker (its gates follow it)
constexpr int kFusedFloats = 1024;   // one fused 4-qubit block: the 32x32 real form of a 16x16 complex matrix

// One (circuit, pass) of a level launch; blocks [first_block, next segment's first_block) run it.
struct Seg {
    int64_t first_block;
    int64_t partial_base; // adjoint: base slot of this (circuit, pass) in the partial-sum array
    int32_t circ;
    int32_t pass;
    int32_t first;        // 1: first pass of the circuit -- the tile starts as |0...0> instead of a load
    int32_t last;         // adjoint: 1 for the circuit's first pass (undone last) -- psi and lambda are not
                          // needed afterwards, so the tile is not written back
    int64_t wait;         // persistent launch: tiles of this circuit that must be finished first
    int64_t tile_off;     // tile number of the segment's first block (a pass's tiles may span two launches)
};

// Expectation work: one Pauli x-mask group of one circuit. Blocks [first_block, ...) cover its chunks.
struct DevGroup {
    uint64_t xmask;
    int64_t first_block;
    int64_t partial_base; // partials[partial_base + chunk * n_terms + j]
    int32_t circ;
    int32_t n_terms;
    int32_t term_begin;   // into DevTerm array
    int32_t chunk_log2;   // pairs (or amplitudes when xmask == 0) per block
};

struct DevTerm {
    uint64_t zmask;
    int32_t ny;           // popcount(x & z) mod 4
    int32_t pad;
};

// Where the partial sums of one output value live: sum over c < count of partials[base + c * stride].
struct PartialRef {
    int64_t base;
    int32_t count;
    int32_t stride;
};

// Term of an observable, as used to seed the adjoint vector lambda = w H psi.
struct DevObsTerm {
    uint64_t xmask, zmask;
    double coeff;
    int32_t ny;
    int32_t pad;
};

// Launch parameters for one level of tile passes.
struct LevelArgs {
    const Seg *segs;
    int32_t n_segs;
    int32_t lds_t;        // largest tile of the level (LDS sizing)
    int64_t n_blocks;
    const DevPass *passes;
    const DevOp *ops;
    const DevSeg *rsegs;  // register segments of the passes
    int32_t max_train;    // largest n_train of the level's passes (LDS for the adjoint partial sums)
    int32_t tab_bits;     // largest t - lowc of the level's passes: the LDS run-offset table has 2^tab_bits entries
    const DevCirc *circs;
    const qv_gate *gates;
    const double *theta;
    const void *mats;     // per circuit and plan op: its 2x2 matrix (8 reals, R precision), built from theta
    const void *smats;    // per circuit of the launch: the matrix of its shifted gate (parameter-shift variants)
    const float *fmats;   // fused blocks: kFusedFloats per block, in the order the MFMA A operand reads them
    void *psi;
    void *lam;
    double *partials;
    int32_t chunk;        // register-tiled levels: consecutive tiles per workgroup (set by the launcher)
    int32_t stream;       // 1: the batch's states total at least kStreamBatchBytes (stride passes use
                          // non-temporal accesses)
};

// One persistent launch runs every level of a direction: workgroups claim items (level blocks in level
// order) from a queue; an item waits until its circuit's earlier passes are complete.
struct PersistLevel {
    int64_t first_item;   // items [first_item, next level's first_item) are this level's blocks
    int64_t seg_off;
    int32_t n_segs;
    int32_t pad;
};

struct PersistArgs {
    LevelArgs base;              // segs/n_segs are taken per level; lds_t, tab_bits, max_train are maxima
    const PersistLevel *levels;
    int32_t n_levels;
    int32_t chunk;               // consecutive items a workgroup claims at once (set by the launcher)
    int64_t n_items;
    unsigned long long *head;    // queue head, zero before the launch
    unsigned long long *done;    // finished tiles per circuit, zero before the launch
    int32_t *error;              // set to 1 if a wait runs out; later items then skip their work
    int64_t wait_ticks;          // longest wait, in ticks of the device's constant-rate wall clock
    int64_t wait_extra;          // added to every nonzero dependency count (0; a test sets it to force time-outs)
};

// Gate matrices of a batch: for every gate record, its 2x2 complex matrix at the current parameters.
struct MatArgs {
    const qv_gate *gates;
    const int32_t *gate_circ;   // circuit of each matrix-table entry
    const DevOp *ops;           // plans: entry gate_off + j of the table is the circuit's op op_base + j
    const DevCirc *circs;
    const double *theta;
    void *mats;
    int64_t n_gates;
};

// Shifted-gate matrices of a set of parameter-shift variants: entry c is the 2x2 matrix of circuit c's
// shifted gate at its moved angle (circuits without a shift are skipped).
struct ShiftMatArgs {
    const DevCirc *circs;
    const qv_gate *gates;
    const double *theta;
    void *smats;
    int64_t n_circ;
};

// One circuit's final state made textbook: the kernels build RZ(a) as e^{ia/2} RZ(a), so the state is
// multiplied by exp(-i/2 sum of the circuit's RZ angles) on its way out.
struct StatePhaseArgs {
    const qv_gate *gates;   // the circuit's gate records
    const double *theta;    // the circuit's parameters (gate.param indexes them)
    int64_t n_gates;
    const void *src;        // amplitudes to copy (a range of the circuit's state)
    void *dst;              // device destination of the scaled copy
    int64_t n_amps;
    double *phase;          // two doubles of device memory: cos and sin of the restoring phase
};

struct ExpArgs {
    const DevGroup *groups;
    int32_t n_groups;
    int32_t stream;       // 1: the largest state has at least kStreamStateBytes (non-temporal reads)
    int64_t n_blocks;
    const DevTerm *terms;
    const DevCirc *circs;
    const void *psi;
    double *partials;
};

struct FinalizeArgs {
    int32_t n_circ;
    int64_t n_terms;             // output terms of all circuits (tv_begin[n_circ])
    const int64_t *tv_begin;     // [n_circ + 1] output term ranges
    const PartialRef *term_refs; // per output term
    const double *coeff;         // per output term
    const PartialRef *norm_refs; // per circuit
    const double *partials;      // expectation partial sums
    double *term_values;         // out
    double *energies;            // out
    double *norms;               // out (may be NULL)
};

struct LambdaArgs {
    const DevCirc *circs;
    int32_t n_circ;
    const int64_t *first_block;  // [n_circ + 1] block prefix (4096 amplitudes per block)
    const int64_t *obs_begin;    // [n_circ + 1] ranges into obs
    const DevObsTerm *obs;
    const double *upstream;      // [B] or NULL (weights 1)
    const void *psi;
    void *lam;
    int64_t n_blocks;
};

struct GradReduceArgs {
    int32_t n_out;
    const int64_t *ref_begin;    // [n_out + 1]
    const PartialRef *refs;
    const double *partials;
    double *grad;
};

// Parameter-shift combination: grad[g] = sum over its occurrences of w_b (E+ - E-) / 2.
struct ShiftCombineArgs {
    int32_t n_out;
    const int64_t *occ_begin;    // [n_out + 1]
    const int32_t *occ_plus;     // variant index of E+
    const int32_t *occ_minus;    // variant index of E-
    const int32_t *occ_circ;     // batch circuit of the occurrence (for the upstream weight)
    const double *energies;      // variant energies
    const double *upstream;      // [B] or NULL
    double *grad;
};

// Launchers (kernels.hip). All return hipSuccess or the launch error.
int launch_level(const LevelArgs &a, int precision, int adjoint, void *stream);
int launch_stride_level(const LevelArgs &a, int precision, int adjoint, void *stream);
int launch_rlevel(const LevelArgs &a, int precision, int adjoint, void *stream);
// The same level through a generated kernel of its pass (fn: a hipFunction_t; its LDS is static).
int launch_rlevel_gen(const LevelArgs &a, int adjoint, void *fn, void *stream);
int launch_persistent(const PersistArgs &a, int precision, int adjoint, void *stream);
int persistent_blocks(int precision, int adjoint, int lds_t, int tab_bits, int max_train, int *blocks);
// 1 when one persistent launch can hold the largest tile of the given passes in LDS.
int persistent_fits(int precision, int adjoint, int lds_t, int tab_bits, int max_train);
int launch_zero_u64(unsigned long long *p, int64_t n, void *stream);
int launch_init_states(void *psi, const DevCirc *circs, const int64_t *first_block, int32_t n_circ,
                       int64_t n_blocks, int precision, void *stream);
int launch_expectation(const ExpArgs &a, int precision, void *stream);
int launch_finalize(const FinalizeArgs &a, void *stream);
int launch_lambda(const LambdaArgs &a, int precision, void *stream);
int launch_grad_reduce(const GradReduceArgs &a, void *stream);
int launch_shift_combine(const ShiftCombineArgs &a, void *stream);

// Probability path (Section 4.2). Blocks of 4096 amplitudes; first_block is the per-circuit block prefix.
struct ProbArgs {
    const DevCirc *circs;
    int32_t n_circ;
    const int64_t *first_block;  // [n_circ + 1]
    int64_t n_blocks;
    const void *psi;
    const double *target;        // [pool amplitudes] target distributions, or NULL (no divergence)
    double *probs;               // [pool amplitudes] |psi|^2, or NULL
    double *w;                   // [pool amplitudes] dJS/dP_theta, written when target is given
    double *partials;            // [n_blocks] Jensen-Shannon partial sums (before the factor 1/2)
};

// Expectations of, or the adjoint seed for, the diagonal observable diag(w): w is indexed through the base
// circuit of each entry (a parameter-shift variant uses its base circuit's weights).
struct DiagArgs {
    const DevCirc *circs;
    int32_t n_circ;
    const int64_t *first_block;  // [n_circ + 1]
    int64_t n_blocks;
    const DevCirc *base_circs;   // the batch's circuits (state offsets of w)
    const double *w;
    const double *upstream;      // seed only: [B] weights, or NULL (1)
    const void *psi;
    void *lam;                   // seed only
    double *partials;            // expectation only: [n_blocks]
};

// out[c] = scale * sum of partials[first_block[c] .. first_block[c + 1]), fixed summation order.
struct SegSumArgs {
    const int64_t *first_block;
    const double *partials;
    double *out;
    int32_t n;
    double scale;
};

// Shots from the output distributions. The distribution of circuit c (probs, pool layout) is split into the
// probability path's blocks of kSampleBlock amplitudes (first_block as for ProbArgs). C(x), the running sum
// of the distribution in bit-string order, is held as a block offset (sum of the earlier blocks) plus a
// prefix within the block; a shot with uniform u is the first x with C(x) > u * C(last).
constexpr int kSampleBlock = 4096;

struct SampleArgs {
    const DevCirc *circs;
    int32_t n_circ;
    const int64_t *first_block;  // [n_circ + 1]
    int64_t n_blocks;
    const double *probs;         // [pool amplitudes] the distributions
    double *local;               // [pool amplitudes] prefix sums within each block
    double *bsum;                // [n_blocks] block totals
    double *boff;                // [n_blocks] sums of the circuit's earlier blocks
    double *total;               // [n_circ] C(last)
    int64_t shots;               // per circuit
    const double *uniforms;      // [n_circ * shots]
    int64_t *samples;            // [n_circ * shots] bit string of every shot
    uint32_t *hist;              // [pool amplitudes] shots per bit string (zero before the draw)
    int64_t *nnz;                // [n_blocks] distinct sampled bit strings per block
    int64_t *noff;               // [n_blocks] of the circuit's earlier blocks
    int64_t *n_distinct;         // [n_circ]
    uint64_t *bits;              // [n_circ * shots] circuit c's distinct bit strings from c * shots on
    int64_t *counts;             // [n_circ * shots] their counts
};

int launch_sample(const SampleArgs &a, void *stream);
int launch_zero_hist(uint32_t *p, int64_t n, void *stream);

int launch_probs(const ProbArgs &a, int precision, void *stream);
int launch_diag_seed(const DiagArgs &a, int precision, void *stream);
int launch_diag_expect(const DiagArgs &a, int precision, void *stream);
int launch_segment_sum(const SegSumArgs &a, void *stream);
int launch_fill(double *p, int64_t n, double v, void *stream);
int launch_matrices(const MatArgs &a, int precision, void *stream);
int launch_shift_matrices(const ShiftMatArgs &a, int precision, void *stream);
int launch_rlevel_lam(const LevelArgs &a, int precision, void *stream);  // adjoint tiles where psi is zero
int launch_rz_phase(const StatePhaseArgs &a, void *stream);            // writes a.phase
int launch_scale_copy(const StatePhaseArgs &a, int precision, void *stream);  // dst = phase * src

// Fused 4-qubit blocks: for every circuit and block, the product of the block's gates (16x16 complex),
// written as the 32x32 real matrix [[Re, -Im], [Im, Re]] interleaved per amplitude, in MFMA A order.
struct FuseArgs {
    const DevOp *ops;
    const DevCirc *circs;
    const int64_t *first_block;  // [n_circ + 1]: blocks of circuit c are [first_block[c], first_block[c+1])
    int32_t n_circ;
    int32_t pad;
    const int64_t *fused_ops;    // global op index of each plan's markers
    const void *mats;            // 2x2 matrices (complex64)
    float *fmats;
    int64_t n_blocks;
};
int launch_fuse(const FuseArgs &a, void *stream);
int prepare_kernels();  // raises the dynamic-LDS limits; call once per device

// Static scratch of the non-allocating expectation call (a file-scope device array, one per device).
constexpr int64_t kStaticScratchDoubles = (int64_t)1 << 20;  // 8 MiB
constexpr int kMaxStaticDevices = 64;
int static_scratch_setup(int device);  // looks up the array's address on `device`, which must be current
double *static_scratch(int device);    // that address, or NULL before static_scratch_setup

}  // namespace qv
