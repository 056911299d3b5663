// Pass planner: turns a circuit's gate list into passes (see engine.h). Host only.
#pragma once
#include <stdint.h>

#include <vector>

#include "engine.h"

namespace qv {

struct PlanInput {
    int n = 0;
    std::vector<int> kinds, q0, q1;   // q1 = -1 for one-qubit gates
    std::vector<bool> trainable;
};

// A fused-block marker (kind kFusedKind, declared with the device op layout) heads a fused block: the
// next fused_count ops of the segment are its gates.

struct PlanOp {
    int gate;        // index in the circuit (fused-block markers: 0, unused)
    int kind;        // qv_gate_kind, or kFusedKind for a fused-block marker
    int q0, q1;      // qubits (global)
    int train_slot;  // position among the pass's trainable gates, -1 if fixed
    int fused_count = 0;   // markers: number of gates in the block
    int fused_index = -1;  // markers: block number within the plan
};

// A register segment of a pass (see DevSeg in engine.h): positions are local.
struct PlanSeg {
    std::vector<int> rpos;  // register bit -> local position
    std::vector<int> tpos;  // thread bit -> local position
    int op_begin = 0;       // first op of the segment in the pass's (reordered) op list
    int n_ops = 0;
    // CNOT runs folded into the segment's LDS addressing (they permute the tile's amplitudes): `lead` runs
    // before the segment's ops, `trail` after them, each in program order.
    std::vector<PlanOp> lead, trail;
};

// Most CNOTs one segment boundary may fold (per run; longer runs keep the rest as ops).
constexpr int kMaxFoldedCnots = 8;

struct PlanPass {
    uint64_t local_mask = 0;
    int t = 0;
    int lowc = 0;     // local qubits 0..lowc-1 are qubits 0..lowc-1 (contiguous runs in memory)
    int stride = 0;   // 1: a single gate applied straight from global memory
    int n_train = 0;
    std::vector<int> lq;      // local position -> qubit (ascending)
    std::vector<PlanOp> ops;  // in program order (register-tiled passes: in segment order)
    std::vector<PlanSeg> segs;  // empty: the pass runs op by op in LDS
};

struct Plan {
    std::vector<PlanPass> passes;
};

// Most trainable gates one pass may hold (their adjoint partial sums live in LDS).
constexpr int kMaxTrainPerPass = 256;

// LDS tile plan with tiles of at most `tile_qubits` qubits, the lowest `lowc` qubits always local.
// reg_bits > 0 splits every pass of at least reg_bits qubits into register segments of 2^reg_bits
// amplitudes per thread.
// fuse_min > 0 turns every run of at least fuse_min consecutive gates of a segment that act on register
// qubits only into a fused block (a marker op followed by the run).
// fold > 0 folds the CNOT runs at register-segment boundaries into the segments' addressing.
Plan plan_tiled(const PlanInput &in, int tile_qubits, int lowc, int reg_bits = 0, int fuse_min = 0, int fold = 1);

// Splits one pass into register segments (reorders its ops; dependencies are kept).
void segment_pass(PlanPass &pp, int reg_bits);

// Moves the CNOT runs at the two ends of every register segment out of its op list into its lead / trail
// lists (a segment left without ops hands its CNOTs to a neighbour).
void fold_boundary_cnots(PlanPass &pp);

// Gates of a pass in execution order (folded CNOTs included, fused-block markers left out).
std::vector<int> pass_gate_order(const PlanPass &pp);

// Gates of a pass: its ops other than fused-block markers, plus its folded CNOTs.
int pass_gate_count(const PlanPass &pp);

// Inserts fused-block markers into the segments of a plan's passes; numbers the blocks plan-wide.
void fuse_segments(Plan &pl, int fuse_min);

// Number of fused blocks of a plan.
int fused_blocks(const Plan &pl);

// One stride pass per gate.
Plan plan_stride(const PlanInput &in);

// Per pass: the qubits outside its tile that no earlier pass touches (folded CNOTs included). They are still
// |0> when the pass runs, so a tile with one of them at 1 holds zeros throughout it.
std::vector<uint64_t> pass_zero_masks(const Plan &pl);

// Appends a plan's passes and ops in device form.
void lower_plan(const Plan &pl, std::vector<DevPass> &passes, std::vector<DevOp> &ops,
                std::vector<DevSeg> &segs);

}  // namespace qv
