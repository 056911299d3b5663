// Pass planner. A pass may contain any gate whose qubits are all in the pass's local set and which does
// not have to wait for an earlier gate that stays behind (gates on disjoint qubits commute, so a gate
// can move ahead of unscheduled gates it shares no qubit with). The greedy loop below walks the
// unscheduled gates in program order, growing the local set while it has room; once a gate cannot join,
// its qubits are blocked for the rest of the pass so that later gates on them keep their order.
#include "planner.h"

#include <algorithm>

namespace qv {

static bool two_qubit(int kind) { return kind == QV_CNOT || kind == QV_CZ; }

static void finish_pass(PlanPass &pp, int n)
{
    pp.lq.clear();
    for (int q = 0; q < n; q++)
        if (pp.local_mask >> q & 1ull) pp.lq.push_back(q);
    pp.t = (int)pp.lq.size();
    pp.lowc = 0;
    while (pp.lowc < pp.t && pp.lq[pp.lowc] == pp.lowc) pp.lowc++;
    int slot = 0;
    for (PlanOp &op : pp.ops) op.train_slot = op.train_slot >= 0 ? slot++ : -1;
    pp.n_train = slot;
}

Plan plan_tiled(const PlanInput &in, int tile_qubits, int lowc)
{
    Plan pl;
    const int n = in.n;
    const int G = (int)in.kinds.size();
    const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    auto mk_op = [&](int g) {
        PlanOp op;
        op.gate = g;
        op.kind = in.kinds[g];
        op.q0 = in.q0[g];
        op.q1 = in.q1[g];
        op.train_slot = in.trainable[g] ? 0 : -1;
        return op;
    };
    if (n <= tile_qubits) {
        PlanPass pp;
        pp.local_mask = full;
        for (int g = 0; g < G; g++) pp.ops.push_back(mk_op(g));
        finish_pass(pp, n);
        pl.passes.push_back(pp);
        return pl;
    }
    lowc = std::min(lowc, n);
    std::vector<char> done(G, 0);
    int remaining = G;
    int first = 0;
    while (remaining > 0) {
        PlanPass pp;
        uint64_t L = (1ull << lowc) - 1ull;
        int cnt = lowc;
        uint64_t blocked = 0;
        while (first < G && done[first]) first++;
        for (int g = first; g < G; g++) {
            if (done[g]) continue;
            const uint64_t qs = (1ull << in.q0[g]) | (two_qubit(in.kinds[g]) ? (1ull << in.q1[g]) : 0ull);
            if (qs & blocked) { blocked |= qs; continue; }
            const uint64_t need = qs & ~L;
            const int add = __builtin_popcountll(need);
            if (cnt + add <= tile_qubits) {
                L |= need;
                cnt += add;
                done[g] = 1;
                remaining--;
                pp.ops.push_back(mk_op(g));
            } else {
                blocked |= qs;
            }
        }
        // pad the tile with the lowest unused qubits (fewer, larger tiles; longer contiguous runs)
        for (int q = 0; q < n && cnt < tile_qubits; q++)
            if (!(L >> q & 1ull)) { L |= 1ull << q; cnt++; }
        pp.local_mask = L;
        finish_pass(pp, n);
        pl.passes.push_back(pp);
    }
    return pl;
}

Plan plan_stride(const PlanInput &in)
{
    Plan pl;
    const int G = (int)in.kinds.size();
    for (int g = 0; g < G; g++) {
        PlanPass pp;
        PlanOp op;
        op.gate = g;
        op.kind = in.kinds[g];
        op.q0 = in.q0[g];
        op.q1 = in.q1[g];
        op.train_slot = in.trainable[g] ? 0 : -1;
        pp.ops.push_back(op);
        pp.local_mask = (1ull << op.q0) | (two_qubit(op.kind) ? (1ull << op.q1) : 0ull);
        pp.stride = 1;
        finish_pass(pp, in.n);
        pl.passes.push_back(pp);
    }
    return pl;
}

void lower_plan(const Plan &pl, std::vector<DevPass> &passes, std::vector<DevOp> &ops)
{
    for (const PlanPass &pp : pl.passes) {
        DevPass d{};
        d.local_mask = pp.local_mask;
        d.t = pp.t;
        d.op_begin = (int32_t)ops.size();
        d.n_ops = (int32_t)pp.ops.size();
        d.n_train = pp.n_train;
        d.stride = pp.stride;
        d.pad = pp.lowc;
        for (int i = 0; i < 16; i++) d.lq[i] = i < (int)pp.lq.size() ? (int8_t)pp.lq[i] : (int8_t)-1;
        int pos[64];
        for (int i = 0; i < 64; i++) pos[i] = -1;
        for (size_t i = 0; i < pp.lq.size(); i++) pos[pp.lq[i]] = (int)i;
        for (const PlanOp &op : pp.ops) {
            DevOp o{};
            o.gate = op.gate;
            o.kind = (uint8_t)op.kind;
            if (pp.stride) {
                o.p0 = (uint8_t)op.q0;
                o.p1 = (uint8_t)(op.q1 >= 0 ? op.q1 : 0);
            } else {
                o.p0 = (uint8_t)pos[op.q0];
                o.p1 = (uint8_t)(op.q1 >= 0 ? pos[op.q1] : 0);
            }
            o.flags = op.train_slot >= 0 ? OP_TRAIN : 0;
            o.train_slot = op.train_slot;
            o.pad = 0;
            ops.push_back(o);
        }
        passes.push_back(d);
    }
}

}  // namespace qv
