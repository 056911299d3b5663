// Pass planner. A pass may contain any gate whose qubits are all in the pass's local set and which does
// not have to wait for an earlier gate that stays behind (gates on disjoint qubits commute, so a gate
// can move ahead of unscheduled gates it shares no qubit with). The greedy loop below walks the
// unscheduled gates in program order, growing the local set while it has room; once a gate cannot join,
// its qubits are blocked for the rest of the pass so that later gates on them keep their order.
// Register segments split a pass the same way one level down: a segment holds 2^reg_bits amplitudes
// per thread, and a gate joins it when the qubit it mixes (a rotation's qubit, a CNOT's target) is one of
// the segment's register qubits.
#include "planner.h"

#include <algorithm>
#include <climits>
#include <cstdlib>

namespace qv {

static bool two_qubit(int kind) { return kind == QV_CNOT || kind == QV_CZ; }

static bool diagonal(int kind)
{
    return kind == QV_Z || kind == QV_S || kind == QV_T || kind == QV_RZ || kind == QV_CZ;
}

static void number_train_slots(PlanPass &pp)
{
    int slot = 0;
    for (PlanOp &op : pp.ops) op.train_slot = op.train_slot >= 0 ? slot++ : -1;
    pp.n_train = slot;
}

static void finish_pass(PlanPass &pp, int n)
{
    pp.lq.clear();
    for (int q = 0; q < n; q++)
        if (pp.local_mask >> q & 1ull) pp.lq.push_back(q);
    pp.t = (int)pp.lq.size();
    pp.lowc = 0;
    while (pp.lowc < pp.t && pp.lq[pp.lowc] == pp.lowc) pp.lowc++;
    number_train_slots(pp);
}

void segment_pass(PlanPass &pp, int reg_bits)
{
    pp.segs.clear();
    if (reg_bits <= 0 || pp.t < reg_bits || pp.stride) return;
    int pos[64];
    for (int i = 0; i < 64; i++) pos[i] = -1;
    for (size_t i = 0; i < pp.lq.size(); i++) pos[pp.lq[i]] = (int)i;
    const int G = (int)pp.ops.size();
    std::vector<char> done(G, 0);
    std::vector<PlanOp> order;
    order.reserve(G);
    int remaining = G, first = 0;
    while (remaining > 0) {
        PlanSeg sg;
        sg.op_begin = (int)order.size();
        uint32_t R = 0, blocked = 0;
        int nr = 0;
        while (first < G && done[first]) first++;
        for (int g = first; g < G; g++) {
            if (done[g]) continue;
            const PlanOp &op = pp.ops[g];
            const int a = pos[op.q0], b = two_qubit(op.kind) ? pos[op.q1] : -1;
            const uint32_t qs = (1u << a) | (b >= 0 ? (1u << b) : 0u);
            if (qs & blocked) { blocked |= qs; continue; }
            uint32_t need = 0;
            if (op.kind == QV_CNOT) need = 1u << b;
            else if (!diagonal(op.kind)) need = 1u << a;
            need &= ~R;
            const int add = __builtin_popcount(need);
            if (nr + add <= reg_bits) {
                R |= need;
                nr += add;
                done[g] = 1;
                remaining--;
                order.push_back(op);
            } else {
                blocked |= qs;
            }
        }
        sg.n_ops = (int)order.size() - sg.op_begin;
        // register qubits: the ones the segment needs, then the lowest free positions
        for (int p = 0; p < pp.t; p++)
            if (R >> p & 1u) sg.rpos.push_back(p);
        for (int p = 0; p < pp.t && (int)sg.rpos.size() < reg_bits; p++)
            if (!(R >> p & 1u)) { sg.rpos.push_back(p); R |= 1u << p; }
        // thread bits: the four lowest lanes on positions with distinct (position mod 4), so a quarter
        // wave's LDS accesses fall in distinct banks under the tile's XOR swizzle; the rest ascending
        std::vector<int> rest;
        for (int p = 0; p < pp.t; p++)
            if (!(R >> p & 1u)) rest.push_back(p);
        uint32_t used_mod = 0;
        for (int m = 0; m < 4 && !rest.empty(); m++) {
            size_t pick = 0;
            bool found = false;
            for (size_t i = 0; i < rest.size(); i++)
                if (!(used_mod >> (rest[i] & 3) & 1u)) { pick = i; found = true; break; }
            if (!found) break;
            used_mod |= 1u << (rest[pick] & 3);
            sg.tpos.push_back(rest[pick]);
            rest.erase(rest.begin() + (long)pick);
        }
        for (int p : rest) sg.tpos.push_back(p);
        pp.segs.push_back(sg);
    }
    pp.ops = order;
    number_train_slots(pp);
}

Plan plan_tiled(const PlanInput &in, int tile_qubits, int lowc, int reg_bits, int fuse_min, int fold)
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
    lowc = std::min(lowc, n);
    std::vector<char> done(G, 0);
    std::vector<uint64_t> qmask(G);
    for (int g = 0; g < G; g++)
        qmask[g] = (1ull << in.q0[g]) | (two_qubit(in.kinds[g]) ? (1ull << in.q1[g]) : 0ull);
    int remaining = G;
    int first = 0;
    const bool whole = n <= tile_qubits;
    // Gates a pass with local set L can take: in program order, each unscheduled gate whose qubits are
    // local and not blocked by an earlier gate left behind.
    auto schedulable = [&](uint64_t L, std::vector<int> *out) {
        uint64_t blocked = 0;
        int cnt = 0, ntrain = 0;
        for (int g = first; g < G; g++) {
            if (done[g]) continue;
            const uint64_t qs = qmask[g];
            if (qs & blocked) { blocked |= qs; continue; }
            if ((qs & ~L) || (in.trainable[g] && ntrain >= kMaxTrainPerPass)) { blocked |= qs; continue; }
            cnt++;
            ntrain += in.trainable[g] ? 1 : 0;
            if (out) out->push_back(g);
        }
        return cnt;
    };
    while (remaining > 0) {
        PlanPass pp;
        while (first < G && done[first]) first++;
        // 1. grow the local set greedily in program order
        uint64_t L = whole ? full : (1ull << lowc) - 1ull;
        int cnt = whole ? n : lowc;
        {
            uint64_t blocked = 0;
            for (int g = first; g < G && cnt < tile_qubits; g++) {
                if (done[g]) continue;
                const uint64_t qs = qmask[g];
                if (qs & blocked) { blocked |= qs; continue; }
                const uint64_t need = qs & ~L;
                const int add = __builtin_popcountll(need);
                if (cnt + add <= tile_qubits) { L |= need; cnt += add; }
                else blocked |= qs;
            }
            for (int q = 0; q < n && cnt < tile_qubits; q++)
                if (!(L >> q & 1ull)) { L |= 1ull << q; cnt++; }
        }
        // 2. local search: swap one free qubit in and one out while that lets the pass take more gates
        if (!whole) {
            int best = schedulable(L, nullptr);
            for (int round = 0; round < 64; round++) {
                bool improved = false;
                for (int qi = lowc; qi < n && !improved; qi++) {
                    if (L >> qi & 1ull) continue;
                    for (int qo = lowc; qo < n; qo++) {
                        if (!(L >> qo & 1ull)) continue;
                        const uint64_t L2 = (L | (1ull << qi)) & ~(1ull << qo);
                        const int c2 = schedulable(L2, nullptr);
                        if (c2 > best) { best = c2; L = L2; improved = true; break; }
                    }
                }
                if (!improved) break;
            }
        }
        std::vector<int> take;
        schedulable(L, &take);
        for (int g : take) {
            done[g] = 1;
            remaining--;
            pp.ops.push_back(mk_op(g));
        }
        pp.local_mask = L;
        finish_pass(pp, n);
        segment_pass(pp, reg_bits);
        if (fold) fold_boundary_cnots(pp);
        pl.passes.push_back(pp);
    }
    if (fuse_min > 0) fuse_segments(pl, fuse_min);
    return pl;
}

void fold_boundary_cnots(PlanPass &pp)
{
    if (pp.segs.empty()) return;
    std::vector<PlanSeg> segs;
    std::vector<PlanOp> ops;
    for (size_t s = 0; s < pp.segs.size(); s++) {
        PlanSeg sg = pp.segs[s];
        const int b = sg.op_begin, e = sg.op_begin + sg.n_ops;
        int i = b, j = e;
        while (i < j && pp.ops[i].kind == QV_CNOT && (int)sg.lead.size() < kMaxFoldedCnots) sg.lead.push_back(pp.ops[i++]);
        if (i == j) {
            // only CNOTs: they run between the neighbouring segments
            if (!segs.empty() && (int)(segs.back().trail.size() + sg.lead.size()) <= kMaxFoldedCnots) {
                for (const PlanOp &op : sg.lead) segs.back().trail.push_back(op);
                continue;
            }
            if (s + 1 < pp.segs.size()) {
                // hand them to the next segment's leading run (checked against the cap there)
                PlanSeg &nx = pp.segs[s + 1];
                std::vector<PlanOp> merged = sg.lead;
                const int nb = nx.op_begin, ne = nx.op_begin + nx.n_ops;
                int k = nb;
                while (k < ne && pp.ops[k].kind == QV_CNOT) merged.push_back(pp.ops[k++]);
                if ((int)merged.size() <= kMaxFoldedCnots) {
                    nx.lead = merged;
                    nx.n_ops -= k - nb;
                    nx.op_begin = k;
                    continue;
                }
            }
            // no neighbour can take them: keep the last one as an op, so the segment is not empty
            sg.lead.pop_back();
            i--;
        }
        std::vector<PlanOp> tail;
        while (j - 1 > i && pp.ops[j - 1].kind == QV_CNOT && (int)tail.size() < kMaxFoldedCnots) tail.push_back(pp.ops[--j]);
        std::reverse(tail.begin(), tail.end());
        sg.trail = tail;
        sg.op_begin = (int)ops.size();
        for (int k = i; k < j; k++) ops.push_back(pp.ops[k]);
        sg.n_ops = j - i;
        segs.push_back(sg);
    }
    pp.ops = ops;
    pp.segs = segs;
    number_train_slots(pp);
}

std::vector<int> pass_gate_order(const PlanPass &pp)
{
    std::vector<int> g;
    if (pp.segs.empty()) {
        for (const PlanOp &op : pp.ops)
            if (op.kind != kFusedKind) g.push_back(op.gate);
        return g;
    }
    for (const PlanSeg &sg : pp.segs) {
        for (const PlanOp &op : sg.lead) g.push_back(op.gate);
        for (int k = 0; k < sg.n_ops; k++)
            if (pp.ops[sg.op_begin + k].kind != kFusedKind) g.push_back(pp.ops[sg.op_begin + k].gate);
        for (const PlanOp &op : sg.trail) g.push_back(op.gate);
    }
    return g;
}

int pass_gate_count(const PlanPass &pp)
{
    int n = 0;
    for (const PlanOp &op : pp.ops) n += op.kind != kFusedKind ? 1 : 0;
    for (const PlanSeg &sg : pp.segs) n += (int)(sg.lead.size() + sg.trail.size());
    return n;
}

void fuse_segments(Plan &pl, int fuse_min)
{
    int next = 0;
    for (PlanPass &pp : pl.passes) {
        if (pp.segs.empty()) continue;
        std::vector<PlanOp> out;
        std::vector<PlanSeg> segs = pp.segs;
        for (PlanSeg &sg : segs) {
            uint32_t R = 0;
            int pos[64];
            for (int i = 0; i < 64; i++) pos[i] = -1;
            for (size_t i = 0; i < pp.lq.size(); i++) pos[pp.lq[i]] = (int)i;
            for (int p : sg.rpos) R |= 1u << p;
            auto local = [&](const PlanOp &op) {
                if (!(R >> pos[op.q0] & 1u)) return false;
                if (two_qubit(op.kind) && !(R >> pos[op.q1] & 1u)) return false;
                return true;
            };
            const int b = sg.op_begin, e = sg.op_begin + sg.n_ops;
            const int new_begin = (int)out.size();
            for (int i = b; i < e;) {
                int j = i;
                while (j < e && local(pp.ops[j])) j++;
                if (j - i >= fuse_min && next < 65535) {   // block numbers are 16-bit in the device op
                    PlanOp m;
                    m.gate = 0;
                    m.kind = kFusedKind;
                    m.q0 = pp.ops[i].q0;
                    m.q1 = -1;
                    m.train_slot = -1;
                    m.fused_count = j - i;
                    m.fused_index = next++;
                    out.push_back(m);
                    for (int k = i; k < j; k++) out.push_back(pp.ops[k]);
                    i = j;
                } else {
                    out.push_back(pp.ops[i]);
                    i++;
                }
            }
            sg.op_begin = new_begin;
            sg.n_ops = (int)out.size() - new_begin;
        }
        pp.ops = out;
        pp.segs = segs;
    }
}

int fused_blocks(const Plan &pl)
{
    int n = 0;
    for (const PlanPass &pp : pl.passes)
        for (const PlanOp &op : pp.ops)
            if (op.kind == kFusedKind) n++;
    return n;
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

std::vector<uint64_t> pass_zero_masks(const Plan &pl)
{
    std::vector<uint64_t> out;
    uint64_t touched = 0;  // qubits acted on by the passes before this one
    auto touch = [&](const PlanOp &op) {
        if (op.kind == kFusedKind) return;
        touched |= 1ull << op.q0;
        if (op.q1 >= 0) touched |= 1ull << op.q1;
    };
    for (const PlanPass &pp : pl.passes) {
        out.push_back(~pp.local_mask & ~touched);  // bits at or above the circuit's width never occur in a base
        for (const PlanOp &op : pp.ops) touch(op);
        for (const PlanSeg &sg : pp.segs) {
            for (const PlanOp &op : sg.lead) touch(op);
            for (const PlanOp &op : sg.trail) touch(op);
        }
    }
    return out;
}

void lower_plan(const Plan &pl, std::vector<DevPass> &passes, std::vector<DevOp> &ops, std::vector<DevSeg> &segs)
{
    const std::vector<uint64_t> zero = pass_zero_masks(pl);
    for (const PlanPass &pp : pl.passes) {
        DevPass d{};
        d.local_mask = pp.local_mask;
        d.zero_mask = zero[(size_t)(&pp - pl.passes.data())];
        d.t = pp.t;
        d.op_begin = (int32_t)ops.size();
        d.n_ops = (int32_t)pp.ops.size();
        d.n_train = pp.n_train;
        d.stride = pp.stride;
        d.pad = pp.lowc;
        d.seg_begin = (int32_t)segs.size();
        d.n_seg = (int32_t)pp.segs.size();
        for (int i = 0; i < 16; i++) d.lq[i] = i < (int)pp.lq.size() ? (int8_t)pp.lq[i] : (int8_t)-1;
        int pos[64];
        for (int i = 0; i < 64; i++) pos[i] = -1;
        for (size_t i = 0; i < pp.lq.size(); i++) pos[pp.lq[i]] = (int)i;
        // register index of each local position, per segment
        std::vector<int> seg_of(pp.ops.size(), -1);
        for (size_t s = 0; s < pp.segs.size(); s++)
            for (int k = 0; k < pp.segs[s].n_ops; k++) seg_of[pp.segs[s].op_begin + k] = (int)s;
        for (size_t i = 0; i < pp.ops.size(); i++) {
            const PlanOp &op = pp.ops[i];
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
            o.k0 = -1;
            o.k1 = -1;
            if (op.kind == kFusedKind) {
                // marker: block number in p0 | p1 << 8, block size in pad
                o.kind = (uint8_t)kFusedKind;
                o.p0 = (uint8_t)(op.fused_index & 0xFF);
                o.p1 = (uint8_t)((op.fused_index >> 8) & 0xFF);
                o.pad = (int16_t)op.fused_count;
                o.flags = (uint8_t)(OC_FUSED << kOpCodeShift);
                o.train_slot = -1;
                ops.push_back(o);
                continue;
            }
            if (seg_of[i] >= 0) {
                const PlanSeg &sg = pp.segs[seg_of[i]];
                for (size_t k = 0; k < sg.rpos.size(); k++) {
                    if (sg.rpos[k] == o.p0) o.k0 = (int8_t)k;
                    if (op.q1 >= 0 && sg.rpos[k] == o.p1) o.k1 = (int8_t)k;
                }
                int code = OC_NONE;
                switch (op.kind) {
                case QV_RY: code = OC_RY + o.k0; break;
                case QV_RZ: case QV_Z: case QV_S: case QV_T: code = o.k0 >= 0 ? OC_DIAG + o.k0 : OC_DIAG_T; break;
                case QV_CNOT: code = o.k0 >= 0 ? OC_CNOT_RR + 4 * o.k0 + o.k1 : OC_CNOT_TR + o.k1; break;
                case QV_CZ: code = OC_CZ; break;
                default: code = OC_GEN + o.k0; break;  // H, X, Y, RX: the qubit is a register qubit
                }
                o.flags = (uint8_t)(o.flags | (code << kOpCodeShift));
            }
            o.pad = 0;
            ops.push_back(o);
        }
        d.first_train = INT32_MAX;
        for (size_t i = 0; i < pp.ops.size(); i++)
            if (pp.ops[i].kind != kFusedKind && pp.ops[i].train_slot >= 0) {
                d.first_train = d.op_begin + (int32_t)i;
                break;
            }
        d.adj_last_nseg = 0;
        for (const PlanSeg &sg : pp.segs)
            if (d.op_begin + sg.op_begin + sg.n_ops > d.first_train) d.adj_last_nseg++;
        for (const PlanSeg &sg : pp.segs) {
            DevSeg ds{};
            ds.op_begin = d.op_begin + sg.op_begin;
            ds.n_ops = sg.n_ops;
            for (int k = 0; k < 8; k++) ds.rpos[k] = k < (int)sg.rpos.size() ? (int8_t)sg.rpos[k] : (int8_t)-1;
            for (int m = 0; m < 16; m++) ds.tpos[m] = m < (int)sg.tpos.size() ? (int8_t)sg.tpos[m] : (int8_t)-1;
            auto pack = [&](const std::vector<PlanOp> &run, uint64_t &out) {
                // positions index the tile (< t <= 15), so the folded map stays inside it
                if (run.size() > (size_t)kMaxFoldedCnots) std::abort();
                out = ~0ull;  // unused entries: 0xFF, a no-op on tile indices (< 2^15)
                for (size_t k = 0; k < run.size(); k++) {
                    const int c = pos[run[k].q0], t = pos[run[k].q1];
                    if (c < 0 || t < 0 || c >= pp.t || t >= pp.t || c == t || pp.t > 15) std::abort();
                    out &= ~(0xFFull << (8 * k));
                    out |= (uint64_t)(c | (t << 4)) << (8 * k);
                }
                return (int8_t)run.size();
            };
            ds.n_lead = pack(sg.lead, ds.lead);
            ds.n_trail = pack(sg.trail, ds.trail);
            auto apply = [&](uint32_t e, const std::vector<PlanOp> &run, bool rev) {
                for (size_t i = 0; i < run.size(); i++) {
                    const PlanOp &op = run[rev ? run.size() - 1 - i : i];
                    e ^= ((e >> pos[op.q0]) & 1u) << pos[op.q1];
                }
                return e;
            };
            for (int k = 0; k < 4; k++) {
                const uint32_t bit = k < (int)sg.rpos.size() ? 1u << sg.rpos[k] : 0u;
                ds.rimg_lead[k] = (uint16_t)apply(bit, sg.lead, true);
                ds.rimg_trail[k] = (uint16_t)apply(bit, sg.trail, false);
            }
            segs.push_back(ds);
        }
        passes.push_back(d);
    }
}

}  // namespace qv
