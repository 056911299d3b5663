// Test driver (CPU only, no GPU): plans one circuit read from stdin, writes the source of every kernel the
// library would generate for its register-tiled passes, compiles each with hipRTC for gfx950 and stores the
// code objects in the directory given as argv[1]. Input: "n tile lowc reg_bits fuse_min precision inner_f64"
// and then one gate per line, "kind q0 q1 trainable".
#include <cstdio>
#include <fstream>
#include <iostream>

#include "jit.h"
#include "planner.h"

using namespace qv;

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    PlanInput in;
    int tile, lowc, rb, fuse, prec, inner_f64;
    if (!(std::cin >> in.n >> tile >> lowc >> rb >> fuse >> prec >> inner_f64)) return 2;
    int k, a, b, t;
    while (std::cin >> k >> a >> b >> t) {
        in.kinds.push_back(k);
        in.q0.push_back(a);
        in.q1.push_back(b);
        in.trainable.push_back(t != 0);
    }
    const Plan pl = plan_tiled(in, tile, lowc, rb, fuse, 1);
    std::vector<DevPass> passes;
    std::vector<DevOp> ops;
    std::vector<DevSeg> segs;
    lower_plan(pl, passes, ops, segs);
    int bad = 0;
    for (size_t p = 0; p < passes.size(); p++) {
        if (passes[p].n_seg == 0) continue;
        for (int adj = 0; adj < 2; adj++) {
            GenPassDesc d;
            d.pass = passes[p];
            d.segs.assign(segs.begin() + d.pass.seg_begin, segs.begin() + d.pass.seg_begin + d.pass.n_seg);
            d.ops.assign(ops.begin() + d.pass.op_begin, ops.begin() + d.pass.op_begin + d.pass.n_ops);
            d.precision = prec;
            d.adjoint = adj;
            d.lds_t = d.pass.t;
            d.tab_bits = d.pass.t - d.pass.pad;
            d.max_train = d.pass.n_train;
            d.inner_f64 = inner_f64;
            std::string err;
            const std::string code = gen_compile(gen_pass_source(d), err);
            const std::string name = std::string(argv[1]) + "/pass" + std::to_string(p) + (adj ? "_adj" : "_fwd") + ".co";
            if (code.empty()) {
                std::cout << "FAIL " << name << "\n" << err << "\n";
                bad++;
                continue;
            }
            std::ofstream(name, std::ios::binary).write(code.data(), (std::streamsize)code.size());
            std::cout << "OK " << name << " ops " << d.ops.size() << " segs " << d.pass.n_seg << "\n";
        }
    }
    return bad ? 1 : 0;
}
