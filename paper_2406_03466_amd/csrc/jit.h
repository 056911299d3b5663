// Tile passes specialised at run time: the ops of one register-tiled pass written out as straight-line
// code (a generated op program for tile_device.h), compiled for gfx950 with hipRTC and loaded as a module.
// Host only.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "engine.h"

namespace qv {

// What one generated kernel needs to know about its pass and level.
struct GenPassDesc {
    DevPass pass;                 // the pass (op and segment ranges index the two arrays below)
    std::vector<DevSeg> segs;     // its register segments, in order
    std::vector<DevOp> ops;       // its ops, in order (fused-block markers included)
    int precision;                // QV_C64 / QV_C128
    int adjoint;                  // 0: forward sweep, 1: reverse sweep
    int lds_t, tab_bits, max_train;  // the level's LDS layout (equal to the pass's when it is alone)
    int inner_f64 = 0;            // complex64 adjoint: inner products formed and summed in FP64
};

// Name of a generated pass's kernel: qv_gen_fwd (forward sweep) or qv_gen_adj (reverse sweep).
const char *gen_kernel_name(int adjoint);

// HIP C++ source of the kernel gen_kernel_name(d.adjoint) for one pass and direction.
std::string gen_pass_source(const GenPassDesc &d);

// hipRTC alone (no device): the code object of one generated source, or an empty string and err.
std::string gen_compile(const std::string &src, std::string &err);

// Compiles (or finds in the in-process or on-disk cache) every source for the current device and returns
// its kernel handles (hipFunction_t) in fns. Compilations run on several host threads. Returns 0, or a
// HIP error code with a message in err.
int gen_kernels(const std::vector<std::string> &srcs, std::vector<void *> &fns, std::string &err);

}  // namespace qv
