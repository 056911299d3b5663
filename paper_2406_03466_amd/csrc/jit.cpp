// Tile passes specialised at run time (see jit.h). The generated op program writes every op of a pass as
// one call of gen_fwd_op / gen_adj_op (tile_device.h) with the op's code, kind, qubits, register bits,
// gate index and partial-sum slot as template constants, segment by segment; the tile body around it (LDS
// loads, register segments, folded CNOT addressing, prefetch, stores) is the same device code the
// precompiled kernels use. Compiled with hipRTC for gfx950 (packed FP32 instructions off, as for the
// library itself), loaded as a module, and kept per device in this process and on disk.
#include "jit.h"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <thread>

#include "jit_headers.inc"  // kGenHeaderNames / kGenHeaderText: tile_device.h, engine.h, qvpu.h (build step)

namespace qv {

namespace {

const char *const kGenOptions[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                                   "-Xclang", "-packed-fp32-ops"};

size_t lds_bytes(const GenPassDesc &d)
{
    // the layout rtile_body carves: tile(s), run-offset table, reduction area, adjoint partial sums
    const size_t amp = d.precision == QV_C64 ? 8 : 16;
    size_t b = (size_t)(d.adjoint ? 2 : 1) * ((size_t)1 << d.lds_t) * amp + ((size_t)8 << d.tab_bits) +
               sizeof(double) * (kBlock / 64);
    if (d.adjoint) b += sizeof(double) * (kRtileThreads / 64) * (size_t)d.max_train;
    return b;
}

// Written after every op: the compiler may not move instructions across it, which keeps each op's
// loads and arithmetic together instead of spread over the whole straight-line program.
const char *const kOpFence = "        __builtin_amdgcn_sched_barrier(0);\n";

void op_args(std::ostringstream &o, const DevOp &op)
{
    o << (op.flags >> kOpCodeShift) << ", " << (int)op.kind << ", " << (int)op.p0 << ", " << (int)op.p1 << ", "
      << (int)op.k0 << ", " << (int)op.k1 << ", " << op.gate;
}

void emit_fwd(std::ostringstream &o, const GenPassDesc &d, const DevSeg &S, int rel0)
{
    // A fused block's gates run one by one here (they follow its marker). With the block's MFMA product
    // in the same straight-line program, the forward pass needs about 200 registers a lane: at the
    // 128 of two workgroups per CU the register set is spilled around every segment, and at one
    // workgroup per CU the pass is slower than the general kernel with its blocks, so a level takes
    // whichever of the two kernels times faster.
    for (int j = 0; j < S.n_ops; j++) {
        const DevOp &op = d.ops[rel0 + j];
        if (op.kind == kFusedKind) continue;
        o << "        gen_fwd_op<R, RB, ";
        op_args(o, op);
        o << ">(a, C, circ, mp, " << j << ", Et, v);\n" << kOpFence;
    }
}

void emit_adj(std::ostringstream &o, const GenPassDesc &d, const DevSeg &S, int rel0)
{
    for (int j = S.n_ops - 1; j >= 0; j--) {
        const DevOp &op = d.ops[rel0 + j];
        if (op.kind == kFusedKind) continue;  // the adjoint undoes a block's gates one by one
        // a circuit's first pass is undone only down to its first trainable op (rtile_body's stop_early)
        const bool below = d.pass.first_train >= 0 && S.op_begin + j < d.pass.first_train;
        o << (below ? "        if (!stop_early) gen_adj_op<R, RB, NT, " : "        gen_adj_op<R, RB, NT, ");
        op_args(o, op);
        o << ", " << ((op.flags & OP_TRAIN) ? 1 : 0) << ", " << op.train_slot
          << ">(a, C, circ, mp, " << j << ", Et, active, lane, wave, red, av, lv);\n" << kOpFence;
    }
}

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t source_key(const std::string &src)
{
    uint64_t h = fnv1a(src);
    for (const char *opt : kGenOptions) h = fnv1a(opt, h);
    for (int i = 0; i < kGenHeaderCount; i++) h = fnv1a(kGenHeaderText[i], h);
    return h;
}

std::string cache_path(uint64_t key)
{
    const char *dir = getenv("QV_GEN_CACHE");
    std::string d;
    if (dir && *dir) d = dir;
    else {
        const char *home = getenv("HOME");
        d = std::string(home && *home ? home : "/tmp") + "/.cache/qvpu_gen";
    }
    char name[40];
    snprintf(name, sizeof name, "/%016llx.co", (unsigned long long)key);
    return d + name;
}

bool read_file(const std::string &path, std::string &out)
{
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::ostringstream ss;
    ss << f.rdbuf();
    out = ss.str();
    return !out.empty();
}

void write_file(const std::string &path, const std::string &data)
{
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); i++)  // create the parent directories one level at a time
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>()(
                                                std::this_thread::get_id()));
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f.write(data.data(), (std::streamsize)data.size());
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

std::string compile(const std::string &src, std::string &err);

}  // namespace

std::string gen_compile(const std::string &src, std::string &err) { return compile(src, err); }

namespace {

// hipRTC: source -> code object for gfx950; returns an empty string and sets err on failure.
std::string compile(const std::string &src, std::string &err)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "qv_gen.hip", kGenHeaderCount, kGenHeaderText,
                            kGenHeaderNames) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return {};
    }
    const int nopt = (int)(sizeof kGenOptions / sizeof kGenOptions[0]);
    const hiprtcResult r = hiprtcCompileProgram(prog, nopt, kGenOptions);
    std::string code;
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        err = std::string("generated tile pass did not compile: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
    } else {
        size_t n = 0;
        hiprtcGetCodeSize(prog, &n);
        code.resize(n);
        hiprtcGetCode(prog, &code[0]);
    }
    hiprtcDestroyProgram(&prog);
    return code;
}

struct Loaded {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, uint64_t>, Loaded> g_loaded;  // (device, source key) -> module

}  // namespace

const char *gen_kernel_name(int adjoint) { return adjoint ? "qv_gen_adj" : "qv_gen_fwd"; }

std::string gen_pass_source(const GenPassDesc &d)
{
    std::ostringstream o;
    const bool c64 = d.precision == QV_C64;
    o << "// generated: one register-tiled pass, " << (d.adjoint ? "reverse" : "forward") << " sweep, "
      << (c64 ? "complex64" : "complex128") << "\n" << (d.inner_f64 ? "#define QV_ADJ_INNER_F64 1\n" : "")
      << "#include \"tile_device.h\"\n\nnamespace qv {\n\n"
      << "struct GenProg {\n    static constexpr bool kGenerated = true;\n\n";
    o << "    template <typename R, int RB, int NT>\n"
         "    static __device__ __forceinline__ void fwd(int si, const LevelArgs &a, const DevCirc &C, int circ,\n"
         "                                               const M2<R> *mp, uint32_t Et, int lane, Regs<R, 1 << RB> &v)\n"
         "    {\n";
    if (!d.adjoint) {
        o << "        switch (si) {\n";
        for (size_t si = 0; si < d.segs.size(); si++) {
            o << "        case " << si << ": {\n";
            emit_fwd(o, d, d.segs[si], d.segs[si].op_begin - d.pass.op_begin);
            o << "        } break;\n";
        }
        o << "        default: break;\n        }\n";
    }
    o << "    }\n\n";
    o << "    template <typename R, int RB, int NT>\n"
         "    static __device__ __forceinline__ void adj(int si, bool stop_early, const LevelArgs &a, const DevCirc &C,\n"
         "                                               int circ, const M2<R> *mp, uint32_t Et, bool active, int lane,\n"
         "                                               int wave, double *red, Regs<R, 1 << RB> &av,\n"
         "                                               Regs<R, 1 << RB> &lv)\n"
         "    {\n";
    if (d.adjoint) {
        o << "        switch (si) {\n";
        for (size_t si = 0; si < d.segs.size(); si++) {
            o << "        case " << si << ": {\n";
            emit_adj(o, d, d.segs[si], d.segs[si].op_begin - d.pass.op_begin);
            o << "        } break;\n";
        }
        o << "        default: break;\n        }\n";
    }
    o << "    }\n};\n\n}  // namespace qv\n\n";
    o << "extern \"C\" __global__ __launch_bounds__(" << kRtileThreads << ")"
      << (d.adjoint ? "" : " __attribute__((amdgpu_waves_per_eu(4)))") << " void " << gen_kernel_name(d.adjoint)
      << "(qv::LevelArgs a)\n{\n"
      << "    __shared__ __align__(16) unsigned char smem[" << lds_bytes(d) << "];\n"
      << "    qv::rtile_tiles<" << (c64 ? "float" : "double") << ", " << (d.adjoint ? "true" : "false") << ", "
      << (c64 ? kRegBitsC64 : kRegBitsC128) << ", " << kRtileThreads << ", qv::GenProg>(a, smem);\n}\n";
    return o.str();
}

int gen_kernels(const std::vector<std::string> &srcs, std::vector<void *> &fns, std::string &err)
{
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return he;
    fns.assign(srcs.size(), nullptr);
    std::vector<uint64_t> keys(srcs.size());
    std::vector<size_t> todo;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (size_t i = 0; i < srcs.size(); i++) {
            keys[i] = source_key(srcs[i]);
            auto it = g_loaded.find({dev, keys[i]});
            if (it != g_loaded.end()) fns[i] = it->second.fn;
            else todo.push_back(i);
        }
    }
    if (todo.empty()) return 0;
    // code objects: from the disk cache, else compiled (several programs at once)
    std::vector<std::string> code(srcs.size()), errs(srcs.size());
    std::vector<size_t> compile_list;
    for (size_t i : todo)
        if (!read_file(cache_path(keys[i]), code[i])) compile_list.push_back(i);
    if (!compile_list.empty()) {
        const char *env = getenv("QV_GEN_THREADS");
        // default: one compiler thread per host CPU, at most 16
        const size_t hw = std::max(1u, std::thread::hardware_concurrency());
        size_t nthreads = env ? (size_t)std::max(1, atoi(env)) : std::min<size_t>(hw, 16);
        nthreads = std::min(nthreads, compile_list.size());
        std::vector<std::thread> pool;
        std::mutex next_mu;
        size_t next = 0;
        for (size_t t = 0; t < nthreads; t++)
            pool.emplace_back([&] {
                for (;;) {
                    size_t k;
                    {
                        std::lock_guard<std::mutex> lk(next_mu);
                        if (next >= compile_list.size()) return;
                        k = compile_list[next++];
                    }
                    code[k] = compile(srcs[k], errs[k]);
                    if (!code[k].empty()) write_file(cache_path(keys[k]), code[k]);
                }
            });
        for (auto &th : pool) th.join();
    }
    for (size_t i : todo) {
        if (code[i].empty()) {
            err = errs[i].empty() ? "generated tile pass: no code" : errs[i];
            return hipErrorInvalidKernelFile;
        }
        Loaded ld;
        he = hipModuleLoadData(&ld.mod, code[i].data());
        if (he != hipSuccess) {
            err = "hipModuleLoadData failed for a generated tile pass";
            return he;
        }
        // the source names its kernel for its direction
        const char *name = gen_kernel_name(srcs[i].find(std::string(" void ") + gen_kernel_name(1) + "(") !=
                                           std::string::npos);
        he = hipModuleGetFunction(&ld.fn, ld.mod, name);
        if (he != hipSuccess) {
            (void)hipModuleUnload(ld.mod);
            err = std::string("generated tile pass has no kernel ") + name;
            return he;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        auto ins = g_loaded.emplace(std::make_pair(dev, keys[i]), ld);
        if (!ins.second) (void)hipModuleUnload(ld.mod);  // another thread loaded it meanwhile
        fns[i] = ins.first->second.fn;
    }
    return 0;
}

}  // namespace qv
