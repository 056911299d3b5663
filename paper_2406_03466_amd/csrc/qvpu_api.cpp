// Host side of the qvpu C interface: validation, pass planning, device layout of a batch, hipGraph
// capture and replay. Every arithmetic step of the path runs in the HIP kernels of kernels.hip; this
// file only decides what to launch and in which order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "jit.h"
#include "planner.h"
#include "qvpu.h"

using namespace qv;

// ---------------------------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------------------------
static thread_local std::string g_err;

static qv_status fail(qv_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

static qv_status ok()
{
    g_err.clear();
    return QV_OK;
}

#define HIPRET(expr)                                    \
    do {                                                \
        hipError_t e_ = (hipError_t)(expr);             \
        if (e_ != hipSuccess) return e_;                \
    } while (0)

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (hipError_t)(expr);                                                            \
        if (e_ != hipSuccess) return fail(QV_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------------------------------------
// Options: a flat JSON object with string, number and boolean values.
// ---------------------------------------------------------------------------------------------------------
static bool parse_options(const char *js, std::map<std::string, std::string> &out, std::string &err)
{
    if (!js) return true;
    const char *p = js;
    auto ws = [&]() { while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') p++; };
    auto str = [&](std::string &s) -> bool {
        if (*p != '"') return false;
        p++;
        while (*p && *p != '"') s.push_back(*p++);
        if (*p != '"') return false;
        p++;
        return true;
    };
    ws();
    if (*p == 0) return true;
    if (*p != '{') { err = "options must be a JSON object"; return false; }
    p++;
    ws();
    if (*p == '}') return true;
    for (;;) {
        ws();
        std::string k, v;
        if (!str(k)) { err = "expected a quoted key"; return false; }
        ws();
        if (*p != ':') { err = "expected ':' after key " + k; return false; }
        p++;
        ws();
        if (*p == '"') {
            if (!str(v)) { err = "unterminated string for key " + k; return false; }
        } else {
            while (*p && *p != ',' && *p != '}' && *p != ' ' && *p != '\n') v.push_back(*p++);
            if (v.empty()) { err = "missing value for key " + k; return false; }
        }
        out[k] = v;
        ws();
        if (*p == ',') { p++; continue; }
        if (*p == '}') { p++; break; }
        err = "expected ',' or '}'";
        return false;
    }
    ws();
    if (*p) { err = "trailing characters after the options object"; return false; }
    return true;
}

// ---------------------------------------------------------------------------------------------------------
// Context and batch objects
// ---------------------------------------------------------------------------------------------------------
constexpr int kSpecializeTimed = 4;                // "specialize" bit: choose per level by timing
constexpr int kTimingSweeps = 4;                   // reverse sweeps timed, alternating general / generated
constexpr int kFuseAuto = -1;                      // "fusion": "auto": the autotuner picks the minimum run
constexpr int kFuseCandidates[] = {0, 4, 6, 8};    // minimum run lengths it times (0: no fused blocks)
constexpr int kFuseDefault = 8;                    // its choice before (or without) a search

// Makes `device` current and clears the runtime's last-error slot, so that the launch checks of this call
// (which read that slot) report only this call's launches, not an earlier failure another call ignored.
static hipError_t enter_device(int device)
{
    const hipError_t e = hipSetDevice(device);
    (void)hipGetLastError();
    return e;
}

struct qv_ctx_s {
    std::atomic<int> refs{1};   // the caller's reference plus one per live batch
    int device = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int engine = 0;             // 0: register tiles, 1: op-by-op LDS tiles, 2: one global pass per gate
    int tile_qubits = 0;        // 0: automatic
    int graph = 1;
    int n_vqpu = 0;             // 0: all circuits in flight
    int launch_events = 0;      // 1: record a HIP event pair around every launch (eager mode)
    int contig = 0;             // qubits 0..contig-1 always local (0: 4 for complex64, 3 for complex128)
    int autotune = 1;           // 0 off, 1 cached (use a stored choice), 2 search (time candidates once)
    int persistent = 0;         // 1: one persistent work-queue launch per direction instead of one per level
    int wait_ms = 4000;         // persistent launches: longest dependency wait
    int persist_chunk = 0;      // persistent launches: items a workgroup claims at once (0: the launcher's choice)
    int wait_extra = 0;         // persistent launches: added to every dependency count (tests of the time-out)
    int fuse_min = 0;           // >0: fuse runs of at least this many register-local gates into MFMA blocks
    int fold_cnots = 1;         // 1: CNOT runs at register-segment boundaries fold into the LDS addressing
    int specialize = 0;         // register-tiled levels of one pass run a kernel generated for that pass:
                                // bit 0 in forward sweeps, bit 1 in reverse (adjoint) sweeps, and with
                                // kSpecializeTimed only where timing shows it faster than the general one
    int inner_f64 = 0;          // 1: generated complex64 adjoint passes form their inner products in FP64
    hipStream_t stream() const { return user_stream; }  // NULL is the device's default stream
};

// A device buffer owned by a batch.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DBuf &operator=(DBuf &&o) noexcept
    {
        if (this != &o) {
            if (p) (void)hipFree(p);
            p = o.p; bytes = o.bytes;
            o.p = nullptr; o.bytes = 0;
        }
        return *this;
    }
    ~DBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t b)
    {
        if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
        if (b == 0) b = 8;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    template <typename T>
    hipError_t upload(const std::vector<T> &v)
    {
        hipError_t e = alloc(v.size() * sizeof(T));
        if (e != hipSuccess) return e;
        if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        return e;
    }
    template <typename T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

// LK_LAM: the tiles of a register-tiled reverse pass where psi is zero (lambda alone, k_rtile_lam)
enum LevelKind { LK_RTILE = 0, LK_TILE = 1, LK_STRIDE = 2, LK_LAM = 3 };

struct Level {
    int64_t seg_off;
    int32_t n_segs;
    int64_t n_blocks;
    int32_t lds_t;
    int32_t kind;     // LevelKind
    int64_t bytes;    // algorithmic state bytes moved by the launch (read + write)
    double flops;     // algorithmic floating-point operations of the launch (op_flops per amplitude)
    int32_t max_train;
    int32_t tab_bits; // largest (tile qubits - contiguous low qubits) of the level's passes
    void *gen = nullptr;  // register-tiled level of a single pass: the kernel generated for it, if any
};

// Algorithmic flops per amplitude of a gate, by what the gate's matrix needs, averaged over the two
// amplitudes of a pair: RX and RY mix a pair with real weights (two real-times-complex products and one
// complex add per output, 6); RZ (built as diag(1, e^{ia})) and T multiply one of the two by a phase (3);
// H adds and subtracts the pair and scales by a real (4); X, Y, Z, S, CNOT and CZ only move amplitudes or
// flip signs (0). Fused-block markers add nothing (their gates are counted).
static double op_flops(int kind)
{
    switch (kind) {
    case QV_RX: case QV_RY: return 6.0;
    case QV_H: return 4.0;
    case QV_RZ: case QV_T: return 3.0;
    default: return 0.0;
    }
}

// Per amplitude: forward applies each gate once; the adjoint un-applies it from psi and lambda and, per
// trainable gate, takes the imaginary part of one complex product per amplitude (4), or for RZ of the
// amplitudes with the gate's bit set only (2). The adjoint's sweep over a circuit's first register-tiled
// pass (last_rev) stops at its first trainable gate, so the gates below it count nothing.
static double pass_flops(const PlanPass &pp, bool adjoint, bool last_rev = false)
{
    size_t from = 0;
    if (adjoint && last_rev && !pp.segs.empty()) {
        from = pp.ops.size();
        for (size_t i = 0; i < pp.ops.size(); i++)
            if (pp.ops[i].kind != kFusedKind && pp.ops[i].train_slot >= 0) { from = i; break; }
    }
    double f = 0.0, inner = 0.0;
    for (size_t i = from; i < pp.ops.size(); i++) {
        f += op_flops(pp.ops[i].kind);
        if (adjoint && pp.ops[i].kind != kFusedKind && pp.ops[i].train_slot >= 0)
            inner += pp.ops[i].kind == QV_RZ ? 2.0 : 4.0;
    }
    return adjoint ? 2.0 * f + inner : f;
}

static int pass_kind(const PlanPass &pp)
{
    if (pp.stride) return LK_STRIDE;
    return pp.segs.empty() ? LK_TILE : LK_RTILE;
}

// Per-launch HIP event log (context option "launch_events"; eager launches only, no graph).
struct LaunchLog {
    std::vector<hipEvent_t> pool;
    std::vector<qv_launch_rec> recs;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    ~LaunchLog() { for (auto e : pool) (void)hipEventDestroy(e); }
    void clear() { recs.clear(); ev.clear(); used = 0; }
    hipEvent_t next()
    {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};

template <typename F>
static int logged(LaunchLog *log, hipStream_t s, int kernel, int level, int64_t bytes, F launch,
                  double flops = 0.0)
{
    if (!log) return launch();
    hipEvent_t a = log->next(), b = log->next();
    if (!a || !b) return launch();
    (void)hipEventRecord(a, s);
    int e = launch();
    (void)hipEventRecord(b, s);
    qv_launch_rec r;
    r.kernel = kernel;
    r.level = level;
    r.bytes = bytes;
    r.ms = 0.0;
    r.flops = flops;
    log->recs.push_back(r);
    log->ev.emplace_back(a, b);
    return e;
}

// Everything needed to run one set of device circuits (the batch itself, or a chunk of parameter-shift
// variants): per-circuit records, the launch levels, and the expectation / gradient reductions.
struct ExecSet {
    int n_circ = 0;
    std::vector<DevCirc> circs;
    std::vector<int> plan_of;                  // plan id per device circuit
    int64_t state_amps = 0;                    // amplitudes in this set's pool
    // forward and reverse levels
    std::vector<Seg> segs;
    std::vector<Level> fwd, rev;
    int64_t partial_count = 0;                 // adjoint partial sums
    // init
    std::vector<int64_t> init_first_block;
    int64_t init_blocks = 0;
    // expectation
    std::vector<DevGroup> groups;
    std::vector<DevTerm> terms;
    int64_t exp_blocks = 0;
    int64_t exp_partials = 0;
    std::vector<int64_t> tv_begin;
    std::vector<PartialRef> term_refs, norm_refs;
    std::vector<double> out_coeff;
    // adjoint seed
    std::vector<int64_t> lam_first_block, obs_begin;
    std::vector<DevObsTerm> obs;
    int64_t lam_blocks = 0;
    // gradient reduction
    std::vector<int64_t> gref_begin;
    std::vector<PartialRef> grefs;
    int64_t algo_bytes_fwd = 0, algo_bytes_rev = 0, passes_fwd = 0, passes_rev = 0;
    bool gen_ready[2] = {false, false};  // generated kernels looked up for the forward / reverse levels
    bool gen_timed[2] = {false, false};  // forward / reverse levels: generated or general kernel chosen by timing
    int64_t init_bytes = 0, exp_bytes = 0, lam_bytes = 0;

    // device copies
    DBuf d_circs, d_segs, d_init_fb, d_groups, d_terms, d_tv_begin, d_term_refs, d_norm_refs, d_coeff;
    DBuf d_lam_fb, d_obs_begin, d_obs, d_gref_begin, d_grefs;
    DBuf d_exp_partials, d_adj_partials;
    // parameter-shift variants: the matrix of each circuit's shifted gate, rebuilt from theta per call
    bool has_shift = false;
    DBuf d_smats;
    // persistent launches (one per direction), built when every level of the direction is register-tiled
    std::vector<PersistLevel> p_fwd, p_rev;
    int64_t p_fwd_items = 0, p_rev_items = 0;
    int p_fwd_ok = 0, p_rev_ok = 0;
    int32_t p_lds_t[2] = {0, 0}, p_tab_bits[2] = {0, 0}, p_max_train[2] = {0, 0};
    DBuf d_p_fwd, d_p_rev, d_p_head, d_p_done, d_p_error;
    // probability path: per-circuit block prefix and partial sums of diagonal-observable expectations
    std::vector<int64_t> diag_fb;
    DBuf d_diag_fb, d_diag_part;
};

// Device form of a batch's plans (shared by all its circuits and parameter-shift variants).
struct DevPlans {
    DBuf passes, ops, rsegs, fused_ops;
    std::vector<DevPass> h_passes;      // host copies (for generating specialised kernels)
    std::vector<DevOp> h_ops;
    std::vector<DevSeg> h_rsegs;
    std::vector<int> pass_base;
    std::vector<int64_t> op_count;      // ops per plan (fused-block markers included)
    std::vector<int64_t> fused_base;    // per plan: first entry in fused_ops
    std::vector<int64_t> fused_count;   // per plan: fused blocks
};

struct qv_batch_s {
    qv_ctx ctx = nullptr;
    int B = 0;
    qv_precision prec = QV_C64;
    int amp_bytes = 8;
    int stream_levels = 0;  // states total >= kStreamBatchBytes (LevelArgs::stream)
    int stream_expect = 0;  // largest state >= kStreamStateBytes (ExpArgs::stream)
    std::vector<int32_t> nq;
    std::vector<int64_t> goff;
    std::vector<qv_gate> gates;
    std::vector<int32_t> nparams;
    int params_shared = 0;
    int64_t n_theta = 0, n_grad = 0;
    std::vector<int64_t> toff;
    std::vector<uint64_t> xm, zm;
    std::vector<double> cf;
    int obs_shared = 0;
    int64_t n_tv = 0;

    std::vector<Plan> plans;
    std::vector<int> plan_of;          // per circuit
    int tile_qubits = 0;
    int contig = 0;
    std::unique_ptr<DevPlans> dp;
    int tuned = 0;                     // 1 once the autotuner (or its cache) has chosen the configuration
    int fuse_min = 0;                  // minimum run length of fused blocks in this batch's plans (0: none)

    ExecSet main;
    // parameter-shift chunks
    std::vector<std::unique_ptr<ExecSet>> ps_chunks;
    std::vector<int64_t> ps_chunk_var0;    // first variant index of each chunk
    int64_t n_occ = 0;
    std::vector<int64_t> occ_begin;
    std::vector<int32_t> occ_plus, occ_minus, occ_circ;
    bool ps_ready = false;

    DBuf d_gates, d_theta, d_psi, d_lam, d_energies, d_tv, d_norms, d_grad, d_upstream;
    DBuf d_state_phase, d_state_stage;  // qv_batch_state: the restoring phase; staging for host outputs
    DBuf d_gate_circ, d_mats;   // circuit of each matrix-table entry; 2x2 matrix of each circuit's plan ops
    DBuf d_fmats, d_fuse_fb;    // fused-block matrices; per-circuit block prefix for k_fuse
    int64_t n_mats = 0, n_fused = 0;
    DBuf d_ps_psi, d_ps_energies, d_ps_tv, d_occ_begin, d_occ_plus, d_occ_minus, d_occ_circ;

    bool theta_set = false;
    bool fwd_valid = false;

    // probability path: block prefix of the batch's circuits, output distributions, target distributions,
    // divergence weights dJS/dP_theta, divergence partial sums and values
    std::vector<int64_t> pfb;
    DBuf d_pfb, d_probs, d_target, d_w, d_js_part, d_js;
    DBuf d_slocal, d_bsum, d_boff, d_stotal, d_uni, d_samples, d_hist, d_nnz, d_noff, d_ndist, d_bits, d_counts;

    hipGraphExec_t g_fwd = nullptr, g_adj = nullptr, g_ps = nullptr, g_js_adj = nullptr, g_js_ps = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    LaunchLog log;
    qv_stats last{};
};

// ---------------------------------------------------------------------------------------------------------
// Validation (host only)
// ---------------------------------------------------------------------------------------------------------
static bool is_rotation(int k) { return k == QV_RX || k == QV_RY || k == QV_RZ; }
static bool is_two_qubit(int k) { return k == QV_CNOT || k == QV_CZ; }

static qv_status validate(int32_t B, const int32_t *nq, const int64_t *goff, const qv_gate *gates,
                          const int32_t *np, int32_t params_shared, const int64_t *toff, const uint64_t *xm,
                          const uint64_t *zm, const double *cf, int32_t obs_shared, qv_precision prec)
{
    if (B < 1) return fail(QV_E_INVALID, "n_circuits must be >= 1 (got %d)", B);
    if (!nq || !goff || !np || !toff) return fail(QV_E_INVALID, "n_qubits, gate_offsets, n_params and term_offsets must not be NULL");
    if (prec != QV_C64 && prec != QV_C128) return fail(QV_E_INVALID, "precision must be QV_C64 or QV_C128 (got %d)", (int)prec);
    if (goff[0] != 0) return fail(QV_E_INVALID, "gate_offsets[0] must be 0 (got %lld)", (long long)goff[0]);
    for (int b = 0; b < B; b++) {
        if (nq[b] < 1 || nq[b] > 34) return fail(QV_E_INVALID, "circuit %d: n_qubits must be in [1, 34] (got %d)", b, nq[b]);
        if (goff[b + 1] < goff[b]) return fail(QV_E_INVALID, "gate_offsets must be non-decreasing (circuit %d)", b);
        if (np[b] < 0) return fail(QV_E_INVALID, "circuit %d: n_params must be >= 0", b);
        if (params_shared && np[b] != np[0]) return fail(QV_E_INVALID, "params_shared requires equal n_params (circuit %d)", b);
    }
    if (goff[B] > 0 && !gates) return fail(QV_E_INVALID, "gates must not be NULL");
    for (int b = 0; b < B; b++) {
        const int n = nq[b];
        for (int64_t k = goff[b]; k < goff[b + 1]; k++) {
            const qv_gate &g = gates[k];
            const long long kl = (long long)(k - goff[b]);
            if (g.kind < QV_H || g.kind > QV_CZ) return fail(QV_E_INVALID, "circuit %d gate %lld: unknown kind %d", b, kl, g.kind);
            if (g.q0 < 0 || g.q0 >= n) return fail(QV_E_INVALID, "circuit %d gate %lld: qubit %d out of range [0, %d)", b, kl, g.q0, n);
            if (is_two_qubit(g.kind)) {
                if (g.q1 < 0 || g.q1 >= n) return fail(QV_E_INVALID, "circuit %d gate %lld: qubit %d out of range [0, %d)", b, kl, g.q1, n);
                if (g.q1 == g.q0) return fail(QV_E_INVALID, "circuit %d gate %lld: both qubits are %d", b, kl, g.q0);
            }
            if (is_rotation(g.kind)) {
                if (g.param < -1 || g.param >= np[b])
                    return fail(QV_E_INVALID, "circuit %d gate %lld: param %d out of range [-1, %d)", b, kl, g.param, np[b]);
                if (g.param == -1 && !std::isfinite(g.angle))
                    return fail(QV_E_INVALID, "circuit %d gate %lld: non-finite angle", b, kl);
            } else if (g.param != -1) {
                return fail(QV_E_INVALID, "circuit %d gate %lld: only RX/RY/RZ take a parameter", b, kl);
            }
        }
    }
    const int nto = obs_shared ? 1 : B;
    if (toff[0] < 0) return fail(QV_E_INVALID, "term_offsets[0] must be >= 0");
    for (int i = 0; i < nto; i++)
        if (toff[i + 1] < toff[i]) return fail(QV_E_INVALID, "term_offsets must be non-decreasing");
    const int64_t tt = toff[nto];
    if (tt > toff[0] && (!xm || !zm || !cf)) return fail(QV_E_INVALID, "xmask, zmask and coeff must not be NULL");
    for (int b = 0; b < B; b++) {
        const int64_t t0 = obs_shared ? toff[0] : toff[b], t1 = obs_shared ? toff[1] : toff[b + 1];
        const uint64_t lim = nq[b] >= 64 ? ~0ull : ((1ull << nq[b]) - 1ull);
        for (int64_t t = t0; t < t1; t++) {
            if ((xm[t] & ~lim) || (zm[t] & ~lim))
                return fail(QV_E_INVALID, "term %lld has a qubit outside circuit %d's %d qubits", (long long)t, b, nq[b]);
            if (!std::isfinite(cf[t])) return fail(QV_E_INVALID, "term %lld: non-finite coefficient", (long long)t);
        }
    }
    return QV_OK;
}

// ---------------------------------------------------------------------------------------------------------
// ExecSet construction
// ---------------------------------------------------------------------------------------------------------
static int64_t tiles_of(const DevCirc &c, const Plan &pl, int p)
{
    const PlanPass &pp = pl.passes[p];
    if (pp.stride) {
        const int k = pp.t;
        const int64_t groups = (int64_t)1 << (c.n - k);
        return (groups + kStrideGroupsPerBlock - 1) / kStrideGroupsPerBlock;
    }
    return (int64_t)1 << (c.n - pp.t);
}

// Tiles a forward launch runs for pass p of circuit c. A register-tiled pass after the circuit's first
// leaves out the tiles with a qubit of its zero mask at 1: they hold the zeros earlier passes wrote
// (rtile_body numbers the rest first). zero: pass_zero_masks of the circuit's plan.
static int64_t fwd_tiles(const DevCirc &c, const Plan &pl, int p, const std::vector<uint64_t> &zero)
{
    const PlanPass &pp = pl.passes[p];
    if (p == 0 || pass_kind(pp) != LK_RTILE) return tiles_of(c, pl, p);
    const uint64_t full = c.n >= 64 ? ~0ull : ((1ull << c.n) - 1ull);
    const uint64_t outside = full & ~pp.local_mask;
    return (int64_t)1 << __builtin_popcountll(outside & ~zero[(size_t)p]);
}

// Builds the launch levels (forward and reverse) and the adjoint partial-sum layout of a set.
// Circuits are launched in waves of at most `wave` circuits; every wave runs all its levels before the
// next wave starts. Results do not depend on the wave size.
static void build_levels(ExecSet &es, const std::vector<Plan> &plans, const std::vector<int> &pass_base, int wave,
                         int amp_bytes, bool split_zero = false)
{
    es.gen_ready[0] = es.gen_ready[1] = false;
    es.gen_timed[0] = es.gen_timed[1] = false;
    es.segs.clear(); es.fwd.clear(); es.rev.clear();
    es.partial_count = 0;
    es.algo_bytes_fwd = es.algo_bytes_rev = es.passes_fwd = es.passes_rev = 0;
    const int N = es.n_circ;
    if (wave <= 0 || wave > N) wave = N;
    // zero masks per plan
    std::vector<std::vector<uint64_t>> zero(plans.size());
    for (size_t i = 0; i < plans.size(); i++) zero[i] = pass_zero_masks(plans[i]);
    // partial bases per (circuit, pass)
    std::vector<std::vector<int64_t>> pbase(N);
    for (int c = 0; c < N; c++) {
        const Plan &pl = plans[es.plan_of[c]];
        pbase[c].resize(pl.passes.size());
        const int64_t S = ((int64_t)1 << es.circs[c].n) * amp_bytes;
        for (size_t p = 0; p < pl.passes.size(); p++) {
            pbase[c][p] = es.partial_count;
            es.partial_count += tiles_of(es.circs[c], pl, (int)p) * pl.passes[p].n_train;
            // the tiles a forward pass leaves out are neither read nor written
            es.algo_bytes_fwd += 2 * S / tiles_of(es.circs[c], pl, (int)p) *
                                 fwd_tiles(es.circs[c], pl, (int)p, zero[(size_t)es.plan_of[c]]);
        }
        es.algo_bytes_rev += 4 * S * (int64_t)pl.passes.size();
        es.passes_fwd += (int64_t)pl.passes.size();
        es.passes_rev += (int64_t)pl.passes.size();
    }
    // One launch per (depth, kernel kind): passes of the same depth that need different kernels (register
    // tiles, op-by-op LDS tiles for tiny tiles, stride passes) go to separate launches of that depth.
    for (int w0 = 0; w0 < N; w0 += wave) {
        const int w1 = std::min(N, w0 + wave);
        int maxp = 0;
        for (int c = w0; c < w1; c++) maxp = std::max(maxp, (int)plans[es.plan_of[c]].passes.size());
        for (int dir = 0; dir < 2; dir++) {
            for (int L = 0; L < maxp; L++) {
                for (int kind = 0; kind < 4; kind++) {
                    Level lv{(int64_t)es.segs.size(), 0, 0, 0, kind, 0, 0.0, 0, 0};
                    for (int c = w0; c < w1; c++) {
                        const Plan &pl = plans[es.plan_of[c]];
                        const int np = (int)pl.passes.size();
                        if (L >= np) continue;
                        const int p = dir == 0 ? L : np - 1 - L;
                        const PlanPass &pp = pl.passes[p];
                        const std::vector<uint64_t> &zm = zero[(size_t)es.plan_of[c]];
                        // a register-tiled reverse pass after the circuit's first, with tiles where psi is
                        // zero: those (numbered last) go to the LK_LAM launch of its depth
                        const int64_t all = tiles_of(es.circs[c], pl, p);
                        const int64_t live = dir == 1 && split_zero && p > 0 && pass_kind(pp) == LK_RTILE
                                                 ? fwd_tiles(es.circs[c], pl, p, zm) : all;
                        if (kind == LK_LAM ? live == all : pass_kind(pp) != kind) continue;
                        Seg s;
                        s.first_block = lv.n_blocks;
                        s.partial_base = pbase[c][p];
                        s.circ = c;
                        s.pass = pass_base[es.plan_of[c]] + p;
                        s.first = (dir == 0 && p == 0 && !pp.stride) ? 1 : 0;
                        s.last = (dir == 1 && p == 0) ? 1 : 0;
                        s.wait = 0;
                        s.tile_off = kind == LK_LAM ? live : 0;
                        if (dir == 0) {
                            for (int q = 0; q < p; q++) s.wait += fwd_tiles(es.circs[c], pl, q, zm);
                        } else {
                            for (int q = p + 1; q < np; q++) s.wait += tiles_of(es.circs[c], pl, q);
                        }
                        es.segs.push_back(s);
                        lv.n_segs++;
                        const int64_t run = dir == 0 ? fwd_tiles(es.circs[c], pl, p, zm)
                                                     : (kind == LK_LAM ? all - live : live);
                        lv.n_blocks += run;
                        lv.lds_t = std::max(lv.lds_t, pp.t);
                        lv.max_train = std::max(lv.max_train, pp.n_train);
                        lv.tab_bits = std::max(lv.tab_bits, pp.t - pp.lowc);
                        // forward: read + write (first pass: write only); adjoint: psi and lambda read + write
                        // (the circuit's last reverse pass: read only). Register-tiled first passes compute
                        // only tile 0 (rtile_body): the forward writes the other tiles' zeros, the adjoint
                        // leaves them alone.
                        const int64_t S = ((int64_t)1 << es.circs[c].n) * amp_bytes;
                        const bool rt = pass_kind(pp) == LK_RTILE;
                        const int64_t work = (rt && p == 0) ? 1 : run;
                        // LK_LAM: lambda alone read, undone once and written
                        lv.bytes += dir == 0 ? (s.first ? S : 2 * (S / all) * run)
                                             : (s.last ? 2 * (S / all) * work
                                                       : (kind == LK_LAM ? 2 : 4) * (S / all) * run);
                        lv.flops += pass_flops(pp, dir == 1 && kind != LK_LAM, s.last != 0) *
                                    (double)((int64_t)1 << es.circs[c].n) * ((double)work / (double)all);
                    }
                    if (lv.n_segs) (dir == 0 ? es.fwd : es.rev).push_back(lv);
                }
            }
        }
    }
    // |0...0> is written by k_init only for circuits whose first pass does not generate it
    es.init_first_block.assign(N + 1, 0);
    es.init_bytes = 0;
    for (int c = 0; c < N; c++) {
        const Plan &pl = plans[es.plan_of[c]];
        const bool needs = pl.passes.empty() || pl.passes[0].stride;
        const int64_t amps = (int64_t)1 << es.circs[c].n;
        es.init_first_block[c + 1] = es.init_first_block[c] + (needs ? (amps + 4095) / 4096 : 0);
        if (needs) es.init_bytes += amps * amp_bytes;
    }
    es.init_blocks = es.init_first_block[N];
    for (int dir = 0; dir < 2; dir++) {
        const std::vector<Level> &lvs = dir == 0 ? es.fwd : es.rev;
        std::vector<PersistLevel> &pl = dir == 0 ? es.p_fwd : es.p_rev;
        int64_t items = 0;
        int ok = 1;
        pl.clear();
        es.p_lds_t[dir] = es.p_tab_bits[dir] = es.p_max_train[dir] = 0;
        for (const Level &lv : lvs) {
            if (lv.kind != LK_RTILE) ok = 0;
            PersistLevel p;
            p.first_item = items;
            p.seg_off = lv.seg_off;
            p.n_segs = lv.n_segs;
            p.pad = 0;
            pl.push_back(p);
            items += lv.n_blocks;
            es.p_lds_t[dir] = std::max(es.p_lds_t[dir], lv.lds_t);
            es.p_tab_bits[dir] = std::max(es.p_tab_bits[dir], lv.tab_bits);
            es.p_max_train[dir] = std::max(es.p_max_train[dir], lv.max_train);
        }
        (dir == 0 ? es.p_fwd_items : es.p_rev_items) = items;
        ok = ok && !lvs.empty() &&
             persistent_fits(amp_bytes == 8 ? QV_C64 : QV_C128, dir, es.p_lds_t[dir], es.p_tab_bits[dir],
                             es.p_max_train[dir]);
        (dir == 0 ? es.p_fwd_ok : es.p_rev_ok) = ok;
    }
    es.algo_bytes_fwd = es.init_bytes;
    for (const Level &lv : es.fwd) es.algo_bytes_fwd += lv.bytes;
}

struct ObsView {
    const int64_t *toff;
    const uint64_t *xm, *zm;
    const double *cf;
    int obs_shared;
};

// Expectation work items of a set. Terms of a circuit are grouped by x-mask (first appearance order),
// each group split into items of at most kMaxGroupTerms terms; an identity term carries the norm.
// out_base[c] is the first output slot of device circuit c; obs_of[c] the batch circuit whose terms it uses.
static void build_expectation(ExecSet &es, const ObsView &ov, const std::vector<int> &obs_of,
                              const std::vector<int64_t> &out_base, int64_t n_out, bool with_norm, int amp_bytes)
{
    es.exp_bytes = 0;
    es.groups.clear(); es.terms.clear(); es.term_refs.assign(n_out, PartialRef{0, 0, 1});
    es.norm_refs.assign(es.n_circ, PartialRef{0, 0, 1});
    es.out_coeff.assign(n_out, 0.0);
    es.tv_begin.assign(es.n_circ + 1, 0);
    es.exp_blocks = 0;
    es.exp_partials = 0;
    for (int c = 0; c < es.n_circ; c++) {
        const int b = obs_of[c];
        const int n = es.circs[c].n;
        const int64_t t0 = ov.obs_shared ? ov.toff[0] : ov.toff[b];
        const int64_t t1 = ov.obs_shared ? ov.toff[1] : ov.toff[b + 1];
        es.tv_begin[c] = out_base[c];
        es.tv_begin[c + 1] = out_base[c] + (t1 - t0);
        // group terms by xmask; -1 marks the norm
        std::vector<uint64_t> gx;
        std::vector<std::vector<int64_t>> gt;
        std::unordered_map<uint64_t, int> gi;
        auto add = [&](uint64_t x, int64_t t) {
            auto it = gi.find(x);
            int id;
            if (it == gi.end()) { id = (int)gx.size(); gi[x] = id; gx.push_back(x); gt.emplace_back(); }
            else id = it->second;
            gt[id].push_back(t);
        };
        for (int64_t t = t0; t < t1; t++) add(ov.xm[t], t);
        if (with_norm) add(0, -1);
        for (size_t g = 0; g < gx.size(); g++) {
            const uint64_t x = gx[g];
            const int clog = std::min(kExpChunkLog2, x ? n - 1 : n);
            const int64_t items = x ? ((int64_t)1 << (n - 1)) : ((int64_t)1 << n);
            const int64_t nchunks = std::max<int64_t>(1, items >> clog);
            for (size_t j0 = 0; j0 < gt[g].size(); j0 += kMaxGroupTerms) {
                const int nt = (int)std::min<size_t>(kMaxGroupTerms, gt[g].size() - j0);
                DevGroup G;
                G.xmask = x;
                G.first_block = es.exp_blocks;
                G.partial_base = es.exp_partials;
                G.circ = c;
                G.n_terms = nt;
                G.term_begin = (int32_t)es.terms.size();
                G.chunk_log2 = clog;
                for (int j = 0; j < nt; j++) {
                    const int64_t t = gt[g][j0 + j];
                    const uint64_t z = t >= 0 ? ov.zm[t] : 0;
                    DevTerm dt;
                    dt.zmask = z;
                    dt.ny = __builtin_popcountll(x & z) & 3;
                    dt.pad = 0;
                    es.terms.push_back(dt);
                    PartialRef r{G.partial_base + j, (int32_t)nchunks, nt};
                    if (t >= 0) {
                        const int64_t o = out_base[c] + (t - t0);
                        es.term_refs[o] = r;
                        es.out_coeff[o] = ov.cf[t];
                    } else {
                        es.norm_refs[c] = r;
                    }
                }
                es.groups.push_back(G);
                es.exp_blocks += nchunks;
                es.exp_bytes += ((int64_t)1 << n) * amp_bytes;
                es.exp_partials += nchunks * nt;
            }
        }
    }
}

static void build_lambda(ExecSet &es, const ObsView &ov, const std::vector<int> &obs_of, int amp_bytes)
{
    es.lam_bytes = 0;
    es.lam_first_block.assign(es.n_circ + 1, 0);
    es.obs_begin.assign(es.n_circ + 1, 0);
    es.obs.clear();
    for (int c = 0; c < es.n_circ; c++) {
        const int b = obs_of[c];
        const int64_t t0 = ov.obs_shared ? ov.toff[0] : ov.toff[b];
        const int64_t t1 = ov.obs_shared ? ov.toff[1] : ov.toff[b + 1];
        // terms ordered by x-mask (stable), so that k_lambda reads psi[o ^ x] once per distinct mask
        std::vector<int64_t> order;
        for (int64_t t = t0; t < t1; t++) order.push_back(t);
        std::stable_sort(order.begin(), order.end(), [&](int64_t u, int64_t v) { return ov.xm[u] < ov.xm[v]; });
        for (int64_t t : order) {
            DevObsTerm o;
            o.xmask = ov.xm[t];
            o.zmask = ov.zm[t];
            o.coeff = ov.cf[t];
            o.ny = __builtin_popcountll(ov.xm[t] & ov.zm[t]) & 3;
            o.pad = 0;
            es.obs.push_back(o);
        }
        es.obs_begin[c + 1] = (int64_t)es.obs.size();
        es.lam_bytes += (1 + (t1 - t0)) * (((int64_t)1 << es.circs[c].n) * amp_bytes);
        es.lam_first_block[c + 1] = es.lam_first_block[c] + ((((int64_t)1 << es.circs[c].n) + 4095) / 4096);
    }
    es.lam_blocks = es.lam_first_block[es.n_circ];
}

// Gradient references: for output g, every trainable gate occurrence that reads it.
static void build_grad_refs(ExecSet &es, const qv_batch_s &bt, const std::vector<int> &pass_base)
{
    (void)pass_base;
    std::vector<std::vector<PartialRef>> per(bt.n_grad);
    // reconstruct partial bases in the same order as build_levels
    int64_t base = 0;
    for (int c = 0; c < es.n_circ; c++) {
        const Plan &pl = bt.plans[es.plan_of[c]];
        const int b = es.circs[c].base_circ;
        for (size_t p = 0; p < pl.passes.size(); p++) {
            const PlanPass &pp = pl.passes[p];
            const int64_t tiles = tiles_of(es.circs[c], pl, (int)p);
            for (const PlanOp &op : pp.ops) {
                if (op.train_slot < 0) continue;
                const qv_gate &g = bt.gates[bt.goff[b] + op.gate];
                int64_t out = g.param;
                if (!bt.params_shared) {
                    int64_t pb = 0;
                    for (int i = 0; i < b; i++) pb += bt.nparams[i];
                    out += pb;
                }
                per[out].push_back(PartialRef{base + op.train_slot, (int32_t)tiles, pp.n_train});
            }
            base += tiles * pp.n_train;
        }
    }
    es.gref_begin.assign(bt.n_grad + 1, 0);
    es.grefs.clear();
    for (int64_t g = 0; g < bt.n_grad; g++) {
        for (auto &r : per[g]) es.grefs.push_back(r);
        es.gref_begin[g + 1] = (int64_t)es.grefs.size();
    }
}

static hipError_t upload_set(ExecSet &es, bool adjoint_parts)
{
    hipError_t e;
    if ((e = es.d_circs.upload(es.circs)) != hipSuccess) return e;
    if ((e = es.d_segs.upload(es.segs)) != hipSuccess) return e;
    if ((e = es.d_init_fb.upload(es.init_first_block)) != hipSuccess) return e;
    if ((e = es.d_groups.upload(es.groups)) != hipSuccess) return e;
    if ((e = es.d_terms.upload(es.terms)) != hipSuccess) return e;
    if ((e = es.d_tv_begin.upload(es.tv_begin)) != hipSuccess) return e;
    if ((e = es.d_term_refs.upload(es.term_refs)) != hipSuccess) return e;
    if ((e = es.d_norm_refs.upload(es.norm_refs)) != hipSuccess) return e;
    if ((e = es.d_coeff.upload(es.out_coeff)) != hipSuccess) return e;
    if ((e = es.d_exp_partials.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, es.exp_partials))) != hipSuccess) return e;
    if ((e = es.d_p_fwd.upload(es.p_fwd)) != hipSuccess) return e;
    if ((e = es.d_p_rev.upload(es.p_rev)) != hipSuccess) return e;
    if ((e = es.d_p_head.alloc(sizeof(unsigned long long))) != hipSuccess) return e;
    if ((e = es.d_p_done.alloc(sizeof(unsigned long long) * (size_t)std::max(1, es.n_circ))) != hipSuccess) return e;
    if ((e = es.d_p_error.alloc(sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMemset(es.d_p_error.p, 0, sizeof(int32_t))) != hipSuccess) return e;
    if (adjoint_parts) {
        if ((e = es.d_lam_fb.upload(es.lam_first_block)) != hipSuccess) return e;
        if ((e = es.d_obs_begin.upload(es.obs_begin)) != hipSuccess) return e;
        if ((e = es.d_obs.upload(es.obs)) != hipSuccess) return e;
        if ((e = es.d_gref_begin.upload(es.gref_begin)) != hipSuccess) return e;
        if ((e = es.d_grefs.upload(es.grefs)) != hipSuccess) return e;
        if ((e = es.d_adj_partials.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, es.partial_count))) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------------------------------------
// Launch sequences
// ---------------------------------------------------------------------------------------------------------


static LevelArgs level_args(const qv_batch_s &bt, const ExecSet &es, const DevPlans &dp, const Level &lv,
                            void *psi, void *lam)
{
    LevelArgs a;
    a.segs = es.d_segs.as<Seg>() + lv.seg_off;
    a.n_segs = lv.n_segs;
    a.lds_t = lv.lds_t;
    a.n_blocks = lv.n_blocks;
    a.passes = dp.passes.as<DevPass>();
    a.ops = dp.ops.as<DevOp>();
    a.circs = es.d_circs.as<DevCirc>();
    a.gates = bt.d_gates.as<qv_gate>();
    a.theta = bt.d_theta.as<double>();
    a.mats = bt.d_mats.p;
    a.smats = es.d_smats.p;
    a.fmats = bt.d_fmats.as<float>();
    a.psi = psi;
    a.lam = lam;
    a.partials = es.d_adj_partials.as<double>();
    a.rsegs = dp.rsegs.as<DevSeg>();
    a.max_train = lv.max_train;
    a.tab_bits = lv.tab_bits;
    a.chunk = 0;
    a.stream = bt.stream_levels;
    return a;
}

static int launch_kind(const Level &lv, const LevelArgs &a, int prec, int adjoint, hipStream_t s)
{
    if (lv.kind == LK_STRIDE) return launch_stride_level(a, prec, adjoint, s);
    if (lv.kind == LK_LAM) return launch_rlevel_lam(a, prec, s);
    if (lv.kind == LK_RTILE && lv.gen) return launch_rlevel_gen(a, adjoint, lv.gen, s);
    if (lv.kind == LK_RTILE) return launch_rlevel(a, prec, adjoint, s);
    return launch_level(a, prec, adjoint, s);
}

static int log_id(const Level &lv, int adjoint)
{
    if (lv.kind == LK_STRIDE) return adjoint ? QV_K_STRIDE_ADJ : QV_K_STRIDE;
    if (lv.kind == LK_LAM) return QV_K_RTILE_LAM;
    if (lv.kind == LK_RTILE && lv.gen) return adjoint ? QV_K_RTILE_ADJ_GEN : QV_K_RTILE_GEN;
    if (lv.kind == LK_RTILE) return adjoint ? QV_K_RTILE_ADJ : QV_K_RTILE;
    return adjoint ? QV_K_TILE_ADJ : QV_K_TILE;
}

// Kernels generated for the register-tiled levels of one direction of an execution set: a level whose
// segments all run one plan pass gets a kernel with that pass's ops as straight-line code (compiled once
// per distinct pass, cached). Runs before any graph capture; the autotuner's timing runs leave it out.
static qv_status ensure_generated(qv_batch_s *bt, ExecSet &es, int dir)
{
    if (!(bt->ctx->specialize >> dir & 1) || es.gen_ready[dir]) return QV_OK;
    std::vector<Level> &lvs = dir ? es.rev : es.fwd;
    const DevPlans &dp = *bt->dp;
    std::vector<std::string> srcs;
    std::vector<size_t> level_of;
    for (size_t L = 0; L < lvs.size(); L++) {
        Level &lv = lvs[L];
        lv.gen = nullptr;
        if (lv.kind != LK_RTILE || lv.n_segs <= 0) continue;
        const int pass = es.segs[(size_t)lv.seg_off].pass;
        bool one = true;
        for (int i = 1; i < lv.n_segs && one; i++) one = es.segs[(size_t)lv.seg_off + i].pass == pass;
        if (!one) continue;
        GenPassDesc d;
        d.pass = dp.h_passes[(size_t)pass];
        d.segs.assign(dp.h_rsegs.begin() + d.pass.seg_begin, dp.h_rsegs.begin() + d.pass.seg_begin + d.pass.n_seg);
        d.ops.assign(dp.h_ops.begin() + d.pass.op_begin, dp.h_ops.begin() + d.pass.op_begin + d.pass.n_ops);
        d.precision = bt->prec;
        d.adjoint = dir;
        d.lds_t = lv.lds_t;
        d.tab_bits = lv.tab_bits;
        d.max_train = lv.max_train;
        d.inner_f64 = bt->ctx->inner_f64;
        srcs.push_back(gen_pass_source(d));
        level_of.push_back(L);
    }
    std::vector<void *> fns;
    std::string err;
    const int e = gen_kernels(srcs, fns, err);
    if (e) return fail(QV_E_DEVICE, "%s", err.empty() ? hipGetErrorString((hipError_t)e) : err.c_str());
    for (size_t i = 0; i < level_of.size(); i++) lvs[level_of[i]].gen = fns[i];
    es.gen_ready[dir] = true;
    return QV_OK;
}

static int enqueue_matrices(const qv_batch_s &bt, hipStream_t s, LaunchLog *log)
{
    MatArgs ma;
    ma.gates = bt.d_gates.as<qv_gate>();
    ma.gate_circ = bt.d_gate_circ.as<int32_t>();
    ma.ops = bt.dp->ops.as<DevOp>();
    ma.circs = bt.main.d_circs.as<DevCirc>();
    ma.theta = bt.d_theta.as<double>();
    ma.mats = bt.d_mats.p;
    ma.n_gates = bt.n_mats;
    int e = logged(log, s, QV_K_MATRICES, -1, 0, [&] { return launch_matrices(ma, bt.prec, s); });
    if (e || bt.n_fused == 0) return e;
    FuseArgs fa;
    fa.ops = bt.dp->ops.as<DevOp>();
    fa.circs = bt.main.d_circs.as<DevCirc>();
    fa.first_block = bt.d_fuse_fb.as<int64_t>();
    fa.n_circ = bt.B;
    fa.pad = 0;
    fa.fused_ops = bt.dp->fused_ops.as<int64_t>();
    fa.mats = bt.d_mats.p;
    fa.fmats = bt.d_fmats.as<float>();
    fa.n_blocks = bt.n_fused;
    return logged(log, s, QV_K_FUSE, -1, 0, [&] { return launch_fuse(fa, s); });
}

// Longest dependency wait of a persistent launch in ticks of the device's constant-rate wall clock (default
// 4 s: a pass over the largest state that fits takes well under a second).
static int64_t wait_ticks(int device, int ms)
{
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
    return (int64_t)khz * ms;
}

// One persistent launch for all levels of a direction (see k_rtile_*_persist).
static int enqueue_persistent(const qv_batch_s &bt, ExecSet &es, const DevPlans &dp, int dir, void *psi, void *lam,
                              hipStream_t s, LaunchLog *log)
{
    const std::vector<Level> &lvs = dir == 0 ? es.fwd : es.rev;
    int e = launch_zero_u64(es.d_p_head.as<unsigned long long>(), 1, s);
    if (!e) e = launch_zero_u64(es.d_p_done.as<unsigned long long>(), es.n_circ, s);
    if (e) return e;
    PersistArgs pa;
    pa.base = level_args(bt, es, dp, lvs[0], psi, lam);
    pa.base.segs = es.d_segs.as<Seg>();
    pa.base.lds_t = es.p_lds_t[dir];
    pa.base.tab_bits = es.p_tab_bits[dir];
    pa.base.max_train = es.p_max_train[dir];
    pa.levels = (dir == 0 ? es.d_p_fwd : es.d_p_rev).as<PersistLevel>();
    pa.n_levels = (int32_t)lvs.size();
    pa.chunk = bt.ctx->persist_chunk;
    pa.n_items = dir == 0 ? es.p_fwd_items : es.p_rev_items;
    pa.head = es.d_p_head.as<unsigned long long>();
    pa.done = es.d_p_done.as<unsigned long long>();
    pa.error = es.d_p_error.as<int32_t>();
    pa.wait_ticks = wait_ticks(bt.ctx->device, bt.ctx->wait_ms);
    pa.wait_extra = bt.ctx->wait_extra;
    int64_t bytes = 0;
    double flops = 0.0;
    for (const Level &lv : lvs) { bytes += lv.bytes; flops += lv.flops; }
    return logged(log, s, dir == 0 ? QV_K_RTILE_PERSIST : QV_K_RTILE_ADJ_PERSIST, -1, bytes,
                  [&] { return launch_persistent(pa, bt.prec, dir, s); }, flops);
}

static int enqueue_forward(const qv_batch_s &bt, ExecSet &es, const DevPlans &dp, void *psi, double *energies,
                           double *tv, double *norms, hipStream_t s, LaunchLog *log, double *partials = nullptr)
{
    if (!partials) partials = es.d_exp_partials.as<double>();
    int e = logged(log, s, QV_K_INIT, -1, es.init_bytes, [&] {
        return launch_init_states(psi, es.d_circs.as<DevCirc>(), es.d_init_fb.as<int64_t>(), es.n_circ,
                                  es.init_blocks, bt.prec, s);
    });
    if (e) return e;
    if (es.has_shift) {
        ShiftMatArgs sa;
        sa.circs = es.d_circs.as<DevCirc>();
        sa.gates = bt.d_gates.as<qv_gate>();
        sa.theta = bt.d_theta.as<double>();
        sa.smats = es.d_smats.p;
        sa.n_circ = es.n_circ;
        e = logged(log, s, QV_K_MATRICES, -1, 0, [&] { return launch_shift_matrices(sa, bt.prec, s); });
        if (e) return e;
    }
    if (bt.ctx->persistent && es.p_fwd_ok) {
        e = enqueue_persistent(bt, es, dp, 0, psi, nullptr, s, log);
        if (e) return e;
    } else {
        for (size_t L = 0; L < es.fwd.size(); L++) {
            const Level &lv = es.fwd[L];
            LevelArgs a = level_args(bt, es, dp, lv, psi, nullptr);
            e = logged(log, s, log_id(lv, 0), (int)L, lv.bytes, [&] { return launch_kind(lv, a, bt.prec, 0, s); },
                       lv.flops);
            if (e) return e;
        }
    }
    ExpArgs ea;
    ea.groups = es.d_groups.as<DevGroup>();
    ea.n_groups = (int32_t)es.groups.size();
    ea.stream = bt.stream_expect;
    ea.n_blocks = es.exp_blocks;
    ea.terms = es.d_terms.as<DevTerm>();
    ea.circs = es.d_circs.as<DevCirc>();
    ea.psi = psi;
    ea.partials = partials;
    e = logged(log, s, QV_K_EXPECT, -1, es.exp_bytes, [&] { return launch_expectation(ea, bt.prec, s); });
    if (e) return e;
    FinalizeArgs fa;
    fa.n_circ = es.n_circ;
    fa.n_terms = (int64_t)es.term_refs.size();
    fa.tv_begin = es.d_tv_begin.as<int64_t>();
    fa.term_refs = es.d_term_refs.as<PartialRef>();
    fa.coeff = es.d_coeff.as<double>();
    fa.norm_refs = norms ? es.d_norm_refs.as<PartialRef>() : nullptr;
    fa.partials = partials;
    fa.term_values = tv;
    fa.energies = energies;
    fa.norms = norms;
    return logged(log, s, QV_K_FINALIZE, -1, 0, [&] { return launch_finalize(fa, s); });
}

static int enqueue_reverse(const qv_batch_s &bt, ExecSet &es, const DevPlans &dp, hipStream_t s, LaunchLog *log);

static int enqueue_adjoint(const qv_batch_s &bt, ExecSet &es, const DevPlans &dp, hipStream_t s, LaunchLog *log)
{
    LambdaArgs la;
    la.circs = es.d_circs.as<DevCirc>();
    la.n_circ = es.n_circ;
    la.first_block = es.d_lam_fb.as<int64_t>();
    la.obs_begin = es.d_obs_begin.as<int64_t>();
    la.obs = es.d_obs.as<DevObsTerm>();
    la.upstream = bt.d_upstream.as<double>();
    la.psi = bt.d_psi.p;
    la.lam = bt.d_lam.p;
    la.n_blocks = es.lam_blocks;
    const int e = logged(log, s, QV_K_LAMBDA, -1, es.lam_bytes, [&] { return launch_lambda(la, bt.prec, s); });
    if (e) return e;
    return enqueue_reverse(bt, es, dp, s, log);
}

// The reverse sweep from seeded psi and lambda, then the gradient reduction.
static int enqueue_reverse(const qv_batch_s &bt, ExecSet &es, const DevPlans &dp, hipStream_t s, LaunchLog *log)
{
    int e = 0;
    if (bt.ctx->persistent && es.p_rev_ok) {
        e = enqueue_persistent(bt, es, dp, 1, bt.d_psi.p, bt.d_lam.p, s, log);
        if (e) return e;
    } else {
        for (size_t L = 0; L < es.rev.size(); L++) {
            const Level &lv = es.rev[L];
            LevelArgs a = level_args(bt, es, dp, lv, bt.d_psi.p, bt.d_lam.p);
            e = logged(log, s, log_id(lv, 1), (int)L, lv.bytes, [&] { return launch_kind(lv, a, bt.prec, 1, s); },
                       lv.flops);
            if (e) return e;
        }
    }
    GradReduceArgs ga;
    ga.n_out = (int32_t)bt.n_grad;
    ga.ref_begin = es.d_gref_begin.as<int64_t>();
    ga.refs = es.d_grefs.as<PartialRef>();
    ga.partials = es.d_adj_partials.as<double>();
    ga.grad = bt.d_grad.as<double>();
    return logged(log, s, QV_K_GRAD_REDUCE, -1, 0, [&] { return launch_grad_reduce(ga, s); });
}

// "specialize": "auto": sweeps of one direction alternately with the general kernels and with the generated
// ones (kTimingSweeps in all, eager, with per-launch events), then every level of that direction keeps the
// kernel with the lower of its two times. `sweep` enqueues one timed sweep and logs the levels of direction
// `dir` (a reverse sweep runs after its own forward pass, whose levels keep their kernels). Once per
// execution set and direction; it leaves no valid final states behind.
template <class Sweep>
static qv_status time_generated(qv_batch_s *bt, ExecSet &es, int dir, Sweep &&sweep)
{
    if (!(bt->ctx->specialize & kSpecializeTimed) || es.gen_timed[dir] || bt->ctx->persistent) return QV_OK;
    es.gen_timed[dir] = true;
    std::vector<Level> &lvs = dir ? es.rev : es.fwd;
    std::vector<void *> gens;
    bool any = false;
    for (const Level &lv : lvs) {
        gens.push_back(lv.gen);
        any |= lv.gen != nullptr;
    }
    if (!any) return QV_OK;
    const int k_general = dir ? QV_K_RTILE_ADJ : QV_K_RTILE, k_gen = dir ? QV_K_RTILE_ADJ_GEN : QV_K_RTILE_GEN;
    hipStream_t s = bt->ctx->stream();
    std::vector<double> ms[2];
    ms[0].assign(lvs.size(), 1e300);
    ms[1].assign(lvs.size(), 1e300);
    for (int run = 0; run < kTimingSweeps; run++) {
        const int variant = run & 1;
        for (size_t L = 0; L < lvs.size(); L++) lvs[L].gen = variant ? gens[L] : nullptr;
        LaunchLog log;
        const int e = sweep(s, &log);
        if (e) return fail(QV_E_DEVICE, "timing launch failed: %s", hipGetErrorString((hipError_t)e));
        HIPCHK(hipStreamSynchronize(s));
        for (size_t i = 0; i < log.recs.size(); i++) {
            const qv_launch_rec &r = log.recs[i];
            if (r.level < 0 || (size_t)r.level >= lvs.size()) continue;
            if (r.kernel != k_general && r.kernel != k_gen) continue;
            float f = 0.f;
            HIPCHK(hipEventElapsedTime(&f, log.ev[i].first, log.ev[i].second));
            ms[variant][(size_t)r.level] = std::min(ms[variant][(size_t)r.level], (double)f);
        }
    }
    for (size_t L = 0; L < lvs.size(); L++) lvs[L].gen = (gens[L] && ms[1][L] < ms[0][L]) ? gens[L] : nullptr;
    bt->fwd_valid = false;
    return QV_OK;
}

// The reverse levels of the main execution set, each sweep after its own forward pass.
static qv_status time_generated_reverse(qv_batch_s *bt, ExecSet &es)
{
    const DevPlans &dp = *bt->dp;
    return time_generated(bt, es, 1, [&](hipStream_t s, LaunchLog *log) {
        int e = enqueue_matrices(*bt, s, nullptr);
        if (!e)
            e = enqueue_forward(*bt, es, dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                                bt->d_norms.as<double>(), s, nullptr);
        if (!e) e = enqueue_adjoint(*bt, es, dp, s, log);
        return e;
    });
}

// The forward levels of the main execution set and of every parameter-shift chunk (kernels generated for
// them first). A chunk's sweeps write the variants' scratch states and energies, as its real sweep does.
static qv_status generated_forward(qv_batch_s *bt, bool with_chunks)
{
    const DevPlans &dp = *bt->dp;
    qv_status st = ensure_generated(bt, bt->main, 0);
    if (st != QV_OK) return st;
    st = time_generated(bt, bt->main, 0, [&](hipStream_t s, LaunchLog *log) {
        const int e = enqueue_matrices(*bt, s, nullptr);
        if (e) return e;
        return enqueue_forward(*bt, bt->main, dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                               bt->d_norms.as<double>(), s, log);
    });
    if (st != QV_OK || !with_chunks) return st;
    for (size_t i = 0; i < bt->ps_chunks.size(); i++) {
        ExecSet &es = *bt->ps_chunks[i];
        if ((st = ensure_generated(bt, es, 0)) != QV_OK) return st;
        st = time_generated(bt, es, 0, [&](hipStream_t s, LaunchLog *log) {
            const int e = enqueue_matrices(*bt, s, nullptr);
            if (e) return e;
            return enqueue_forward(*bt, es, dp, bt->d_ps_psi.p, bt->d_ps_energies.as<double>() + bt->ps_chunk_var0[i],
                                   bt->d_ps_tv.as<double>(), nullptr, s, log);
        });
        if (st != QV_OK) return st;
    }
    return QV_OK;
}

// ---------------------------------------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------------------------------------
// Exported functions (C linkage comes from their declarations in qvpu.h).

const char *qv_last_error(void) { return g_err.c_str(); }

const char *qv_version(void) { return "qvpu 0.1 (gfx950)"; }

qv_status qv_ctx_create(int32_t device, void *hip_stream, const char *options_json, qv_ctx *out)
{
    if (!out) return fail(QV_E_INVALID, "out must not be NULL");
    *out = nullptr;
    std::map<std::string, std::string> opt;
    std::string perr;
    if (!parse_options(options_json, opt, perr)) return fail(QV_E_INVALID, "options_json: %s", perr.c_str());
    auto c = std::make_unique<qv_ctx_s>();
    for (auto &kv : opt) {
        const std::string &k = kv.first, &v = kv.second;
        if (k == "n-virtual-qpus") {
            int n = atoi(v.c_str());
            if (n < 1) return fail(QV_E_INVALID, "n-virtual-qpus must be >= 1");
            c->n_vqpu = n;
        } else if (k == "engine") {
            if (v == "tiled") c->engine = 0;
            else if (v == "lds") c->engine = 1;
            else if (v == "stride") c->engine = 2;
            else return fail(QV_E_INVALID, "engine must be \"tiled\", \"lds\" or \"stride\"");
        } else if (k == "tile_qubits") {
            if (v == "auto") c->tile_qubits = 0;
            else {
                int t = atoi(v.c_str());
                if (t < 6 || t > kMaxTileQubits) return fail(QV_E_INVALID, "tile_qubits must be in [6, %d] or \"auto\"", kMaxTileQubits);
                c->tile_qubits = t;
            }
        } else if (k == "graph") {
            c->graph = (v == "true" || v == "1");
        } else if (k == "contig_qubits") {
            int cq = atoi(v.c_str());
            if (cq < 1 || cq > 6) return fail(QV_E_INVALID, "contig_qubits must be in [1, 6]");
            c->contig = cq;
        } else if (k == "launch_events") {
            c->launch_events = (v == "true" || v == "1");
        } else if (k == "launch") {
            if (v == "levels") c->persistent = 0;
            else if (v == "persistent") c->persistent = 1;
            else return fail(QV_E_INVALID, "launch must be \"levels\" or \"persistent\"");
        } else if (k == "wait_ms") {
            const int w = atoi(v.c_str());
            if (w < 0 || w > 600000) return fail(QV_E_INVALID, "wait_ms must be in [0, 600000]");
            c->wait_ms = w;
        } else if (k == "persist_chunk") {
            const int w = atoi(v.c_str());
            if (w < 0 || w > 64) return fail(QV_E_INVALID, "persist_chunk must be in [0, 64]");
            c->persist_chunk = w;
        } else if (k == "wait_extra") {
            const int w = atoi(v.c_str());
            if (w < 0) return fail(QV_E_INVALID, "wait_extra must be >= 0");
            c->wait_extra = w;
        } else if (k == "autotune") {
            if (v == "off") c->autotune = 0;
            else if (v == "cached") c->autotune = 1;
            else if (v == "search") c->autotune = 2;
            else return fail(QV_E_INVALID, "autotune must be \"off\", \"cached\" or \"search\"");
        } else if (k == "fusion") {
            if (v == "off" || v == "0") c->fuse_min = 0;
            else if (v == "on") c->fuse_min = 6;
            else if (v == "auto") c->fuse_min = kFuseAuto;
            else {
                const int fm = atoi(v.c_str());
                if (fm < 1 || fm > 64)
                    return fail(QV_E_INVALID, "fusion must be \"off\", \"on\", \"auto\" or a minimum run length 1..64");
                c->fuse_min = fm;
            }
        } else if (k == "specialize") {
            if (v == "on" || v == "1" || v == "true") c->specialize = 3;
            else if (v == "adjoint") c->specialize = 2;
            else if (v == "auto") c->specialize = 3 | kSpecializeTimed;
            else if (v == "off" || v == "0" || v == "false") c->specialize = 0;
            else return fail(QV_E_INVALID, "specialize must be \"on\", \"adjoint\", \"auto\" or \"off\"");
        } else if (k == "adjoint_inner") {
            if (v == "f64") c->inner_f64 = 1;
            else if (v == "f32") c->inner_f64 = 0;
            else return fail(QV_E_INVALID, "adjoint_inner must be \"f32\" or \"f64\"");
        } else if (k == "fold_cnots") {
            if (v == "on" || v == "1" || v == "true") c->fold_cnots = 1;
            else if (v == "off" || v == "0" || v == "false") c->fold_cnots = 0;
            else return fail(QV_E_INVALID, "fold_cnots must be \"on\" or \"off\"");
        } else if (k == "fusion_k" || k == "precision" || k == "deterministic") {
            /* accepted for compatibility; the current planner ignores them */
        } else {
            return fail(QV_E_INVALID, "unknown option \"%s\"", k.c_str());
        }
    }
    if (c->inner_f64 && !(c->specialize & 2))
        return fail(QV_E_INVALID, "\"adjoint_inner\": \"f64\" applies to generated adjoint passes: give \"specialize\": "
                                  "\"on\" or \"adjoint\"");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(QV_E_INVALID, "device %d out of range (%d devices)", device, ndev);
    c->device = device;
    HIPCHK(enter_device(device));
    int e = prepare_kernels();
    if (e) return fail(QV_E_DEVICE, "kernel setup failed: %s", hipGetErrorString((hipError_t)e));
    if ((e = static_scratch_setup(device)) != 0)
        return fail(QV_E_DEVICE, "static scratch lookup failed: %s", hipGetErrorString((hipError_t)e));
    c->user_stream = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    *out = c.release();
    return ok();
}

qv_status qv_ctx_set_stream(qv_ctx ctx, void *hip_stream)
{
    if (!ctx) return fail(QV_E_INVALID, "ctx must not be NULL");
    ctx->user_stream = reinterpret_cast<hipStream_t>(hip_stream);
    return ok();
}

// Drops one reference; the last one frees the context (its capture stream).
static void ctx_release(qv_ctx ctx)
{
    if (ctx->refs.fetch_sub(1) != 1) return;
    if (hipSetDevice(ctx->device) == hipSuccess && ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    (void)hipGetLastError();  // a failure here must not be reported by the next call's launch checks
    delete ctx;
}

qv_status qv_ctx_destroy(qv_ctx ctx)
{
    if (!ctx) return fail(QV_E_INVALID, "ctx must not be NULL");
    ctx_release(ctx);
    return ok();
}

qv_status qv_validate_batch(int32_t n_circuits, const int32_t *n_qubits, const int64_t *gate_offsets,
                            const qv_gate *gates, const int32_t *n_params, int32_t params_shared,
                            const int64_t *term_offsets, const uint64_t *xmask, const uint64_t *zmask,
                            const double *coeff, int32_t obs_shared, qv_precision precision)
{
    qv_status st = validate(n_circuits, n_qubits, gate_offsets, gates, n_params, params_shared, term_offsets, xmask,
                            zmask, coeff, obs_shared, precision);
    if (st == QV_OK) return ok();
    return st;
}

static int default_tile_qubits(qv_precision p, bool adjoint)
{
    const char *env = getenv("QV_TILE_QUBITS");
    int t = env ? atoi(env) : 0;
    if (t < 6 || t > kMaxTileQubits) t = (p == QV_C64) ? 13 : 12;
    if (adjoint) t -= 1;
    if (p == QV_C128 && t > 13) t = 13;
    if (adjoint && p == QV_C128 && t > 12) t = 12;
    if (adjoint && p == QV_C64 && t > 13) t = 13;
    return t;
}

static void drop_graphs(qv_batch_s *bt)
{
    if (bt->g_fwd) (void)hipGraphExecDestroy(bt->g_fwd);
    if (bt->g_adj) (void)hipGraphExecDestroy(bt->g_adj);
    if (bt->g_ps) (void)hipGraphExecDestroy(bt->g_ps);
    if (bt->g_js_adj) (void)hipGraphExecDestroy(bt->g_js_adj);
    if (bt->g_js_ps) (void)hipGraphExecDestroy(bt->g_js_ps);
    bt->g_fwd = bt->g_adj = bt->g_ps = bt->g_js_adj = bt->g_js_ps = nullptr;
    bt->ps_chunks.clear();
    bt->ps_chunk_var0.clear();
    bt->ps_ready = false;
    bt->fwd_valid = false;
}

// (Re)builds the plans, their device form and the batch's launch structure for a tile size and a
// contiguous-run length. Cached graphs and parameter-shift chunks are dropped; state buffers are kept.
static hipError_t configure(qv_batch_s *bt, int tile_qubits, int contig)
{
    qv_ctx ctx = bt->ctx;
    const int B = bt->B;
    const qv_precision prec = bt->prec;
    const int32_t *nq = bt->nq.data();
    const int64_t *goff = bt->goff.data();
    const qv_gate *gates = bt->gates.data();
    const int32_t *np = bt->nparams.data();
    const int params_shared = bt->params_shared;
    const int obs_shared = bt->obs_shared;
    drop_graphs(bt);
    bt->plans.clear();
    bt->main = ExecSet{};
    // plans: circuits with the same structure share one
    // The adjoint sweep holds two tiles (psi and lambda) in LDS, so a plan's tiles are capped at
    // 2^13 amplitudes for complex64 and 2^12 for complex128 (2 x 64 KiB plus the index table).
    bt->tile_qubits = tile_qubits ? tile_qubits : default_tile_qubits(prec, false);
    bt->tile_qubits = std::min(bt->tile_qubits, prec == QV_C64 ? 13 : 12);
    bt->contig = contig ? contig : (prec == QV_C64 ? 4 : 3);
    std::unordered_map<std::string, int> sig2plan;
    bt->plan_of.resize(B);
    for (int b = 0; b < B; b++) {
        std::string sig((const char *)&nq[b], sizeof(int32_t));
        for (int64_t k = goff[b]; k < goff[b + 1]; k++) {
            const qv_gate &g = gates[k];
            int32_t rec[4] = {g.kind, g.q0, is_two_qubit(g.kind) ? g.q1 : -1, (is_rotation(g.kind) && g.param >= 0) ? 1 : 0};
            sig.append((const char *)rec, sizeof rec);
        }
        auto it = sig2plan.find(sig);
        if (it != sig2plan.end()) { bt->plan_of[b] = it->second; continue; }
        const int id = (int)bt->plans.size();
        sig2plan.emplace(sig, id);
        bt->plan_of[b] = id;
        PlanInput pin;
        pin.n = nq[b];
        for (int64_t k = goff[b]; k < goff[b + 1]; k++) {
            const qv_gate &g = gates[k];
            pin.kinds.push_back(g.kind);
            pin.q0.push_back(g.q0);
            pin.q1.push_back(is_two_qubit(g.kind) ? g.q1 : -1);
            pin.trainable.push_back(is_rotation(g.kind) && g.param >= 0);
        }
        const int lowc = bt->contig;
        const int rb = ctx->engine == 0 ? (prec == QV_C64 ? kRegBitsC64 : kRegBitsC128) : 0;
        const int fm = (ctx->engine == 0) ? bt->fuse_min : 0;
        bt->plans.push_back(ctx->engine == 2 ? plan_stride(pin)
                                              : plan_tiled(pin, bt->tile_qubits, lowc, rb, fm, ctx->fold_cnots));
    }
    // device plan arrays
    auto dp = std::make_unique<DevPlans>();
    std::vector<DevPass> passes;
    std::vector<DevOp> ops;
    std::vector<DevSeg> rsegs;
    std::vector<int64_t> plan_op_base;
    std::vector<int64_t> fused_ops;
    for (const Plan &pl : bt->plans) {
        dp->pass_base.push_back((int)passes.size());
        plan_op_base.push_back((int64_t)ops.size());
        const size_t before = ops.size();
        lower_plan(pl, passes, ops, rsegs);
        dp->op_count.push_back((int64_t)(ops.size() - before));
        dp->fused_base.push_back((int64_t)fused_ops.size());
        std::vector<int64_t> mk(fused_blocks(pl), -1);
        for (size_t i = before; i < ops.size(); i++)
            if (ops[i].kind == kFusedKind) mk[ops[i].p0 | (ops[i].p1 << 8)] = (int64_t)i;
        for (int64_t v : mk) fused_ops.push_back(v);
        dp->fused_count.push_back((int64_t)mk.size());
    }
    HIPRET(dp->fused_ops.upload(fused_ops));
    HIPRET(dp->passes.upload(passes));
    HIPRET(dp->ops.upload(ops));
    HIPRET(dp->rsegs.upload(rsegs));
    dp->h_passes = passes;
    dp->h_ops = ops;
    dp->h_rsegs = rsegs;

    // main set
    ExecSet &es = bt->main;
    es.n_circ = B;
    es.circs.resize(B);
    es.plan_of = bt->plan_of;
    int64_t off = 0, pb = 0;
    for (int b = 0; b < B; b++) {
        DevCirc &c = es.circs[b];
        c.state_off = off;
        c.gate_off = goff[b];
        c.param_base = params_shared ? 0 : pb;
        c.n = nq[b];
        c.shift_gate = -1;
        c.shift = 0.0;
        c.base_circ = b;
        c.pad = 0;
        c.op_base = plan_op_base[bt->plan_of[b]];
        c.mat_off = 0;
        c.fused_off = 0;
        c.fused_ops = dp->fused_base[bt->plan_of[b]];
        off += (int64_t)1 << nq[b];
        pb += np[b];
    }
    es.state_amps = off;
    // matrix table: one entry per circuit and plan op; fused blocks: one per circuit and block
    {
        int64_t mo = 0, fo = 0;
        std::vector<int32_t> mat_circ;
        std::vector<int64_t> ffb(B + 1, 0);
        for (int b = 0; b < B; b++) {
            const int pl = bt->plan_of[b];
            es.circs[b].mat_off = mo;
            es.circs[b].fused_off = fo;
            for (int64_t k = 0; k < dp->op_count[pl]; k++) mat_circ.push_back(b);
            mo += dp->op_count[pl];
            const int64_t nf = prec == QV_C64 ? dp->fused_count[pl] : 0;
            fo += nf;
            ffb[b + 1] = ffb[b] + nf;
        }
        bt->n_mats = mo;
        bt->n_fused = fo;
        HIPRET(bt->d_gate_circ.upload(mat_circ));
        HIPRET(bt->d_mats.alloc((size_t)std::max<int64_t>(1, mo) * 8 * (bt->amp_bytes / 2)));
        HIPRET(bt->d_fmats.alloc(sizeof(float) * (size_t)std::max<int64_t>(1, fo) * kFusedFloats));
        HIPRET(bt->d_fuse_fb.upload(ffb));
    }
    build_levels(es, bt->plans, dp->pass_base, ctx->n_vqpu, bt->amp_bytes, ctx->persistent == 0);
    ObsView ov{bt->toff.data(), bt->xm.data(), bt->zm.data(), bt->cf.data(), bt->obs_shared};
    std::vector<int> obs_of(B);
    std::vector<int64_t> out_base(B);
    const int64_t Tsh = obs_shared ? bt->toff[1] - bt->toff[0] : 0;
    for (int b = 0; b < B; b++) {
        obs_of[b] = b;
        out_base[b] = obs_shared ? (int64_t)b * Tsh : bt->toff[b];
    }
    build_expectation(es, ov, obs_of, out_base, bt->n_tv, true, bt->amp_bytes);
    build_lambda(es, ov, obs_of, bt->amp_bytes);
    build_grad_refs(es, *bt, dp->pass_base);
    HIPRET(upload_set(es, true));

    bt->dp = std::move(dp);
    return hipSuccess;
}

qv_status qv_batch_create(qv_ctx ctx, int32_t B, const int32_t *nq, const int64_t *goff, const qv_gate *gates,
                          const int32_t *np, int32_t params_shared, const int64_t *toff, const uint64_t *xm,
                          const uint64_t *zm, const double *cf, int32_t obs_shared, qv_precision prec,
                          qv_batch *out)
{
    if (!ctx) return fail(QV_E_INVALID, "ctx must not be NULL");
    if (!out) return fail(QV_E_INVALID, "out must not be NULL");
    *out = nullptr;
    qv_status st = validate(B, nq, goff, gates, np, params_shared, toff, xm, zm, cf, obs_shared, prec);
    if (st != QV_OK) return st;
    HIPCHK(enter_device(ctx->device));
    auto bt = std::make_unique<qv_batch_s>();
    bt->ctx = ctx;
    bt->B = B;
    bt->prec = prec;
    bt->amp_bytes = prec == QV_C64 ? 8 : 16;
    bt->nq.assign(nq, nq + B);
    {
        int64_t total = 0, largest = 0;
        for (int b = 0; b < B; b++) {
            total += (int64_t)bt->amp_bytes << nq[b];
            largest = std::max(largest, (int64_t)bt->amp_bytes << nq[b]);
        }
        bt->stream_levels = total >= kStreamBatchBytes;
        bt->stream_expect = largest >= kStreamStateBytes;
    }
    bt->goff.assign(goff, goff + B + 1);
    bt->gates.assign(gates, gates + goff[B]);
    bt->nparams.assign(np, np + B);
    bt->params_shared = params_shared ? 1 : 0;
    bt->n_theta = 0;
    if (params_shared) bt->n_theta = np[0];
    else for (int b = 0; b < B; b++) bt->n_theta += np[b];
    bt->n_grad = bt->n_theta;
    bt->obs_shared = obs_shared ? 1 : 0;
    const int nto = obs_shared ? 1 : B;
    bt->toff.assign(toff, toff + nto + 1);
    const int64_t T0 = toff[0], T1 = toff[nto];
    bt->xm.assign(xm ? xm + T0 : nullptr, xm ? xm + T1 : nullptr);
    bt->zm.assign(zm ? zm + T0 : nullptr, zm ? zm + T1 : nullptr);
    bt->cf.assign(cf ? cf + T0 : nullptr, cf ? cf + T1 : nullptr);
    for (auto &v : bt->toff) v -= T0;
    bt->n_tv = obs_shared ? (int64_t)B * (bt->toff[1] - bt->toff[0]) : bt->toff[B];

    // memory check: states of the batch
    int64_t amps = 0;
    for (int b = 0; b < B; b++) amps += (int64_t)1 << nq[b];
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const double need = (double)amps * bt->amp_bytes;
    if (need > 0.92 * (double)freeb)
        return fail(QV_E_OOM, "states need %.2f GiB, device has %.2f GiB free", need / 1073741824.0, freeb / 1073741824.0);

    bt->fuse_min = ctx->fuse_min == kFuseAuto ? (prec == QV_C64 ? kFuseDefault : 0) : ctx->fuse_min;
    HIPCHK(configure(bt.get(), ctx->tile_qubits, ctx->contig));

    HIPCHK(bt->d_gates.upload(bt->gates));
    HIPCHK(bt->d_theta.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, bt->n_theta)));
    HIPCHK(bt->d_psi.alloc((size_t)bt->main.state_amps * bt->amp_bytes));
    HIPCHK(bt->d_energies.alloc(sizeof(double) * B));
    HIPCHK(bt->d_tv.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, bt->n_tv)));
    HIPCHK(bt->d_norms.alloc(sizeof(double) * B));
    HIPCHK(bt->d_grad.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, bt->n_grad)));
    HIPCHK(bt->d_upstream.alloc(sizeof(double) * B));
    HIPCHK(hipEventCreate(&bt->ev0));
    HIPCHK(hipEventCreate(&bt->ev1));
    if (bt->n_theta == 0) bt->theta_set = true;
    ctx->refs.fetch_add(1);  // the context stays alive until this batch is destroyed
    *out = bt.release();
    return ok();
}

qv_status qv_batch_set_params(qv_batch bt, const double *theta, int32_t on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (bt->n_theta == 0) { bt->theta_set = true; return ok(); }
    if (!theta) return fail(QV_E_INVALID, "theta must not be NULL");
    if (!on_device)
        for (int64_t i = 0; i < bt->n_theta; i++)
            if (!std::isfinite(theta[i])) return fail(QV_E_INVALID, "theta[%lld] is not finite", (long long)i);
    HIPCHK(enter_device(bt->ctx->device));
    hipStream_t s = bt->ctx->stream();
    HIPCHK(hipMemcpyAsync(bt->d_theta.p, theta, sizeof(double) * (size_t)bt->n_theta,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (!on_device) HIPCHK(hipStreamSynchronize(s));
    bt->theta_set = true;
    bt->fwd_valid = false;
    return ok();
}

// Runs `fn` either directly on the stream or through a cached graph captured on the context's capture stream.
template <typename F>
static qv_status run_graph(qv_batch bt, hipGraphExec_t &cache, F fn)
{
    hipStream_t s = bt->ctx->stream();
    if (!bt->ctx->graph) {
        int e = fn(s, bt->ctx->launch_events ? &bt->log : nullptr);
        if (e) return fail(QV_E_DEVICE, "launch failed: %s", hipGetErrorString((hipError_t)e));
        return QV_OK;
    }
    if (!cache) {
        hipStream_t cs = bt->ctx->cap_stream;
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        int e = fn(cs, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e) { if (g) (void)hipGraphDestroy(g); return fail(QV_E_DEVICE, "launch failed during capture: %s", hipGetErrorString((hipError_t)e)); }
        if (e2 != hipSuccess) return fail(QV_E_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
        hipError_t e3 = hipGraphInstantiate(&cache, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) { cache = nullptr; return fail(QV_E_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e3)); }
    }
    HIPCHK(hipGraphLaunch(cache, s));
    return QV_OK;
}

// ---------------------------------------------------------------------------------------------------------
// Autotuner: picks the tile size and the contiguous-run length of a batch by timing one forward pass per
// candidate on the device, and remembers the choice in a small text cache keyed by device architecture,
// precision, engine and the batch's shape (circuits, largest register, distinct structures, largest gate
// count). Explicit "tile_qubits" / "contig_qubits" options always win.
// ---------------------------------------------------------------------------------------------------------
static std::string tune_path()
{
    const char *p = getenv("QV_TUNE_CACHE");
    if (p && *p) return p;
    const char *h = getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/qvpu_tune.txt";
}

static std::string tune_key(const qv_batch_s *bt)
{
    int nmax = 0;
    int64_t gmax = 0;
    for (int b = 0; b < bt->B; b++) {
        nmax = std::max(nmax, bt->nq[b]);
        gmax = std::max<int64_t>(gmax, bt->goff[b + 1] - bt->goff[b]);
    }
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, bt->ctx->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    char buf[256];
    char fz[16];
    if (bt->ctx->fuse_min == kFuseAuto) snprintf(fz, sizeof fz, "auto");
    else snprintf(fz, sizeof fz, "%d", bt->ctx->fuse_min);
    snprintf(buf, sizeof buf, "%s/%s/%s/B%d/n%d/s%d/g%lld/f%s", arch.c_str(), bt->prec == QV_C64 ? "c64" : "c128",
             bt->ctx->engine == 0 ? "tiled" : "lds", bt->B, nmax, (int)bt->plans.size(), (long long)gmax, fz);
    return buf;
}

// Cache lines: key, tile qubits, contiguous qubits, fused-block width (register qubits, 4), minimum run
// length of a fused block (0: none), forward time in ms.
static bool tune_lookup(const std::string &key, int &T, int &contig, int &fm)
{
    FILE *f = fopen(tune_path().c_str(), "r");
    if (!f) return false;
    char line[512], k[256];
    int t = 0, c = 0, w = 0, m = 0;
    double ms = 0;
    bool found = false;
    while (fgets(line, sizeof line, f))
        if (sscanf(line, "%255s %d %d %d %d %lf", k, &t, &c, &w, &m, &ms) == 6 && key == k) {
            T = t;
            contig = c;
            fm = m;
            found = true;
        }
    fclose(f);
    return found;
}

static void tune_store(const std::string &key, int T, int contig, int fm, double ms)
{
    const std::string path = tune_path();
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;  // the cache is an optimisation only
    fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), T, contig, kRegBitsC64, fm, ms);
    fclose(f);
}

static qv_status time_forward(qv_batch bt, double &ms)
{
    hipStream_t s = bt->ctx->stream();
    DevPlans &dp = *bt->dp;
    for (int rep = 0; rep < 2; rep++) {
        if (rep == 1) HIPCHK(hipEventRecord(bt->ev0, s));
        int e = enqueue_matrices(*bt, s, nullptr);
        if (!e) e = enqueue_forward(*bt, bt->main, dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                                    bt->d_norms.as<double>(), s, nullptr);
        if (e) return fail(QV_E_DEVICE, "autotune launch failed: %s", hipGetErrorString((hipError_t)e));
    }
    HIPCHK(hipEventRecord(bt->ev1, s));
    HIPCHK(hipEventSynchronize(bt->ev1));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, bt->ev0, bt->ev1));
    ms = f;
    return QV_OK;
}

// The autotuner's candidates for a batch: tile sizes and contiguous-run lengths when some circuit needs
// more than one pass and none is given explicitly, fused-block minimum runs under "fusion": "auto"
// (complex64, register tiles). One candidate each: nothing to choose.
struct TuneSpace {
    std::vector<int> T, C, FM;
    bool trivial() const { return T.size() * C.size() * FM.size() <= 1; }
};

static TuneSpace tune_space(const qv_batch_s *bt)
{
    const qv_ctx ctx = bt->ctx;
    TuneSpace sp;
    int nmax = 0;
    for (int b = 0; b < bt->B; b++) nmax = std::max(nmax, bt->nq[b]);
    const int tmax = bt->prec == QV_C64 ? 13 : 12, c_hi = bt->prec == QV_C64 ? 4 : 3;
    const bool tiles = ctx->engine != 2 && !ctx->tile_qubits && !ctx->contig && nmax > tmax;
    if (tiles) sp.T = {tmax, tmax - 1, tmax - 2}, sp.C = {c_hi, c_hi - 1};
    else sp.T = {bt->tile_qubits}, sp.C = {bt->contig};
    if (ctx->fuse_min == kFuseAuto && ctx->engine == 0 && bt->prec == QV_C64)
        sp.FM.assign(std::begin(kFuseCandidates), std::end(kFuseCandidates));
    else
        sp.FM = {bt->fuse_min};
    return sp;
}

// True when autotune() would leave the launch configuration as it is (no re-planning, no allocation).
static bool tune_settled(qv_batch bt)
{
    if (bt->tuned || bt->ctx->autotune == 0) return true;
    if (tune_space(bt).trivial()) return true;
    int T = 0, contig = 0, fm = 0;
    if (tune_lookup(tune_key(bt), T, contig, fm))
        return T == bt->tile_qubits && contig == bt->contig && fm == bt->fuse_min;
    return bt->ctx->autotune != 2;
}

static qv_status autotune(qv_batch bt)
{
    bt->tuned = 1;
    if (bt->ctx->autotune == 0) return QV_OK;
    const TuneSpace sp = tune_space(bt);
    if (sp.trivial()) return QV_OK;
    const std::string key = tune_key(bt);
    int T = 0, contig = 0, fm = 0;
    if (tune_lookup(key, T, contig, fm)) {
        if (T != bt->tile_qubits || contig != bt->contig || fm != bt->fuse_min) {
            bt->fuse_min = fm;
            HIPCHK(configure(bt, T, contig));
        }
        return QV_OK;
    }
    if (bt->ctx->autotune != 2) return QV_OK;
    double best = 1e300;
    int bT = bt->tile_qubits, bc = bt->contig, bf = bt->fuse_min;
    for (int t : sp.T)
        for (int c : sp.C)
            for (int f : sp.FM) {
                bt->fuse_min = f;
                HIPCHK(configure(bt, t, c));
                double ms = 0.0;
                qv_status st = time_forward(bt, ms);
                if (st != QV_OK) return st;
                if (ms < best) { best = ms; bT = t; bc = c; bf = f; }
            }
    bt->fuse_min = bf;
    HIPCHK(configure(bt, bT, bc));
    tune_store(key, bT, bc, bf, best);
    return QV_OK;
}

static qv_status forward(qv_batch bt)
{
    if (!bt->tuned) {
        qv_status st = autotune(bt);
        if (st != QV_OK) return st;
    }
    DevPlans &dp = *bt->dp;
    qv_status st = generated_forward(bt, false);
    if (st != QV_OK) return st;
    st = run_graph(bt, bt->g_fwd, [&](hipStream_t s, LaunchLog *log) {
        const int e = enqueue_matrices(*bt, s, log);
        if (e) return e;
        return enqueue_forward(*bt, bt->main, dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                               bt->d_norms.as<double>(), s, log);
    });
    if (st != QV_OK) return st;
    bt->fwd_valid = true;
    bt->last = qv_stats{};
    bt->last.passes = bt->main.passes_fwd;
    bt->last.launches = 3 + (int64_t)bt->main.fwd.size();
    bt->last.algorithmic_bytes = bt->main.algo_bytes_fwd;
    return QV_OK;
}

// A persistent launch whose wait ran out leaves a flag behind; report it once.
static qv_status check_persist_error(qv_batch bt)
{
    std::vector<ExecSet *> sets{&bt->main};
    for (auto &c : bt->ps_chunks) sets.push_back(c.get());
    for (ExecSet *es : sets) {
        if (!es->d_p_error.p) continue;
        int32_t flag = 0;
        HIPCHK(hipMemcpy(&flag, es->d_p_error.p, sizeof flag, hipMemcpyDeviceToHost));
        if (flag) {
            HIPCHK(hipMemset(es->d_p_error.p, 0, sizeof(int32_t)));
            return fail(QV_E_DEVICE, "a persistent launch gave up waiting for a dependency; its results are invalid");
        }
    }
    return QV_OK;
}

static qv_status copy_out(qv_batch bt, void *dst, const void *src, size_t bytes, int on_device)
{
    if (!dst || bytes == 0) return QV_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, bt->ctx->stream()));
    return QV_OK;
}

qv_status qv_batch_expectations(qv_batch bt, double *energies, double *term_values, int32_t out_on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!bt->theta_set) return fail(QV_E_STATE, "qv_batch_set_params must be called first");
    HIPCHK(enter_device(bt->ctx->device));
    HIPCHK(hipEventRecord(bt->ev0, bt->ctx->stream()));
    qv_status st = forward(bt);
    if (st != QV_OK) return st;
    HIPCHK(hipEventRecord(bt->ev1, bt->ctx->stream()));
    bt->timed = true;
    if ((st = copy_out(bt, energies, bt->d_energies.p, sizeof(double) * bt->B, out_on_device)) != QV_OK) return st;
    if ((st = copy_out(bt, term_values, bt->d_tv.p, sizeof(double) * (size_t)bt->n_tv, out_on_device)) != QV_OK) return st;
    if (!out_on_device) {
        HIPCHK(hipStreamSynchronize(bt->ctx->stream()));
        if ((st = check_persist_error(bt)) != QV_OK) return st;
    }
    return ok();
}


// The non-allocating form of qv_batch_expectations: the same kernels, launched eagerly (no graph), with
// the expectation partial sums in the static scratch array instead of the batch's buffer. Every call on a
// device shares that device's array (calls that overlap on one device race); the partial sums are written
// in full before they are read, so nothing needs clearing.
qv_status qv_batch_expectations_static(qv_batch bt, double *energies, double *term_values, int32_t out_on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!bt->theta_set) return fail(QV_E_STATE, "qv_batch_set_params must be called first");
    ExecSet &es = bt->main;
    if (es.exp_partials > kStaticScratchDoubles)
        return fail(QV_E_INVALID, "the batch's expectations need %lld partial sums, more than the %lld of the static "
                                  "scratch; use qv_batch_expectations", (long long)es.exp_partials,
                    (long long)kStaticScratchDoubles);
    if (!tune_settled(bt))
        return fail(QV_E_STATE, "the autotuner has still to choose this batch's tiles (which allocates): call "
                                "qv_batch_expectations once first, or use \"autotune\": \"off\" or fixed tile sizes");
    bt->tuned = 1;
    double *scr = static_scratch(bt->ctx->device);
    if (!scr) return fail(QV_E_STATE, "the static scratch of device %d is not set up", bt->ctx->device);
    HIPCHK(enter_device(bt->ctx->device));
    hipStream_t s = bt->ctx->stream();
    HIPCHK(hipEventRecord(bt->ev0, s));
    int e = enqueue_matrices(*bt, s, nullptr);
    if (!e)
        e = enqueue_forward(*bt, es, *bt->dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                            bt->d_norms.as<double>(), s, nullptr, scr);
    if (e) return fail(QV_E_DEVICE, "launch failed: %s", hipGetErrorString((hipError_t)e));
    HIPCHK(hipEventRecord(bt->ev1, s));
    bt->timed = true;
    bt->fwd_valid = true;
    bt->last = qv_stats{};
    bt->last.passes = es.passes_fwd;
    bt->last.launches = 3 + (int64_t)es.fwd.size();
    bt->last.algorithmic_bytes = es.algo_bytes_fwd;
    qv_status st;
    if ((st = copy_out(bt, energies, bt->d_energies.p, sizeof(double) * bt->B, out_on_device)) != QV_OK) return st;
    if ((st = copy_out(bt, term_values, bt->d_tv.p, sizeof(double) * (size_t)bt->n_tv, out_on_device)) != QV_OK) return st;
    if (!out_on_device) {
        HIPCHK(hipStreamSynchronize(s));
        if ((st = check_persist_error(bt)) != QV_OK) return st;
    }
    return ok();
}

static qv_status ensure_lambda(qv_batch bt)
{
    if (bt->d_lam.p) return QV_OK;
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const double need = (double)bt->main.state_amps * bt->amp_bytes;
    if (need > 0.92 * (double)freeb)
        return fail(QV_E_OOM, "adjoint vectors need %.2f GiB, device has %.2f GiB free", need / 1073741824.0, freeb / 1073741824.0);
    HIPCHK(bt->d_lam.alloc((size_t)bt->main.state_amps * bt->amp_bytes));
    return QV_OK;
}

// Parameter-shift variants: every trainable gate occurrence (b, k) gives variants 2i (+pi/2), 2i+1 (-pi/2).
static qv_status ensure_param_shift(qv_batch bt)
{
    if (bt->ps_ready) return QV_OK;
    DevPlans &dp = *bt->dp;
    struct Occ { int b; int k; int64_t out; };
    std::vector<Occ> occ;
    std::vector<int64_t> pbase(bt->B + 1, 0);
    for (int b = 0; b < bt->B; b++) pbase[b + 1] = pbase[b] + bt->nparams[b];
    for (int b = 0; b < bt->B; b++)
        for (int64_t k = bt->goff[b]; k < bt->goff[b + 1]; k++) {
            const qv_gate &g = bt->gates[k];
            if (is_rotation(g.kind) && g.param >= 0)
                occ.push_back({b, (int)(k - bt->goff[b]), bt->params_shared ? g.param : pbase[b] + g.param});
        }
    bt->n_occ = (int64_t)occ.size();
    // CSR by output index
    std::vector<std::vector<int>> by_out(bt->n_grad);
    for (size_t i = 0; i < occ.size(); i++) by_out[occ[i].out].push_back((int)i);
    bt->occ_begin.assign(bt->n_grad + 1, 0);
    bt->occ_plus.clear(); bt->occ_minus.clear(); bt->occ_circ.clear();
    for (int64_t g = 0; g < bt->n_grad; g++) {
        for (int i : by_out[g]) {
            bt->occ_plus.push_back(2 * i);
            bt->occ_minus.push_back(2 * i + 1);
            bt->occ_circ.push_back(occ[i].b);
        }
        bt->occ_begin[g + 1] = (int64_t)bt->occ_plus.size();
    }
    // chunk variants so that a chunk's states stay within a budget
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const char *envb = getenv("QV_PS_BUDGET_MB");
    double budget = envb ? atof(envb) * 1048576.0 : std::min(8.0 * 1073741824.0, 0.5 * (double)freeb);
    const int64_t nvar = 2 * bt->n_occ;
    bt->ps_chunks.clear();
    bt->ps_chunk_var0.clear();
    int64_t v = 0, max_amps = 0;
    int64_t maxT = 0;
    for (int b = 0; b < bt->B; b++) {
        const int64_t T = bt->obs_shared ? bt->toff[1] - bt->toff[0] : bt->toff[b + 1] - bt->toff[b];
        maxT = std::max(maxT, T);
    }
    ObsView ov{bt->toff.data(), bt->xm.data(), bt->zm.data(), bt->cf.data(), bt->obs_shared};
    int64_t max_chunk_var = 0;
    while (v < nvar) {
        auto es = std::make_unique<ExecSet>();
        int64_t amps = 0;
        std::vector<int> obs_of;
        while (v < nvar) {
            const Occ &o = occ[v / 2];
            const int64_t a = (int64_t)1 << bt->nq[o.b];
            if (es->n_circ > 0 && (double)(amps + a) * bt->amp_bytes > budget) break;
            DevCirc c = bt->main.circs[o.b];
            c.state_off = amps;
            c.shift_gate = o.k;
            c.shift = (v % 2 == 0) ? M_PI / 2.0 : -M_PI / 2.0;
            c.base_circ = o.b;
            es->circs.push_back(c);
            es->plan_of.push_back(bt->plan_of[o.b]);
            obs_of.push_back(o.b);
            es->n_circ++;
            amps += a;
            v++;
        }
        es->state_amps = amps;
        max_amps = std::max(max_amps, amps);
        build_levels(*es, bt->plans, dp.pass_base, bt->ctx->n_vqpu, bt->amp_bytes);
        std::vector<int64_t> out_base(es->n_circ);
        int64_t ob = 0;
        for (int c = 0; c < es->n_circ; c++) {
            out_base[c] = ob;
            const int b = obs_of[c];
            ob += bt->obs_shared ? bt->toff[1] - bt->toff[0] : bt->toff[b + 1] - bt->toff[b];
        }
        build_expectation(*es, ov, obs_of, out_base, ob, false, bt->amp_bytes);
        HIPCHK(upload_set(*es, false));
        es->has_shift = true;
        HIPCHK(es->d_smats.alloc((size_t)es->n_circ * 8 * (bt->amp_bytes / 2)));
        bt->ps_chunk_var0.push_back(v - es->n_circ);
        max_chunk_var = std::max<int64_t>(max_chunk_var, es->n_circ);
        bt->ps_chunks.push_back(std::move(es));
    }
    HIPCHK(bt->d_ps_psi.alloc((size_t)std::max<int64_t>(1, max_amps) * bt->amp_bytes));
    HIPCHK(bt->d_ps_energies.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, nvar)));
    HIPCHK(bt->d_ps_tv.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, max_chunk_var * std::max<int64_t>(1, maxT))));
    HIPCHK(bt->d_occ_begin.upload(bt->occ_begin));
    HIPCHK(bt->d_occ_plus.upload(bt->occ_plus));
    HIPCHK(bt->d_occ_minus.upload(bt->occ_minus));
    HIPCHK(bt->d_occ_circ.upload(bt->occ_circ));
    bt->ps_ready = true;
    return QV_OK;
}

qv_status qv_batch_gradient(qv_batch bt, qv_grad_method method, const double *upstream, double *grad,
                            double *energies, int32_t on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!grad) return fail(QV_E_INVALID, "grad must not be NULL");
    if (method != QV_ADJOINT && method != QV_PARAM_SHIFT) return fail(QV_E_INVALID, "unknown gradient method %d", (int)method);
    if (!bt->theta_set) return fail(QV_E_STATE, "qv_batch_set_params must be called first");
    HIPCHK(enter_device(bt->ctx->device));
    hipStream_t s = bt->ctx->stream();
    if (upstream) {
        if (!on_device)
            for (int b = 0; b < bt->B; b++)
                if (!std::isfinite(upstream[b])) return fail(QV_E_INVALID, "upstream[%d] is not finite", b);
        HIPCHK(hipMemcpyAsync(bt->d_upstream.p, upstream, sizeof(double) * bt->B,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    } else {
        int e = launch_fill(bt->d_upstream.as<double>(), bt->B, 1.0, s);
        if (e) return fail(QV_E_DEVICE, "fill failed: %s", hipGetErrorString((hipError_t)e));
    }
    DevPlans &dp = *bt->dp;
    qv_status st;
    HIPCHK(hipEventRecord(bt->ev0, s));
    if (method == QV_ADJOINT) {
        if ((st = ensure_lambda(bt)) != QV_OK) return st;
        if ((st = ensure_generated(bt, bt->main, 1)) != QV_OK) return st;
        if ((st = time_generated_reverse(bt, bt->main)) != QV_OK) return st;
        // The reverse sweep starts from the final states of a forward pass with the current parameters;
        // run one first unless the last call left them in place.
        int64_t passes = 0, bytes = 0, launches = 0;
        if (!bt->fwd_valid) {
            if ((st = forward(bt)) != QV_OK) return st;
            passes += bt->last.passes;
            bytes += bt->last.algorithmic_bytes;
            launches += bt->last.launches;
        }
        st = run_graph(bt, bt->g_adj,
                       [&](hipStream_t cs, LaunchLog *log) { return enqueue_adjoint(*bt, bt->main, dp, cs, log); });
        if (st != QV_OK) return st;
        bt->fwd_valid = false;  // the reverse sweep has un-applied the circuit from psi
        bt->last = qv_stats{};
        bt->last.passes = passes + bt->main.passes_rev;
        bt->last.launches = launches + 2 + (int64_t)bt->main.rev.size();
        bt->last.algorithmic_bytes = bytes + bt->main.algo_bytes_rev;
    } else {
        if ((st = ensure_param_shift(bt)) != QV_OK) return st;
        if ((st = generated_forward(bt, true)) != QV_OK) return st;
        st = run_graph(bt, bt->g_ps, [&](hipStream_t cs, LaunchLog *log) {
            int e = enqueue_matrices(*bt, cs, log);
            if (e) return e;
            e = enqueue_forward(*bt, bt->main, dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                                    bt->d_norms.as<double>(), cs, log);
            if (e) return e;
            for (size_t i = 0; i < bt->ps_chunks.size(); i++) {
                ExecSet &es = *bt->ps_chunks[i];
                e = enqueue_forward(*bt, es, dp, bt->d_ps_psi.p, bt->d_ps_energies.as<double>() + bt->ps_chunk_var0[i],
                                    bt->d_ps_tv.as<double>(), nullptr, cs, log);
                if (e) return e;
            }
            ShiftCombineArgs sa;
            sa.n_out = (int32_t)bt->n_grad;
            sa.occ_begin = bt->d_occ_begin.as<int64_t>();
            sa.occ_plus = bt->d_occ_plus.as<int32_t>();
            sa.occ_minus = bt->d_occ_minus.as<int32_t>();
            sa.occ_circ = bt->d_occ_circ.as<int32_t>();
            sa.energies = bt->d_ps_energies.as<double>();
            sa.upstream = bt->d_upstream.as<double>();
            sa.grad = bt->d_grad.as<double>();
            return logged(log, cs, QV_K_SHIFT_COMBINE, -1, 0, [&] { return launch_shift_combine(sa, cs); });
        });
        if (st != QV_OK) return st;
        bt->fwd_valid = true;
        bt->last = qv_stats{};
        int64_t passes = bt->main.passes_fwd, bytes = bt->main.algo_bytes_fwd, launches = 4 + (int64_t)bt->main.fwd.size();
        for (auto &c : bt->ps_chunks) {
            passes += c->passes_fwd;
            bytes += c->algo_bytes_fwd;
            launches += 3 + (int64_t)c->fwd.size();
        }
        bt->last.passes = passes;
        bt->last.launches = launches;
        bt->last.algorithmic_bytes = bytes;
    }
    HIPCHK(hipEventRecord(bt->ev1, s));
    bt->timed = true;
    if ((st = copy_out(bt, grad, bt->d_grad.p, sizeof(double) * (size_t)bt->n_grad, on_device)) != QV_OK) return st;
    if ((st = copy_out(bt, energies, bt->d_energies.p, sizeof(double) * bt->B, on_device)) != QV_OK) return st;
    if (!on_device) {
        HIPCHK(hipStreamSynchronize(s));
        if ((st = check_persist_error(bt)) != QV_OK) return st;
    }
    return ok();
}

// ---------------------------------------------------------------------------------------------------------
// Probability path (Section 4.2): output distributions and the Jensen-Shannon divergence of Eq. 3
// ---------------------------------------------------------------------------------------------------------
static void diag_prefix(const std::vector<DevCirc> &circs, std::vector<int64_t> &fb)
{
    fb.assign(circs.size() + 1, 0);
    for (size_t c = 0; c < circs.size(); c++) fb[c + 1] = fb[c] + ((((int64_t)1 << circs[c].n) + 4095) / 4096);
}

static qv_status alloc_bytes(DBuf &d, size_t bytes, const char *what)
{
    if (d.p && d.bytes >= bytes) return QV_OK;
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    if ((double)bytes > 0.92 * (double)freeb)
        return fail(QV_E_OOM, "%s need %.2f GiB, device has %.2f GiB free", what, bytes / 1073741824.0,
                    freeb / 1073741824.0);
    HIPCHK(d.alloc(bytes));
    return QV_OK;
}

static qv_status alloc_doubles(DBuf &d, int64_t n, const char *what)
{
    return alloc_bytes(d, sizeof(double) * (size_t)std::max<int64_t>(1, n), what);
}

static qv_status ensure_prob_blocks(qv_batch bt)
{
    if (!bt->pfb.empty()) return QV_OK;
    std::vector<int64_t> fb;
    diag_prefix(bt->main.circs, fb);
    HIPCHK(bt->d_pfb.upload(fb));
    bt->pfb = std::move(fb);
    return QV_OK;
}

static ProbArgs prob_args(const qv_batch_s &bt)
{
    ProbArgs a{};
    a.circs = bt.main.d_circs.as<DevCirc>();
    a.n_circ = bt.B;
    a.first_block = bt.d_pfb.as<int64_t>();
    a.n_blocks = bt.pfb[bt.B];
    a.psi = bt.d_psi.p;
    return a;
}

qv_status qv_batch_probabilities(qv_batch bt, double *probs, int32_t out_on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!probs) return fail(QV_E_INVALID, "probs must not be NULL");
    if (!bt->theta_set) return fail(QV_E_STATE, "qv_batch_set_params must be called first");
    HIPCHK(enter_device(bt->ctx->device));
    qv_status st;
    if ((st = ensure_prob_blocks(bt)) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_probs, bt->main.state_amps, "output distributions")) != QV_OK) return st;
    hipStream_t s = bt->ctx->stream();
    HIPCHK(hipEventRecord(bt->ev0, s));
    if ((st = forward(bt)) != QV_OK) return st;
    ProbArgs a = prob_args(*bt);
    a.probs = bt->d_probs.as<double>();
    const int64_t bytes = bt->main.state_amps * (bt->amp_bytes + (int64_t)sizeof(double));
    const int e = logged(bt->ctx->launch_events ? &bt->log : nullptr, s, QV_K_PROBS, -1, bytes,
                         [&] { return launch_probs(a, bt->prec, s); });
    if (e) return fail(QV_E_DEVICE, "probabilities launch failed: %s", hipGetErrorString((hipError_t)e));
    HIPCHK(hipEventRecord(bt->ev1, s));
    bt->timed = true;
    bt->last.launches += 1;
    bt->last.algorithmic_bytes += bytes;
    if ((st = copy_out(bt, probs, bt->d_probs.p, sizeof(double) * (size_t)bt->main.state_amps, out_on_device)) != QV_OK)
        return st;
    if (!out_on_device) HIPCHK(hipStreamSynchronize(s));
    return ok();
}

qv_status qv_batch_sample(qv_batch bt, int64_t shots, const double *uniforms, int64_t *samples,
                          uint64_t *bitstrings, int64_t *counts, int64_t *n_distinct, int32_t on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!uniforms) return fail(QV_E_INVALID, "uniforms must not be NULL");
    if (shots < 1 || shots > (int64_t)INT32_MAX) return fail(QV_E_INVALID, "shots must be in [1, 2^31 - 1]");
    const bool want_counts = bitstrings || counts || n_distinct;
    if (want_counts && !(bitstrings && counts && n_distinct))
        return fail(QV_E_INVALID, "bitstrings, counts and n_distinct must be given together");
    if (!want_counts && !samples) return fail(QV_E_INVALID, "nothing to return: give samples or the counts");
    const int64_t nshots = (int64_t)bt->B * shots;
    if (nshots > ((int64_t)1 << 40)) return fail(QV_E_INVALID, "too many shots in total");
    if (!on_device)
        for (int64_t i = 0; i < nshots; i++)
            if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0))
                return fail(QV_E_INVALID, "uniforms[%lld] = %g is not in [0, 1)", (long long)i, uniforms[i]);
    if (!bt->theta_set) return fail(QV_E_STATE, "qv_batch_set_params must be called first");
    HIPCHK(enter_device(bt->ctx->device));
    qv_status st;
    if ((st = ensure_prob_blocks(bt)) != QV_OK) return st;
    const int64_t amps = bt->main.state_amps, nb = bt->pfb[bt->B];
    if ((st = alloc_doubles(bt->d_probs, amps, "output distributions")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_slocal, amps, "running sums")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_bsum, nb, "block sums")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_boff, nb, "block offsets")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_stotal, bt->B, "distribution totals")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_uni, nshots, "uniforms")) != QV_OK) return st;
    if ((st = alloc_bytes(bt->d_samples, sizeof(int64_t) * (size_t)nshots, "samples")) != QV_OK) return st;
    if ((st = alloc_bytes(bt->d_hist, sizeof(uint32_t) * (size_t)std::max<int64_t>(1, amps), "counts per bit string")) != QV_OK)
        return st;
    if ((st = alloc_bytes(bt->d_nnz, sizeof(int64_t) * (size_t)std::max<int64_t>(1, nb), "block counts")) != QV_OK) return st;
    if ((st = alloc_bytes(bt->d_noff, sizeof(int64_t) * (size_t)std::max<int64_t>(1, nb), "block count offsets")) != QV_OK)
        return st;
    if ((st = alloc_bytes(bt->d_ndist, sizeof(int64_t) * (size_t)bt->B, "distinct counts")) != QV_OK) return st;
    if ((st = alloc_bytes(bt->d_bits, sizeof(uint64_t) * (size_t)nshots, "drawn bit strings")) != QV_OK) return st;
    if ((st = alloc_bytes(bt->d_counts, sizeof(int64_t) * (size_t)nshots, "drawn counts")) != QV_OK) return st;
    hipStream_t s = bt->ctx->stream();
    HIPCHK(hipMemcpyAsync(bt->d_uni.p, uniforms, sizeof(double) * (size_t)nshots,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(bt->ev0, s));
    if ((st = forward(bt)) != QV_OK) return st;
    ProbArgs pa = prob_args(*bt);
    pa.probs = bt->d_probs.as<double>();
    LaunchLog *log = bt->ctx->launch_events ? &bt->log : nullptr;
    int e = logged(log, s, QV_K_PROBS, -1, amps * (bt->amp_bytes + (int64_t)sizeof(double)),
                   [&] { return launch_probs(pa, bt->prec, s); });
    if (e) return fail(QV_E_DEVICE, "probabilities launch failed: %s", hipGetErrorString((hipError_t)e));
    SampleArgs sa{};
    sa.circs = bt->main.d_circs.as<DevCirc>();
    sa.n_circ = bt->B;
    sa.first_block = bt->d_pfb.as<int64_t>();
    sa.n_blocks = nb;
    sa.probs = bt->d_probs.as<double>();
    sa.local = bt->d_slocal.as<double>();
    sa.bsum = bt->d_bsum.as<double>();
    sa.boff = bt->d_boff.as<double>();
    sa.total = bt->d_stotal.as<double>();
    sa.shots = shots;
    sa.uniforms = bt->d_uni.as<double>();
    sa.samples = bt->d_samples.as<int64_t>();
    sa.hist = bt->d_hist.as<uint32_t>();
    sa.nnz = bt->d_nnz.as<int64_t>();
    sa.noff = bt->d_noff.as<int64_t>();
    sa.n_distinct = bt->d_ndist.as<int64_t>();
    sa.bits = bt->d_bits.as<uint64_t>();
    sa.counts = bt->d_counts.as<int64_t>();
    // probabilities read, running sums written and read back, the histogram cleared, counted and scanned
    const int64_t bytes = amps * (3 * (int64_t)sizeof(double) + 3 * (int64_t)sizeof(uint32_t)) + nshots * 40;
    e = logged(log, s, QV_K_SAMPLE, -1, bytes, [&] {
        const int z = launch_zero_hist(sa.hist, amps, s);
        return z ? z : launch_sample(sa, s);
    });
    if (e) return fail(QV_E_DEVICE, "sampling launch failed: %s", hipGetErrorString((hipError_t)e));
    HIPCHK(hipEventRecord(bt->ev1, s));
    bt->timed = true;
    if ((st = copy_out(bt, samples, bt->d_samples.p, sizeof(int64_t) * (size_t)nshots, on_device)) != QV_OK) return st;
    if ((st = copy_out(bt, bitstrings, bt->d_bits.p, sizeof(uint64_t) * (size_t)nshots, on_device)) != QV_OK) return st;
    if ((st = copy_out(bt, counts, bt->d_counts.p, sizeof(int64_t) * (size_t)nshots, on_device)) != QV_OK) return st;
    if ((st = copy_out(bt, n_distinct, bt->d_ndist.p, sizeof(int64_t) * (size_t)bt->B, on_device)) != QV_OK) return st;
    if (!on_device) HIPCHK(hipStreamSynchronize(s));
    return ok();
}

qv_status qv_batch_js_gradient(qv_batch bt, qv_grad_method method, const double *target, const double *upstream,
                               double *js, double *grad, int32_t on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!target) return fail(QV_E_INVALID, "target must not be NULL");
    if (!grad && !js) return fail(QV_E_INVALID, "js and grad must not both be NULL");
    if (method != QV_ADJOINT && method != QV_PARAM_SHIFT) return fail(QV_E_INVALID, "unknown gradient method %d", (int)method);
    if (!bt->theta_set) return fail(QV_E_STATE, "qv_batch_set_params must be called first");
    const int64_t n = bt->main.state_amps;
    if (!on_device) {
        for (int64_t i = 0; i < n; i++)
            if (!(target[i] >= 0.0) || !std::isfinite(target[i]))
                return fail(QV_E_INVALID, "target[%lld] = %g is not a finite probability", (long long)i, target[i]);
        if (upstream)
            for (int b = 0; b < bt->B; b++)
                if (!std::isfinite(upstream[b])) return fail(QV_E_INVALID, "upstream[%d] is not finite", b);
    }
    HIPCHK(enter_device(bt->ctx->device));
    qv_status st;
    if ((st = ensure_prob_blocks(bt)) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_target, n, "target distributions")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_w, n, "divergence weights")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_js_part, bt->pfb[bt->B], "divergence partial sums")) != QV_OK) return st;
    if ((st = alloc_doubles(bt->d_js, bt->B, "divergences")) != QV_OK) return st;
    hipStream_t s = bt->ctx->stream();
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(bt->d_target.p, target, sizeof(double) * (size_t)n, kind, s));
    if (upstream) {
        HIPCHK(hipMemcpyAsync(bt->d_upstream.p, upstream, sizeof(double) * bt->B, kind, s));
    } else {
        const int e = launch_fill(bt->d_upstream.as<double>(), bt->B, 1.0, s);
        if (e) return fail(QV_E_DEVICE, "fill failed: %s", hipGetErrorString((hipError_t)e));
    }
    DevPlans &dp = *bt->dp;
    const int64_t js_bytes = n * (bt->amp_bytes + 2 * (int64_t)sizeof(double));
    // output distributions, divergences and their weights dJS/dP_theta from the batch's final states
    auto divergence = [&](hipStream_t cs, LaunchLog *log) {
        ProbArgs a = prob_args(*bt);
        a.target = bt->d_target.as<double>();
        a.w = bt->d_w.as<double>();
        a.partials = bt->d_js_part.as<double>();
        int e = logged(log, cs, QV_K_PROBS, -1, js_bytes, [&] { return launch_probs(a, bt->prec, cs); });
        if (e) return e;
        SegSumArgs sa{bt->d_pfb.as<int64_t>(), bt->d_js_part.as<double>(), bt->d_js.as<double>(), bt->B, 0.5};
        return logged(log, cs, QV_K_SEGMENT_SUM, -1, 0, [&] { return launch_segment_sum(sa, cs); });
    };
    HIPCHK(hipEventRecord(bt->ev0, s));
    if (!grad) {
        // divergences only: one forward pass, whose final states stay for a following gradient call
        if ((st = forward(bt)) != QV_OK) return st;
        const int e = divergence(s, bt->ctx->launch_events ? &bt->log : nullptr);
        if (e) return fail(QV_E_DEVICE, "divergence launch failed: %s", hipGetErrorString((hipError_t)e));
        bt->last.launches += 2;
        bt->last.algorithmic_bytes += js_bytes;
    } else if (method == QV_ADJOINT) {
        if ((st = ensure_lambda(bt)) != QV_OK) return st;
        if ((st = ensure_generated(bt, bt->main, 1)) != QV_OK) return st;
        if ((st = time_generated_reverse(bt, bt->main)) != QV_OK) return st;
        int64_t passes = 0, bytes = 0, launches = 0;
        if (!bt->fwd_valid) {
            if ((st = forward(bt)) != QV_OK) return st;
            passes += bt->last.passes;
            bytes += bt->last.algorithmic_bytes;
            launches += bt->last.launches;
        }
        if ((st = generated_forward(bt, false)) != QV_OK) return st;
        st = run_graph(bt, bt->g_js_adj, [&](hipStream_t cs, LaunchLog *log) {
            int e = divergence(cs, log);
            if (e) return e;
            DiagArgs d{};
            d.circs = bt->main.d_circs.as<DevCirc>();
            d.n_circ = bt->B;
            d.first_block = bt->d_pfb.as<int64_t>();
            d.n_blocks = bt->pfb[bt->B];
            d.base_circs = bt->main.d_circs.as<DevCirc>();
            d.w = bt->d_w.as<double>();
            d.upstream = bt->d_upstream.as<double>();
            d.psi = bt->d_psi.p;
            d.lam = bt->d_lam.p;
            e = logged(log, cs, QV_K_DIAG_SEED, -1, n * (2 * bt->amp_bytes + (int64_t)sizeof(double)),
                       [&] { return launch_diag_seed(d, bt->prec, cs); });
            if (e) return e;
            return enqueue_reverse(*bt, bt->main, dp, cs, log);
        });
        if (st != QV_OK) return st;
        bt->fwd_valid = false;
        bt->last = qv_stats{};
        bt->last.passes = passes + bt->main.passes_rev;
        bt->last.launches = launches + 4 + (int64_t)bt->main.rev.size();
        bt->last.algorithmic_bytes = bytes + js_bytes + bt->main.algo_bytes_rev;
    } else {
        if ((st = ensure_param_shift(bt)) != QV_OK) return st;
        for (auto &c : bt->ps_chunks) {
            if (!c->diag_fb.empty()) continue;
            diag_prefix(c->circs, c->diag_fb);
            HIPCHK(c->d_diag_fb.upload(c->diag_fb));
            HIPCHK(c->d_diag_part.alloc(sizeof(double) * (size_t)std::max<int64_t>(1, c->diag_fb.back())));
        }
        if ((st = generated_forward(bt, true)) != QV_OK) return st;
        st = run_graph(bt, bt->g_js_ps, [&](hipStream_t cs, LaunchLog *log) {
            int e = enqueue_matrices(*bt, cs, log);
            if (e) return e;
            e = enqueue_forward(*bt, bt->main, dp, bt->d_psi.p, bt->d_energies.as<double>(), bt->d_tv.as<double>(),
                                bt->d_norms.as<double>(), cs, log);
            if (e) return e;
            if ((e = divergence(cs, log))) return e;
            // each variant's <diag(w)> with its base circuit's weights replaces its energy in the combination
            for (size_t i = 0; i < bt->ps_chunks.size(); i++) {
                ExecSet &es = *bt->ps_chunks[i];
                double *ev = bt->d_ps_energies.as<double>() + bt->ps_chunk_var0[i];
                e = enqueue_forward(*bt, es, dp, bt->d_ps_psi.p, ev, bt->d_ps_tv.as<double>(), nullptr, cs, log);
                if (e) return e;
                DiagArgs d{};
                d.circs = es.d_circs.as<DevCirc>();
                d.n_circ = es.n_circ;
                d.first_block = es.d_diag_fb.as<int64_t>();
                d.n_blocks = es.diag_fb.back();
                d.base_circs = bt->main.d_circs.as<DevCirc>();
                d.w = bt->d_w.as<double>();
                d.psi = bt->d_ps_psi.p;
                d.partials = es.d_diag_part.as<double>();
                e = logged(log, cs, QV_K_DIAG_EXPECT, -1, es.state_amps * (bt->amp_bytes + (int64_t)sizeof(double)),
                           [&] { return launch_diag_expect(d, bt->prec, cs); });
                if (e) return e;
                SegSumArgs sa{es.d_diag_fb.as<int64_t>(), es.d_diag_part.as<double>(), ev, es.n_circ, 1.0};
                e = logged(log, cs, QV_K_SEGMENT_SUM, -1, 0, [&] { return launch_segment_sum(sa, cs); });
                if (e) return e;
            }
            ShiftCombineArgs sa;
            sa.n_out = (int32_t)bt->n_grad;
            sa.occ_begin = bt->d_occ_begin.as<int64_t>();
            sa.occ_plus = bt->d_occ_plus.as<int32_t>();
            sa.occ_minus = bt->d_occ_minus.as<int32_t>();
            sa.occ_circ = bt->d_occ_circ.as<int32_t>();
            sa.energies = bt->d_ps_energies.as<double>();
            sa.upstream = bt->d_upstream.as<double>();
            sa.grad = bt->d_grad.as<double>();
            return logged(log, cs, QV_K_SHIFT_COMBINE, -1, 0, [&] { return launch_shift_combine(sa, cs); });
        });
        if (st != QV_OK) return st;
        bt->fwd_valid = true;
        bt->last = qv_stats{};
        int64_t passes = bt->main.passes_fwd, bytes = bt->main.algo_bytes_fwd + js_bytes;
        int64_t launches = 6 + (int64_t)bt->main.fwd.size();
        for (auto &c : bt->ps_chunks) {
            passes += c->passes_fwd;
            bytes += c->algo_bytes_fwd + c->state_amps * (bt->amp_bytes + (int64_t)sizeof(double));
            launches += 5 + (int64_t)c->fwd.size();
        }
        bt->last.passes = passes;
        bt->last.launches = launches;
        bt->last.algorithmic_bytes = bytes;
    }
    HIPCHK(hipEventRecord(bt->ev1, s));
    bt->timed = true;
    if (grad && (st = copy_out(bt, grad, bt->d_grad.p, sizeof(double) * (size_t)bt->n_grad, on_device)) != QV_OK)
        return st;
    if ((st = copy_out(bt, js, bt->d_js.p, sizeof(double) * bt->B, on_device)) != QV_OK) return st;
    if (!on_device) {
        HIPCHK(hipStreamSynchronize(s));
        if ((st = check_persist_error(bt)) != QV_OK) return st;
    }
    return ok();
}

qv_status qv_batch_state(qv_batch bt, int32_t circuit, void *out, int32_t out_on_device)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    if (!out) return fail(QV_E_INVALID, "out must not be NULL");
    if (circuit < 0 || circuit >= bt->B) return fail(QV_E_INVALID, "circuit %d out of range [0, %d)", circuit, bt->B);
    if (!bt->fwd_valid) return fail(QV_E_STATE, "no forward state: call qv_batch_expectations first");
    HIPCHK(enter_device(bt->ctx->device));
    const DevCirc &c = bt->main.circs[circuit];
    hipStream_t s = bt->ctx->stream();
    // the kernels' states lack the phase exp(-i/2 sum of RZ angles) (gate_matrix builds RZ as diag(1, e^{ia})):
    // copied out through a kernel that multiplies it back, in chunks through a staging buffer for host outputs
    if (!bt->d_state_phase.p) HIPCHK(bt->d_state_phase.alloc(2 * sizeof(double)));
    StatePhaseArgs pa;
    pa.gates = bt->d_gates.as<qv_gate>() + c.gate_off;
    pa.theta = bt->d_theta.as<double>() + c.param_base;
    pa.n_gates = bt->goff[(size_t)circuit + 1] - bt->goff[(size_t)circuit];
    pa.phase = bt->d_state_phase.as<double>();
    int e = launch_rz_phase(pa, s);
    if (e) return fail(QV_E_DEVICE, "phase launch failed: %s", hipGetErrorString((hipError_t)e));
    const int64_t n_amps = (int64_t)1 << c.n;
    const char *src = (const char *)bt->d_psi.p + (size_t)c.state_off * bt->amp_bytes;
    if (out_on_device) {
        pa.src = src;
        pa.dst = out;
        pa.n_amps = n_amps;
        e = launch_scale_copy(pa, bt->prec, s);
        if (e) return fail(QV_E_DEVICE, "state copy failed: %s", hipGetErrorString((hipError_t)e));
        return ok();
    }
    const int64_t chunk = std::min<int64_t>(n_amps, ((int64_t)64 << 20) / bt->amp_bytes);
    if (bt->d_state_stage.bytes < (size_t)(chunk * bt->amp_bytes))
        HIPCHK(bt->d_state_stage.alloc((size_t)(chunk * bt->amp_bytes)));
    for (int64_t i = 0; i < n_amps; i += chunk) {
        pa.src = src + (size_t)i * bt->amp_bytes;
        pa.dst = bt->d_state_stage.p;
        pa.n_amps = std::min(chunk, n_amps - i);
        e = launch_scale_copy(pa, bt->prec, s);
        if (e) return fail(QV_E_DEVICE, "state copy failed: %s", hipGetErrorString((hipError_t)e));
        HIPCHK(hipMemcpyAsync((char *)out + (size_t)i * bt->amp_bytes, bt->d_state_stage.p,
                              (size_t)pa.n_amps * bt->amp_bytes, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return ok();
}

qv_status qv_batch_stats(qv_batch bt, qv_stats *out)
{
    if (!bt || !out) return fail(QV_E_INVALID, "batch and out must not be NULL");
    HIPCHK(enter_device(bt->ctx->device));
    if (bt->timed) {
        HIPCHK(hipEventSynchronize(bt->ev1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, bt->ev0, bt->ev1));
        bt->last.kernel_ms = ms;
    }
    if (bt->fwd_valid || bt->d_norms.p) {
        std::vector<double> nrm(bt->B);
        HIPCHK(hipMemcpy(nrm.data(), bt->d_norms.p, sizeof(double) * bt->B, hipMemcpyDeviceToHost));
        double m = 0.0;
        for (double v : nrm) m = std::max(m, std::fabs(v - 1.0));
        bt->last.norm_err_max = m;
    }
    qv_status pst = check_persist_error(bt);
    if (pst != QV_OK) return pst;
    *out = bt->last;
    out->tile_qubits = bt->tile_qubits;
    out->contig_qubits = bt->contig;
    int pmax = 0;
    for (const Plan &pl : bt->plans) pmax = std::max(pmax, (int)pl.passes.size());
    out->passes_per_circuit_max = pmax;
    out->fuse_min_run = bt->ctx->engine == 0 ? bt->fuse_min : 0;
    return ok();
}

qv_status qv_batch_destroy(qv_batch bt)
{
    if (!bt) return fail(QV_E_INVALID, "batch must not be NULL");
    qv_ctx ctx = bt->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream());
    drop_graphs(bt);
    if (bt->ev0) (void)hipEventDestroy(bt->ev0);
    if (bt->ev1) (void)hipEventDestroy(bt->ev1);
    delete bt;
    (void)hipGetLastError();  // failures while tearing down are not reported by a later call
    ctx_release(ctx);
    return ok();
}



qv_status qv_batch_launch_log(qv_batch bt, qv_launch_rec *out, int32_t max_records, int32_t *n_records)
{
    if (!bt || !n_records) return fail(QV_E_INVALID, "batch and n_records must not be NULL");
    if (max_records > 0 && !out) return fail(QV_E_INVALID, "out must not be NULL when max_records > 0");
    HIPCHK(enter_device(bt->ctx->device));
    const int32_t n = (int32_t)bt->log.recs.size();
    *n_records = n;
    if (n == 0) return ok();
    HIPCHK(hipEventSynchronize(bt->log.ev.back().second));
    for (int32_t i = 0; i < n && i < max_records; i++) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, bt->log.ev[i].first, bt->log.ev[i].second));
        out[i] = bt->log.recs[i];
        out[i].ms = ms;
    }
    if (max_records >= n) bt->log.clear();
    return ok();
}

qv_status qv_plan_circuit(int32_t n_qubits, int64_t n_gates, const qv_gate *gates, int32_t tile_qubits,
                          qv_precision precision, int32_t engine, int32_t fuse_min, int32_t max_passes,
                          qv_pass_info *out, int32_t *n_passes, int32_t *order)
{
    if (!n_passes) return fail(QV_E_INVALID, "n_passes must not be NULL");
    if (max_passes > 0 && !out) return fail(QV_E_INVALID, "out must not be NULL when max_passes > 0");
    if (engine < 0 || engine > 2) return fail(QV_E_INVALID, "engine must be 0 (tiled), 1 (lds) or 2 (stride)");
    const int64_t goff[2] = {0, n_gates};
    const int32_t nq[1] = {n_qubits};
    int32_t np = 0;
    for (int64_t k = 0; k < n_gates; k++)
        if (gates && gates[k].param >= np) np = gates[k].param + 1;
    const int64_t toff[2] = {0, 0};
    qv_status st = validate(1, nq, goff, gates, &np, 1, toff, nullptr, nullptr, nullptr, 1, precision);
    if (st != QV_OK) return st;
    int t = tile_qubits > 0 ? tile_qubits : default_tile_qubits(precision, false);
    if (t < 6 || t > kMaxTileQubits) return fail(QV_E_INVALID, "tile_qubits must be in [6, %d]", kMaxTileQubits);
    t = std::min(t, precision == QV_C64 ? 13 : 12);
    PlanInput pin;
    pin.n = n_qubits;
    for (int64_t k = 0; k < n_gates; k++) {
        pin.kinds.push_back(gates[k].kind);
        pin.q0.push_back(gates[k].q0);
        pin.q1.push_back(is_two_qubit(gates[k].kind) ? gates[k].q1 : -1);
        pin.trainable.push_back(is_rotation(gates[k].kind) && gates[k].param >= 0);
    }
    const int lowc = precision == QV_C64 ? 4 : 3;
    const int rb = engine == 0 ? (precision == QV_C64 ? kRegBitsC64 : kRegBitsC128) : 0;
    const Plan pl = engine == 2 ? plan_stride(pin) : plan_tiled(pin, t, lowc, rb, engine == 0 ? fuse_min : 0);
    *n_passes = (int32_t)pl.passes.size();
    const std::vector<uint64_t> zero = pass_zero_masks(pl);
    const uint64_t width = n_qubits >= 64 ? ~0ull : ((1ull << n_qubits) - 1ull);
    for (int32_t i = 0; i < *n_passes && i < max_passes; i++) {
        const PlanPass &pp = pl.passes[i];
        qv_pass_info &o = out[i];
        o.local_mask = pp.local_mask;
        o.zero_mask = zero[(size_t)i] & width;
        o.qubits = pp.t;
        int32_t nf = 0;
        for (const PlanOp &op : pp.ops) nf += op.kind == kFusedKind ? 1 : 0;
        o.n_ops = (int32_t)pass_gate_count(pp);
        o.n_fused = nf;
        o.n_folded = 0;
        for (const PlanSeg &sg : pp.segs) o.n_folded += (int32_t)(sg.lead.size() + sg.trail.size());
        o.n_trainable = pp.n_train;
        o.n_segments = (int32_t)pp.segs.size();
        const std::vector<int> g = pass_gate_order(pp);
        o.first_gate = g.empty() ? -1 : g[0];
        o.contiguous_low = pp.lowc;
    }
    if (order) {
        int64_t k = 0;
        for (const PlanPass &pp : pl.passes)
            for (int gi : pass_gate_order(pp)) order[k++] = gi;
    }
    return ok();
}
