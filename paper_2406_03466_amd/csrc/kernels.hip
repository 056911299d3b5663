// HIP kernels for gfx950 (MI355X): gate passes over batches of state vectors, Pauli-string expectation
// reductions in FP64, the adjoint seed lambda = w H psi, and the deterministic reductions behind
// gradients.
//
// What the kernels compute (the paper's Eq. 1 evaluated directly, Section 4.1):
//   * a one-qubit gate U on qubit q maps every amplitude pair (i, i | 2^q) with bit q of i clear to
//     (u00 a + u01 b, u10 a + u11 b); CNOT swaps the pair where the control bit is set; CZ negates
//     amplitudes where both bits are set;
//   * <P> for P = (x, z) is sum_b conj(psi[b ^ x]) i^{ny} (-1)^{popcount(b & z)} psi[b], taken over
//     pairs {b, b ^ x} as 2 Re[...] when x != 0;
//   * the adjoint sweep (Jones and Gacon 2020) un-applies gates from psi and lambda and adds
//     Im <lambda| G |psi> for every trainable gate exp(-i a G / 2).
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"
#include "tile_device.h"

namespace qv {

// ------------------------------------------------------------------------------------------------------
// LDS tile pass. One workgroup owns one tile: the 2^t amplitudes whose non-local bits equal the tile's
// index. The lowest `lowc` local qubits are qubits 0..lowc-1, so each run of 2^lowc amplitudes is
// contiguous in HBM and the gather/scatter is coalesced.
// ------------------------------------------------------------------------------------------------------
template <typename R, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_tile(LevelArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t blk = (int64_t)blockIdx.x;
    const Seg sg = a.segs[find_block(a.segs, a.n_segs, blk)];
    const int64_t tile = blk - sg.first_block;
    const DevPass P = a.passes[sg.pass];
    const DevCirc C = a.circs[sg.circ];
    const int n = C.n, t = P.t, lowc = P.pad;
    const uint32_t T = 1u << t;
    const int TL = 1 << (a.lds_t);

    Cx<R> *sp = reinterpret_cast<Cx<R> *>(smem);
    Cx<R> *sl = sp + (ADJ ? TL : 0);
    uint64_t *segtab = reinterpret_cast<uint64_t *>(sp + (ADJ ? 2 * TL : TL));
    double *red = reinterpret_cast<double *>(segtab + (1 << a.tab_bits));

    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint64_t base = deposit((uint64_t)tile, full & ~P.local_mask);
    const uint64_t himask = P.local_mask & ~((1ull << lowc) - 1ull);
    const uint32_t nh = 1u << (t - lowc);
    for (uint32_t h = threadIdx.x; h < nh; h += kBlock) segtab[h] = deposit(h, himask);
    __syncthreads();

    Cx<R> *gpsi = reinterpret_cast<Cx<R> *>(a.psi) + C.state_off;
    Cx<R> *glam = ADJ ? reinterpret_cast<Cx<R> *>(a.lam) + C.state_off : nullptr;
    const uint32_t lmask = (1u << lowc) - 1u;
    for (uint32_t e = threadIdx.x; e < T; e += kBlock) {
        if (!ADJ && sg.first) {
            // first pass of the circuit: the tile of |0...0> is zero except amplitude 0 of tile 0
            Cx<R> z;
            z.re = (R)((base == 0 && e == 0) ? 1 : 0);
            z.im = (R)0;
            sp[e] = z;
            continue;
        }
        const uint64_t g = base | segtab[e >> lowc] | (e & lmask);
        sp[e] = gpsi[g];
        if (ADJ) sl[e] = glam[g];
    }
    __syncthreads();

    for (int k0 = 0; k0 < P.n_ops; k0++) {
        const int k = ADJ ? P.n_ops - 1 - k0 : k0;
        const DevOp op = a.ops[P.op_begin + k];
        const int kind = op.kind;
        if (kind == QV_CNOT || kind == QV_CZ) {
            const uint32_t bc = 1u << op.p0, bt = 1u << op.p1;
            const int plo = op.p0 < op.p1 ? op.p0 : op.p1, phi = op.p0 < op.p1 ? op.p1 : op.p0;
            for (uint32_t i = threadIdx.x; i < (T >> 2); i += kBlock) {
                const uint32_t i00 = insert0(insert0(i, plo), phi);
                if (kind == QV_CNOT) {
                    const uint32_t i10 = i00 | bc, i11 = i00 | bc | bt;
                    Cx<R> x = sp[i10]; sp[i10] = sp[i11]; sp[i11] = x;
                    if (ADJ) { Cx<R> y = sl[i10]; sl[i10] = sl[i11]; sl[i11] = y; }
                } else {
                    const uint32_t i11 = i00 | bc | bt;
                    sp[i11].re = -sp[i11].re; sp[i11].im = -sp[i11].im;
                    if (ADJ) { sl[i11].re = -sl[i11].re; sl[i11].im = -sl[i11].im; }
                }
            }
        } else {
            const int p = op.p0;
            const uint32_t bit = 1u << p;
            if (ADJ && (op.flags & OP_TRAIN)) {
                double acc = 0.0;
                for (uint32_t i = threadIdx.x; i < (T >> 1); i += kBlock) {
                    const uint32_t i0 = insert0(i, p), i1 = i0 | bit;
                    acc += gen_inner<R>(kind, sp[i0], sp[i1], sl[i0], sl[i1]);
                }
                const double s = block_sum(acc, red);
                if (threadIdx.x == 0) a.partials[sg.partial_base + tile * P.n_train + op.train_slot] = s;
            }
            M2<R> m = op_matrix<R>(a, C, sg.circ, op, P.op_begin + k);
            if (ADJ) m = dagger_r(m);
            for (uint32_t i = threadIdx.x; i < (T >> 1); i += kBlock) {
                const uint32_t i0 = insert0(i, p), i1 = i0 | bit;
                Cx<R> x = sp[i0], y = sp[i1];
                apply2(m, x, y);
                sp[i0] = x; sp[i1] = y;
                if (ADJ) {
                    Cx<R> u = sl[i0], v = sl[i1];
                    apply2(m, u, v);
                    sl[i0] = u; sl[i1] = v;
                }
            }
        }
        __syncthreads();
    }

    for (uint32_t e = threadIdx.x; e < T; e += kBlock) {
        const uint64_t g = base | segtab[e >> lowc] | (e & lmask);
        gpsi[g] = sp[e];
        if (ADJ) glam[g] = sl[e];
    }
}


// Forward passes ask for two workgroups per CU (at most 128 VGPRs); the adjoint keeps psi and lambda in
// registers and runs one workgroup per CU.
template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rtile_fwd(LevelArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    rtile_tiles<R, false, RB, NT>(a, smem);
}

template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) void k_rtile_adj(LevelArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    rtile_tiles<R, true, RB, NT>(a, smem);
}

// The tiles of an adjoint pass where psi is zero: lambda alone, with the forward's LDS layout and register
// budget (two workgroups per CU).
template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rtile_lam(LevelArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    rtile_tiles<R, true, RB, NT, InterpProg, true>(a, smem);
}

// A value every lane of the workgroup holds (read back from LDS after a barrier), made wave-uniform for the
// compiler, so that control flow depending on it is uniform.
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Persistent form: workgroups stay resident and claim items from a queue. Items are the blocks of all
// levels in level order, so every item an item waits for was claimed earlier by a running workgroup and
// every wait ends. A workgroup claims `chunk` consecutive items at a time and runs them in order; where the
// next item of its chunk is the next tile of the same (circuit, pass), the current tile's last register
// segment loads it straight into LDS, as in the level kernels, and the next item needs no wait of its own
// (it shares its predecessor's dependency). A finished tile is published once every wave's stores have
// completed (a wait on the vector memory counter), a barrier, thread 0's device-scope release fence and the
// increment of its circuit's counter; a waiting workgroup acquires after it has seen the count.
//
// The loop keeps every thread of a workgroup on the same path: all work of thread 0 for one step
// (publishing the finished item, claiming the next chunk when this one is used up, waiting for the next
// item's dependency) is one region between two barriers, and the loop reads the next item, the chunk end and
// the run flag back as wave-uniform values. (With the claim at the top of the loop and the publication at
// its bottom, each under its own `threadIdx.x == 0` test, the compiler joins the two regions across the
// loop's back edge and turns the loop into two nested loops whose inner one lets wave 0's other lanes
// return to the top barrier without lane 0, re-read the old item and run it again, forever.)
//
// A wait is bounded by wait_ticks of the constant-rate wall clock. A wait that runs out sets *error; from
// then on every workgroup skips the work of the items it claims (it still counts them finished, so no
// other wait blocks on them) and the host reports the launch's results as invalid.
struct PersistItem {
    LevelArgs a;
    int64_t blk, next_blk;
    Seg sg;
};

// Level, block and segment of an item; next_blk is the item's successor tile in the same (circuit, pass)
// when the item after it (below `end`) is that tile, else -1.
__device__ __forceinline__ PersistItem persist_item(const PersistArgs &pa, int64_t item, int64_t end)
{
    int lo = 0, hi = pa.n_levels - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pa.levels[mid].first_item <= item) lo = mid; else hi = mid - 1;
    }
    const PersistLevel lv = pa.levels[lo];
    PersistItem it;
    it.a = pa.base;
    it.a.segs = pa.base.segs + lv.seg_off;
    it.a.n_segs = lv.n_segs;
    it.blk = item - lv.first_item;
    const int si = find_block(it.a.segs, it.a.n_segs, it.blk);
    it.sg = it.a.segs[si];
    const int64_t level_blocks = (lo + 1 < pa.n_levels ? pa.levels[lo + 1].first_item : pa.n_items) - lv.first_item;
    const int64_t send = si + 1 < it.a.n_segs ? it.a.segs[si + 1].first_block : level_blocks;
    it.next_blk = (item + 1 < end && it.blk + 1 < send) ? it.blk + 1 : -1;
    return it;
}

// Thread 0: waits until the circuit of `sg` has finished sg.wait tiles; false when the wait ran out or an
// earlier one did.
__device__ __forceinline__ bool persist_wait(const PersistArgs &pa, const Seg &sg)
{
    bool run = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    if (run && sg.wait > 0) {
        const int64_t need = sg.wait + pa.wait_extra;
        const int64_t t0 = wall_clock64();
        while ((int64_t)__hip_atomic_load(pa.done + sg.circ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            __builtin_amdgcn_s_sleep(2);
            if (wall_clock64() - t0 > pa.wait_ticks) {
                atomicOr(pa.error, 1);
                run = false;
                break;
            }
        }
    }
    __threadfence();
    return run;
}

template <typename R, bool ADJ, int RB, int NT>
__device__ __forceinline__ void persistent_body(const PersistArgs &pa)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long item_s, end_s;
    __shared__ int run_s;
    const int64_t K = pa.chunk;
    if (threadIdx.x == 0) {
        const int64_t first = (int64_t)atomicAdd(pa.head, (unsigned long long)K);
        item_s = first;
        end_s = first + K < pa.n_items ? first + K : pa.n_items;
        run_s = first < pa.n_items ? (int)persist_wait(pa, persist_item(pa, first, end_s).sg) : 0;
    }
    __syncthreads();
    int64_t item = uniform_i64(item_s);
    int64_t end = uniform_i64(end_s);
    bool run = uniform_i64(run_s) != 0;
    bool pre = false;
    while (item < pa.n_items) {
        const PersistItem it = persist_item(pa, item, end);
        // the adjoint's tiles where psi is zero run the lambda-only code, as their own launch does in levels mode
        bool lam = false;
        if constexpr (ADJ) lam = run && lam_tile(it.a, it.blk, it.sg);
        if (!run) pre = false;
        else if (lam) pre = rtile_body<R, ADJ, RB, NT, InterpProg, true>(it.a, smem, it.blk, it.sg, pre, it.next_blk);
        else pre = rtile_body<R, ADJ, RB, NT>(it.a, smem, it.blk, it.sg, pre, it.next_blk);
        // every wave's stores of the tile have reached the L2 (vmcnt 0; expcnt and lgkmcnt left alone), so
        // thread 0's device-scope release below (one L2 write-back) covers them all
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(pa.done + it.sg.circ, 1ull);
            int64_t next = item + 1, nend = end;
            if (next >= end) {
                next = (int64_t)atomicAdd(pa.head, (unsigned long long)K);
                nend = next + K < pa.n_items ? next + K : pa.n_items;
            }
            // a prefetched successor shares this item's dependency and run flag
            int r = run ? 1 : 0;
            if (!pre && next < pa.n_items) r = (int)persist_wait(pa, persist_item(pa, next, nend).sg);
            item_s = next;
            end_s = nend;
            run_s = r;
        }
        __syncthreads();
        item = uniform_i64(item_s);
        end = uniform_i64(end_s);
        run = uniform_i64(run_s) != 0;
    }
}

template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rtile_fwd_persist(PersistArgs pa)
{
    persistent_body<R, false, RB, NT>(pa);
}

template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) void k_rtile_adj_persist(PersistArgs pa)
{
    persistent_body<R, true, RB, NT>(pa);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ------------------------------------------------------------------------------------------------------
// Stride pass: one gate straight from global memory. Each block handles kStrideGroupsPerBlock amplitude
// pairs (one-qubit gates) or quads (two-qubit gates); op.p0/op.p1 hold the gate's qubits.
// ------------------------------------------------------------------------------------------------------

// 16 bytes of amplitudes: two complex64 or one complex128, moved as one vector load or store.
template <typename R>
struct Vec16 {
    typedef float T __attribute__((ext_vector_type(4)));
    static constexpr int E = 2;
    __device__ static Cx<R> get(const T &v, int e) { return e ? Cx<R>{v.z, v.w} : Cx<R>{v.x, v.y}; }
    __device__ static void put(T &v, int e, const Cx<R> &c)
    {
        if (e) { v.z = c.re; v.w = c.im; } else { v.x = c.re; v.y = c.im; }
    }
    __device__ static T shfl_xor(const T &v, int d)
    {
        return T{__shfl_xor(v.x, d, 64), __shfl_xor(v.y, d, 64), __shfl_xor(v.z, d, 64), __shfl_xor(v.w, d, 64)};
    }
};
template <>
struct Vec16<double> {
    typedef double T __attribute__((ext_vector_type(2)));
    static constexpr int E = 1;
    __device__ static Cx<double> get(const T &v, int) { return Cx<double>{v.x, v.y}; }
    __device__ static void put(T &v, int, const Cx<double> &c) { v.x = c.re; v.y = c.im; }
    __device__ static T shfl_xor(const T &v, int d) { return T{__shfl_xor(v.x, d, 64), __shfl_xor(v.y, d, 64)}; }
};

// A one-qubit gate on qubit p as a stream over the state: every byte is read once and written once, in
// 16-byte vectors, each thread issuing all loads of a round before its first store; with NT (states larger
// than the caches) the accesses carry the non-temporal hint. Vector index j holds amplitudes
// E*j .. E*j+E-1, so qubit p is bit pb = p - log2(E) of j. When pb < 6 the partner vector (j ^ 2^pb) is in the same wave: every lane reads the vector at its
// own index, consecutive lanes consecutive vectors, and gets its partner from lane ^ 2^pb by a shuffle
// (pb < 0, complex64 with p = 0: both amplitudes of a pair are in one vector). Otherwise a lane reads a
// vector and its partner 2^pb vectors on (runs of at least 64 vectors per wave). The adjoint moves lambda
// the same way and adds the pair's inner-product term where the generator's sum needs it (one lane per pair).
template <bool NT, typename T>
__device__ __forceinline__ T ld_vec(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st_vec(const T &v, T *p)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename R, bool ADJ, bool NT>
__device__ __forceinline__ double stride_one_qubit(Cx<R> *gpsi, Cx<R> *glam, int n, int p, int kind, bool train,
                                                   const M2<R> &m, int64_t chunk)
{
    using V = Vec16<R>;
    using VT = typename V::T;
    constexpr int E = V::E, LE = E == 2 ? 1 : 0;
    constexpr int UR = 4;                                    // vectors per round and thread
    const int64_t nv = (int64_t)1 << (n - LE);
    VT *vp = reinterpret_cast<VT *>(gpsi);
    VT *vl = reinterpret_cast<VT *>(glam);
    const int pb = p - LE;
    double acc = 0.0;
    if (pb < 6) {
        constexpr int VB = 2 * kStrideGroupsPerBlock / E;   // the block's vectors: its groups' amplitudes
        for (int r = 0; r < VB / kBlock; r += UR) {
            // loads are not branched around (lanes past the end of a small state read its last vector and
            // store nothing), so the compiler keeps them all in flight together
            VT x[UR], l[UR];
            int64_t j[UR];
#pragma unroll
            for (int k = 0; k < UR; k++) {
                j[k] = chunk * VB + (int64_t)(r + k) * kBlock + threadIdx.x;
                const int64_t jc = j[k] < nv ? j[k] : nv - 1;
                x[k] = ld_vec<NT>(vp + jc);
                if (ADJ) l[k] = ld_vec<NT>(vl + jc);
            }
#pragma unroll
            for (int k = 0; k < UR; k++) {
                VT o = x[k], ol = ADJ ? l[k] : x[k];
                const bool live = j[k] < nv;   // lanes past the end hold a copy of the last vector
                if (pb < 0) {
                    Cx<R> a0 = V::get(x[k], 0), a1 = V::get(x[k], 1);
                    if (ADJ) {
                        Cx<R> u0 = V::get(l[k], 0), u1 = V::get(l[k], 1);
                        if (train && live) acc += gen_inner<R>(kind, a0, a1, u0, u1);
                        apply2(m, u0, u1);
                        V::put(ol, 0, u0);
                        V::put(ol, 1, u1);
                    }
                    apply2(m, a0, a1);
                    V::put(o, 0, a0);
                    V::put(o, 1, a1);
                } else {
                    const int d = 1 << pb;
                    const VT w = V::shfl_xor(x[k], d);
                    VT wl = w;
                    if (ADJ) wl = V::shfl_xor(l[k], d);
                    const bool hi = (j[k] >> pb) & 1;   // this lane holds the pairs' |1> side
#pragma unroll
                    for (int e = 0; e < E; e++) {
                        Cx<R> a0 = V::get(hi ? w : x[k], e), a1 = V::get(hi ? x[k] : w, e);
                        if (ADJ) {
                            Cx<R> u0 = V::get(hi ? wl : l[k], e), u1 = V::get(hi ? l[k] : wl, e);
                            if (train && live && !hi) acc += gen_inner<R>(kind, a0, a1, u0, u1);
                            apply2(m, u0, u1);
                            V::put(ol, e, hi ? u1 : u0);
                        }
                        apply2(m, a0, a1);
                        V::put(o, e, hi ? a1 : a0);
                    }
                }
                if (live) {
                    st_vec<NT>(o, vp + j[k]);
                    if (ADJ) st_vec<NT>(ol, vl + j[k]);
                }
            }
        }
        return acc;
    }
    constexpr int UB = kStrideGroupsPerBlock / E;            // the block's vector pairs
    constexpr int UU = UR / 2;                               // pairs per round and thread
    const int64_t nu = nv >> 1, half = (int64_t)1 << pb;
    for (int r = 0; r < UB / kBlock; r += UU) {
        VT x[UU], y[UU], lx[UU], ly[UU];
        int64_t ia[UU];
        bool in[UU];
#pragma unroll
        for (int k = 0; k < UU; k++) {
            const int64_t u = chunk * UB + (int64_t)(r + k) * kBlock + threadIdx.x;
            in[k] = u < nu;
            ia[k] = (int64_t)insert0_64((uint64_t)(in[k] ? u : nu - 1), pb);
            x[k] = ld_vec<NT>(vp + ia[k]);
            y[k] = ld_vec<NT>(vp + ia[k] + half);
            if (ADJ) {
                lx[k] = ld_vec<NT>(vl + ia[k]);
                ly[k] = ld_vec<NT>(vl + ia[k] + half);
            }
        }
#pragma unroll
        for (int k = 0; k < UU; k++) {
            if (!in[k]) continue;
#pragma unroll
            for (int e = 0; e < E; e++) {
                Cx<R> a0 = V::get(x[k], e), a1 = V::get(y[k], e);
                if (ADJ) {
                    Cx<R> u0 = V::get(lx[k], e), u1 = V::get(ly[k], e);
                    if (train) acc += gen_inner<R>(kind, a0, a1, u0, u1);
                    apply2(m, u0, u1);
                    V::put(lx[k], e, u0);
                    V::put(ly[k], e, u1);
                }
                apply2(m, a0, a1);
                V::put(x[k], e, a0);
                V::put(y[k], e, a1);
            }
            st_vec<NT>(x[k], vp + ia[k]);
            st_vec<NT>(y[k], vp + ia[k] + half);
            if (ADJ) {
                st_vec<NT>(lx[k], vl + ia[k]);
                st_vec<NT>(ly[k], vl + ia[k] + half);
            }
        }
    }
    return acc;
}

template <typename R, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_stride(LevelArgs a)
{
    __shared__ double red[kBlock / 64];
    const int64_t blk = (int64_t)blockIdx.x;
    const Seg sg = a.segs[find_block(a.segs, a.n_segs, blk)];
    const int64_t chunk = blk - sg.first_block;
    const DevPass P = a.passes[sg.pass];
    const DevCirc C = a.circs[sg.circ];
    const int n = C.n;
    const DevOp op = a.ops[P.op_begin];
    const int kind = op.kind;
    Cx<R> *gpsi = reinterpret_cast<Cx<R> *>(a.psi) + C.state_off;
    Cx<R> *glam = ADJ ? reinterpret_cast<Cx<R> *>(a.lam) + C.state_off : nullptr;
    const uint64_t g0 = (uint64_t)chunk * kStrideGroupsPerBlock;
    if (kind == QV_CNOT || kind == QV_CZ) {
        const uint64_t ngroups = 1ull << (n - 2);
        const uint64_t bc = 1ull << op.p0, bt = 1ull << op.p1;
        const int plo = op.p0 < op.p1 ? op.p0 : op.p1, phi = op.p0 < op.p1 ? op.p1 : op.p0;
        for (uint32_t e = threadIdx.x; e < kStrideGroupsPerBlock; e += kBlock) {
            const uint64_t gi = g0 + e;
            if (gi >= ngroups) break;
            const uint64_t i00 = insert0_64(insert0_64(gi, plo), phi);
            if (kind == QV_CNOT) {
                const uint64_t i10 = i00 | bc, i11 = i00 | bc | bt;
                Cx<R> x = gpsi[i10], y = gpsi[i11];
                gpsi[i10] = y; gpsi[i11] = x;
                if (ADJ) { Cx<R> u = glam[i10], v = glam[i11]; glam[i10] = v; glam[i11] = u; }
            } else {
                const uint64_t i11 = i00 | bc | bt;
                Cx<R> x = gpsi[i11]; x.re = -x.re; x.im = -x.im; gpsi[i11] = x;
                if (ADJ) { Cx<R> u = glam[i11]; u.re = -u.re; u.im = -u.im; glam[i11] = u; }
            }
        }
        return;
    }
    M2<R> m = op_matrix<R>(a, C, sg.circ, op, P.op_begin);
    if (ADJ) m = dagger_r(m);
    const bool train = (op.flags & OP_TRAIN) != 0;
    const double acc = a.stream ? stride_one_qubit<R, ADJ, true>(gpsi, glam, n, op.p0, kind, train, m, chunk)
                                : stride_one_qubit<R, ADJ, false>(gpsi, glam, n, op.p0, kind, train, m, chunk);
    if (ADJ && (op.flags & OP_TRAIN)) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) a.partials[sg.partial_base + chunk * P.n_train + op.train_slot] = s;
    }
}

// Matrix table: the 2x2 matrix of every one-qubit gate record at the current parameters (FP64 angles and
// trigonometry, rounded to the state precision).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_matrices(MatArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n_gates) return;
    const DevCirc C = a.circs[a.gate_circ[i]];
    const DevOp op = a.ops[C.op_base + (i - C.mat_off)];
    M2d md;
    if (op.kind == kFusedKind) {
        gate_matrix(-1, 0.0, md);
        reinterpret_cast<M2<R> *>(a.mats)[i] = narrow<R>(md);
        return;
    }
    const qv_gate g = a.gates[C.gate_off + op.gate];
    if (g.kind == QV_CNOT || g.kind == QV_CZ) {
        gate_matrix(-1, 0.0, md);
    } else {
        const double ang = g.param >= 0 ? a.theta[C.param_base + g.param] : g.angle;
        gate_matrix(g.kind, ang, md);
    }
    reinterpret_cast<M2<R> *>(a.mats)[i] = narrow<R>(md);
}

// Shifted-gate matrices of parameter-shift variants (FP64 angle and trigonometry, rounded to the state
// precision), one thread per circuit.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_shift_matrices(ShiftMatArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n_circ) return;
    const DevCirc C = a.circs[i];
    if (C.shift_gate < 0) return;
    const qv_gate g = a.gates[C.gate_off + C.shift_gate];
    const double ang = (g.param >= 0 ? a.theta[C.param_base + g.param] : g.angle) + C.shift;
    M2d md;
    gate_matrix(g.kind, ang, md);
    reinterpret_cast<M2<R> *>(a.smats)[i] = narrow<R>(md);
}

// The restoring phase of one circuit's state (one workgroup): exp(-i/2 sum of its RZ angles), each angle
// taken modulo 4 pi first (the period of e^{-ia/2}).
__global__ __launch_bounds__(kBlock) void k_rz_phase(StatePhaseArgs a)
{
    __shared__ double red[kBlock / 64];
    const double period = 4.0 * 3.14159265358979323846;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < a.n_gates; i += kBlock) {
        const qv_gate g = a.gates[i];
        if (g.kind == QV_RZ) acc += fmod(g.param >= 0 ? a.theta[g.param] : g.angle, period);
    }
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) {
        double sn, cs;
        sincos(-0.5 * sum, &sn, &cs);
        a.phase[0] = cs;
        a.phase[1] = sn;
    }
}

// dst = phase * src over a range of one circuit's amplitudes (grid-stride).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_scale_copy(StatePhaseArgs a)
{
    const R c = (R)a.phase[0], s = (R)a.phase[1];
    const Cx<R> *src = reinterpret_cast<const Cx<R> *>(a.src);
    Cx<R> *dst = reinterpret_cast<Cx<R> *>(a.dst);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n_amps; i += (int64_t)gridDim.x * kBlock) {
        const Cx<R> x = src[i];
        Cx<R> y;
        y.re = c * x.re - s * x.im;
        y.im = c * x.im + s * x.re;
        dst[i] = y;
    }
}

// Fused-block matrices: one workgroup per (circuit, block) multiplies the block's gates into a 16x16
// complex matrix in LDS (thread (r, c) owns entry r, c; each gate acts on the rows of its register bits),
// then writes the 32x32 real form in the order fused_mfma reads it: entry s*64 + l is A[l % 32][2s + l / 32].
__global__ __launch_bounds__(256) void k_fuse(FuseArgs a)
{
    __shared__ float ur[256], ui[256];
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const int64_t f = blk - a.first_block[c];
    const int64_t mk = a.fused_ops[C.fused_ops + f];
    const DevOp marker = a.ops[mk];
    const int m = marker.pad;
    const int r = threadIdx.x >> 4, col = threadIdx.x & 15;
    ur[threadIdx.x] = r == col ? 1.f : 0.f;
    ui[threadIdx.x] = 0.f;
    __syncthreads();
    const M2<float> *mt = reinterpret_cast<const M2<float> *>(a.mats) + (C.mat_off - C.op_base);
    for (int j = 1; j <= m; j++) {
        const DevOp op = a.ops[mk + j];
        float nr, ni;
        if (op.kind == QV_CNOT) {
            const int src = ((r >> op.k0) & 1) ? (r ^ (1 << op.k1)) : r;
            nr = ur[src * 16 + col];
            ni = ui[src * 16 + col];
        } else if (op.kind == QV_CZ) {
            const float sg = (((r >> op.k0) & 1) && ((r >> op.k1) & 1)) ? -1.f : 1.f;
            nr = sg * ur[threadIdx.x];
            ni = sg * ui[threadIdx.x];
        } else {
            const M2<float> g = mt[mk + j];
            const int b = (r >> op.k0) & 1;
            const int r0 = r & ~(1 << op.k0), r1 = r | (1 << op.k0);
            const float g0r = g.re[2 * b], g0i = g.im[2 * b], g1r = g.re[2 * b + 1], g1i = g.im[2 * b + 1];
            const float x0r = ur[r0 * 16 + col], x0i = ui[r0 * 16 + col];
            const float x1r = ur[r1 * 16 + col], x1i = ui[r1 * 16 + col];
            nr = g0r * x0r - g0i * x0i + g1r * x1r - g1i * x1i;
            ni = g0r * x0i + g0i * x0r + g1r * x1i + g1i * x1r;
        }
        __syncthreads();
        ur[threadIdx.x] = nr;
        ui[threadIdx.x] = ni;
        __syncthreads();
    }
    float *out = a.fmats + (C.fused_off + f) * (int64_t)kFusedFloats;
    for (int e = threadIdx.x; e < kFusedFloats; e += 256) {
        const int s = e >> 6, l = e & 63;
        const int i = l & 31, k = 2 * s + (l >> 5);
        const int rr = i >> 1, pr = i & 1, cc = k >> 1, pc = k & 1;
        const float re = ur[rr * 16 + cc], im = ui[rr * 16 + cc];
        out[e] = pr == pc ? re : (pr == 0 ? -im : im);
    }
}

// psi_b = |0...0> for every circuit; blocks cover 4096 amplitudes each.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_init(Cx<R> *psi, const DevCirc *circs, const int64_t *first_block,
                                                 int32_t n_circ)
{
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(first_block, n_circ, blk);
    const DevCirc C = circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t e0 = (uint64_t)(blk - first_block[c]) * 4096ull;
    Cx<R> *st = psi + C.state_off;
    for (uint32_t e = threadIdx.x; e < 4096u; e += kBlock) {
        const uint64_t i = e0 + e;
        if (i >= dim) break;
        Cx<R> v;
        v.re = (i == 0) ? (R)1 : (R)0;
        v.im = (R)0;
        st[i] = v;
    }
}

// ------------------------------------------------------------------------------------------------------
// Pauli expectations. A block handles 2^chunk_log2 pairs {b, b ^ x} (or amplitudes when x == 0) of one
// x-mask group and writes one FP64 partial sum per term of the group.
// ------------------------------------------------------------------------------------------------------
// A block's items (amplitudes, or pairs when x != 0) are i = i0 | tid | (k << 8): i0 the block's first item
// (a multiple of its chunk), tid the thread, k the loop step, which is the same for the whole wave. The
// sign (-1)^{popcount(b & z)} of a term therefore splits into a thread part, taken once, and a part that
// depends on k alone, computed in scalar registers, so each term costs one FP64 fused multiply-add per
// item (two for pairs: the real and imaginary parts of conj(psi[b ^ x]) psi[b], one of whose weights is 0).
// When x != 0, b = i with a zero inserted at bit h (the top bit of x), so popcount(b & z) = popcount(i & z'),
// z' being z with bit h removed.
// One amplitude, with the non-temporal hint when NT (a large state is read once per group and cannot stay
// cached between groups; a small one is re-read from the caches by its other groups).
template <bool NT, typename R>
__device__ __forceinline__ Cx<R> ld_amp(const Cx<R> *p)
{
    typedef R V2 __attribute__((ext_vector_type(2)));
    const V2 v = ld_vec<NT>(reinterpret_cast<const V2 *>(p));
    return Cx<R>{v.x, v.y};
}

// The group's TERMS accumulators (1, 2, 4 or 8; those past the group's n_terms have weight zero, so no
// term test sits in the loops). Loop steps whose 256 items all lie in the block's chunk run U at a time with
// no bounds tests; the remaining steps run one at a time, an item past the end reading the chunk's last
// item with weight zero. The block then writes one partial per term: wave sums, one barrier, and a fixed
// order over the waves.
template <typename R, bool NT, int TERMS>
__device__ __forceinline__ void expect_group(const ExpArgs &a, const DevGroup &G, int64_t chunk, double *red)
{
    const DevCirc C = a.circs[G.circ];
    const Cx<R> *st = reinterpret_cast<const Cx<R> *>(a.psi) + C.state_off;
    const int nt = G.n_terms;
    const uint64_t x = G.xmask;
    const int h = x ? 63 - __clzll(x) : 0;
    const uint32_t per = 1u << G.chunk_log2;
    const uint64_t i0 = (uint64_t)chunk << G.chunk_log2;
    const uint64_t items = x ? (1ull << (C.n - 1)) : (1ull << C.n);
    const uint32_t lim = (uint32_t)(items - i0 < (uint64_t)per ? items - i0 : (uint64_t)per);
    const uint32_t nk = (lim + kBlock - 1) / kBlock, nfull = lim / kBlock;
    uint32_t zk[TERMS];   // the loop-step part of each term's z (item bits 8 and up, within the chunk)
    double fr[TERMS], fi[TERMS];  // weights of Re w and Im w (the same for every thread)
    double ts[TERMS], acc[TERMS];  // the thread's part of the sign; its sum
#pragma unroll
    for (int j = 0; j < TERMS; j++) {
        const uint64_t z = j < nt ? a.terms[G.term_begin + j].zmask : 0;
        const int q = j < nt ? a.terms[G.term_begin + j].ny : 0;
        const uint64_t zs = x ? ((z & ((1ull << h) - 1ull)) | ((z >> (h + 1)) << h)) : z;
        zk[j] = (uint32_t)(zs >> 8) & ((per - 1u) >> 8);
        // Re[i^q w] = wr, -wi, -wr, wi for q = 0..3; a pair counts twice
        const double w2 = j < nt ? (x ? 2.0 : 1.0) : 0.0;
        fr[j] = q == 0 ? w2 : q == 2 ? -w2 : 0.0;
        fi[j] = q == 1 ? -w2 : q == 3 ? w2 : 0.0;
        ts[j] = parity64((i0 | (uint64_t)threadIdx.x) & zs) ? -1.0 : 1.0;
        acc[j] = 0.0;
    }
    if (x == 0) {
        constexpr uint32_t U = 8;
        uint32_t k0 = 0;
        for (; k0 + U <= nfull; k0 += U) {
            double w[U];
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const Cx<R> v = ld_amp<NT>(st + i0 + threadIdx.x + (k0 + u) * kBlock);
                w[u] = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; u++)
#pragma unroll
                for (int j = 0; j < TERMS; j++)
                    acc[j] = fma(__popc((k0 + u) & zk[j]) & 1 ? -fr[j] : fr[j], w[u], acc[j]);
        }
        for (; k0 < nk; k0++) {
            const uint32_t e = threadIdx.x + k0 * kBlock;
            const Cx<R> v = ld_amp<NT>(st + i0 + (e < lim ? e : lim - 1));
            const double w = (e < lim ? 1.0 : 0.0) * ((double)v.re * (double)v.re + (double)v.im * (double)v.im);
#pragma unroll
            for (int j = 0; j < TERMS; j++) acc[j] = fma(__popc(k0 & zk[j]) & 1 ? -fr[j] : fr[j], w, acc[j]);
        }
    } else {
        // w = conj(psi[b ^ x]) psi[b] for the pair's lower index b (item i with a zero inserted at bit h)
        constexpr uint32_t U = 4;
        uint32_t k0 = 0;
        for (; k0 + U <= nfull; k0 += U) {
            double wr[U], wi[U];
#pragma unroll
            for (uint32_t u = 0; u < U; u++) {
                const uint64_t b = insert0_64(i0 + threadIdx.x + (k0 + u) * kBlock, h);
                const Cx<R> a0 = ld_amp<NT>(st + b), a1 = ld_amp<NT>(st + (b ^ x));
                wr[u] = (double)a1.re * (double)a0.re + (double)a1.im * (double)a0.im;
                wi[u] = (double)a1.re * (double)a0.im - (double)a1.im * (double)a0.re;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; u++)
#pragma unroll
                for (int j = 0; j < TERMS; j++) {
                    const bool neg = __popc((k0 + u) & zk[j]) & 1;
                    acc[j] = fma(neg ? -fr[j] : fr[j], wr[u], acc[j]);
                    acc[j] = fma(neg ? -fi[j] : fi[j], wi[u], acc[j]);
                }
        }
        for (; k0 < nk; k0++) {
            const uint32_t e = threadIdx.x + k0 * kBlock;
            const uint64_t b = insert0_64(i0 + (e < lim ? e : lim - 1), h);
            const Cx<R> a0 = ld_amp<NT>(st + b), a1 = ld_amp<NT>(st + (b ^ x));
            const double keep = e < lim ? 1.0 : 0.0;
            const double wr = keep * ((double)a1.re * (double)a0.re + (double)a1.im * (double)a0.im);
            const double wi = keep * ((double)a1.re * (double)a0.im - (double)a1.im * (double)a0.re);
#pragma unroll
            for (int j = 0; j < TERMS; j++) {
                const bool neg = __popc(k0 & zk[j]) & 1;
                acc[j] = fma(neg ? -fr[j] : fr[j], wr, acc[j]);
                acc[j] = fma(neg ? -fi[j] : fi[j], wi, acc[j]);
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < TERMS; j++) {
        double v = ts[j] * acc[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave * TERMS + j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nt) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; w++) s += red[w * TERMS + threadIdx.x];
        a.partials[G.partial_base + chunk * nt + threadIdx.x] = s;
    }
}

template <typename R, bool NT>
__device__ __forceinline__ void expect_terms(const ExpArgs &a, const DevGroup &G, int64_t chunk, double *red)
{
    static_assert(kMaxGroupTerms == 8, "accumulator counts below cover groups of up to 8 terms");
    if (G.n_terms <= 1) expect_group<R, NT, 1>(a, G, chunk, red);
    else if (G.n_terms <= 2) expect_group<R, NT, 2>(a, G, chunk, red);
    else if (G.n_terms <= 4) expect_group<R, NT, 4>(a, G, chunk, red);
    else expect_group<R, NT, 8>(a, G, chunk, red);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_expect(ExpArgs a)
{
    __shared__ double red[(kBlock / 64) * kMaxGroupTerms];
    const int64_t blk = (int64_t)blockIdx.x;
    const DevGroup G = a.groups[find_block(a.groups, a.n_groups, blk)];
    const int64_t chunk = blk - G.first_block;
    if (a.stream) expect_terms<R, true>(a, G, chunk, red);
    else expect_terms<R, false>(a, G, chunk, red);
}

// Second stage of the expectation reduction: one workgroup per output (a term value, or a circuit's norm)
// sums that output's partials -- a fixed strided share per thread, then a fixed tree -- so the result does
// not depend on scheduling.
__global__ __launch_bounds__(kBlock) void k_finalize_refs(FinalizeArgs a)
{
    __shared__ double red[kBlock / 64];
    const int64_t o = (int64_t)blockIdx.x;
    const bool term = o < a.n_terms;
    const PartialRef r = term ? a.term_refs[o] : a.norm_refs[o - a.n_terms];
    double s = 0.0;
    for (int32_t c = threadIdx.x; c < r.count; c += kBlock) s += a.partials[r.base + (int64_t)c * r.stride];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        if (term) a.term_values[o] = s;
        else a.norms[o - a.n_terms] = s;
    }
}

// E_b = sum_t c_t <P_t>, in term order.
__global__ __launch_bounds__(kBlock) void k_finalize_energies(FinalizeArgs a)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= a.n_circ) return;
    double e = 0.0;
    for (int64_t o = a.tv_begin[b]; o < a.tv_begin[b + 1]; o++) e += a.coeff[o] * a.term_values[o];
    a.energies[b] = e;
}

// lambda_b[o] = w_b sum_t c_t (P_t psi_b)[o], (P psi)[o] = i^{ny} (-1)^{popcount((o^x) & z)} psi[o ^ x].
// A block covers 4096 consecutive amplitudes of one circuit, a thread kLambdaPer of them,
// o = o0 | tid | (j << 8), in rounds of kLambdaRound. Each round walks the terms in the host's x-mask order:
// at each new mask the thread reads psi[o ^ x] for the round's amplitudes at once, then adds every term of
// that mask. A term's sign splits like the expectation's: (-1)^popcount(x & z) and the thread's part
// (o0 | tid) & z once per term, the part of j from the wave-uniform z.
constexpr int kLambdaPer = 4096 / kBlock;
constexpr int kLambdaRound = 8;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_lambda(LambdaArgs a)
{
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * 4096ull;
    const Cx<R> *st = reinterpret_cast<const Cx<R> *>(a.psi) + C.state_off;
    Cx<R> *lam = reinterpret_cast<Cx<R> *>(a.lam) + C.state_off;
    const double w = a.upstream ? a.upstream[C.base_circ] : 1.0;
    const int64_t tb = a.obs_begin[c], te = a.obs_begin[c + 1];
    const uint64_t ot = o0 | (uint64_t)threadIdx.x;
    for (int h = 0; h < kLambdaPer; h += kLambdaRound) {
        double ar[kLambdaRound], ai[kLambdaRound];
        Cx<R> v[kLambdaRound];
#pragma unroll
        for (int j = 0; j < kLambdaRound; j++) {
            ar[j] = ai[j] = 0.0;
            v[j].re = v[j].im = (R)0;
        }
        uint64_t px = ~0ull;
        for (int64_t t = tb; t < te; t++) {
            const DevObsTerm term = ldu(a.obs + t);
            if (term.xmask != px) {
                px = term.xmask;
#pragma unroll
                for (int j = 0; j < kLambdaRound; j++) {
                    const uint64_t o = ot | ((uint64_t)(h + j) << 8);
                    v[j] = st[(o < dim ? o : 0ull) ^ px];   // past a small state's end: a valid amplitude
                }
            }
            // c i^ny as a complex weight, signed by the parts of the sign that do not depend on j
            const double c0 =
                (parity64(term.xmask & term.zmask) ^ parity64(ot & term.zmask)) ? -term.coeff : term.coeff;
            const double wr = (term.ny & 1) ? 0.0 : ((term.ny & 2) ? -c0 : c0);
            const double wi = (term.ny & 1) ? ((term.ny & 2) ? -c0 : c0) : 0.0;
            const uint32_t zj = (uint32_t)(term.zmask >> 8) & (uint32_t)(kLambdaPer - 1);
#pragma unroll
            for (int j = 0; j < kLambdaRound; j++) {
                const bool neg = __popc((uint32_t)(h + j) & zj) & 1;
                const double sr = neg ? -wr : wr, si = neg ? -wi : wi;
                const double xr = (double)v[j].re, xi = (double)v[j].im;
                ar[j] = fma(sr, xr, fma(-si, xi, ar[j]));
                ai[j] = fma(sr, xi, fma(si, xr, ai[j]));
            }
        }
#pragma unroll
        for (int j = 0; j < kLambdaRound; j++) {
            const uint64_t o = ot | ((uint64_t)(h + j) << 8);
            if (o < dim) {
                Cx<R> out;
                out.re = (R)(w * ar[j]);
                out.im = (R)(w * ai[j]);
                lam[o] = out;
            }
        }
    }
}

// grad[g] = sum over refs of g of sum_c partials[base + c * stride], one block per output.
__global__ __launch_bounds__(kBlock) void k_grad_reduce(GradReduceArgs a)
{
    __shared__ double red[kBlock / 64];
    const int g = blockIdx.x;
    double s = 0.0;
    for (int64_t r = a.ref_begin[g]; r < a.ref_begin[g + 1]; r++) {
        const PartialRef ref = a.refs[r];
        for (int32_t c = threadIdx.x; c < ref.count; c += kBlock) s += a.partials[ref.base + (int64_t)c * ref.stride];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) a.grad[g] = s;
}

__global__ void k_shift_combine(ShiftCombineArgs a)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_out) return;
    double s = 0.0;
    for (int64_t k = a.occ_begin[g]; k < a.occ_begin[g + 1]; k++) {
        const double w = a.upstream ? a.upstream[a.occ_circ[k]] : 1.0;
        s += w * 0.5 * (a.energies[a.occ_plus[k]] - a.energies[a.occ_minus[k]]);
    }
    a.grad[g] = s;
}

// ------------------------------------------------------------------------------------------------------
// Probability path (Section 4.2): the output distribution P_theta(b) = |psi_b|^2 over all bit strings, the
// Jensen-Shannon divergence of Eq. 3 against a target distribution P, and its derivative. With M = (P + Q)/2
// and Q = P_theta, dJS/dQ(b) = log(Q(b)/M(b)) / 2; a bit string with Q(b) = 0 gets weight 0 (Q is at its
// minimum there, so dQ/dtheta = 0) and 0 log 0 counts as 0. The gradient of the divergence is then the
// gradient of the diagonal observable diag(w) at fixed w, by either rule.
// ------------------------------------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_probs(ProbArgs a)
{
    __shared__ double red[kBlock / 64];
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * 4096ull;
    const Cx<R> *st = reinterpret_cast<const Cx<R> *>(a.psi) + C.state_off;
    double js = 0.0;
    for (uint32_t e = threadIdx.x; e < 4096u; e += kBlock) {
        const uint64_t o = o0 + e;
        if (o >= dim) break;
        const Cx<R> v = st[o];
        const double vr = v.re, vi = v.im;
        const double q = vr * vr + vi * vi;
        const int64_t i = C.state_off + (int64_t)o;
        if (a.probs) a.probs[i] = q;
        if (a.target) {
            const double p = a.target[i];
            const double m = 0.5 * (p + q);
            if (p > 0.0) js += p * log(p / m);
            if (q > 0.0) js += q * log(q / m);
            a.w[i] = q > 0.0 ? 0.5 * log(q / m) : 0.0;
        }
    }
    if (a.partials) {
        js = block_sum(js, red);
        if (threadIdx.x == 0) a.partials[blk] = js;
    }
}

// lambda = u_b diag(w) psi: the adjoint seed of the diagonal observable.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag_seed(DiagArgs a)
{
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * 4096ull;
    const Cx<R> *st = reinterpret_cast<const Cx<R> *>(a.psi) + C.state_off;
    Cx<R> *lam = reinterpret_cast<Cx<R> *>(a.lam) + C.state_off;
    const double *w = a.w + a.base_circs[C.base_circ].state_off;
    const double u = a.upstream ? a.upstream[C.base_circ] : 1.0;
    for (uint32_t e = threadIdx.x; e < 4096u; e += kBlock) {
        const uint64_t o = o0 + e;
        if (o >= dim) break;
        const Cx<R> v = st[o];
        const double f = u * w[o];
        Cx<R> out;
        out.re = (R)(f * (double)v.re);
        out.im = (R)(f * (double)v.im);
        lam[o] = out;
    }
}

// Per-block partial sums of <psi|diag(w)|psi> = sum_o w[o] |psi[o]|^2 (FP64).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag_expect(DiagArgs a)
{
    __shared__ double red[kBlock / 64];
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * 4096ull;
    const Cx<R> *st = reinterpret_cast<const Cx<R> *>(a.psi) + C.state_off;
    const double *w = a.w + a.base_circs[C.base_circ].state_off;
    double s = 0.0;
    for (uint32_t e = threadIdx.x; e < 4096u; e += kBlock) {
        const uint64_t o = o0 + e;
        if (o >= dim) break;
        const Cx<R> v = st[o];
        const double vr = v.re, vi = v.im;
        s += w[o] * (vr * vr + vi * vi);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) a.partials[blk] = s;
}

// One workgroup per output: a fixed strided share per thread, then a fixed tree.
__global__ __launch_bounds__(kBlock) void k_segment_sum(SegSumArgs a)
{
    __shared__ double red[kBlock / 64];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t j = a.first_block[c] + threadIdx.x; j < a.first_block[c + 1]; j += kBlock) s += a.partials[j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) a.out[c] = a.scale * s;
}

__global__ void k_fill(double *p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------------------------------------------
// Shots and bit-string counts (Section 3.1: a circuit's execution yields a table of observed bit strings
// and their counts; Section 4.2 works on those counts). Every sum below runs in a fixed order, so the
// draws are reproducible: a thread owns kSampleBlock / kBlock consecutive entries of a block and sums them
// left to right, thread 0 scans the thread totals, and the block's prefixes are the thread's running sum
// plus its offset.
// ------------------------------------------------------------------------------------------------------
constexpr int kSamplePer = kSampleBlock / kBlock;  // 16 entries per thread

// Exclusive prefix of the kBlock values tot[] in thread order, in place; returns the block total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T *tot)
{
    __syncthreads();
    __shared__ T total_s;
    if (threadIdx.x == 0) {
        T run = 0;
        for (int t = 0; t < kBlock; t++) {
            const T v = tot[t];
            tot[t] = run;
            run += v;
        }
        total_s = run;
    }
    __syncthreads();
    return total_s;
}

// Per block: prefix sums of the distribution within the block (local) and the block total (bsum).
__global__ __launch_bounds__(kBlock) void k_cdf_local(SampleArgs a)
{
    __shared__ double q[kSampleBlock];
    __shared__ double tot[kBlock];
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * kSampleBlock;
    const uint32_t lim = (uint32_t)(dim - o0 < (uint64_t)kSampleBlock ? dim - o0 : (uint64_t)kSampleBlock);
    const double *pr = a.probs + C.state_off + o0;
    for (uint32_t e = threadIdx.x; e < (uint32_t)kSampleBlock; e += kBlock) q[e] = e < lim ? pr[e] : 0.0;
    __syncthreads();
    const int t0 = threadIdx.x * kSamplePer;
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < kSamplePer; k++) {
        run += q[t0 + k];
        q[t0 + k] = run;
    }
    tot[threadIdx.x] = run;
    const double total = block_exclusive_scan(tot);
    const double off = tot[threadIdx.x];
    double *lo = a.local + C.state_off + o0;
#pragma unroll
    for (int k = 0; k < kSamplePer; k++)
        if ((uint32_t)(t0 + k) < lim) lo[t0 + k] = off + q[t0 + k];
    if (threadIdx.x == 0) a.bsum[blk] = total;
}

// One workgroup per circuit: exclusive prefix of its block totals (boff) and the circuit's total.
template <typename T>
__device__ __forceinline__ T segment_exclusive_scan(const T *in, T *out, int64_t b0, int64_t b1)
{
    __shared__ T tot[kBlock];
    const int64_t nb = b1 - b0;
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t j0 = b0 + (int64_t)threadIdx.x * per;
    const int64_t j1 = j0 + per < b1 ? j0 + per : b1;
    T run = 0;
    for (int64_t j = j0; j < j1; j++) run += in[j];
    tot[threadIdx.x] = run;
    const T total = block_exclusive_scan(tot);
    T acc = tot[threadIdx.x];
    for (int64_t j = j0; j < j1; j++) {
        const T v = in[j];
        out[j] = acc;
        acc += v;
    }
    return total;
}

__global__ __launch_bounds__(kBlock) void k_cdf_blocks(SampleArgs a)
{
    const int c = blockIdx.x;
    const double t = segment_exclusive_scan<double>(a.bsum, a.boff, a.first_block[c], a.first_block[c + 1]);
    if (threadIdx.x == 0) a.total[c] = t;
}

// One thread per shot: the first bit string x with C(x) > u * C(last), by binary search over the circuit's
// blocks and then within the block; the shot is counted in the histogram.
__global__ __launch_bounds__(kBlock) void k_draw(SampleArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (int64_t)a.n_circ * a.shots) return;
    const int c = (int)(s / a.shots);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    double u = a.uniforms[s];
    u = u >= 0.0 ? u : 0.0;
    u = u < 1.0 ? u : 0x1.fffffffffffffp-1;
    const double target = u * a.total[c];
    int64_t lo = a.first_block[c], hi = a.first_block[c + 1] - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.boff[mid] + a.bsum[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    const uint64_t o0 = (uint64_t)(lo - a.first_block[c]) * kSampleBlock;
    const double off = a.boff[lo];
    const double *loc = a.local + C.state_off + o0;
    int64_t e0 = 0, e1 = (int64_t)(dim - o0 < (uint64_t)kSampleBlock ? dim - o0 : (uint64_t)kSampleBlock) - 1;
    while (e0 < e1) {
        const int64_t mid = (e0 + e1) >> 1;
        if (off + loc[mid] > target) e1 = mid;
        else e0 = mid + 1;
    }
    const uint64_t x = o0 + (uint64_t)e0;
    if (a.samples) a.samples[s] = (int64_t)x;
    atomicAdd(a.hist + C.state_off + x, 1u);
}

// Per block: how many bit strings were drawn at least once.
__global__ __launch_bounds__(kBlock) void k_hist_nnz(SampleArgs a)
{
    __shared__ double red[kBlock / 64];
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * kSampleBlock;
    double n = 0.0;
    for (uint32_t e = threadIdx.x; e < (uint32_t)kSampleBlock; e += kBlock)
        if (o0 + e < dim && a.hist[C.state_off + o0 + e] != 0u) n += 1.0;
    n = block_sum(n, red);
    if (threadIdx.x == 0) a.nnz[blk] = (int64_t)n;
}

__global__ __launch_bounds__(kBlock) void k_hist_offsets(SampleArgs a)
{
    const int c = blockIdx.x;
    const int64_t t = segment_exclusive_scan<int64_t>(a.nnz, a.noff, a.first_block[c], a.first_block[c + 1]);
    if (threadIdx.x == 0) a.n_distinct[c] = t;
}

// Per block: its drawn bit strings and counts, in increasing order, after those of earlier blocks.
__global__ __launch_bounds__(kBlock) void k_hist_emit(SampleArgs a)
{
    __shared__ int64_t tot[kBlock];
    const int64_t blk = (int64_t)blockIdx.x;
    const int c = find_prefix(a.first_block, a.n_circ, blk);
    const DevCirc C = a.circs[c];
    const uint64_t dim = 1ull << C.n;
    const uint64_t o0 = (uint64_t)(blk - a.first_block[c]) * kSampleBlock;
    const int t0 = threadIdx.x * kSamplePer;
    const uint32_t *h = a.hist + C.state_off + o0;
    int64_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kSamplePer; k++)
        if (o0 + (uint64_t)(t0 + k) < dim && h[t0 + k] != 0u) cnt++;
    tot[threadIdx.x] = cnt;
    block_exclusive_scan(tot);
    int64_t pos = (int64_t)c * a.shots + a.noff[blk] + tot[threadIdx.x];
#pragma unroll
    for (int k = 0; k < kSamplePer; k++) {
        const uint64_t x = o0 + (uint64_t)(t0 + k);
        if (x < dim && h[t0 + k] != 0u) {
            a.bits[pos] = x;
            a.counts[pos] = (int64_t)h[t0 + k];
            pos++;
        }
    }
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------------
// LDS of a tile launch: the tile (twice for the adjoint), the table of 2^tab_bits run offsets, and a
// small reduction area.
static size_t tile_lds_bytes(int lds_t, int tab_bits, int amp_bytes, int adjoint)
{
    return (size_t)(adjoint ? 2 : 1) * ((size_t)1 << lds_t) * amp_bytes + ((size_t)8 << tab_bits) +
           sizeof(double) * (kBlock / 64);
}

// Dynamic LDS the persistent kernels may use: the whole 160 KiB less their static work-item slot.
constexpr int kLdsLimit = 160 * 1024;
constexpr int kPersistStaticLds = 64;

static hipError_t allow_lds(const void *fn, int bytes)
{
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

int prepare_kernels()
{
    const int lim = kLdsLimit, plim = kLdsLimit - kPersistStaticLds;
    const struct { const void *fn; int bytes; } ks[] = {
        {reinterpret_cast<const void *>(&k_tile<float, false>), lim},
        {reinterpret_cast<const void *>(&k_tile<float, true>), lim},
        {reinterpret_cast<const void *>(&k_tile<double, false>), lim},
        {reinterpret_cast<const void *>(&k_tile<double, true>), lim},
        {reinterpret_cast<const void *>(&k_rtile_fwd<float, kRegBitsC64, kRtileThreads>), lim},
        {reinterpret_cast<const void *>(&k_rtile_adj<float, kRegBitsC64, kRtileThreads>), lim},
        {reinterpret_cast<const void *>(&k_rtile_fwd<double, kRegBitsC128, kRtileThreads>), lim},
        {reinterpret_cast<const void *>(&k_rtile_adj<double, kRegBitsC128, kRtileThreads>), lim},
        {reinterpret_cast<const void *>(&k_rtile_lam<float, kRegBitsC64, kRtileThreads>), lim},
        {reinterpret_cast<const void *>(&k_rtile_lam<double, kRegBitsC128, kRtileThreads>), lim},
        {reinterpret_cast<const void *>(&k_rtile_fwd_persist<float, kRegBitsC64, kRtileThreads>), plim},
        {reinterpret_cast<const void *>(&k_rtile_adj_persist<float, kRegBitsC64, kRtileThreads>), plim},
        {reinterpret_cast<const void *>(&k_rtile_fwd_persist<double, kRegBitsC128, kRtileThreads>), plim},
        {reinterpret_cast<const void *>(&k_rtile_adj_persist<double, kRegBitsC128, kRtileThreads>), plim},
    };
    for (const auto &k : ks) {
        const hipError_t e = allow_lds(k.fn, k.bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static size_t rtile_lds_bytes(int precision, int adjoint, int lds_t, int tab_bits, int max_train)
{
    const int amp = precision == QV_C64 ? 8 : 16;
    return tile_lds_bytes(lds_t, tab_bits, amp, adjoint) +
           (adjoint ? sizeof(double) * (kRtileThreads / 64) * (size_t)max_train : 0);
}

int persistent_fits(int precision, int adjoint, int lds_t, int tab_bits, int max_train)
{
    return rtile_lds_bytes(precision, adjoint, lds_t, tab_bits, max_train) <=
           (size_t)(kLdsLimit - kPersistStaticLds);
}

int persistent_blocks(int precision, int adjoint, int lds_t, int tab_bits, int max_train, int *blocks)
{
    const size_t lds = rtile_lds_bytes(precision, adjoint, lds_t, tab_bits, max_train) + 64;
    if (lds > (size_t)kLdsLimit) return hipErrorInvalidValue;
    const void *k = precision == QV_C64
                        ? (adjoint ? reinterpret_cast<const void *>(&k_rtile_adj_persist<float, kRegBitsC64, kRtileThreads>)
                                   : reinterpret_cast<const void *>(&k_rtile_fwd_persist<float, kRegBitsC64, kRtileThreads>))
                        : (adjoint ? reinterpret_cast<const void *>(&k_rtile_adj_persist<double, kRegBitsC128, kRtileThreads>)
                                   : reinterpret_cast<const void *>(&k_rtile_fwd_persist<double, kRegBitsC128, kRtileThreads>));
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kRtileThreads, lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    *blocks = (per_cu < 1 ? 1 : per_cu) * cus;
    return hipSuccess;
}

int launch_persistent(const PersistArgs &a, int precision, int adjoint, void *stream)
{
    if (a.n_items <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t lds = rtile_lds_bytes(precision, adjoint, a.base.lds_t, a.base.tab_bits, a.base.max_train);
    if (lds > (size_t)(kLdsLimit - kPersistStaticLds)) return hipErrorInvalidValue;
    int blocks = 0;
    hipError_t e = (hipError_t)persistent_blocks(precision, adjoint, a.base.lds_t, a.base.tab_bits, a.base.max_train,
                                                 &blocks);
    if (e != hipSuccess) return e;
    // items claimed at once: as requested, else the level kernels' tile chunk halved until every
    // workgroup gets a claim
    PersistArgs pa = a;
    int64_t chunk = a.chunk;
    if (chunk <= 0) {
        chunk = adjoint ? tile_chunk<true>() : tile_chunk<false>();
        while (chunk > 1 && (a.n_items + chunk - 1) / chunk < blocks) chunk >>= 1;
    }
    pa.chunk = (int32_t)chunk;
    if ((int64_t)blocks > (a.n_items + chunk - 1) / chunk) blocks = (int)((a.n_items + chunk - 1) / chunk);
    const dim3 grid((unsigned)blocks), block(kRtileThreads);
    if (precision == QV_C64) {
        if (adjoint) hipLaunchKernelGGL((k_rtile_adj_persist<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, pa);
        else hipLaunchKernelGGL((k_rtile_fwd_persist<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, pa);
    } else {
        if (adjoint) hipLaunchKernelGGL((k_rtile_adj_persist<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, pa);
        else hipLaunchKernelGGL((k_rtile_fwd_persist<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, pa);
    }
    return hipGetLastError();
}

int launch_zero_u64(unsigned long long *p, int64_t n, void *stream)
{
    if (n <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// Scratch of qv_batch_expectations_static: the expectation partial sums of one call, at most
// kStaticScratchDoubles of them. Every device the library runs on holds its own copy until the process
// ends. The host-side name `scratch` is not a device address: host code uses the address looked up per
// device by static_scratch_setup, never the name itself.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

static double *g_scratch_addr[kMaxStaticDevices];
static std::mutex g_scratch_mu;

int static_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_addr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = static_cast<double *>(ptr);
    return hipSuccess;
}

double *static_scratch(int device)
{
    if (device < 0 || device >= kMaxStaticDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_addr[device];
}

// Compute units of the current device (cached per device).
static int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

int launch_rlevel_gen(const LevelArgs &a_in, int adjoint, void *fn, void *stream)
{
    if (a_in.n_blocks <= 0) return hipSuccess;
    LevelArgs a = a_in;
    const int64_t resident = (int64_t)device_cus() * (adjoint ? 1 : 2);
    int64_t chunk = adjoint ? tile_chunk<true>() : tile_chunk<false>();
    while (chunk > 1 && (a.n_blocks + chunk - 1) / chunk < resident) chunk >>= 1;
    a.chunk = (int32_t)chunk;
    void *args[] = {&a};
    return hipModuleLaunchKernel(reinterpret_cast<hipFunction_t>(fn), (unsigned)((a.n_blocks + chunk - 1) / chunk),
                                 1, 1, kRtileThreads, 1, 1, 0, reinterpret_cast<hipStream_t>(stream), args, nullptr);
}

int launch_rlevel(const LevelArgs &a_in, int precision, int adjoint, void *stream)
{
    if (a_in.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int amp = precision == QV_C64 ? 8 : 16;
    const size_t lds = tile_lds_bytes(a_in.lds_t, a_in.tab_bits, amp, adjoint) +
                       (adjoint ? sizeof(double) * (kRtileThreads / 64) * (size_t)a_in.max_train : 0);
    if (lds > (size_t)kLdsLimit) return hipErrorInvalidValue;
    // one workgroup per chunk of tiles; chunks shrink until every resident workgroup (two per CU forward,
    // one adjoint) has one
    LevelArgs a = a_in;
    const int64_t resident = (int64_t)device_cus() * (adjoint ? 1 : 2);
    int64_t chunk = adjoint ? tile_chunk<true>() : tile_chunk<false>();
    while (chunk > 1 && (a.n_blocks + chunk - 1) / chunk < resident) chunk >>= 1;
    a.chunk = (int32_t)chunk;
    dim3 grid((unsigned)((a.n_blocks + chunk - 1) / chunk)), block(kRtileThreads);
    if (precision == QV_C64) {
        if (adjoint) hipLaunchKernelGGL((k_rtile_adj<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_rtile_fwd<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, a);
    } else {
        if (adjoint) hipLaunchKernelGGL((k_rtile_adj<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_rtile_fwd<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

int launch_rlevel_lam(const LevelArgs &a_in, int precision, void *stream)
{
    if (a_in.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int amp = precision == QV_C64 ? 8 : 16;
    const size_t lds = tile_lds_bytes(a_in.lds_t, a_in.tab_bits, amp, 0);
    if (lds > (size_t)kLdsLimit) return hipErrorInvalidValue;
    LevelArgs a = a_in;
    const int64_t resident = (int64_t)device_cus() * 2;
    int64_t chunk = tile_chunk<false>();
    while (chunk > 1 && (a.n_blocks + chunk - 1) / chunk < resident) chunk >>= 1;
    a.chunk = (int32_t)chunk;
    dim3 grid((unsigned)((a.n_blocks + chunk - 1) / chunk)), block(kRtileThreads);
    if (precision == QV_C64) hipLaunchKernelGGL((k_rtile_lam<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_rtile_lam<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, a);
    return hipGetLastError();
}

int launch_level(const LevelArgs &a, int precision, int adjoint, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int amp = precision == QV_C64 ? 8 : 16;
    const size_t lds = tile_lds_bytes(a.lds_t, a.tab_bits, amp, adjoint);
    if (lds > (size_t)kLdsLimit) return hipErrorInvalidValue;
    dim3 grid((unsigned)a.n_blocks), block(kBlock);
    if (precision == QV_C64) {
        if (adjoint) hipLaunchKernelGGL((k_tile<float, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_tile<float, false>), grid, block, lds, s, a);
    } else {
        if (adjoint) hipLaunchKernelGGL((k_tile<double, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_tile<double, false>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

int launch_stride_level(const LevelArgs &a, int precision, int adjoint, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    dim3 grid((unsigned)a.n_blocks), block(kBlock);
    if (precision == QV_C64) {
        if (adjoint) hipLaunchKernelGGL((k_stride<float, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_stride<float, false>), grid, block, 0, s, a);
    } else {
        if (adjoint) hipLaunchKernelGGL((k_stride<double, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_stride<double, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

int launch_init_states(void *psi, const DevCirc *circs, const int64_t *first_block, int32_t n_circ,
                       int64_t n_blocks, int precision, void *stream)
{
    if (n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == QV_C64)
        hipLaunchKernelGGL((k_init<float>), dim3((unsigned)n_blocks), dim3(kBlock), 0, s,
                           reinterpret_cast<Cx<float> *>(psi), circs, first_block, n_circ);
    else
        hipLaunchKernelGGL((k_init<double>), dim3((unsigned)n_blocks), dim3(kBlock), 0, s,
                           reinterpret_cast<Cx<double> *>(psi), circs, first_block, n_circ);
    return hipGetLastError();
}

int launch_expectation(const ExpArgs &a, int precision, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == QV_C64)
        hipLaunchKernelGGL((k_expect<float>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_expect<double>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_finalize(const FinalizeArgs &a, void *stream)
{
    if (a.n_circ <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t outs = a.n_terms + ((a.norm_refs && a.norms) ? a.n_circ : 0);
    if (outs > 0) hipLaunchKernelGGL(k_finalize_refs, dim3((unsigned)outs), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_finalize_energies, dim3((unsigned)((a.n_circ + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_lambda(const LambdaArgs &a, int precision, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == QV_C64)
        hipLaunchKernelGGL((k_lambda<float>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_lambda<double>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_grad_reduce(const GradReduceArgs &a, void *stream)
{
    if (a.n_out <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)a.n_out), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_shift_combine(const ShiftCombineArgs &a, void *stream)
{
    if (a.n_out <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_shift_combine, dim3((unsigned)((a.n_out + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int launch_matrices(const MatArgs &a, int precision, void *stream)
{
    if (a.n_gates <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)((a.n_gates + kBlock - 1) / kBlock));
    if (precision == QV_C64) hipLaunchKernelGGL((k_matrices<float>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_matrices<double>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_rz_phase(const StatePhaseArgs &a, void *stream)
{
    hipLaunchKernelGGL(k_rz_phase, dim3(1), dim3(kBlock), 0, reinterpret_cast<hipStream_t>(stream), a);
    return hipGetLastError();
}

int launch_scale_copy(const StatePhaseArgs &a, int precision, void *stream)
{
    if (a.n_amps <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t blocks = std::min<int64_t>((a.n_amps + kBlock - 1) / kBlock, (int64_t)device_cus() * 16);
    if (precision == QV_C64) hipLaunchKernelGGL((k_scale_copy<float>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_scale_copy<double>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_shift_matrices(const ShiftMatArgs &a, int precision, void *stream)
{
    if (a.n_circ <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)((a.n_circ + kBlock - 1) / kBlock));
    if (precision == QV_C64) hipLaunchKernelGGL((k_shift_matrices<float>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_shift_matrices<double>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_fuse(const FuseArgs &a, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_fuse, dim3((unsigned)a.n_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

int launch_probs(const ProbArgs &a, int precision, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    if (a.target && !a.w) return hipErrorInvalidValue;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == QV_C64) hipLaunchKernelGGL((k_probs<float>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_probs<double>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_diag_seed(const DiagArgs &a, int precision, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == QV_C64) hipLaunchKernelGGL((k_diag_seed<float>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_diag_seed<double>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_diag_expect(const DiagArgs &a, int precision, void *stream)
{
    if (a.n_blocks <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == QV_C64) hipLaunchKernelGGL((k_diag_expect<float>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_diag_expect<double>), dim3((unsigned)a.n_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_segment_sum(const SegSumArgs &a, void *stream)
{
    if (a.n <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_segment_sum, dim3((unsigned)a.n), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_fill(double *p, int64_t n, double v, void *stream)
{
    if (n <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}


// Shots and counts: block prefixes, block offsets, the draw, then the compaction of the histogram. The
// histogram (one 32-bit count per amplitude of the pool) is cleared by a kernel, not a memset, so the
// sequence can sit in a captured graph.
int launch_sample(const SampleArgs &a, void *stream)
{
    if (a.n_blocks <= 0 || a.n_circ <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)a.n_blocks;
    hipLaunchKernelGGL(k_cdf_local, dim3(nb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_cdf_blocks, dim3((unsigned)a.n_circ), dim3(kBlock), 0, s, a);
    const int64_t nshots = (int64_t)a.n_circ * a.shots;
    hipLaunchKernelGGL(k_draw, dim3((unsigned)((nshots + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_hist_nnz, dim3(nb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_hist_offsets, dim3((unsigned)a.n_circ), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_hist_emit, dim3(nb), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int launch_zero_hist(uint32_t *p, int64_t n, void *stream)
{
    if (n <= 0) return hipSuccess;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace qv
