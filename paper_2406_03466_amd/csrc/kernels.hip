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

namespace qv {

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
    R re, im;
};

struct M2d {  // 2x2 complex matrix in double: m[row*2+col]
    double re[4], im[4];
};

__device__ __forceinline__ uint32_t insert0(uint32_t x, int p)
{
    return ((x >> p) << (p + 1)) | (x & ((1u << p) - 1u));
}

__device__ __forceinline__ uint64_t insert0_64(uint64_t x, int p)
{
    return ((x >> p) << (p + 1)) | (x & ((1ull << p) - 1ull));
}

// Scatters the low bits of v into the set bits of mask (lowest first).
__device__ __forceinline__ uint64_t deposit(uint64_t v, uint64_t mask)
{
    uint64_t r = 0;
    while (mask) {
        uint64_t low = mask & (~mask + 1);
        if (v & 1) r |= low;
        v >>= 1;
        mask &= mask - 1;
    }
    return r;
}

__device__ __forceinline__ int parity64(uint64_t v) { return __popcll(v) & 1; }

// Matrix of a one-qubit gate (textbook definitions; rotations are exp(-i a sigma / 2)).
__device__ inline void gate_matrix(int kind, double a, M2d &m)
{
    for (int k = 0; k < 4; k++) { m.re[k] = 0.0; m.im[k] = 0.0; }
    double s, c;
    sincos(0.5 * a, &s, &c);
    const double r = 0.70710678118654752440;
    switch (kind) {
    case QV_H: m.re[0] = r; m.re[1] = r; m.re[2] = r; m.re[3] = -r; break;
    case QV_X: m.re[1] = 1; m.re[2] = 1; break;
    case QV_Y: m.im[1] = -1; m.im[2] = 1; break;
    case QV_Z: m.re[0] = 1; m.re[3] = -1; break;
    case QV_S: m.re[0] = 1; m.im[3] = 1; break;
    case QV_T: m.re[0] = 1; m.re[3] = r; m.im[3] = r; break;
    case QV_RX: m.re[0] = c; m.im[1] = -s; m.im[2] = -s; m.re[3] = c; break;
    case QV_RY: m.re[0] = c; m.re[1] = -s; m.re[2] = s; m.re[3] = c; break;
    case QV_RZ: m.re[0] = c; m.im[0] = -s; m.re[3] = c; m.im[3] = s; break;
    default: m.re[0] = 1; m.re[3] = 1; break;
    }
}

// Conjugate transpose in place.
__device__ inline void dagger(M2d &m)
{
    double r1 = m.re[1], i1 = m.im[1];
    m.re[1] = m.re[2]; m.im[1] = -m.im[2];
    m.re[2] = r1; m.im[2] = -i1;
    m.im[0] = -m.im[0];
    m.im[3] = -m.im[3];
}

template <typename R>
struct M2 {
    R re[4], im[4];
};

// Read-only tables indexed by workgroup-uniform values: loads through the constant address space, so
// they become scalar loads.
template <typename T>
__device__ __forceinline__ T ldu(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "whole words only");
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) w[i] = q[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

template <typename R>
__device__ __forceinline__ M2<R> narrow(const M2d &m)
{
    M2<R> o;
    for (int k = 0; k < 4; k++) { o.re[k] = (R)m.re[k]; o.im[k] = (R)m.im[k]; }
    return o;
}

template <typename R>
__device__ __forceinline__ void apply2(const M2<R> &m, Cx<R> &a, Cx<R> &b)
{
    Cx<R> x = a, y = b;
    a.re = m.re[0] * x.re - m.im[0] * x.im + m.re[1] * y.re - m.im[1] * y.im;
    a.im = m.re[0] * x.im + m.im[0] * x.re + m.re[1] * y.im + m.im[1] * y.re;
    b.re = m.re[2] * x.re - m.im[2] * x.im + m.re[3] * y.re - m.im[3] * y.im;
    b.im = m.re[2] * x.im + m.im[2] * x.re + m.re[3] * y.im + m.im[3] * y.re;
}

// Im <lambda| G |psi> restricted to one amplitude pair (a0, a1) of psi and (l0, l1) of lambda, where G is
// the generator (X, Y or Z) of a rotation on the pair's qubit. FP64.
template <typename R>
__device__ __forceinline__ double gen_inner(int kind, Cx<R> a0, Cx<R> a1, Cx<R> l0, Cx<R> l1)
{
    const double a0r = a0.re, a0i = a0.im, a1r = a1.re, a1i = a1.im;
    const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
    if (kind == QV_RX)
        return (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r);
    if (kind == QV_RY)
        return -(l0r * a1r + l0i * a1i) + (l1r * a0r + l1i * a0i);
    return (l0r * a0i - l0i * a0r) - (l1r * a1i - l1i * a1r);
}

// DPP move of a double: both 32-bit halves go through the same lane permutation. Lanes of rows outside
// row_mask are left undefined (callers only use lanes that every step writes).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave with DPP lane moves (no LDS); the total ends up in lane 63 (other lanes
// hold partial or undefined values).
// quad_perm [1,0,3,2] and [2,3,0,1] sum each quad, row_half_mirror each 8 lanes, row_mirror each row of
// 16; row_bcast15 adds row 0 into row 1 and row 2 into row 3; row_bcast31 adds lane 31 into rows 2 and 3.
__device__ __forceinline__ double wave_sum_to_63(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);
    v += dpp_f64<0x4E, 0xF>(v);
    v += dpp_f64<0x141, 0xF>(v);
    v += dpp_f64<0x140, 0xF>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
    return v;
}

// Sum over the workgroup (kBlock threads); the result is valid in thread 0. red holds kBlock/64 doubles.
__device__ inline double block_sum(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; w++) s += red[w];
    __syncthreads();
    return s;
}

template <typename T>
__device__ __forceinline__ int find_block(const T *arr, int n, int64_t blk)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (arr[mid].first_block <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_prefix(const int64_t *pre, int n, int64_t blk)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Matrix of op for circuit `circ` (record C) of a launch: from the batch's matrix table, or, for the one gate
// whose angle a parameter-shift variant moves, from the launch's shifted-gate table.
// The table is laid out in plan order (entry mat_off + o - op_base for the plan's op o, fused-block markers
// included), so an op's matrix can be fetched without first reading the op record.
template <typename R>
__device__ __forceinline__ M2<R> op_matrix(const LevelArgs &a, const DevCirc &C, int circ, const DevOp &op, int64_t oi)
{
    if (op.gate == C.shift_gate) return reinterpret_cast<const M2<R> *>(a.smats)[circ];
    return reinterpret_cast<const M2<R> *>(a.mats)[C.mat_off + (oi - C.op_base)];
}

template <typename R>
__device__ __forceinline__ M2<R> dagger_r(const M2<R> &m)
{
    M2<R> o;
    o.re[0] = m.re[0]; o.im[0] = -m.im[0];
    o.re[1] = m.re[2]; o.im[1] = -m.im[2];
    o.re[2] = m.re[1]; o.im[2] = -m.im[1];
    o.re[3] = m.re[3]; o.im[3] = -m.im[3];
    return o;
}


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

// ------------------------------------------------------------------------------------------------------
// Register-tiled pass. The tile sits in LDS (XOR-swizzled so that any quarter wave touches distinct
// banks); each register segment loads 2^RB amplitudes per thread into registers, runs its ops there and
// stores them back. A rotation or CNOT target is always a register qubit of its segment, so those ops
// need no data exchange; diagonal ops and CNOT controls on thread qubits use the thread's own index bits.
// ------------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t swz(uint32_t e)
{
    return e ^ (((e >> 4) ^ (e >> 8) ^ (e >> 12)) & 15u);
}

// Bit j of reg_pattern(k) is bit k of j: the registers whose index has register bit k set.
__device__ __forceinline__ uint32_t reg_pattern(int k)
{
    return k == 0 ? 0xAAAAAAAAu : k == 1 ? 0xCCCCCCCCu : k == 2 ? 0xF0F0F0F0u : k == 3 ? 0xFF00FF00u : 0xFFFF0000u;
}

// Runs STMT with the compile-time register bit K equal to the runtime value k (0 <= k < RB).
#define WITH_K(RB_, k, STMT)                                                 \
    switch (k) {                                                             \
    case 0: { constexpr int K = 0; STMT; } break;                            \
    case 1: { constexpr int K = 1; STMT; } break;                            \
    case 2: { constexpr int K = 2; STMT; } break;                            \
    case 3: { constexpr int K = (RB_) > 3 ? 3 : 0; if constexpr ((RB_) > 3) { STMT; } } break; \
    default: __builtin_unreachable();                                        \
    }

// A thread's 2^RB register amplitudes as one vector value (re, im interleaved). Every update below uses
// compile-time element indices, so the vector stays in one fixed block of registers across the op loop and
// its branches instead of being copied between them.
template <typename R, int N>
struct Regs {
    typedef R V __attribute__((ext_vector_type(2 * N)));
    V d;
    __device__ __forceinline__ Cx<R> get(int j) const
    {
        Cx<R> c;
        c.re = d[2 * j];
        c.im = d[2 * j + 1];
        return c;
    }
    __device__ __forceinline__ void set(int j, R re, R im)
    {
        d[2 * j] = re;
        d[2 * j + 1] = im;
    }
    __device__ __forceinline__ void set(int j, Cx<R> c) { set(j, c.re, c.im); }
};

// [[c, -s], [s, c]] on register bit K (RY and its inverse).
template <int K, int N, typename R>
__device__ __forceinline__ void r_real(Regs<R, N> &v, R c, R s)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (j & (1 << K)) continue;
        const int j1 = j | (1 << K);
        const Cx<R> x = v.get(j), y = v.get(j1);
        v.set(j, c * x.re - s * y.re, c * x.im - s * y.im);
        v.set(j1, s * x.re + c * y.re, s * x.im + c * y.im);
    }
}

template <int K, int N, typename R>
__device__ __forceinline__ void r_gen(Regs<R, N> &v, const M2<R> &m)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (j & (1 << K)) continue;
        const int j1 = j | (1 << K);
        Cx<R> x = v.get(j), y = v.get(j1);
        apply2(m, x, y);
        v.set(j, x);
        v.set(j1, y);
    }
}

// diag(d0, d1) on register bit K.
template <int K, int N, typename R>
__device__ __forceinline__ void r_diag(Regs<R, N> &v, R d0r, R d0i, R d1r, R d1i)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        const R dr = (j & (1 << K)) ? d1r : d0r, di = (j & (1 << K)) ? d1i : d0i;
        const Cx<R> x = v.get(j);
        v.set(j, dr * x.re - di * x.im, dr * x.im + di * x.re);
    }
}

template <int N, typename R>
__device__ __forceinline__ void t_scale(Regs<R, N> &v, R dr, R di)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        const Cx<R> x = v.get(j);
        v.set(j, dr * x.re - di * x.im, dr * x.im + di * x.re);
    }
}

// CNOT with target register bit KT and control register bit KC: a fixed permutation of the registers.
template <int KC, int KT, int N, typename R>
__device__ __forceinline__ void r_cnot(Regs<R, N> &v)
{
    if constexpr (KC == KT) return;
#pragma unroll
    for (int j = 0; j < N; j++) {
        if ((j & (1 << KT)) || !(j & (1 << KC))) continue;
        const int j1 = j | (1 << KT);
        const Cx<R> x = v.get(j), y = v.get(j1);
        v.set(j, y);
        v.set(j1, x);
    }
}


// CNOT with target register bit KT, control given per thread.
template <int KT, int N, typename R>
__device__ __forceinline__ void t_cnot(Regs<R, N> &v, bool ctl)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (j & (1 << KT)) continue;
        const int j1 = j | (1 << KT);
        const Cx<R> x = v.get(j), y = v.get(j1);
        v.set(j, ctl ? y : x);
        v.set(j1, ctl ? x : y);
    }
}

// Negates register j where bit j of m is set.
template <int N, typename R>
__device__ __forceinline__ void neg_mask(Regs<R, N> &v, uint32_t m)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        const Cx<R> x = v.get(j);
        const bool f = (m >> j) & 1u;
        v.set(j, f ? -x.re : x.re, f ? -x.im : x.im);
    }
}

// Im <l| G |a> over the register pairs of bit K, G the generator of rotation kind GEN (RX: X, RY: Y, RZ: Z):
// a thread's products are summed in R precision (two interleaved accumulators), the result in FP64.
template <int K, int GEN, int N, typename R>
__device__ __forceinline__ double r_inner(const Regs<R, N> &a, const Regs<R, N> &l)
{
    R acc[2] = {(R)0, (R)0};
#pragma unroll
    for (int j = 0, n = 0; j < N; j++) {
        if (j & (1 << K)) continue;
        const int j1 = j | (1 << K);
        const Cx<R> a0 = a.get(j), a1 = a.get(j1), l0 = l.get(j), l1 = l.get(j1);
        R &s = acc[n++ & 1];
        if constexpr (GEN == QV_RX) {
            // conj(l0) (-i a1) + conj(l1) (-i a0)
            s += l0.re * a1.im - l0.im * a1.re + l1.re * a0.im - l1.im * a0.re;
        } else if constexpr (GEN == QV_RY) {
            // conj(l0) (-i a1) + conj(l1) (i a0)
            s += l1.re * a0.re + l1.im * a0.im - l0.re * a1.re - l0.im * a1.im;
        } else {
            // conj(l0) a0 - conj(l1) a1
            s += l0.re * a0.im - l0.im * a0.re - l1.re * a1.im + l1.im * a1.re;
        }
    }
    return (double)acc[0] + (double)acc[1];
}

// Im <l| Z_p |a> when qubit p is a thread bit with value `bit`.
template <int N, typename R>
__device__ __forceinline__ double t_inner_z(const Regs<R, N> &a, const Regs<R, N> &l, int bit)
{
    R acc[2] = {(R)0, (R)0};
#pragma unroll
    for (int j = 0; j < N; j++) {
        const Cx<R> x = a.get(j), y = l.get(j);
        acc[j & 1] += y.re * x.im - y.im * x.re;
    }
    const double t = (double)acc[0] + (double)acc[1];
    return bit ? -t : t;
}

// Adjoint step for one op on psi (a) and lambda (l) together on register bit K: Im <l| G |a> when the op
// is trainable (returned through ip), then the inverse op on both.
template <int K, int N, typename R>
__device__ __forceinline__ void adj_real(Regs<R, N> &a, Regs<R, N> &l, R c, R s, bool train, double &ip)
{
    if (train) ip = r_inner<K, QV_RY>(a, l);
    r_real<K>(a, c, s);
    r_real<K>(l, c, s);
}

template <int K, int N, typename R>
__device__ __forceinline__ void adj_diag(Regs<R, N> &a, Regs<R, N> &l, R d0r, R d0i, R d1r, R d1i, bool train,
                                         double &ip)
{
    // of the diagonal kinds only RZ carries a parameter
    if (train) ip = r_inner<K, QV_RZ>(a, l);
    r_diag<K>(a, d0r, d0i, d1r, d1i);
    r_diag<K>(l, d0r, d0i, d1r, d1i);
}

template <int K, int N, typename R>
__device__ __forceinline__ void adj_gen(Regs<R, N> &a, Regs<R, N> &l, const M2<R> &m, bool train, double &ip)
{
    // of the dense kinds only RX carries a parameter
    if (train) ip = r_inner<K, QV_RX>(a, l);
    r_gen<K>(a, m);
    r_gen<K>(l, m);
}

// Register-bit cases of an op-code switch: BASE + k runs STMT with the compile-time register bit K = k
// (codes for register bits the kernel does not have are never generated).
#define K4_CASES(BASE, STMT)                                                                  \
    case (BASE) + 0: { constexpr int K = 0; STMT; } break;                                    \
    case (BASE) + 1: { constexpr int K = 1; if constexpr (K < RB) { STMT; } } break;          \
    case (BASE) + 2: { constexpr int K = 2; if constexpr (K < RB) { STMT; } } break;          \
    case (BASE) + 3: { constexpr int K = 3; if constexpr (K < RB) { STMT; } } break;
#define CNOT_CASE(KC_, KT_, STMT)                                                             \
    case OC_CNOT_RR + 4 * (KC_) + (KT_): {                                                    \
        constexpr int KC = KC_, KT = KT_;                                                     \
        if constexpr (KC < RB && KT < RB && KC != KT) { STMT; }                               \
    } break;
#define CNOT_CASES(STMT)                                                                      \
    CNOT_CASE(0, 1, STMT) CNOT_CASE(0, 2, STMT) CNOT_CASE(0, 3, STMT)                         \
    CNOT_CASE(1, 0, STMT) CNOT_CASE(1, 2, STMT) CNOT_CASE(1, 3, STMT)                         \
    CNOT_CASE(2, 0, STMT) CNOT_CASE(2, 1, STMT) CNOT_CASE(2, 3, STMT)                         \
    CNOT_CASE(3, 0, STMT) CNOT_CASE(3, 1, STMT) CNOT_CASE(3, 2, STMT)

// One register-segment op on v by its op code (the inverse when INV).
template <bool INV, int RB, typename R>
__device__ __forceinline__ void code_apply(Regs<R, 1 << RB> &v, int code, const DevOp &op, const M2<R> &mat,
                                           uint32_t Et)
{
    const R cr = mat.re[0], sr = INV ? -mat.re[2] : mat.re[2];
    const R d0r = mat.re[0], d1r = mat.re[3];
    const R d0i = INV ? -mat.im[0] : mat.im[0], d1i = INV ? -mat.im[3] : mat.im[3];
    switch (code) {
    K4_CASES(OC_RY, (r_real<K>(v, cr, sr)))
    K4_CASES(OC_DIAG, (r_diag<K>(v, d0r, d0i, d1r, d1i)))
    case OC_DIAG_T: {
        const bool b = (Et >> op.p0) & 1u;
        t_scale(v, b ? d1r : d0r, b ? d1i : d0i);
    } break;
    K4_CASES(OC_GEN, (r_gen<K>(v, INV ? dagger_r(mat) : mat)))
    CNOT_CASES((r_cnot<KC, KT>(v)))
    K4_CASES(OC_CNOT_TR, (t_cnot<K>(v, ((Et >> op.p0) & 1u) != 0)))
    case OC_CZ: {
        const uint32_t ma = op.k0 >= 0 ? reg_pattern(op.k0) : (((Et >> op.p0) & 1u) ? 0xFFFFFFFFu : 0u);
        const uint32_t mb = op.k1 >= 0 ? reg_pattern(op.k1) : (((Et >> op.p1) & 1u) ? 0xFFFFFFFFu : 0u);
        neg_mask(v, ma & mb);
    } break;
    default: break;
    }
}

// One adjoint register-segment op by its op code: Im <l| G |a> when the op is trainable, then the inverse
// op on a and l.
template <int RB, typename R>
__device__ __forceinline__ double code_adjoint(Regs<R, 1 << RB> &a, Regs<R, 1 << RB> &l, int code, const DevOp &op,
                                               const M2<R> &mat, uint32_t Et)
{
    const bool train = (op.flags & OP_TRAIN) != 0;
    double ip = 0.0;
    const R cr = mat.re[0], sr = -mat.re[2];
    const R d0r = mat.re[0], d1r = mat.re[3], d0i = -mat.im[0], d1i = -mat.im[3];
    switch (code) {
    K4_CASES(OC_RY, (adj_real<K>(a, l, cr, sr, train, ip)))
    K4_CASES(OC_DIAG, (adj_diag<K>(a, l, d0r, d0i, d1r, d1i, train, ip)))
    case OC_DIAG_T: {
        const bool b = (Et >> op.p0) & 1u;
        if (train) ip = t_inner_z(a, l, (int)b);
        t_scale(a, b ? d1r : d0r, b ? d1i : d0i);
        t_scale(l, b ? d1r : d0r, b ? d1i : d0i);
    } break;
    K4_CASES(OC_GEN, (adj_gen<K>(a, l, dagger_r(mat), train, ip)))
    CNOT_CASES((r_cnot<KC, KT>(a), r_cnot<KC, KT>(l)))
    K4_CASES(OC_CNOT_TR, (t_cnot<K>(a, ((Et >> op.p0) & 1u) != 0), t_cnot<K>(l, ((Et >> op.p0) & 1u) != 0)))
    case OC_CZ: {
        const uint32_t ma = op.k0 >= 0 ? reg_pattern(op.k0) : (((Et >> op.p0) & 1u) ? 0xFFFFFFFFu : 0u);
        const uint32_t mb = op.k1 >= 0 ? reg_pattern(op.k1) : (((Et >> op.p1) & 1u) ? 0xFFFFFFFFu : 0u);
        neg_mask(a, ma & mb);
        neg_mask(l, ma & mb);
    } break;
    default: break;
    }
    return ip;
}

typedef float v16f __attribute__((ext_vector_type(16)));

// A fused 4-qubit block on the 16 register amplitudes of every lane, as one wave-wide real GEMM on MFMA:
// Y (32 x 64) = A (32 x 32) X (32 x 64), where column l of X is lane l's amplitudes as 32 reals
// (re, im interleaved) and A is the block's [[Re, -Im], [Im, Re]] form. v_mfma_f32_32x32x2_f32 takes B
// row k from lane half k, so permlane32 swaps pair rows 2s and 2s+1 across the lane halves: one swap
// yields the B operand of both 32-column halves. Its result holds, per lane half, rows 8i+4h+r of a
// column; swapping the two halves' accumulators gives every lane its own column back.
__device__ __forceinline__ void fused_mfma(Regs<float, 16> &v, const float *__restrict__ A, int lane)
{
    // all 16 A-operand loads are issued before the first product, so their latencies overlap
    v16f am;
#pragma unroll
    for (int s = 0; s < 16; s++) am[s] = A[s * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
    v16f acc0, acc1;
#pragma unroll
    for (int q = 0; q < 16; q++) { acc0[q] = 0.f; acc1[q] = 0.f; }
#pragma unroll
    for (int s = 0; s < 16; s++) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(v.d[2 * s]), __float_as_uint(v.d[2 * s + 1]),
                                                         false, false);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(am[s], __uint_as_float(sw[0]), acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(am[s], __uint_as_float(sw[1]), acc1, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc0[q]), __float_as_uint(acc1[q]), false,
                                                         false);
        const int rlo = 8 * (q / 4) + (q % 4);
        v.d[rlo] = __uint_as_float(sw[0]);
        v.d[rlo + 4] = __uint_as_float(sw[1]);
    }
}

// Position in a register segment's op list: index k of n, the op record and matrix of op k already
// loaded (one op ahead), and its global index oi.
template <typename R>
struct OpCursor {
    int k, n;
    int64_t oi;
    DevOp op;
    M2<R> mat;
};

// Waits for the scalar loads that produced x right here. A parameter-shift variant's shifted matrix is loaded
// on a rare path; waiting inside that path keeps the wait (which covers every outstanding scalar load,
// including the next op's prefetch) out of the common path where the two meet.
template <typename T>
__device__ __forceinline__ void scalar_wait(const T &x)
{
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) asm volatile("" ::"s"(w[i]));
}

// Moves the cursor `by` ops on (forward: up the list; adjoint: down) and fetches that op's record and matrix.
template <typename R, bool ADJ>
__device__ __forceinline__ void cursor_advance(const LevelArgs &a, const M2<R> *mtab, OpCursor<R> &oc, int by = 1)
{
    oc.k += by;
    if (oc.k < oc.n) {
        oc.oi += ADJ ? -by : by;
        oc.op = ldu(a.ops + oc.oi);
        oc.mat = ldu(mtab + oc.oi);
    }
}

// Moves the cursor past fused-block markers (scalar work only).
template <typename R, bool ADJ>
__device__ __forceinline__ void cursor_skip_markers(const LevelArgs &a, const M2<R> *mtab, OpCursor<R> &oc)
{
    while (oc.k < oc.n && oc.op.kind == kFusedKind) cursor_advance<R, ADJ>(a, mtab, oc);
}

// The register-segment op loops below run two steps per iteration, reading one register set and writing
// the other (vi -> vo, then vo -> vi), so no branch of the gate dispatch has to leave its result in the
// registers it read. The forward loop stores from whichever set holds the result; the adjoint loop moves it
// into the first set at its exit.

// One forward step: the next op (or fused block) applied to vi, result in vo. FUSE: fused-block markers
// are executed (complex64 with 16 amplitudes per thread); otherwise the caller keeps the cursor off them.
template <typename R, int RB, bool FUSE>
__device__ __forceinline__ void fwd_step(const LevelArgs &a, const DevCirc &C, int circ, const M2<R> *mtab,
                                         OpCursor<R> &oc, uint32_t Et, int lane, const Regs<R, 1 << RB> &vi,
                                         Regs<R, 1 << RB> &vo)
{
    const DevOp op = oc.op;
    M2<R> mat = oc.mat;
    const int64_t cur = oc.oi;
    cursor_advance<R, false>(a, mtab, oc);
    vo = vi;
    if constexpr (FUSE) {
        if (op.kind == kFusedKind) {
            // A fused block: its product on MFMA and its gates skipped. A block that holds a parameter-shift
            // variant's shifted gate is left to its gates, one by one (the cursor is on its first gate).
            const int m = op.pad;
            bool shifted = false;
            if (C.shift_gate >= 0)
                for (int j = 1; j <= m; j++) shifted |= ldu(a.ops + cur + j).gate == C.shift_gate;
            if (!shifted) {
                fused_mfma(vo, a.fmats + (C.fused_off + (op.p0 | (op.p1 << 8))) * (int64_t)kFusedFloats, lane);
                cursor_advance<R, false>(a, mtab, oc, m);
            }
            return;
        }
    } else {
        (void)cur;
        (void)lane;
    }
    if (op.gate == C.shift_gate) {
        mat = ldu(reinterpret_cast<const M2<R> *>(a.smats) + circ);
        scalar_wait(mat);
    }
    code_apply<false, RB, R>(vo, op.flags >> kOpCodeShift, op, mat, Et);
    if constexpr (!FUSE) cursor_skip_markers<R, false>(a, mtab, oc);
}

// One adjoint step, walking the segment's ops backwards: the next op undone on (ai, li) with its partial
// sum, result in (ao, lo). Fused-block markers carry no adjoint work (the adjoint needs the state at every
// trainable gate, so a block's gates are undone one by one).
template <typename R, int RB, int NT>
__device__ __forceinline__ void adj_step(const LevelArgs &a, const DevCirc &C, int circ, const M2<R> *mtab,
                                         OpCursor<R> &oc, uint32_t Et, bool active, int lane, int wave, double *red,
                                         const Regs<R, 1 << RB> &ai, const Regs<R, 1 << RB> &li,
                                         Regs<R, 1 << RB> &ao, Regs<R, 1 << RB> &lo)
{
    auto advance = [&]() {
        oc.k += 1;
        if (oc.k < oc.n) {
            oc.oi -= 1;
            oc.op = ldu(a.ops + oc.oi);
            oc.mat = ldu(mtab + oc.oi);
        }
    };
    ao = ai;
    lo = li;
    while (oc.k < oc.n && oc.op.kind == kFusedKind) advance();
    if (oc.k >= oc.n) return;
    const DevOp op = oc.op;
    M2<R> mat = oc.mat;
    advance();
    if (op.gate == C.shift_gate) {
        mat = ldu(reinterpret_cast<const M2<R> *>(a.smats) + circ);
        scalar_wait(mat);
    }
    double ip = code_adjoint<RB, R>(ao, lo, op.flags >> kOpCodeShift, op, mat, Et);
    if (op.flags & OP_TRAIN) {
        if (!active) ip = 0.0;
        ip = wave_sum_to_63(ip);
        if (lane == 63) red[op.train_slot * (NT / 64) + wave] = ip;
    }
}

// A run of CNOTs folded into a segment's addressing, applied to a tile index e (e ^= bit c << t for each,
// a linear map on the index bits). w holds the run's eight entries (byte k: control | target << 4; unused
// entries are 0xFF, bit 15 of a tile index being always clear); REV applies them last to first, which is
// the inverse map (every CNOT is its own inverse). Straight-line, with no branch even for an empty run:
// a loop or branch here, next to the op loop, makes the compiler keep the op loop's register sets far
// less tidily (copies in every gate branch).
template <bool REV>
__device__ __forceinline__ uint32_t cnot_run(uint32_t e, uint64_t w)
{
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int k = REV ? 7 - i : i;
        const uint32_t b = (uint32_t)(w >> (8 * k)) & 0xFFu;
        e ^= ((e >> (b & 15u)) & 1u) << (b >> 4);
    }
    return e;
}

// The folded CNOT runs of a segment, by scalar loads: entries, lengths and the register-bit images.
struct SegRuns {
    uint64_t lead, trail;
    int n_lead, n_trail;
    uint32_t rimg_lead[4], rimg_trail[4];
};

__device__ __forceinline__ SegRuns seg_runs(const DevSeg *sp)
{
    static_assert(offsetof(DevSeg, lead) % 8 == 0 && offsetof(DevSeg, trail) == offsetof(DevSeg, lead) + 8 &&
                      offsetof(DevSeg, n_lead) == offsetof(DevSeg, trail) + 8 &&
                      offsetof(DevSeg, n_trail) == offsetof(DevSeg, n_lead) + 1 &&
                      offsetof(DevSeg, rimg_lead) == offsetof(DevSeg, n_lead) + 4 &&
                      offsetof(DevSeg, rimg_trail) == offsetof(DevSeg, rimg_lead) + 8,
                  "DevSeg run layout");
    const uint32_t *w = reinterpret_cast<const uint32_t *>(sp) + offsetof(DevSeg, lead) / 4;
    SegRuns r;
    r.lead = (uint64_t)ldu(w) | ((uint64_t)ldu(w + 1) << 32);
    r.trail = (uint64_t)ldu(w + 2) | ((uint64_t)ldu(w + 3) << 32);
    const uint32_t nn = ldu(w + 4);
    r.n_lead = (int)(nn & 0xFFu);
    r.n_trail = (int)((nn >> 8) & 0xFFu);
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const uint32_t a = ldu(w + 5 + i), b = ldu(w + 7 + i);
        r.rimg_lead[2 * i] = a & 0xFFFFu;
        r.rimg_lead[2 * i + 1] = a >> 16;
        r.rimg_trail[2 * i] = b & 0xFFFFu;
        r.rimg_trail[2 * i + 1] = b >> 16;
    }
    return r;
}

// Amplitudes each thread moves between HBM and LDS per batch of independent loads (or stores).
template <typename R>
constexpr int tile_batch() { return sizeof(R) == 4 ? 16 : 8; }

template <typename R, bool ADJ, int RB, int NT>
__device__ __forceinline__ bool rtile_body(const LevelArgs &a, int64_t blk, const Seg &sg, bool preloaded,
                                           int64_t next_blk)
{
    static_assert(RB >= 1 && RB <= 4, "register-bit dispatch covers register bits 0..3");
    constexpr int N = 1 << RB;
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t tile = blk - sg.first_block;
    const DevPass P = ldu(a.passes + sg.pass);
    const DevCirc C = ldu(a.circs + sg.circ);
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
    const uint32_t lmask = (1u << lowc) - 1u;
    Cx<R> *gpsi = reinterpret_cast<Cx<R> *>(a.psi) + C.state_off;
    Cx<R> *glam = ADJ ? reinterpret_cast<Cx<R> *>(a.lam) + C.state_off : nullptr;
    // The next tile of the same (circuit, pass) is loaded straight into LDS while the last register segment
    // of this one runs (the segment holds the whole tile in registers, so LDS is free); this tile then
    // goes from registers to HBM directly.
    // complex64 moves one float per lane (64 floats = 32 amplitudes per load): the swizzle can put the two
    // floats of an LDS amplitude pair in either order of the HBM pair, so pairs cannot move as one 16-byte
    // unit. complex128 moves one 16-byte amplitude per lane (64 amplitudes per load).
    constexpr int APP = sizeof(R) == 4 ? 32 : 64;
    // The adjoint's sweep over a circuit's first pass stops at its first trainable op (nothing below it is
    // needed): only the last nseg segments run, the lowest of them only down to that op.
    const bool stop_early = ADJ && sg.last;
    const int nseg = stop_early ? P.adj_last_nseg : P.n_seg;
    const bool pf = next_blk >= 0 && !(!ADJ && sg.first) && T >= (uint32_t)APP && nseg > 0;

    if (preloaded) {
        // this tile was loaded by the previous tile's last segment (same pass: the run table is in place)
        __builtin_amdgcn_s_waitcnt(0);
    } else if (!ADJ && sg.first) {
        // first pass of the circuit: the tile of |0...0> is zero except amplitude 0 of tile 0
        for (uint32_t e = threadIdx.x; e < T; e += NT) {
            Cx<R> z;
            z.re = (R)((base == 0 && e == 0) ? 1 : 0);
            z.im = (R)0;
            sp[swz(e)] = z;
        }
    } else {
        for (uint32_t h = threadIdx.x; h < nh; h += NT) segtab[h] = deposit(h, himask);
        __syncthreads();
        // tile_batch<R>() independent loads in flight per thread before any is written to LDS
        constexpr int TB = tile_batch<R>();
        for (uint32_t e0 = threadIdx.x; e0 < T; e0 += TB * NT) {
            Regs<R, TB> bp, bl;
#pragma unroll
            for (int u = 0; u < TB; u++) {
                const uint32_t e = e0 + (uint32_t)u * NT;
                if (e < T) {
                    const uint64_t g = base | segtab[e >> lowc] | (e & lmask);
                    bp.set(u, gpsi[g]);
                    if (ADJ) bl.set(u, glam[g]);
                }
            }
#pragma unroll
            for (int u = 0; u < TB; u++) {
                const uint32_t e = e0 + (uint32_t)u * NT;
                if (e < T) {
                    sp[swz(e)] = bp.get(u);
                    if (ADJ) sl[swz(e)] = bl.get(u);
                }
            }
        }
    }
    __syncthreads();

    const int tbits = t - RB;
    const uint32_t tmask = (1u << tbits) - 1u;
    const bool active = threadIdx.x <= tmask;
    const uint32_t tid = threadIdx.x & tmask;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    for (int s0 = 0; s0 < nseg; s0++) {
        const int si = ADJ ? P.n_seg - 1 - s0 : s0;
        const DevSeg S = ldu(a.rsegs + P.seg_begin + si);
        uint32_t Et = 0;
#pragma unroll
        for (int m = 0; m < 16; m++)
            if (m < tbits && (tid >> m & 1u)) Et |= 1u << S.tpos[m];
        uint32_t rbit[RB];
#pragma unroll
        for (int k = 0; k < RB; k++) rbit[k] = 1u << S.rpos[k];
        // Register j of this thread holds tile element Et | D_j. The segment's folded CNOT runs permute the
        // tile, so the element is read from / written to its permuted position: forward passes read through
        // the inverse of the leading run and write through the trailing run; the adjoint undoes the segment,
        // so it reads through the trailing run and writes through the inverse of the leading run.
        // The store side (ES, rs) is mapped here too, so the runs hold no registers through the op loop.
        Regs<R, N> av, lv;
        uint32_t ES, rs[RB];
        bool remap;  // a folded run moves amplitudes between threads
        {
            const SegRuns sr = seg_runs(a.rsegs + P.seg_begin + si);
            remap = (sr.n_lead | sr.n_trail) != 0;
            ES = ADJ ? cnot_run<true>(Et, sr.lead) : cnot_run<false>(Et, sr.trail);
            const uint32_t PL = swz(ADJ ? cnot_run<false>(Et, sr.trail) : cnot_run<true>(Et, sr.lead));
            uint32_t rl[RB];
#pragma unroll
            for (int k = 0; k < RB; k++) {
                rs[k] = ADJ ? sr.rimg_lead[k] : sr.rimg_trail[k];
                rl[k] = ADJ ? sr.rimg_trail[k] : sr.rimg_lead[k];
            }
#pragma unroll
            for (int j = 0; j < N; j++) {
                uint32_t D = 0;
#pragma unroll
                for (int k = 0; k < RB; k++)
                    if (j >> k & 1) D ^= rl[k];
                const uint32_t addr = PL ^ swz(D);
                av.set(j, sp[addr]);
                if (ADJ) lv.set(j, sl[addr]);
            }
        }
        const bool last_seg = s0 == nseg - 1;
        // With a folded run, a thread's stores may land where another thread loads: every wave loads first.
        if (remap && !(pf && last_seg)) __syncthreads();
        if (pf && last_seg) {
            __syncthreads();  // every wave has its registers: LDS may be overwritten
            const uint64_t nbase = deposit((uint64_t)(next_blk - sg.first_block), full & ~P.local_mask);
            for (uint32_t c = (uint32_t)wave; c < T / APP; c += NT / 64) {
                // load c covers LDS positions [c*APP, (c+1)*APP); position q holds element swz(q)
                if constexpr (sizeof(R) == 4) {
                    const uint32_t d = c * 64 + (uint32_t)lane;  // float d of the tile: part d&1 of position d>>1
                    const uint32_t e = swz(d >> 1);
                    const uint64_t g = nbase | segtab[e >> lowc] | (e & lmask);
                    const float *src = reinterpret_cast<const float *>(gpsi + g) + (d & 1u);
                    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)src,
                                                     (void __attribute__((address_space(3))) *)(sp + c * APP),
                                                     4, 0, 0);
                    if (ADJ) {
                        const float *lsrc = reinterpret_cast<const float *>(glam + g) + (d & 1u);
                        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)lsrc,
                                                         (void __attribute__((address_space(3))) *)(sl + c * APP),
                                                         4, 0, 0);
                    }
                } else {
                    const uint32_t e = swz(c * APP + (uint32_t)lane);
                    const uint64_t g = nbase | segtab[e >> lowc] | (e & lmask);
                    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(gpsi + g),
                                                     (void __attribute__((address_space(3))) *)(sp + c * APP),
                                                     16, 0, 0);
                    if (ADJ)
                        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(glam + g),
                                                         (void __attribute__((address_space(3))) *)(sl + c * APP),
                                                         16, 0, 0);
                }
            }
        }
        // segment result from registers: straight to HBM (last segment of a prefetching tile), else to LDS
        auto store = [&](const Regs<R, N> &v, const Regs<R, N> &l) {
            // recompute the addresses rather than keep 2^RB of them live through the op loop
            uint32_t es = ES, rb2[RB];
            asm volatile("" : "+v"(es));
#pragma unroll
            for (int k = 0; k < RB; k++) {
                rb2[k] = rs[k];
                asm volatile("" : "+s"(rb2[k]));
            }
            if (pf && last_seg) {
                // register j holds tile element es ^ D_j
                if (active && !(ADJ && sg.last)) {
#pragma unroll
                    for (int j = 0; j < N; j++) {
                        uint32_t D = 0;
#pragma unroll
                        for (int k = 0; k < RB; k++)
                            if (j >> k & 1) D ^= rb2[k];
                        const uint32_t e = es ^ D;
                        const uint64_t g = base | segtab[e >> lowc] | (e & lmask);
                        gpsi[g] = v.get(j);
                        if (ADJ) glam[g] = l.get(j);
                    }
                }
            } else if (active) {
                const uint32_t pe = swz(es);
#pragma unroll
                for (int j = 0; j < N; j++) {
                    uint32_t D = 0;
#pragma unroll
                    for (int k = 0; k < RB; k++)
                        if (j >> k & 1) D ^= rb2[k];
                    const uint32_t addr = pe ^ swz(D);
                    sp[addr] = v.get(j);
                    if (ADJ) sl[addr] = l.get(j);
                }
            }
        };
        // op records and matrices are fetched one op ahead, so their latency hides behind the arithmetic
        const M2<R> *mtab = reinterpret_cast<const M2<R> *>(a.mats) + (C.mat_off - C.op_base);
        OpCursor<R> oc;
        oc.k = 0;
        oc.n = S.n_ops;
        if (stop_early && S.op_begin < P.first_train) oc.n = S.op_begin + S.n_ops - P.first_train;
        oc.oi = S.op_begin + (ADJ ? S.n_ops - 1 : 0);
        oc.op = ldu(a.ops + oc.oi);    // a segment holds at least one op
        oc.mat = ldu(mtab + oc.oi);
        if constexpr (ADJ) {
            Regs<R, N> aw, lw;
            while (oc.k < oc.n) {
                adj_step<R, RB, NT>(a, C, sg.circ, mtab, oc, Et, active, lane, wave, red, av, lv, aw, lw);
                if (oc.k >= oc.n) {
                    av = aw;
                    lv = lw;
                    break;
                }
                adj_step<R, RB, NT>(a, C, sg.circ, mtab, oc, Et, active, lane, wave, red, aw, lw, av, lv);
            }
            store(av, lv);
        } else {
            constexpr bool FUSE = RB == 4 && sizeof(R) == 4;
            if constexpr (!FUSE) cursor_skip_markers<R, false>(a, mtab, oc);
            Regs<R, N> aw;
            while (true) {
                if (oc.k >= oc.n) {
                    store(av, av);
                    break;
                }
                fwd_step<R, RB, FUSE>(a, C, sg.circ, mtab, oc, Et, lane, av, aw);
                if (oc.k >= oc.n) {
                    store(aw, aw);
                    break;
                }
                fwd_step<R, RB, FUSE>(a, C, sg.circ, mtab, oc, Et, lane, aw, av);
            }
        }
        __syncthreads();
    }

    if (ADJ) {
        for (int slot = threadIdx.x; slot < P.n_train; slot += NT) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; w++) s += red[slot * (NT / 64) + w];
            a.partials[sg.partial_base + tile * P.n_train + slot] = s;
        }
    }
    if (ADJ && sg.last) return pf;  // psi and lambda of a fully undone circuit are not read again
    if (pf) return true;            // stored from registers in the last segment
    if (sg.first && !ADJ) {
        for (uint32_t h = threadIdx.x; h < nh; h += NT) segtab[h] = deposit(h, himask);
        __syncthreads();
    }
    constexpr int TB = tile_batch<R>();
    typedef unsigned long long GI __attribute__((ext_vector_type(TB)));
    for (uint32_t e0 = threadIdx.x; e0 < T; e0 += TB * NT) {
        Regs<R, TB> bp, bl;
        GI gi;
#pragma unroll
        for (int u = 0; u < TB; u++) {
            const uint32_t e = e0 + (uint32_t)u * NT;
            if (e < T) {
                gi[u] = base | segtab[e >> lowc] | (e & lmask);
                bp.set(u, sp[swz(e)]);
                if (ADJ) bl.set(u, sl[swz(e)]);
            }
        }
#pragma unroll
        for (int u = 0; u < TB; u++) {
            const uint32_t e = e0 + (uint32_t)u * NT;
            if (e < T) {
                gpsi[gi[u]] = bp.get(u);
                if (ADJ) glam[gi[u]] = bl.get(u);
            }
        }
    }
    return false;
}

// A level launch: workgroups take chunks of a.chunk consecutive tiles (grid-stride over chunks); within a
// chunk, a tile whose successor belongs to the same (circuit, pass) prefetches it. Forward passes run two
// workgroups per CU and balance better with shorter chunks (4); the adjoint (one per CU) gains more from
// longer prefetch chains (8; measured on the 20-qubit circuit-learning levels). A level with too few
// tiles to give every resident workgroup a full chunk gets shorter chunks, down to one tile.
template <bool ADJ>
constexpr int tile_chunk() { return ADJ ? 8 : 4; }

template <typename R, bool ADJ, int RB, int NT>
__device__ __forceinline__ void rtile_tiles(const LevelArgs &a)
{
    const int64_t ch = a.chunk;
    const int64_t nchunks = (a.n_blocks + ch - 1) / ch;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t b0 = c * ch, b1 = b0 + ch < a.n_blocks ? b0 + ch : a.n_blocks;
        bool pre = false;
        for (int64_t blk = b0; blk < b1; blk++) {
            const int si = find_block(a.segs, a.n_segs, blk);
            const Seg sg = a.segs[si];
            const int64_t send = si + 1 < a.n_segs ? a.segs[si + 1].first_block : a.n_blocks;
            const int64_t nxt = (blk + 1 < b1 && blk + 1 < send) ? blk + 1 : -1;
            pre = rtile_body<R, ADJ, RB, NT>(a, blk, sg, pre, nxt);
            __syncthreads();
        }
    }
}

// Forward passes ask for two workgroups per CU (at most 128 VGPRs); the adjoint keeps psi and lambda in
// registers and runs one workgroup per CU.
template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rtile_fwd(LevelArgs a)
{
    rtile_tiles<R, false, RB, NT>(a);
}

template <typename R, int RB, int NT>
__global__ __launch_bounds__(NT) void k_rtile_adj(LevelArgs a)
{
    rtile_tiles<R, true, RB, NT>(a);
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
// every wait ends. A finished tile is published with a device-scope release fence before its circuit's
// counter is incremented; a waiting workgroup acquires after it has seen the count.
//
// The claim loop keeps every thread of a workgroup on the same path: the next item is claimed by thread 0
// in the same region that publishes the finished one, fenced by barriers on both sides, and the loop test
// reads the claimed item as a wave-uniform value. (With the claim at the top of the loop and the
// publication at its bottom, each under its own `threadIdx.x == 0` test, the compiler joins the two regions
// across the loop's back edge and turns the loop into two nested loops whose inner one lets wave 0's other
// lanes return to the top barrier without lane 0, re-read the old item and run it again, forever.)
//
// A wait is bounded by wait_ticks of the constant-rate wall clock. A wait that runs out sets *error; from
// then on every workgroup skips the work of the items it claims (it still counts them finished, so no
// other wait blocks on them) and the host reports the launch's results as invalid.
template <typename R, bool ADJ, int RB, int NT>
__device__ __forceinline__ void persistent_body(const PersistArgs &pa)
{
    __shared__ long long item_s;
    __shared__ int run_s;
    if (threadIdx.x == 0) item_s = (long long)atomicAdd(pa.head, 1ull);
    __syncthreads();
    int64_t item = uniform_i64(item_s);
    while (item < pa.n_items) {
        int lo = 0, hi = pa.n_levels - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pa.levels[mid].first_item <= item) lo = mid; else hi = mid - 1;
        }
        const PersistLevel lv = pa.levels[lo];
        LevelArgs a = pa.base;
        a.segs = pa.base.segs + lv.seg_off;
        a.n_segs = lv.n_segs;
        const int64_t blk = item - lv.first_item;
        const Seg sg = a.segs[find_block(a.segs, a.n_segs, blk)];
        if (threadIdx.x == 0) {
            int run = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
            if (run && sg.wait > 0) {
                const int64_t need = sg.wait + pa.wait_extra;
                const int64_t t0 = wall_clock64();
                while ((int64_t)__hip_atomic_load(pa.done + sg.circ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (wall_clock64() - t0 > pa.wait_ticks) {
                        atomicOr(pa.error, 1);
                        run = 0;
                        break;
                    }
                }
            }
            __threadfence();
            run_s = run;
        }
        __syncthreads();
        if (uniform_i64(run_s)) rtile_body<R, ADJ, RB, NT>(a, blk, sg, false, -1);
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(pa.done + sg.circ, 1ull);
            item_s = (long long)atomicAdd(pa.head, 1ull);
        }
        __syncthreads();
        item = uniform_i64(item_s);
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
    const uint64_t ngroups = 1ull << (n - 1);
    const int p = op.p0;
    const uint64_t bit = 1ull << p;
    M2<R> m = op_matrix<R>(a, C, sg.circ, op, P.op_begin);
    if (ADJ) m = dagger_r(m);
    double acc = 0.0;
    for (uint32_t e = threadIdx.x; e < kStrideGroupsPerBlock; e += kBlock) {
        const uint64_t gi = g0 + e;
        if (gi >= ngroups) break;
        const uint64_t i0 = insert0_64(gi, p), i1 = i0 | bit;
        Cx<R> x = gpsi[i0], y = gpsi[i1];
        if (ADJ) {
            Cx<R> u = glam[i0], v = glam[i1];
            if (op.flags & OP_TRAIN) acc += gen_inner<R>(kind, x, y, u, v);
            apply2(m, u, v);
            glam[i0] = u; glam[i1] = v;
        }
        apply2(m, x, y);
        gpsi[i0] = x; gpsi[i1] = y;
    }
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
template <typename R>
__global__ __launch_bounds__(kBlock) void k_expect(ExpArgs a)
{
    __shared__ double red[kBlock / 64];
    const int64_t blk = (int64_t)blockIdx.x;
    const DevGroup G = a.groups[find_block(a.groups, a.n_groups, blk)];
    const int64_t chunk = blk - G.first_block;
    const DevCirc C = a.circs[G.circ];
    const Cx<R> *st = reinterpret_cast<const Cx<R> *>(a.psi) + C.state_off;
    const int nt = G.n_terms;
    uint64_t z[kMaxGroupTerms];
    int ny[kMaxGroupTerms];
    double acc[kMaxGroupTerms];
#pragma unroll
    for (int j = 0; j < kMaxGroupTerms; j++) {
        z[j] = j < nt ? a.terms[G.term_begin + j].zmask : 0;
        ny[j] = j < nt ? a.terms[G.term_begin + j].ny : 0;
        acc[j] = 0.0;
    }
    const uint64_t x = G.xmask;
    const uint32_t per = 1u << G.chunk_log2;
    const uint64_t i0 = (uint64_t)chunk << G.chunk_log2;
    if (x == 0) {
        const uint64_t dim = 1ull << C.n;
        const uint32_t lim = (uint32_t)(dim - i0 < (uint64_t)per ? dim - i0 : (uint64_t)per);
#pragma unroll 4
        for (uint32_t e = threadIdx.x; e < lim; e += kBlock) {
            const uint64_t b = i0 + e;
            const Cx<R> v = st[b];
            const double w = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
#pragma unroll
            for (int j = 0; j < kMaxGroupTerms; j++)
                if (j < nt) acc[j] += parity64(b & z[j]) ? -w : w;
        }
    } else {
        const int h = 63 - __clzll(x);
        const uint64_t npairs = 1ull << (C.n - 1);
        const uint32_t lim = (uint32_t)(npairs - i0 < (uint64_t)per ? npairs - i0 : (uint64_t)per);
#pragma unroll 4
        for (uint32_t e = threadIdx.x; e < lim; e += kBlock) {
            const uint64_t i = i0 + e;
            const uint64_t b = insert0_64(i, h);
            const Cx<R> a0 = st[b], a1 = st[b ^ x];
            // w = conj(psi[b ^ x]) psi[b]
            const double wr = (double)a1.re * (double)a0.re + (double)a1.im * (double)a0.im;
            const double wi = (double)a1.re * (double)a0.im - (double)a1.im * (double)a0.re;
#pragma unroll
            for (int j = 0; j < kMaxGroupTerms; j++) {
                if (j < nt) {
                    const int q = ny[j];
                    double re = (q == 0) ? wr : (q == 1) ? -wi : (q == 2) ? -wr : wi;
                    re *= 2.0;
                    acc[j] += parity64(b & z[j]) ? -re : re;
                }
            }
        }
    }
    for (int j = 0; j < nt; j++) {
        const double s = block_sum(acc[j], red);
        if (threadIdx.x == 0) a.partials[G.partial_base + chunk * nt + j] = s;
    }
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
    for (uint32_t e = threadIdx.x; e < 4096u; e += kBlock) {
        const uint64_t o = o0 + e;
        if (o >= dim) break;
        // diagonal terms (x-mask 0) scale psi[o] itself: their signed coefficients are summed first; the
        // host orders the other terms by x-mask, so terms sharing one read psi[o ^ x] once
        double d = 0.0, sr = 0.0, si = 0.0;
        uint64_t px = 0;
        double vr = 0.0, vi = 0.0;
        for (int64_t t = tb; t < te; t++) {
            const DevObsTerm term = ldu(a.obs + t);
            if (term.xmask == 0) {
                d += parity64(o & term.zmask) ? -term.coeff : term.coeff;
                continue;
            }
            const uint64_t b = o ^ term.xmask;
            if (term.xmask != px) {
                const Cx<R> v = st[b];
                vr = v.re;
                vi = v.im;
                px = term.xmask;
            }
            double pr, pi;
            switch (term.ny) {
            case 0: pr = vr; pi = vi; break;
            case 1: pr = -vi; pi = vr; break;
            case 2: pr = -vr; pi = -vi; break;
            default: pr = vi; pi = -vr; break;
            }
            const double cf = parity64(b & term.zmask) ? -term.coeff : term.coeff;
            sr += cf * pr;
            si += cf * pi;
        }
        const Cx<R> v0 = st[o];
        sr += d * (double)v0.re;
        si += d * (double)v0.im;
        Cx<R> out;
        out.re = (R)(w * sr);
        out.im = (R)(w * si);
        lam[o] = out;
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
    if ((int64_t)blocks > a.n_items) blocks = (int)a.n_items;
    const dim3 grid((unsigned)blocks), block(kRtileThreads);
    if (precision == QV_C64) {
        if (adjoint) hipLaunchKernelGGL((k_rtile_adj_persist<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_rtile_fwd_persist<float, kRegBitsC64, kRtileThreads>), grid, block, lds, s, a);
    } else {
        if (adjoint) hipLaunchKernelGGL((k_rtile_adj_persist<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_rtile_fwd_persist<double, kRegBitsC128, kRtileThreads>), grid, block, lds, s, a);
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
