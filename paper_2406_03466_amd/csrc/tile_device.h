// Device code of the register-tiled gate passes (with the helpers every kernel shares): included by
// kernels.hip for the precompiled kernels, and compiled at run time together with a generated op program
// for the passes the library specialises (see jit.cpp). It holds no host code.
#pragma once
#include <stdint.h>

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

// Matrix of a one-qubit gate: textbook definitions (rotations are exp(-i a sigma / 2)), except RZ, built as
// diag(1, e^{ia}) = e^{ia/2} RZ(a). Every diagonal kind then has 1 as its first entry, so a diagonal op
// multiplies only the amplitudes whose bit is set. A circuit's final state differs from the textbook one by
// the factor e^{ia/2} of each of its RZ gates; every result but the state itself is independent of a global
// phase, and the state is multiplied by the inverse product before it is handed out (k_scale_state).
__device__ inline void gate_matrix(int kind, double a, M2d &m)
{
    for (int k = 0; k < 4; k++) { m.re[k] = 0.0; m.im[k] = 0.0; }
    double s, c;
    sincos(0.5 * a, &s, &c);
    if (kind == QV_RZ) sincos(a, &s, &c);
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
    case QV_RZ: m.re[0] = 1; m.re[3] = c; m.im[3] = s; break;
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

// diag(1, r) on register bit K: only the amplitudes whose bit K is set change.
template <int K, int N, typename R>
__device__ __forceinline__ void r_phase1(Regs<R, N> &v, R rr, R ri)
{
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (!(j & (1 << K))) continue;
        const Cx<R> x = v.get(j);
        v.set(j, rr * x.re - ri * x.im, rr * x.im + ri * x.re);
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
// Precision of the adjoint inner products of complex64 states: 0 sums a thread's products in FP32 and
// everything after that (wave, workgroup, tiles, circuits) in FP64; 1 forms every product of two FP32
// amplitude components in FP64 (exactly: 24 + 24 significant bits fit in 53) and sums in FP64 from there.
#ifndef QV_ADJ_INNER_F64
#define QV_ADJ_INNER_F64 0
#endif

// The accumulator type of a thread's inner-product sum.
template <typename R>
struct InnerAcc {
    typedef R type;
};
#if QV_ADJ_INNER_F64
template <>
struct InnerAcc<float> {
    typedef double type;
};
#endif

template <int K, int GEN, int N, typename R>
__device__ __forceinline__ double r_inner(const Regs<R, N> &a, const Regs<R, N> &l)
{
    typedef typename InnerAcc<R>::type A;
    A acc[2] = {(A)0, (A)0};
#pragma unroll
    for (int j = 0, n = 0; j < N; j++) {
        if (j & (1 << K)) continue;
        const int j1 = j | (1 << K);
        const Cx<R> a0r = a.get(j), a1r = a.get(j1), l0r = l.get(j), l1r = l.get(j1);
        const Cx<A> a0{(A)a0r.re, (A)a0r.im}, a1{(A)a1r.re, (A)a1r.im}, l0{(A)l0r.re, (A)l0r.im},
            l1{(A)l1r.re, (A)l1r.im};
        A &s = acc[n++ & 1];
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

// Im <l| Z_K |a> for register bit K from the amplitudes with bit K set alone: -2 sum Im conj(l1) a1. Over a
// whole state Im <l|a> = 0 (the seed is a Hermitian observable or a real diagonal applied to psi, and the
// sweep applies one unitary to both), so the bit-0 half sums to minus the bit-1 half. Exact for the total
// over all tiles of a circuit, which is what the gradient takes.
template <int K, int N, typename R>
__device__ __forceinline__ double r_inner_z1(const Regs<R, N> &a, const Regs<R, N> &l)
{
    typedef typename InnerAcc<R>::type A;
    A acc[2] = {(A)0, (A)0};
#pragma unroll
    for (int j = 0, n = 0; j < N; j++) {
        if (!(j & (1 << K))) continue;
        const Cx<R> x = a.get(j), y = l.get(j);
        acc[n++ & 1] += (A)y.re * (A)x.im - (A)y.im * (A)x.re;
    }
    return -2.0 * ((double)acc[0] + (double)acc[1]);
}

// Im <l| Z_p |a> when qubit p is a thread bit with value `bit`.
template <int N, typename R>
__device__ __forceinline__ double t_inner_z(const Regs<R, N> &a, const Regs<R, N> &l, int bit)
{
    typedef typename InnerAcc<R>::type A;
    A acc[2] = {(A)0, (A)0};
#pragma unroll
    for (int j = 0; j < N; j++) {
        const Cx<R> x = a.get(j), y = l.get(j);
        acc[j & 1] += (A)y.re * (A)x.im - (A)y.im * (A)x.re;
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

// The inverse of a diagonal op diag(1, d1) (gate_matrix's form of every diagonal kind) on psi and lambda:
// only the amplitudes whose bit K is set change.
template <int K, int N, typename R>
__device__ __forceinline__ void adj_diag(Regs<R, N> &a, Regs<R, N> &l, R d1r, R d1i, bool train, double &ip)
{
    // of the diagonal kinds only RZ carries a parameter
    if (train) ip = r_inner_z1<K>(a, l);
    r_phase1<K>(a, d1r, d1i);
    r_phase1<K>(l, d1r, d1i);
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
    K4_CASES(OC_DIAG, (r_phase1<K>(v, d1r, d1i)))   // diagonal kinds are diag(1, d1) (gate_matrix)
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
    K4_CASES(OC_DIAG, (adj_diag<K>(a, l, d1r, d1i, train, ip)))
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
    static_assert(__builtin_offsetof(DevSeg, lead) % 8 == 0 && __builtin_offsetof(DevSeg, trail) == __builtin_offsetof(DevSeg, lead) + 8 &&
                      __builtin_offsetof(DevSeg, n_lead) == __builtin_offsetof(DevSeg, trail) + 8 &&
                      __builtin_offsetof(DevSeg, n_trail) == __builtin_offsetof(DevSeg, n_lead) + 1 &&
                      __builtin_offsetof(DevSeg, rimg_lead) == __builtin_offsetof(DevSeg, n_lead) + 4 &&
                      __builtin_offsetof(DevSeg, rimg_trail) == __builtin_offsetof(DevSeg, rimg_lead) + 8,
                  "DevSeg run layout");
    const uint32_t *w = reinterpret_cast<const uint32_t *>(sp) + __builtin_offsetof(DevSeg, lead) / 4;
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

// The op program of a tile pass: InterpProg walks each segment's op records on the device (one kernel for
// every pass); a generated program (jit.cpp) holds the ops of one pass as straight-line code, segment by
// segment, with every op's kind, qubits, register bits and partial-sum slot as constants.
struct InterpProg {
    static constexpr bool kGenerated = false;
};

// The matrix of one op of a generated program: from the circuit's table (k: the op's index within its
// segment), or the shifted matrix of a parameter-shift variant's moved gate. The shifted gate's index is
// made opaque at each op: otherwise the compiler hoists every op's test GATE == shift_gate (a 64-bit lane
// mask each) out of the tile loops, and hundreds of live scalar registers spill into vector registers
// (into scratch under the forward's 128-register cap).
template <typename R, int GATE>
__device__ __forceinline__ M2<R> gen_mat(const LevelArgs &a, const DevCirc &C, int circ, const M2<R> *mp, int k)
{
    int shift = C.shift_gate;
    asm volatile("" : "+s"(shift));
    M2<R> mat = ldu(mp + k);
    if (GATE == shift) {
        mat = ldu(reinterpret_cast<const M2<R> *>(a.smats) + circ);
        scalar_wait(mat);
    }
    return mat;
}

// One op of a generated program, forward; the op-code switch of code_apply folds away, its operands being
// constants.
template <typename R, int RB, int CODE, int KIND, int P0, int P1, int K0, int K1, int GATE>
__device__ __forceinline__ void gen_fwd_op(const LevelArgs &a, const DevCirc &C, int circ, const M2<R> *mp, int k,
                                           uint32_t Et, Regs<R, 1 << RB> &v)
{
    M2<R> mat{};
    if constexpr (KIND != QV_CNOT && KIND != QV_CZ) mat = gen_mat<R, GATE>(a, C, circ, mp, k);
    DevOp op;
    op.gate = GATE;
    op.kind = (uint8_t)KIND;
    op.p0 = (uint8_t)P0;
    op.p1 = (uint8_t)P1;
    op.flags = 0;
    op.train_slot = -1;
    op.k0 = (int8_t)K0;
    op.k1 = (int8_t)K1;
    op.pad = 0;
    code_apply<false, RB, R>(v, CODE, op, mat, Et);
}

// One op of a generated program, adjoint: Im <l| G |a> when trainable (wave sum into the slot's LDS
// partials, as adj_step), then the inverse op on a and l in place.
template <typename R, int RB, int NT, int CODE, int KIND, int P0, int P1, int K0, int K1, int GATE, int TRAIN,
          int SLOT>
__device__ __forceinline__ void gen_adj_op(const LevelArgs &a, const DevCirc &C, int circ, const M2<R> *mp, int k,
                                           uint32_t Et, bool active, int lane, int wave, double *red,
                                           Regs<R, 1 << RB> &av, Regs<R, 1 << RB> &lv)
{
    M2<R> mat{};
    if constexpr (KIND != QV_CNOT && KIND != QV_CZ) mat = gen_mat<R, GATE>(a, C, circ, mp, k);
    DevOp op;
    op.gate = GATE;
    op.kind = (uint8_t)KIND;
    op.p0 = (uint8_t)P0;
    op.p1 = (uint8_t)P1;
    op.flags = TRAIN ? (uint8_t)OP_TRAIN : (uint8_t)0;
    op.train_slot = SLOT;
    op.k0 = (int8_t)K0;
    op.k1 = (int8_t)K1;
    op.pad = 0;
    double ip = code_adjoint<RB, R>(av, lv, CODE, op, mat, Et);
    if constexpr (TRAIN != 0) {
        if (!active) ip = 0.0;
        ip = wave_sum_to_63(ip);
        if (lane == 63) red[SLOT * (NT / 64) + wave] = ip;
    }
}

// Whether tile blk of an adjoint segment lies where psi is zero throughout the pass (a qubit of the pass's
// zero mask at 1, in rtile_body's numbering, which puts those tiles last): a tile for the LAM code.
__device__ __forceinline__ bool lam_tile(const LevelArgs &a, int64_t blk, const Seg &sg)
{
    if (sg.last) return false;
    const DevPass P = ldu(a.passes + sg.pass);
    const DevCirc C = ldu(a.circs + sg.circ);
    const uint64_t full = (C.n >= 64) ? ~0ull : ((1ull << C.n) - 1ull);
    const uint64_t outside = full & ~P.local_mask;
    const int live = __popcll(outside & ~(P.zero_mask & outside));
    return ((blk - sg.first_block + sg.tile_off) >> live) != 0;
}

// LAM: an adjoint launch over tiles where psi is zero throughout the pass (a qubit of the pass's zero mask
// at 1): lambda alone is loaded, undone (each op's inverse) and stored, and the partial sums are zero.
template <typename R, bool ADJ, int RB, int NT, class PROG = InterpProg, bool LAM = false>
__device__ __forceinline__ bool rtile_body(const LevelArgs &a, unsigned char *smem, int64_t blk, const Seg &sg,
                                           bool preloaded, int64_t next_blk)
{
    static_assert(RB >= 1 && RB <= 4, "register-bit dispatch covers register bits 0..3");
    constexpr int N = 1 << RB;
    const int64_t tile = blk - sg.first_block + sg.tile_off;
    const DevPass P = ldu(a.passes + sg.pass);
    const DevCirc C = ldu(a.circs + sg.circ);
    const int n = C.n, t = P.t, lowc = P.pad;
    const uint32_t T = 1u << t;
    const int TL = 1 << (a.lds_t);

    Cx<R> *sp = reinterpret_cast<Cx<R> *>(smem);
    // a LAM launch keeps lambda where psi would be (it never touches psi): one tile of LDS, like the forward
    Cx<R> *sl = sp + (ADJ && !LAM ? TL : 0);
    uint64_t *segtab = reinterpret_cast<uint64_t *>(sp + (ADJ && !LAM ? 2 * TL : TL));
    double *red = reinterpret_cast<double *>(segtab + (1 << a.tab_bits));

    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    // Forward passes after a circuit's first: a tile with a qubit of zero_mask at 1 holds zeros, which the
    // earlier passes wrote there (a gate acting on zeros leaves exact zeros), so it is left alone. The
    // circuit's tiles are numbered with those last: tile i < 2^live has base deposit(i, outside & ~zero_mask)
    // and the rest do nothing, which keeps a level's working tiles contiguous.
    const uint64_t outside = full & ~P.local_mask;
    const uint64_t zm = (!ADJ && !sg.first) ? (P.zero_mask & outside) : 0ull;
    // The adjoint numbers the tiles of a pass after the circuit's first the same way, those where psi can
    // be nonzero first (tile i: bits of i below `live` go to outside & ~zero_mask, the rest to zero_mask):
    // the host launches those with the full kernel and the others with the LAM kernel.
    const uint64_t zz = ADJ ? (sg.last ? 0ull : (P.zero_mask & outside)) : zm;
    const int live = __popcll(outside & ~zz);
    if (zm != 0 && (tile >> live) != 0) {
        if (preloaded) __builtin_amdgcn_s_waitcnt(0);  // never the case: no tile prefetches such a tile
        return false;
    }
    auto tile_base = [&](int64_t i) {
        return deposit((uint64_t)i & ((1ull << live) - 1ull), outside & ~zz) | deposit((uint64_t)i >> live, zz);
    };
    const uint64_t base = tile_base(tile);
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
    // A circuit's first pass starts from |0...0> and its gates act on the tile's qubits only, so a tile with
    // a qubit outside the tile set at 1 (base != 0) holds zeros throughout that pass. The forward stores
    // zeros for it; in the adjoint's sweep over that pass psi is zero there, so each of its inner products
    // is zero and psi and lambda are not needed afterwards: the tile only clears its partial sums. Only the
    // circuit's tile 0 then runs the pass, and it prefetches nothing (every later tile is such a tile).
    if (base != 0 && (stop_early || (!ADJ && sg.first))) {
        if (ADJ) {
            for (int slot = threadIdx.x; slot < P.n_train; slot += NT) a.partials[sg.partial_base + tile * P.n_train + slot] = 0.0;
            return false;
        }
        for (uint32_t h = threadIdx.x; h < nh; h += NT) segtab[h] = deposit(h, himask);
        __syncthreads();
        Cx<R> z;
        z.re = (R)0;
        z.im = (R)0;
        for (uint32_t e = threadIdx.x; e < T; e += NT) gpsi[base | segtab[e >> lowc] | (e & lmask)] = z;
        return false;
    }
    // (a tile prefetches only a successor of its own kind: a LAM tile keeps lambda where psi would be)
    const int64_t ntile = next_blk - sg.first_block + sg.tile_off;
    const bool pf = next_blk >= 0 && !(!ADJ && sg.first) && !stop_early && T >= (uint32_t)APP && nseg > 0 &&
                    !(zm != 0 && (ntile >> live) != 0) && (!ADJ || LAM == (zz != 0 && (ntile >> live) != 0));

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
                    if (!LAM) bp.set(u, gpsi[g]);
                    if (ADJ) bl.set(u, glam[g]);
                }
            }
#pragma unroll
            for (int u = 0; u < TB; u++) {
                const uint32_t e = e0 + (uint32_t)u * NT;
                if (e < T) {
                    if (!LAM) sp[swz(e)] = bp.get(u);
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
                if (!LAM) av.set(j, sp[addr]);
                if (ADJ) lv.set(j, sl[addr]);
            }
        }
        const bool last_seg = s0 == nseg - 1;
        // With a folded run, a thread's stores may land where another thread loads: every wave loads first.
        if (remap && !(pf && last_seg)) __syncthreads();
        if (pf && last_seg) {
            __syncthreads();  // every wave has its registers: LDS may be overwritten
            const uint64_t nbase = tile_base(next_blk - sg.first_block + sg.tile_off);
            for (uint32_t c = (uint32_t)wave; c < T / APP; c += NT / 64) {
                // load c covers LDS positions [c*APP, (c+1)*APP); position q holds element swz(q)
                if constexpr (sizeof(R) == 4) {
                    const uint32_t d = c * 64 + (uint32_t)lane;  // float d of the tile: part d&1 of position d>>1
                    const uint32_t e = swz(d >> 1);
                    const uint64_t g = nbase | segtab[e >> lowc] | (e & lmask);
                    const float *src = reinterpret_cast<const float *>(gpsi + g) + (d & 1u);
                    if (!LAM)
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
                    if (!LAM)
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
                        if (!LAM) gpsi[g] = v.get(j);
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
                    if (!LAM) sp[addr] = v.get(j);
                    if (ADJ) sl[addr] = l.get(j);
                }
            }
        };
        // op records and matrices are fetched one op ahead, so their latency hides behind the arithmetic
        const M2<R> *mtab = reinterpret_cast<const M2<R> *>(a.mats) + (C.mat_off - C.op_base);
        if constexpr (PROG::kGenerated) {
            const M2<R> *mp = mtab + S.op_begin;
            if constexpr (ADJ) {
                PROG::template adj<R, RB, NT>(si, stop_early, a, C, sg.circ, mp, Et, active, lane, wave, red, av, lv);
                store(av, lv);
            } else {
                PROG::template fwd<R, RB, NT>(si, a, C, sg.circ, mp, Et, lane, av);
                store(av, av);
            }
            __syncthreads();
            continue;
        }
        OpCursor<R> oc;
        oc.k = 0;
        oc.n = S.n_ops;
        if (stop_early && S.op_begin < P.first_train) oc.n = S.op_begin + S.n_ops - P.first_train;
        oc.oi = S.op_begin + (ADJ ? S.n_ops - 1 : 0);
        oc.op = ldu(a.ops + oc.oi);    // a segment holds at least one op
        oc.mat = ldu(mtab + oc.oi);
        if constexpr (LAM) {
            // lambda alone: each op's inverse in reverse order (fused-block markers are skipped: the block's
            // gates follow them); the next op's record and matrix are fetched while this one runs
            DevOp nop = oc.op;
            M2<R> nmat = oc.mat;
            for (int64_t oi = (int64_t)S.op_begin + S.n_ops - 1; oi >= (int64_t)S.op_begin; oi--) {
                const DevOp op = nop;
                M2<R> mat = nmat;
                if (oi > (int64_t)S.op_begin) {
                    nop = ldu(a.ops + oi - 1);
                    nmat = ldu(mtab + oi - 1);
                }
                if (op.kind == kFusedKind) continue;
                if (op.gate == C.shift_gate) {
                    mat = ldu(reinterpret_cast<const M2<R> *>(a.smats) + sg.circ);
                    scalar_wait(mat);
                }
                code_apply<true, RB, R>(lv, op.flags >> kOpCodeShift, op, mat, Et);
            }
            store(lv, lv);
        } else if constexpr (ADJ) {
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
            if (!LAM)  // a LAM launch has no reduction area: its tiles' inner products are zero
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
                if (!LAM) bp.set(u, sp[swz(e)]);
                if (ADJ) bl.set(u, sl[swz(e)]);
            }
        }
#pragma unroll
        for (int u = 0; u < TB; u++) {
            const uint32_t e = e0 + (uint32_t)u * NT;
            if (e < T) {
                if (!LAM) gpsi[gi[u]] = bp.get(u);
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

// The chunk a workgroup takes when the grid has one workgroup per chunk. The GPU deals workgroups to its 8
// XCDs in turn (workgroup b to XCD b mod 8), so chunk b would put every 8th chunk on one XCD: a level whose
// work is concentrated in every 16th or 32nd chunk (a circuit's first pass, where only each circuit's tile
// 0 runs) would run on one XCD. Instead each XCD takes one contiguous range of the chunks (a bijection of
// [0, n)), which spreads such patterns over all eight. Evenly loaded levels keep chunk b (measured 1-4 %
// faster in that order).
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t n)
{
    constexpr int64_t X = 8;
    const int64_t q = n / X, r = n % X, x = b % X, i = b / X;
    return x * q + (x < r ? x : r) + i;
}

template <typename R, bool ADJ, int RB, int NT, class PROG = InterpProg, bool LAM = false>
__device__ __forceinline__ void rtile_tiles(const LevelArgs &a, unsigned char *smem)
{
    const int64_t ch = a.chunk;
    const int64_t nchunks = (a.n_blocks + ch - 1) / ch;
    // a level of circuits' first passes (judged by its first segment) has its work in each circuit's tile 0
    const Seg s0 = a.segs[0];
    const bool spread = (int64_t)gridDim.x == nchunks && (ADJ ? s0.last : s0.first) != 0;
    for (int64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const int64_t c = spread ? xcd_chunk(c0, nchunks) : c0;
        const int64_t b0 = c * ch, b1 = b0 + ch < a.n_blocks ? b0 + ch : a.n_blocks;
        bool pre = false;
        for (int64_t blk = b0; blk < b1; blk++) {
            const int si = find_block(a.segs, a.n_segs, blk);
            const Seg sg = a.segs[si];
            const int64_t send = si + 1 < a.n_segs ? a.segs[si + 1].first_block : a.n_blocks;
            const int64_t nxt = (blk + 1 < b1 && blk + 1 < send) ? blk + 1 : -1;
            pre = rtile_body<R, ADJ, RB, NT, PROG, LAM>(a, smem, blk, sg, pre, nxt);
            __syncthreads();
        }
    }
}

}  // namespace qv
