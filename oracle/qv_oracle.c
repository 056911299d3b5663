/*
 * ORACLE (test infrastructure only).
 *
 * A plain, slow, complex128 state-vector simulator written from the paper's problem statement:
 * the quantity every circuit execution produces is the expectation value <0|U^dagger(theta) P U(theta)|0>
 * of a Pauli string P (Eq. 1, and Section 4.1 where the Hamiltonian is written as a weighted sum of Pauli
 * strings whose expectations a simulator evaluates directly), and a gradient of the weighted sum with
 * respect to the circuit angles (parameter-shift rule, Section 4.1 and Section 4.2).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load this library.
 * It shares no code, header, table or helper with the GPU library; the two only agree on the flat input
 * format (gate records, Pauli masks), which both sides define independently.
 *
 * Conventions (the paper is silent on them):
 *   - qubit q is bit q of the amplitude index (qubit 0 is the least significant bit);
 *   - RX/RY/RZ(a) = exp(-i a sigma / 2) with sigma = X/Y/Z;
 *   - a Pauli string is (xmask, zmask): X on x-only bits, Z on z-only bits, Y where both are set;
 *   - the state is never renormalised; expectations are <psi|P|psi>.
 *
 * Parity pinning: every function here is checked by the CPU test suite against closed forms, against
 * brute-force Kronecker-product unitaries and Pauli matrices for n <= 6, against central finite
 * differences and against each other (parameter-shift vs adjoint).
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
typedef long double complex lcplx;  /* accumulators of long sums */

/* Gate record layout, 24 bytes: kind, q0, q1, param (-1 = fixed angle), angle. */
typedef struct {
    int32_t kind, q0, q1, param;
    double angle;
} orc_gate;

enum {
    ORC_H = 0, ORC_X = 1, ORC_Y = 2, ORC_Z = 3, ORC_S = 4, ORC_T = 5,
    ORC_RX = 6, ORC_RY = 7, ORC_RZ = 8, ORC_CNOT = 9, ORC_CZ = 10
};

/* ---------------------------------------------------------------------------------------------- */
/* Gate matrices (textbook definitions).                                                           */
/* ---------------------------------------------------------------------------------------------- */

/* Writes the 2x2 matrix m[row][col] of a one-qubit gate of the given kind and angle. Returns 0 if the
 * kind is not a one-qubit gate. */
static int gate_matrix(int kind, double a, cplx m[2][2])
{
    const double r = 1.0 / sqrt(2.0);
    const double c = cos(a / 2.0), s = sin(a / 2.0);
    switch (kind) {
    case ORC_H:  m[0][0] = r;   m[0][1] = r;    m[1][0] = r;    m[1][1] = -r;  return 1;
    case ORC_X:  m[0][0] = 0;   m[0][1] = 1;    m[1][0] = 1;    m[1][1] = 0;   return 1;
    case ORC_Y:  m[0][0] = 0;   m[0][1] = -I;   m[1][0] = I;    m[1][1] = 0;   return 1;
    case ORC_Z:  m[0][0] = 1;   m[0][1] = 0;    m[1][0] = 0;    m[1][1] = -1;  return 1;
    case ORC_S:  m[0][0] = 1;   m[0][1] = 0;    m[1][0] = 0;    m[1][1] = I;   return 1;
    case ORC_T:  m[0][0] = 1;   m[0][1] = 0;    m[1][0] = 0;    m[1][1] = cexp(I * M_PI / 4.0); return 1;
    case ORC_RX: m[0][0] = c;   m[0][1] = -I * s; m[1][0] = -I * s; m[1][1] = c; return 1;
    case ORC_RY: m[0][0] = c;   m[0][1] = -s;   m[1][0] = s;    m[1][1] = c;   return 1;
    case ORC_RZ: m[0][0] = cexp(-I * a / 2.0); m[0][1] = 0; m[1][0] = 0; m[1][1] = cexp(I * a / 2.0); return 1;
    default: return 0;
    }
}

static void apply_matrix_1q(cplx *psi, int n, int q, cplx m[2][2])
{
    const int64_t dim = (int64_t)1 << n, bit = (int64_t)1 << q;
#pragma omp parallel for if (dim >= (1 << 20)) schedule(static)
    for (int64_t i = 0; i < dim; i++) {
        if (i & bit) continue;
        cplx a0 = psi[i], a1 = psi[i | bit];
        psi[i] = m[0][0] * a0 + m[0][1] * a1;
        psi[i | bit] = m[1][0] * a0 + m[1][1] * a1;
    }
}

/* CNOT(control c, target t): swap the pair (bit t = 0, bit t = 1) wherever bit c = 1. */
static void apply_cnot(cplx *psi, int n, int c, int t)
{
    const int64_t dim = (int64_t)1 << n, cb = (int64_t)1 << c, tb = (int64_t)1 << t;
#pragma omp parallel for if (dim >= (1 << 20)) schedule(static)
    for (int64_t i = 0; i < dim; i++) {
        if ((i & cb) && !(i & tb)) {
            cplx tmp = psi[i];
            psi[i] = psi[i | tb];
            psi[i | tb] = tmp;
        }
    }
}

/* CZ: negate every amplitude whose two bits are both 1. */
static void apply_cz(cplx *psi, int n, int a, int b)
{
    const int64_t dim = (int64_t)1 << n, ab = (int64_t)1 << a, bb = (int64_t)1 << b;
#pragma omp parallel for if (dim >= (1 << 20)) schedule(static)
    for (int64_t i = 0; i < dim; i++)
        if ((i & ab) && (i & bb)) psi[i] = -psi[i];
}

/* Rotation angle of gate g given the circuit's parameter vector and an optional shift of this gate. */
static double gate_angle(const orc_gate *g, const double *theta)
{
    return g->param >= 0 ? theta[g->param] : g->angle;
}

/* Applies gate g (or its inverse when inverse != 0) with rotation angle a. */
static void apply_gate(cplx *psi, int n, const orc_gate *g, double a, int inverse)
{
    if (g->kind == ORC_CNOT) { apply_cnot(psi, n, g->q0, g->q1); return; }
    if (g->kind == ORC_CZ) { apply_cz(psi, n, g->q0, g->q1); return; }
    cplx m[2][2];
    gate_matrix(g->kind, a, m);
    if (inverse) {
        cplx h[2][2] = {{conj(m[0][0]), conj(m[1][0])}, {conj(m[0][1]), conj(m[1][1])}};
        apply_matrix_1q(psi, n, g->q0, h);
    } else {
        apply_matrix_1q(psi, n, g->q0, m);
    }
}

/* ---------------------------------------------------------------------------------------------- */
/* Circuit execution and Pauli expectations.                                                      */
/* ---------------------------------------------------------------------------------------------- */

/* psi <- U(theta)|0>, where gate `shift_gate` (if >= 0) has its angle moved by `shift`. */
static void run_circuit(cplx *psi, int n, const orc_gate *g, int64_t ng, const double *theta,
                        int64_t shift_gate, double shift, int shift_param, double param_delta)
{
    const int64_t dim = (int64_t)1 << n;
    memset(psi, 0, (size_t)dim * sizeof(cplx));
    psi[0] = 1.0;
    for (int64_t k = 0; k < ng; k++) {
        double a = gate_angle(&g[k], theta);
        if (k == shift_gate) a += shift;
        if (shift_param >= 0 && g[k].param == shift_param) a += param_delta;
        apply_gate(psi, n, &g[k], a, 0);
    }
}

/* (P psi)[b ^ x] = i^{nY} (-1)^{popcount(b & z)} psi[b]; writes P psi into out. */
static void apply_pauli(const cplx *psi, cplx *out, int n, uint64_t x, uint64_t z)
{
    const int64_t dim = (int64_t)1 << n;
    const int ny = __builtin_popcountll(x & z) & 3;
    const cplx iy[4] = {1, I, -1, -I};
    for (int64_t b = 0; b < dim; b++) {
        cplx ph = iy[ny];
        if (__builtin_popcountll((uint64_t)b & z) & 1) ph = -ph;
        out[(uint64_t)b ^ x] = ph * psi[b];
    }
}

/* <psi|P|psi> summed over all 2^n basis states; the imaginary part is returned through imag_out.
 * Products and the running sum are kept in the host's extended precision (long double), so that the
 * rounding of a sum over millions of amplitudes stays far below the tolerance the results are checked
 * to; the result is rounded to double once. */
static double expect_pauli(const cplx *psi, int n, uint64_t x, uint64_t z, double *imag_out)
{
    const int64_t dim = (int64_t)1 << n;
    const int ny = __builtin_popcountll(x & z) & 3;
    const lcplx iy[4] = {1, I, -1, -I};
    lcplx acc = 0;
    for (int64_t b = 0; b < dim; b++) {
        lcplx ph = iy[ny];
        if (__builtin_popcountll((uint64_t)b & z) & 1) ph = -ph;
        acc += conjl((lcplx)psi[(uint64_t)b ^ x]) * ph * (lcplx)psi[b];
    }
    if (imag_out) *imag_out = (double)cimagl(acc);
    return (double)creall(acc);
}

/* Energy E = sum_t c_t <P_t> for one state. term_values may be NULL. */
static double energy(const cplx *psi, int n, int64_t nt, const uint64_t *xm, const uint64_t *zm,
                     const double *cf, double *term_values, double *max_imag)
{
    double e = 0.0;
    for (int64_t t = 0; t < nt; t++) {
        double im = 0.0;
        double v = expect_pauli(psi, n, xm[t], zm[t], &im);
        if (term_values) term_values[t] = v;
        if (max_imag && fabs(im) > *max_imag) *max_imag = fabs(im);
        e += cf[t] * v;
    }
    return e;
}

/* ---------------------------------------------------------------------------------------------- */
/* Batch entry points. A batch is B circuits; circuit b has n_qubits[b] qubits, gates                */
/* gates[goff[b] .. goff[b+1]) and n_params[b] parameters. When params_shared != 0, all circuits read */
/* one parameter vector theta[0 .. n_params[0]); otherwise circuit b reads theta[pbase_b ..) with     */
/* pbase_b = sum of n_params over earlier circuits. When obs_shared != 0, every circuit uses terms     */
/* toff[0] .. toff[1]; otherwise circuit b uses terms toff[b] .. toff[b+1].                            */
/* ---------------------------------------------------------------------------------------------- */

typedef struct {
    int32_t B;
    const int32_t *n_qubits;
    const int64_t *goff;
    const orc_gate *gates;
    const int32_t *n_params;
    int32_t params_shared;
    const int64_t *toff;
    const uint64_t *xmask, *zmask;
    const double *coeff;
    int32_t obs_shared;
} orc_batch;

static int64_t param_base(const orc_batch *bt, int b)
{
    if (bt->params_shared) return 0;
    int64_t s = 0;
    for (int i = 0; i < b; i++) s += bt->n_params[i];
    return s;
}

static void term_range(const orc_batch *bt, int b, int64_t *t0, int64_t *t1)
{
    if (bt->obs_shared) { *t0 = bt->toff[0]; *t1 = bt->toff[1]; }
    else { *t0 = bt->toff[b]; *t1 = bt->toff[b + 1]; }
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Energies (and per-term expectations, in the caller's term order, concatenated per circuit).
 * Returns the number of threads used; max_imag receives the largest |Im <P>| seen. */
int orc_batch_expectations(int32_t B, const int32_t *n_qubits, const int64_t *goff, const orc_gate *gates,
                           const int32_t *n_params, int32_t params_shared, const double *theta,
                           const int64_t *toff, const uint64_t *xmask, const uint64_t *zmask,
                           const double *coeff, int32_t obs_shared, double *energies, double *term_values,
                           double *max_imag, int32_t nthreads)
{
    orc_batch bt = {B, n_qubits, goff, gates, n_params, params_shared, toff, xmask, zmask, coeff, obs_shared};
    int used = set_threads(nthreads);
    double mi = 0.0;
    int64_t *tv_base = (int64_t *)malloc(sizeof(int64_t) * (size_t)(B + 1));
    tv_base[0] = 0;
    for (int b = 0; b < B; b++) {
        int64_t t0, t1;
        term_range(&bt, b, &t0, &t1);
        tv_base[b + 1] = tv_base[b] + (t1 - t0);
    }
#pragma omp parallel for if (B > 1) schedule(dynamic, 1) reduction(max : mi)
    for (int b = 0; b < B; b++) {
        const int n = n_qubits[b];
        cplx *psi = (cplx *)malloc(sizeof(cplx) * ((size_t)1 << n));
        run_circuit(psi, n, gates + goff[b], goff[b + 1] - goff[b], theta + param_base(&bt, b), -1, 0.0, -1, 0.0);
        int64_t t0, t1;
        term_range(&bt, b, &t0, &t1);
        double lmi = 0.0;
        energies[b] = energy(psi, n, t1 - t0, xmask + t0, zmask + t0, coeff + t0,
                             term_values ? term_values + tv_base[b] : NULL, &lmi);
        if (lmi > mi) mi = lmi;
        free(psi);
    }
    free(tv_base);
    if (max_imag) *max_imag = mi;
    return used;
}

/* Final state of one circuit (for state-level comparisons): psi_out has 2^n complex128 entries. */
int orc_final_state(int32_t n, const orc_gate *gates, int64_t ng, const double *theta, double *psi_out)
{
    run_circuit((cplx *)psi_out, n, gates, ng, theta, -1, 0.0, -1, 0.0);
    return 0;
}

/* Weighted gradient output index for parameter p of circuit b. */
static int64_t grad_index(const orc_batch *bt, int b, int p)
{
    return bt->params_shared ? p : param_base(bt, b) + p;
}

/* Parameter-shift rule: for a gate exp(-i a sigma/2), dE/da = (E(a + pi/2) - E(a - pi/2)) / 2.
 * A parameter that drives several gates gets the sum over those gates (chain rule), each shifted alone.
 * grad[j] = sum_b w_b dE_b/dtheta_j (shared) or dE_b/dtheta_j * w_b per circuit. w = NULL means 1. */
int orc_batch_grad_param_shift(int32_t B, const int32_t *n_qubits, const int64_t *goff, const orc_gate *gates,
                               const int32_t *n_params, int32_t params_shared, const double *theta,
                               const int64_t *toff, const uint64_t *xmask, const uint64_t *zmask,
                               const double *coeff, int32_t obs_shared, const double *upstream,
                               double *grad, int32_t nthreads)
{
    orc_batch bt = {B, n_qubits, goff, gates, n_params, params_shared, toff, xmask, zmask, coeff, obs_shared};
    int used = set_threads(nthreads);
    int64_t ng_out = params_shared ? n_params[0] : param_base(&bt, B);
    memset(grad, 0, sizeof(double) * (size_t)ng_out);
    /* enumerate (circuit, trainable gate) pairs */
    int64_t nitems = 0;
    for (int b = 0; b < B; b++)
        for (int64_t k = goff[b]; k < goff[b + 1]; k++)
            if (gates[k].param >= 0) nitems++;
    int64_t *item_b = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nitems + 1));
    int64_t *item_k = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nitems + 1));
    double *contrib = (double *)malloc(sizeof(double) * (size_t)(nitems + 1));
    int64_t it = 0;
    for (int b = 0; b < B; b++)
        for (int64_t k = goff[b]; k < goff[b + 1]; k++)
            if (gates[k].param >= 0) { item_b[it] = b; item_k[it] = k - goff[b]; it++; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nitems; i++) {
        const int b = (int)item_b[i];
        const int n = n_qubits[b];
        const orc_gate *g = gates + goff[b];
        const int64_t ng = goff[b + 1] - goff[b];
        const double *th = theta + param_base(&bt, b);
        int64_t t0, t1;
        term_range(&bt, b, &t0, &t1);
        cplx *psi = (cplx *)malloc(sizeof(cplx) * ((size_t)1 << n));
        run_circuit(psi, n, g, ng, th, item_k[i], M_PI / 2.0, -1, 0.0);
        double ep = energy(psi, n, t1 - t0, xmask + t0, zmask + t0, coeff + t0, NULL, NULL);
        run_circuit(psi, n, g, ng, th, item_k[i], -M_PI / 2.0, -1, 0.0);
        double em = energy(psi, n, t1 - t0, xmask + t0, zmask + t0, coeff + t0, NULL, NULL);
        free(psi);
        double w = upstream ? upstream[b] : 1.0;
        contrib[i] = w * 0.5 * (ep - em);
    }
    /* fixed-order accumulation */
    for (int64_t i = 0; i < nitems; i++) {
        const int b = (int)item_b[i];
        const orc_gate *g = gates + goff[b] + item_k[i];
        grad[grad_index(&bt, b, g->param)] += contrib[i];
    }
    free(item_b); free(item_k); free(contrib);
    return used;
}

/* Central finite differences in the parameter itself (all gates it drives move together):
 * dE/dtheta_j ~ (E(theta + h e_j) - E(theta - h e_j)) / (2h). */
int orc_batch_grad_fd(int32_t B, const int32_t *n_qubits, const int64_t *goff, const orc_gate *gates,
                      const int32_t *n_params, int32_t params_shared, const double *theta,
                      const int64_t *toff, const uint64_t *xmask, const uint64_t *zmask,
                      const double *coeff, int32_t obs_shared, const double *upstream, double h,
                      double *grad, int32_t nthreads)
{
    orc_batch bt = {B, n_qubits, goff, gates, n_params, params_shared, toff, xmask, zmask, coeff, obs_shared};
    int used = set_threads(nthreads);
    int64_t ng_out = params_shared ? n_params[0] : param_base(&bt, B);
    memset(grad, 0, sizeof(double) * (size_t)ng_out);
    int64_t nitems = 0;
    for (int b = 0; b < B; b++) nitems += n_params[b];
    int64_t *item_b = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nitems + 1));
    int64_t *item_p = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nitems + 1));
    double *contrib = (double *)malloc(sizeof(double) * (size_t)(nitems + 1));
    int64_t it = 0;
    for (int b = 0; b < B; b++)
        for (int p = 0; p < n_params[b]; p++) { item_b[it] = b; item_p[it] = p; it++; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nitems; i++) {
        const int b = (int)item_b[i];
        const int n = n_qubits[b];
        const orc_gate *g = gates + goff[b];
        const int64_t ng = goff[b + 1] - goff[b];
        const double *th = theta + param_base(&bt, b);
        int64_t t0, t1;
        term_range(&bt, b, &t0, &t1);
        cplx *psi = (cplx *)malloc(sizeof(cplx) * ((size_t)1 << n));
        run_circuit(psi, n, g, ng, th, -1, 0.0, (int)item_p[i], h);
        double ep = energy(psi, n, t1 - t0, xmask + t0, zmask + t0, coeff + t0, NULL, NULL);
        run_circuit(psi, n, g, ng, th, -1, 0.0, (int)item_p[i], -h);
        double em = energy(psi, n, t1 - t0, xmask + t0, zmask + t0, coeff + t0, NULL, NULL);
        free(psi);
        double w = upstream ? upstream[b] : 1.0;
        contrib[i] = w * (ep - em) / (2.0 * h);
    }
    for (int64_t i = 0; i < nitems; i++)
        grad[grad_index(&bt, (int)item_b[i], (int)item_p[i])] += contrib[i];
    free(item_b); free(item_p); free(contrib);
    return used;
}

/* Adjoint differentiation (Jones and Gacon, 2020; not part of the paper): with psi the final state
 * and lambda = w H psi, walk the gates backwards; at a trainable gate exp(-i a G/2) add
 * Im <lambda| G |psi> to its parameter's gradient, then un-apply the gate from both vectors. */
int orc_batch_grad_adjoint(int32_t B, const int32_t *n_qubits, const int64_t *goff, const orc_gate *gates,
                           const int32_t *n_params, int32_t params_shared, const double *theta,
                           const int64_t *toff, const uint64_t *xmask, const uint64_t *zmask,
                           const double *coeff, int32_t obs_shared, const double *upstream,
                           double *grad, int32_t nthreads)
{
    orc_batch bt = {B, n_qubits, goff, gates, n_params, params_shared, toff, xmask, zmask, coeff, obs_shared};
    int used = set_threads(nthreads);
    int64_t ng_out = params_shared ? n_params[0] : param_base(&bt, B);
    memset(grad, 0, sizeof(double) * (size_t)ng_out);
    /* per-circuit gradient rows, summed in circuit order afterwards */
    int64_t maxp = 0;
    for (int b = 0; b < B; b++) if (n_params[b] > maxp) maxp = n_params[b];
    double *rows = (double *)calloc((size_t)B * (size_t)(maxp + 1), sizeof(double));
#pragma omp parallel for if (B > 1) schedule(dynamic, 1)
    for (int b = 0; b < B; b++) {
        const int n = n_qubits[b];
        const int64_t dim = (int64_t)1 << n;
        const orc_gate *g = gates + goff[b];
        const int64_t ng = goff[b + 1] - goff[b];
        const double *th = theta + param_base(&bt, b);
        int64_t t0, t1;
        term_range(&bt, b, &t0, &t1);
        const double w = upstream ? upstream[b] : 1.0;
        cplx *psi = (cplx *)malloc(sizeof(cplx) * (size_t)dim);
        cplx *lam = (cplx *)calloc((size_t)dim, sizeof(cplx));
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)dim);
        run_circuit(psi, n, g, ng, th, -1, 0.0, -1, 0.0);
        /* lambda = w * sum_t c_t P_t psi */
        for (int64_t t = t0; t < t1; t++) {
            apply_pauli(psi, tmp, n, xmask[t], zmask[t]);
            for (int64_t i = 0; i < dim; i++) lam[i] += w * coeff[t] * tmp[i];
        }
        double *row = rows + (size_t)b * (size_t)(maxp + 1);
        for (int64_t k = ng - 1; k >= 0; k--) {
            const double a = gate_angle(&g[k], th);
            if (g[k].param >= 0) {
                /* generator of the rotation */
                const int gk = g[k].kind == ORC_RX ? ORC_X : g[k].kind == ORC_RY ? ORC_Y : ORC_Z;
                orc_gate gen = {gk, g[k].q0, -1, -1, 0.0};
                memcpy(tmp, psi, sizeof(cplx) * (size_t)dim);
                apply_gate(tmp, n, &gen, 0.0, 0);
                lcplx ip = 0;  /* extended precision, as in expect_pauli */
                for (int64_t i = 0; i < dim; i++) ip += conjl((lcplx)lam[i]) * (lcplx)tmp[i];
                row[g[k].param] += (double)cimagl(ip);
            }
            apply_gate(psi, n, &g[k], a, 1);
            apply_gate(lam, n, &g[k], a, 1);
        }
        free(psi); free(lam); free(tmp);
    }
    for (int b = 0; b < B; b++)
        for (int p = 0; p < n_params[b]; p++)
            grad[grad_index(&bt, b, p)] += rows[(size_t)b * (size_t)(maxp + 1) + p];
    free(rows);
    return used;
}

/* Returns the number of threads OpenMP would use (for reporting the baseline's core count). */
int orc_max_threads(int32_t nthreads)
{
    return set_threads(nthreads);
}
