"""Seeded synthetic workloads (inputs only: circuits, parameters, Pauli observables, data).

This module draws random numbers and lays out gate records; it holds none of the simulation
arithmetic. Both the GPU library's tests/benchmark and the CPU oracle consume what it produces.

Workloads follow the shapes of the paper's two applications: many slightly different circuits that
share one parameterised structure (parameter-shifted copies for gradients, Section 4.1, Table 1; data-fed
circuits for circuit learning, Section 4.2, Table 2), plus an uneven random batch and a single large
state. The paper's own Hamiltonian coefficients and target distributions are not published, so every
coefficient, angle and data point here is synthetic and seeded.

Gate record (24 bytes): kind, q0, q1, param, angle.
  * one-qubit gates act on q0; CNOT has control q0 and target q1; CZ acts on q0 and q1;
  * param >= 0 selects theta[param] as the rotation angle; param = -1 uses the fixed `angle`.
Qubit q is bit q of the amplitude index. A Pauli string is (xmask, zmask): X where only x is set,
Z where only z is set, Y where both are set.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

H, X, Y, Z, S, T, RX, RY, RZ, CNOT, CZ = range(11)
GATE_NAMES = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "CNOT", "CZ"]
ROTATIONS = (RX, RY, RZ)
TWO_QUBIT = (CNOT, CZ)

GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("param", "<i4"), ("angle", "<f8")])

SEED_BASE = 240603466


@dataclass
class Workload:
    """A batch of circuits plus observables, in the flat layout the library's C interface takes."""

    name: str
    n_qubits: np.ndarray            # int32 [B]
    gate_offsets: np.ndarray        # int64 [B+1]
    gates: np.ndarray               # GATE_DTYPE [G_total]
    n_params: np.ndarray            # int32 [B]
    params_shared: bool
    theta: np.ndarray               # float64 [P] if shared else [sum n_params]
    term_offsets: np.ndarray        # int64 [2] if obs_shared else [B+1]
    xmask: np.ndarray               # uint64 [T_total]
    zmask: np.ndarray               # uint64 [T_total]
    coeff: np.ndarray               # float64 [T_total]
    obs_shared: bool
    extra: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return int(len(self.n_qubits))

    def circuit(self, b: int) -> np.ndarray:
        return self.gates[self.gate_offsets[b]: self.gate_offsets[b + 1]]

    def terms(self, b: int):
        t0, t1 = (self.term_offsets[0], self.term_offsets[1]) if self.obs_shared else \
            (self.term_offsets[b], self.term_offsets[b + 1])
        return self.xmask[t0:t1], self.zmask[t0:t1], self.coeff[t0:t1]

    def theta_of(self, b: int) -> np.ndarray:
        if self.params_shared:
            return self.theta
        base = int(np.sum(self.n_params[:b]))
        return self.theta[base: base + int(self.n_params[b])]

    def n_grad(self) -> int:
        return int(self.n_params[0]) if self.params_shared else int(np.sum(self.n_params))

    def subset(self, idx) -> "Workload":
        """The circuits idx (in that order), with their parameters and terms."""
        idx = [int(i) for i in idx]
        gates = [self.circuit(b) for b in idx]
        goff = np.zeros(len(idx) + 1, np.int64)
        goff[1:] = np.cumsum([len(g) for g in gates])
        if self.params_shared:
            theta = self.theta.copy()
        else:
            theta = np.concatenate([self.theta_of(b) for b in idx]) if idx else np.zeros(0)
        if self.obs_shared:
            toff, xm, zm, cf = self.term_offsets.copy(), self.xmask.copy(), self.zmask.copy(), self.coeff.copy()
        else:
            parts = [self.terms(b) for b in idx]
            toff = np.zeros(len(idx) + 1, np.int64)
            toff[1:] = np.cumsum([len(p[0]) for p in parts])
            xm = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint64)
            zm = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.uint64)
            cf = np.concatenate([p[2] for p in parts]) if parts else np.zeros(0)
        extra = {}
        for k, v in self.extra.items():
            if isinstance(v, np.ndarray) and v.shape[:1] == (self.B,):
                extra[k] = v[idx]
            else:
                extra[k] = v
        return Workload(self.name + "[subset]", self.n_qubits[idx].copy(), goff,
                        np.concatenate(gates) if gates else np.zeros(0, GATE_DTYPE),
                        self.n_params[idx].copy(), self.params_shared, theta, toff,
                        xm.astype(np.uint64), zm.astype(np.uint64), cf, self.obs_shared, extra)


# ------------------------------------------------------------------------------------------------
# Building blocks
# ------------------------------------------------------------------------------------------------

def gate(kind: int, q0: int, q1: int = -1, param: int = -1, angle: float = 0.0):
    return (kind, q0, q1, param, angle)


def hea_layers(n: int, layers: int, first_param: int = 0, rz_fixed: Optional[np.ndarray] = None):
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every qubit, then the CNOT ladder
    q_i -> q_{i+1}. Parameters are numbered layer-major: layer l uses RY params first, then RZ params.
    When rz_fixed is given (shape [layers, n]) the RZ angles are fixed and only RY is trainable."""
    g = []
    p = first_param
    for l in range(layers):
        for q in range(n):
            g.append(gate(RY, q, -1, p, 0.0))
            p += 1
        for q in range(n):
            if rz_fixed is None:
                g.append(gate(RZ, q, -1, p, 0.0))
                p += 1
            else:
                g.append(gate(RZ, q, -1, -1, float(rz_fixed[l, q])))
        for q in range(n - 1):
            g.append(gate(CNOT, q, q + 1))
    return g, p


def pauli_from_letters(letters: np.ndarray):
    """letters[t, q] in {0: I, 1: X, 2: Y, 3: Z} -> (xmask, zmask) per term."""
    T, n = letters.shape
    xm = np.zeros(T, np.uint64)
    zm = np.zeros(T, np.uint64)
    for q in range(n):
        bit = np.uint64(1) << np.uint64(q)
        xm |= np.where((letters[:, q] == 1) | (letters[:, q] == 2), bit, np.uint64(0)).astype(np.uint64)
        zm |= np.where((letters[:, q] == 3) | (letters[:, q] == 2), bit, np.uint64(0)).astype(np.uint64)
    return xm, zm


def pauli_string(xm: int, zm: int, n: int) -> str:
    """Character k describes qubit k."""
    out = []
    for q in range(n):
        xb, zb = (int(xm) >> q) & 1, (int(zm) >> q) & 1
        out.append("IXZY"[xb + 2 * zb])
    return "".join(out)


def parse_pauli(s: str):
    xm = zm = 0
    for q, ch in enumerate(s):
        if ch in "XY":
            xm |= 1 << q
        if ch in "ZY":
            zm |= 1 << q
    return xm, zm


def _pack(name, circuits, nqs, nparams, params_shared, theta, terms, obs_shared, extra=None):
    goff = np.zeros(len(circuits) + 1, np.int64)
    goff[1:] = np.cumsum([len(c) for c in circuits])
    gates = np.array([g for c in circuits for g in c], dtype=GATE_DTYPE) if goff[-1] else np.zeros(0, GATE_DTYPE)
    if obs_shared:
        xm, zm, cf = terms
        toff = np.array([0, len(xm)], np.int64)
    else:
        toff = np.zeros(len(terms) + 1, np.int64)
        toff[1:] = np.cumsum([len(t[0]) for t in terms])
        xm = np.concatenate([t[0] for t in terms]).astype(np.uint64)
        zm = np.concatenate([t[1] for t in terms]).astype(np.uint64)
        cf = np.concatenate([t[2] for t in terms]).astype(np.float64)
    return Workload(name, np.asarray(nqs, np.int32), goff, gates, np.asarray(nparams, np.int32),
                    bool(params_shared), np.asarray(theta, np.float64), toff,
                    np.asarray(xm, np.uint64), np.asarray(zm, np.uint64), np.asarray(cf, np.float64),
                    bool(obs_shared), extra or {})


def random_paulis(rng, T: int, n: int):
    letters = rng.integers(0, 4, size=(T, n))
    xm, zm = pauli_from_letters(letters)
    coeff = rng.normal(0.0, 1.0, size=T)
    return xm, zm, coeff


# ------------------------------------------------------------------------------------------------
# The five workloads
# ------------------------------------------------------------------------------------------------

def hea_vqe(n: int = 10, layers: int = 4, n_terms: int = 20, seed_index: int = 1, name: str = "hea_vqe") -> Workload:
    """One hardware-efficient-ansatz circuit (the base circuit of a parameter-shift gradient) with a
    random Pauli-sum observable. Draw order: theta, Pauli letters (term-major), coefficients."""
    rng = np.random.default_rng(SEED_BASE + seed_index)
    g, P = hea_layers(n, layers)
    theta = rng.uniform(0.0, 2 * np.pi, size=P)
    xm, zm, cf = random_paulis(rng, n_terms, n)
    return _pack(name, [g], [n], [P], True, theta, (xm, zm, cf), True)


def config1() -> Workload:
    """10 qubits, 4 HEA layers (80 params), 20 random Pauli strings with N(0,1) weights."""
    return hea_vqe(10, 4, 20, 1, "hea10_L4_T20")


def config2() -> Workload:
    """16 qubits, 8 HEA layers (256 params), 100 random Pauli strings with N(0,1) weights."""
    return hea_vqe(16, 8, 100, 2, "hea16_L8_T100")


def qcl(n: int = 20, layers: int = 8, samples: int = 64, seed_index: int = 3) -> Workload:
    """Quantum circuit learning: per sample x_k ~ U(-1,1), RY(arcsin x_k) on every qubit, then `layers`
    HEA layers with shared trainable theta; observable Z_0; target y = sin(pi x) + N(0, 0.05).
    Draw order: theta, x, noise."""
    rng = np.random.default_rng(SEED_BASE + seed_index)
    P = 2 * n * layers
    theta = rng.uniform(0.0, 2 * np.pi, size=P)
    x = rng.uniform(-1.0, 1.0, size=samples)
    y = np.sin(np.pi * x) + rng.normal(0.0, 0.05, size=samples)
    body, P2 = hea_layers(n, layers)
    assert P2 == P
    circuits = []
    for k in range(samples):
        enc = [gate(RY, q, -1, -1, float(np.arcsin(x[k]))) for q in range(n)]
        circuits.append(enc + body)
    terms = (np.array([0], np.uint64), np.array([1], np.uint64), np.array([1.0]))
    return _pack(f"qcl{n}_L{layers}_S{samples}", circuits, [n] * samples, [P] * samples, True, theta, terms,
                 True, {"x": x, "y": y})


def config3(layers: int = 8) -> Workload:
    return qcl(20, layers, 64, 3)


def random_batch(n_circuits: int = 1024, n_min: int = 8, n_max: int = 22, g_min: int = 10, g_max: int = 200,
                 n_terms: int = 8, seed_index: int = 4, kinds=None) -> Workload:
    """Uneven batch of random circuits. Per circuit: n ~ U{n_min..n_max}, gate count ~ U{g_min..g_max},
    each gate uniform over `kinds` (default {H, RX, RY, RZ, CNOT, CZ}) on uniform qubits (ordered distinct
    pairs for two-qubit gates); every rotation has its own parameter, theta ~ U[0, 2pi). Then n_terms
    random Pauli strings with N(0,1) weights. Draw order: per circuit (n, G, gates, angles), then all
    observables."""
    rng = np.random.default_rng(SEED_BASE + seed_index)
    kinds = list(kinds) if kinds is not None else [H, RX, RY, RZ, CNOT, CZ]
    circuits, nqs, nps, thetas = [], [], [], []
    for _ in range(n_circuits):
        n = int(rng.integers(n_min, n_max + 1))
        G = int(rng.integers(g_min, g_max + 1))
        ks = rng.integers(0, len(kinds), size=G)
        circ = []
        p = 0
        th = []
        for k in ks:
            kind = kinds[int(k)]
            if kind in TWO_QUBIT:
                a, b = rng.choice(n, size=2, replace=False)
                circ.append(gate(kind, int(a), int(b)))
            else:
                q = int(rng.integers(0, n))
                if kind in ROTATIONS:
                    circ.append(gate(kind, q, -1, p))
                    th.append(float(rng.uniform(0.0, 2 * np.pi)))
                    p += 1
                else:
                    circ.append(gate(kind, q))
        circuits.append(circ)
        nqs.append(n)
        nps.append(p)
        thetas.append(np.array(th, np.float64))
    terms = [random_paulis(rng, n_terms, n) for n in nqs]
    theta = np.concatenate(thetas) if thetas else np.zeros(0)
    return _pack(f"random{n_circuits}_n{n_min}-{n_max}_G{g_min}-{g_max}", circuits, nqs, nps, False, theta,
                 terms, False)


def config4() -> Workload:
    return random_batch()


def large_hea(n: int = 32, layers: int = 10, seed_index: int = 5) -> Workload:
    """One large HEA circuit: RY angles trainable (n*layers params), RZ angles fixed and drawn from the same
    seed; observable sum_{i=0}^{n-2} Z_i Z_{i+1} with unit weights. Draw order: theta, RZ angles."""
    rng = np.random.default_rng(SEED_BASE + seed_index)
    theta = rng.uniform(0.0, 2 * np.pi, size=n * layers)
    rz = rng.uniform(0.0, 2 * np.pi, size=(layers, n))
    g, P = hea_layers(n, layers, rz_fixed=rz)
    assert P == n * layers
    zm = np.array([(1 << i) | (1 << (i + 1)) for i in range(n - 1)], np.uint64)
    terms = (np.zeros(n - 1, np.uint64), zm, np.ones(n - 1))
    return _pack(f"hea{n}_L{layers}_zzchain", [g], [n], [P], True, theta, terms, True)


def config5() -> Workload:
    return large_hea(32, 10, 5)


def cis_prep(c) -> list:
    """Gates preparing sum_A c_A |e_A> (e_A: only qubit A excited) from |0...0>, for a real unit vector c:
    X on qubit 0, then for k = 0..N-2 a Givens rotation between qubits k and k+1 that keeps cos(b_k) of the
    excitation on qubit k and moves sin(b_k) of it to qubit k+1. Each Givens rotation is CNOT(k->k+1),
    RY_{k+1}(-b), CNOT(k->k+1), RY_{k+1}(b), CNOT(k+1->k): a controlled RY(2b) followed by a CNOT back. The
    angles are fixed (not trainable): b_k = atan2(|c_{k+1..}|, c_k), the last one atan2(c_{N-1}, c_{N-2}),
    so that the amplitudes come out as c_0 = cos b_0, c_1 = sin b_0 cos b_1, ... with the signs of c."""
    c = np.asarray(c, np.float64)
    N = len(c)
    g = [gate(X, 0)]
    for k in range(N - 1):
        if k < N - 2:
            b = float(np.arctan2(np.sqrt(np.sum(c[k + 1:] ** 2)), c[k]))
        else:
            b = float(np.arctan2(c[N - 1], c[N - 2]))
        g += [gate(CNOT, k, k + 1), gate(RY, k + 1, -1, -1, -b), gate(CNOT, k, k + 1), gate(RY, k + 1, -1, -1, b),
              gate(CNOT, k + 1, k)]
    return g


def mcvqe_entanglers(n: int, merge: bool = True):
    """The MC-VQE entangler layer (Section 4.1): on each adjacent pair (A, A+1), even pairs first, then odd
    pairs, RY on both qubits, CNOT(A -> A+1), RY on both, CNOT(A -> A+1), RY on both: 6 trainable RY and 2
    CNOTs per pair, 6(n-1) angles. With merge, an RY that directly follows another trainable RY on the same
    qubit (the last RY of one pair's entangler and the first of the next pair's, on the shared qubit) is
    folded into it, RY(a) RY(b) = RY(a + b), which leaves 5n - 4 parameters. Returns (gates, n_params,
    merged_from) where merged_from[p] lists the unmerged parameter indices that parameter p stands for."""
    raw = []
    p = 0
    pairs = [(a, a + 1) for a in range(0, n - 1, 2)] + [(a, a + 1) for a in range(1, n - 1, 2)]
    for a, b in pairs:
        for _ in range(2):
            raw += [gate(RY, a, -1, p), gate(RY, b, -1, p + 1), gate(CNOT, a, b)]
            p += 2
        raw += [gate(RY, a, -1, p), gate(RY, b, -1, p + 1)]
        p += 2
    if not merge:
        return raw, p, [[i] for i in range(p)]
    out = []
    last_on = {}  # qubit -> index in out of the last gate touching it
    new_of = {}
    merged_from = []
    for g in raw:
        kind, q0, q1, par, ang = g
        if kind == RY and par >= 0 and q0 in last_on:
            prev = out[last_on[q0]]
            if prev[0] == RY and prev[3] >= 0:
                new_of[par] = prev[3]
                merged_from[prev[3]].append(par)
                continue
        if kind == RY and par >= 0:
            new_of[par] = len(merged_from)
            merged_from.append([par])
            g = (kind, q0, q1, new_of[par], ang)
        out.append(g)
        last_on[q0] = len(out) - 1
        if q1 >= 0:
            last_on[q1] = len(out) - 1
    return out, len(merged_from), merged_from


def aiem_hamiltonian(rng, n: int):
    """Pauli terms of the ab initio exciton model Hamiltonian (Eq. 2): a constant, X_A and Z_A on every
    monomer A, and XX, XZ, ZX, ZZ on every adjacent pair (A, A+1): 6n - 4 Pauli terms plus the constant,
    which is kept as an identity term (xmask = zmask = 0) at index 0. Coefficients are synthetic N(0, 1)
    (the paper's monomer data are not published); draw order: constant, then term by term as listed."""
    xm, zm = [0], [0]
    for a in range(n):
        xm += [1 << a, 0]
        zm += [0, 1 << a]
    for a in range(n - 1):
        A, B = 1 << a, 1 << (a + 1)
        xm += [A | B, A, B, 0]
        zm += [0, B, A, A | B]
    cf = rng.normal(0.0, 1.0, size=len(xm))
    return np.array(xm, np.uint64), np.array(zm, np.uint64), cf


def mcvqe(n: int = 16, n_states: Optional[int] = None, seed_index: int = 6, merge: bool = True) -> Workload:
    """MC-VQE-shaped batch (Section 4.1): n monomers on n qubits; one circuit per CIS state (n_states of them,
    default n), each its own CIS preparation followed by the shared entangler layer; shared parameters and
    the shared AIEM Hamiltonian, so the mean energy over states and its gradient come from one batch call
    with upstream weights 1/n_states. The CIS vectors are a random orthonormal set (QR of a Gaussian
    matrix; the paper's CIS coefficients are not published). Draw order: theta ~ U[0, 2pi), the Gaussian
    matrix, then the Hamiltonian coefficients."""
    n_states = n if n_states is None else int(n_states)
    rng = np.random.default_rng(SEED_BASE + seed_index)
    ent, P, merged_from = mcvqe_entanglers(n, merge)
    theta = rng.uniform(0.0, 2 * np.pi, size=P)
    q, _ = np.linalg.qr(rng.normal(0.0, 1.0, size=(n, n)))
    cis = q[:, :n_states].T.copy()                      # [n_states, n], orthonormal rows
    xm, zm, cf = aiem_hamiltonian(rng, n)
    circuits = [cis_prep(cis[s]) + ent for s in range(n_states)]
    return _pack(f"mcvqe{n}_S{n_states}", circuits, [n] * n_states, [P] * n_states, True, theta, (xm, zm, cf),
                 True, {"cis": cis, "merged_from": merged_from, "n_hamiltonian_terms": int(len(xm) - 1)})


def ddcl_layers(n: int, layers: int, first_param: int = 0):
    """Data-driven circuit-learning body (Section 4.2): Bell pairs on neighbouring qubits (H on 2i, CNOT
    2i -> 2i+1), then `layers` layers of RZ RY RZ on every qubit, the CNOT ring q -> q+1 (mod n), and RZ RY
    RZ on every qubit again: 6n trainable angles per layer (Table 2: N_theta = 60 N_q at 10 layers)."""
    g = []
    for i in range(0, n - 1, 2):
        g += [gate(H, i), gate(CNOT, i, i + 1)]
    p = first_param
    for _ in range(layers):
        for half in range(2):
            for q in range(n):
                for kind in (RZ, RY, RZ):
                    g.append(gate(kind, q, -1, p))
                    p += 1
            if half == 0 and n > 1:
                g += [gate(CNOT, q, (q + 1) % n) for q in range(n if n > 2 else 1)]
    return g, p - first_param


def ddcl(n: int = 20, layers: int = 10, seed_index: int = 7, sizes=None) -> Workload:
    """DDCL-shaped batch: one circuit per entry of `sizes` (default [n]), each the Bell-pair + layer circuit
    with its own angles theta ~ U[0, 2pi) and its own target distribution: exponential weights on a random
    half of the 2^n bit strings (the rest exactly 0), normalised (the paper's targets are not published).
    No Pauli terms. Draw order per circuit: theta, the support mask, the weights."""
    sizes = [n] if sizes is None else [int(x) for x in sizes]
    rng = np.random.default_rng(SEED_BASE + seed_index)
    circuits, nps, thetas, targets = [], [], [], []
    for m in sizes:
        g, P = ddcl_layers(m, layers)
        thetas.append(rng.uniform(0.0, 2 * np.pi, size=P))
        mask = rng.random(1 << m) < 0.5
        t = rng.exponential(1.0, size=1 << m) * mask
        targets.append(t / t.sum())
        circuits.append(g)
        nps.append(P)
    empty = [(np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0)) for _ in sizes]
    name = f"ddcl{'-'.join(map(str, sizes))}_L{layers}"
    return _pack(name, circuits, sizes, nps, False, np.concatenate(thetas), empty, False,
                 {"target": np.concatenate(targets)})


def ghz(n: int) -> Workload:
    """H on qubit 0 then the CNOT ladder: (|0..0> + |1..1>)/sqrt(2). No parameters, no terms."""
    g = [gate(H, 0)] + [gate(CNOT, q, q + 1) for q in range(n - 1)]
    return _pack(f"ghz{n}", [g], [n], [0], True, np.zeros(0), (np.zeros(0, np.uint64), np.zeros(0, np.uint64),
                                                                  np.zeros(0)), True)


def with_terms(wl: Workload, xm, zm, cf) -> Workload:
    """Same circuits, one shared observable."""
    return Workload(wl.name, wl.n_qubits, wl.gate_offsets, wl.gates, wl.n_params, wl.params_shared, wl.theta,
                    np.array([0, len(xm)], np.int64), np.asarray(xm, np.uint64), np.asarray(zm, np.uint64),
                    np.asarray(cf, np.float64), True, dict(wl.extra))


def with_theta(wl: Workload, theta) -> Workload:
    return Workload(wl.name, wl.n_qubits, wl.gate_offsets, wl.gates, wl.n_params, wl.params_shared,
                    np.asarray(theta, np.float64), wl.term_offsets, wl.xmask, wl.zmask, wl.coeff, wl.obs_shared,
                    dict(wl.extra))


def single(name: str, n: int, gates_list, theta=(), terms=None) -> Workload:
    """One circuit from a list of gate tuples; terms = (xm, zm, coeff) or None."""
    P = 0
    for g in gates_list:
        if g[3] >= 0:
            P = max(P, g[3] + 1)
    if terms is None:
        terms = (np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0))
    return _pack(name, [list(gates_list)], [n], [P], True, np.asarray(theta, np.float64),
                 (np.asarray(terms[0], np.uint64), np.asarray(terms[1], np.uint64),
                  np.asarray(terms[2], np.float64)), True)


def counts(wl: Workload) -> dict:
    """Workload-size bookkeeping (circuits, gates, params, terms)."""
    return {
        "circuits": wl.B,
        "gates": int(wl.gate_offsets[-1]),
        "params": wl.n_grad(),
        "terms": int(len(wl.xmask)),
        "param_shift_circuits": int(np.sum(wl.gates["param"] >= 0)) * 2 + wl.B,
    }
