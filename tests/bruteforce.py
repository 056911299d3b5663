"""Brute-force reference for tiny registers (n <= 6): full 2^n x 2^n unitaries built from Kronecker
products and full Pauli matrices. It pins the oracle's stride-pair gate loops and its mask-formula Pauli
phases with an independent construction (matrix embedding instead of index arithmetic).

Qubit 0 is the rightmost Kronecker factor, so qubit q is bit q of the basis-state index.
"""
import numpy as np

from paper_2406_03466_amd import workloads as W

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)


def one_qubit_matrix(kind, a):
    """Textbook matrices; rotations are exp(-i a sigma / 2) written as cos(a/2) I - i sin(a/2) sigma."""
    c, s = np.cos(a / 2), np.sin(a / 2)
    if kind == W.H:
        return np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
    if kind == W.X:
        return PX
    if kind == W.Y:
        return PY
    if kind == W.Z:
        return PZ
    if kind == W.S:
        return np.diag([1, 1j])
    if kind == W.T:
        return np.diag([1, np.exp(1j * np.pi / 4)])
    if kind == W.RX:
        return c * I2 - 1j * s * PX
    if kind == W.RY:
        return c * I2 - 1j * s * PY
    if kind == W.RZ:
        return c * I2 - 1j * s * PZ
    raise ValueError(kind)


def embed(ops, n):
    """ops: dict qubit -> 2x2 matrix; identity elsewhere. Kronecker order: qubit n-1 ... qubit 0."""
    m = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):
        m = np.kron(m, ops.get(q, I2))
    return m


def gate_unitary(g, n, theta):
    kind, q0, q1, param, angle = int(g["kind"]), int(g["q0"]), int(g["q1"]), int(g["param"]), float(g["angle"])
    a = theta[param] if param >= 0 else angle
    if kind == W.CNOT:
        return embed({q0: P0}, n) + embed({q0: P1, q1: PX}, n)
    if kind == W.CZ:
        return embed({q0: P0}, n) + embed({q0: P1, q1: PZ}, n)
    return embed({q0: one_qubit_matrix(kind, a)}, n)


def circuit_unitary(gates, n, theta):
    U = np.eye(1 << n, dtype=complex)
    for g in gates:
        U = gate_unitary(g, n, theta) @ U
    return U


def final_state(gates, n, theta):
    return circuit_unitary(gates, n, theta)[:, 0]


def pauli_matrix(xm, zm, n):
    ops = {}
    for q in range(n):
        xb, zb = (int(xm) >> q) & 1, (int(zm) >> q) & 1
        ops[q] = [[I2, PZ], [PX, PY]][xb][zb]
    return embed(ops, n)


def expectation(psi, xm, zm, n):
    return np.vdot(psi, pauli_matrix(xm, zm, n) @ psi)
