"""ORACLE (test infrastructure only; only the test suite, the smoke check and the benchmark's CPU leg may
use it): shots drawn from a circuit's output distribution and gathered into bit-string counts, by the
plain definition, in float64 on the CPU.

A circuit's execution yields the distribution of observed bit strings over its 2^n outcomes, kept as a
table from bit string to the number of times it occurred (Section 3.1; Section 4.2, where the circuit
learning application works on exactly these counts). Drawing a shot by inverse transform sampling: with
Q(x) = |<x|U(theta)|0>|^2 in bit-string order (qubit q is bit q of x) and C(x) = Q(0) + ... + Q(x) its
running sum, the uniform u in [0, 1) selects the first x with C(x) > u * C(2^n - 1). The uniforms are
inputs, so the library and this oracle draw the same shots. Counts list the distinct sampled bit strings
in increasing order with how often each occurred.
"""
from __future__ import annotations

import numpy as np

from . import final_state


def distribution(n: int, gates, theta) -> np.ndarray:
    """Q(x) = |psi_x|^2 of one circuit, float64, in bit-string order."""
    psi = final_state(n, gates, theta)
    return psi.real ** 2 + psi.imag ** 2


def cumulative(q) -> np.ndarray:
    """C(x) = Q(0) + ... + Q(x), summed left to right."""
    return np.cumsum(np.asarray(q, np.float64))


def sample_from(q, uniforms) -> np.ndarray:
    """Bit string of every shot: the first x with C(x) > u * C(last)."""
    c = cumulative(q)
    target = np.asarray(uniforms, np.float64) * c[-1]
    return np.searchsorted(c, target, side="right").astype(np.int64)


def counts_of(samples):
    """(distinct bit strings in increasing order, how often each occurs)."""
    bits, cnt = np.unique(np.asarray(samples, np.int64), return_counts=True)
    return bits.astype(np.uint64), cnt.astype(np.int64)


def sample_batch(wl, uniforms, shots: int):
    """Shots of every circuit of a batch: circuit b uses uniforms[b * shots:(b + 1) * shots]. Returns the
    samples in circuit order and, per circuit, its distribution and (bit strings, counts)."""
    u = np.asarray(uniforms, np.float64)
    samples, per = [], []
    for b in range(wl.B):
        q = distribution(int(wl.n_qubits[b]), np.ascontiguousarray(wl.circuit(b)),
                         np.asarray(wl.theta_of(b), np.float64))
        s = sample_from(q, u[b * shots:(b + 1) * shots])
        samples.append(s)
        per.append((q, *counts_of(s)))
    return (np.concatenate(samples) if samples else np.zeros(0, np.int64)), per
