"""CPU checks of the benchmark's unfused ("gate-equivalent") byte count: it follows its definition on a
small hand-counted batch and reproduces the per-workload totals of the circuit-learning and uneven random
batches (2S per gate pass, S per x-mask group, 2S for the adjoint seed and 4S per reverse gate pass)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2406_03466_amd import workloads as W  # noqa: E402


def test_unfused_bytes_by_hand():
    # two circuits: 3 qubits with 4 gates and terms on two x-masks; 2 qubits with 1 gate and one Z term
    g = W.gate
    c0 = [g(W.H, 0), g(W.RY, 1, -1, 0), g(W.CNOT, 0, 2), g(W.RZ, 2, -1, 1)]
    c1 = [g(W.RX, 1, -1, 0)]
    t0 = (np.array([0, 1, 1], np.uint64), np.array([1, 0, 4], np.uint64), np.ones(3))
    t1 = (np.array([0], np.uint64), np.array([1], np.uint64), np.ones(1))
    wl = W._pack("hand", [c0, c1], [3, 2], [2, 1], False, np.zeros(3), [t0, t1], False)
    s0, s1 = 8 * 8, 4 * 8   # complex64 state bytes
    fwd = (2 * 4 + 2) * s0 + (2 * 1 + 1) * s1
    assert bench.unfused_bytes(wl, 8, False) == fwd
    assert bench.unfused_bytes(wl, 8, True) == fwd + (2 + 4 * 4) * s0 + (2 + 4 * 1) * s1


@pytest.mark.parametrize("layers,gb", [(2, 445.6), (4, 825.7), (8, 1585.9)])
def test_unfused_bytes_circuit_learning(layers, gb):
    """64 samples of 20 qubits, 20 + 59 L gates each, one Z term: adjoint gradient bytes in GB."""
    assert abs(bench.unfused_bytes(W.config3(layers), 8, True) / 1e9 - gb) < 0.6


def test_unfused_bytes_uneven_batch():
    """1024 random circuits: gate passes 962 GB plus one read per x-mask group."""
    by = bench.unfused_bytes(W.config4(), 8, False) / 1e9
    assert 962.0 < by < 962.0 + 36.6 + 1.0
