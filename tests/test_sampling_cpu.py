"""Pins of the shot-sampling oracle (oracle/sampling.py) against closed forms and the inverse-transform
law, on the CPU: a point mass, a Bell pair, the uniform distribution of H on every qubit (shot = the
integer part of 2^n u), an equispaced grid of uniforms whose counts must equal 2^20 Q(x) within one, and
a chi-square test of random uniforms against the exact distribution."""
import numpy as np
import pytest
from scipy import stats

from oracle import sampling as OS
from paper_2406_03466_amd import workloads as W


def test_point_mass():
    gates = [W.gate(W.X, 0), W.gate(W.X, 2)]
    q = OS.distribution(4, np.array(gates, W.GATE_DTYPE), np.zeros(0))
    u = np.random.default_rng(1).random(500)
    s = OS.sample_from(q, u)
    assert (s == 5).all()
    bits, cnt = OS.counts_of(s)
    assert bits.tolist() == [5] and cnt.tolist() == [500]


def test_bell_pair_never_draws_zero_probability_strings():
    gates = np.array([W.gate(W.H, 0), W.gate(W.CNOT, 0, 1)], W.GATE_DTYPE)
    q = OS.distribution(2, gates, np.zeros(0))
    np.testing.assert_allclose(q, [0.5, 0, 0, 0.5], atol=1e-15)
    u = np.array([0.0, 0.1, 0.4999, 0.5001, 0.9, 0.999999])
    assert OS.sample_from(q, u).tolist() == [0, 0, 0, 3, 3, 3]


def test_uniform_distribution_is_floor_of_scaled_uniform():
    n = 6
    gates = np.array([W.gate(W.H, k) for k in range(n)], W.GATE_DTYPE)
    q = OS.distribution(n, gates, np.zeros(0))
    rng = np.random.default_rng(2)
    k = rng.integers(0, 1 << n, 2000)
    u = (k + rng.uniform(0.01, 0.99, k.size)) / (1 << n)   # away from the bin edges k / 2^n
    np.testing.assert_array_equal(OS.sample_from(q, u), k)


def test_equispaced_uniforms_reproduce_the_distribution():
    """With u_k = (k + 1/2) / K the shots that land on x are the grid points inside [C(x-1), C(x)) / C(last),
    so count(x) = K Q(x) / C(last) within one."""
    rng = np.random.default_rng(3)
    n = 7
    gates, theta = [], []
    for i in range(40):
        kind = [W.RY, W.RX, W.CNOT, W.RZ, W.H][i % 5]
        if kind == W.CNOT:
            a, b = rng.choice(n, 2, replace=False)
            gates.append(W.gate(kind, int(a), int(b)))
        elif kind == W.H:
            gates.append(W.gate(kind, int(rng.integers(n))))
        else:
            gates.append(W.gate(kind, int(rng.integers(n)), -1, len(theta)))
            theta.append(rng.uniform(0, 2 * np.pi))
    q = OS.distribution(n, np.array(gates, W.GATE_DTYPE), np.array(theta))
    K = 1 << 20
    u = (np.arange(K) + 0.5) / K
    bits, cnt = OS.counts_of(OS.sample_from(q, u))
    full = np.zeros(1 << n, np.int64)
    full[bits.astype(np.int64)] = cnt
    assert np.abs(full - K * q / q.sum()).max() <= 1.0 + 1e-9
    assert full.sum() == K


@pytest.mark.parametrize("seed", [4, 5])
def test_chi_square_against_exact_distribution(seed):
    wl = W.random_batch(1, 6, 6, 30, 30, 1, seed_index=seed)
    shots = 200000
    u = np.random.default_rng(seed).random(shots)
    s, per = OS.sample_batch(wl, u, shots)
    q, bits, cnt = per[0]
    assert cnt.sum() == shots and np.all(np.diff(bits.astype(np.int64)) > 0)
    full = np.zeros(q.size)
    full[bits.astype(np.int64)] = cnt
    exp = shots * q / q.sum()
    keep = exp >= 5
    chi2 = float(np.sum((full[keep] - exp[keep]) ** 2 / exp[keep]))
    assert stats.chi2.sf(chi2, int(keep.sum()) - 1) > 1e-4
    assert (full[q == 0] == 0).all()
