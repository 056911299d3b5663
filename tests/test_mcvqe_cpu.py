"""The MC-VQE-shaped workload (Section 4.1): its sizes against Table 1, its CIS preparation and its
zero-angle energy against closed forms, the RY merge against the unmerged circuit, and the oracle's
gradients on it against two independent rules. CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2406_03466_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mcvqe_table1.json")


@pytest.mark.parametrize("row", json.load(open(GOLDEN))["rows"])
def test_sizes_match_table1(row):
    """N_H = 6N - 4 Pauli terms (constant excluded), N_theta = 5N - 4 after merging, and 2 N_H N_theta
    per-term parameter-shift circuits, as printed in Table 1. Catches a wrong pair list, a missed or extra
    merge, or a wrong term list."""
    nq, nh, nth, circ = row
    wl = W.mcvqe(nq, n_states=1)
    assert wl.extra["n_hamiltonian_terms"] == nh
    assert wl.n_grad() == nth
    assert 2 * wl.extra["n_hamiltonian_terms"] * wl.n_grad() == circ
    # the identity term carries the constant; every other term is X, Z or an adjacent two-qubit product
    xm, zm = wl.xmask.astype(np.int64), wl.zmask.astype(np.int64)
    assert xm[0] == 0 and zm[0] == 0
    support = xm[1:] | zm[1:]
    assert all(bin(int(s)).count("1") in (1, 2) for s in support)
    assert len(set(zip(xm.tolist(), zm.tolist()))) == len(xm)


def test_entangler_structure():
    """6 RY and 2 CNOT per adjacent pair before merging; merging removes exactly one RY per interior qubit."""
    for n in (2, 3, 6, 9):
        raw, P, _ = W.mcvqe_entanglers(n, merge=False)
        kinds = [g[0] for g in raw]
        assert kinds.count(W.RY) == 6 * (n - 1) == P and kinds.count(W.CNOT) == 2 * (n - 1)
        merged, Pm, mf = W.mcvqe_entanglers(n)
        assert Pm == 5 * n - 4 if n > 1 else True
        assert sorted(i for m in mf for i in m) == list(range(P))


@pytest.mark.parametrize("n", [2, 5, 8])
def test_cis_preparation_amplitudes(n):
    """The preparation leaves amplitude c_A on basis state 2^A and nothing elsewhere (closed form of the
    single-excitation state), for every CIS vector of the batch, signs included."""
    wl = W.mcvqe(n)
    for s in range(wl.B):
        c = wl.extra["cis"][s]
        psi = oracle.final_state(n, np.array(W.cis_prep(c), dtype=W.GATE_DTYPE), np.zeros(0))
        want = np.zeros(1 << n, complex)
        want[[1 << a for a in range(n)]] = c
        np.testing.assert_allclose(psi, want, atol=1e-14)


def _cis_energy(c, xm, zm, cf, n):
    """<CIS|H|CIS> for sum_A c_A |e_A>: X_A and X_A Z_B change the excitation number (0); Z_A gives
    1 - 2 c_A^2; Z_A Z_B gives 1 - 2 c_A^2 - 2 c_B^2; X_A X_B swaps e_A and e_B (2 c_A c_B)."""
    e = 0.0
    for x, z, w in zip(xm.tolist(), zm.tolist(), cf):
        xs = [a for a in range(n) if x >> a & 1]
        zs = [a for a in range(n) if z >> a & 1]
        if not xs:
            e += w * (1.0 - 2.0 * sum(c[a] ** 2 for a in zs))
        elif len(xs) == 2 and not zs:
            e += w * 2.0 * c[xs[0]] * c[xs[1]]
    return e


@pytest.mark.parametrize("n", [3, 6])
def test_zero_angle_energy_is_cis_energy(n):
    """All entangler angles zero: each entangler is CNOT CNOT = I, so every circuit's energy is the closed-form
    CIS energy of its vector."""
    wl = W.with_theta(W.mcvqe(n), np.zeros(5 * n - 4))
    e, _, mi, _ = oracle.expectations(wl)
    assert mi < 1e-13
    want = [_cis_energy(wl.extra["cis"][s], wl.xmask, wl.zmask, wl.coeff, n) for s in range(wl.B)]
    np.testing.assert_allclose(e, want, atol=1e-13)


def test_merge_preserves_the_circuit():
    """RY(a) RY(b) = RY(a + b): the merged circuit at the summed angles has the unmerged circuit's state."""
    n = 6
    rng = np.random.default_rng(11)
    raw, P, _ = W.mcvqe_entanglers(n, merge=False)
    merged, Pm, mf = W.mcvqe_entanglers(n)
    th = rng.uniform(0, 2 * np.pi, P)
    thm = np.array([th[m].sum() for m in mf])
    prep = W.cis_prep(W.mcvqe(n).extra["cis"][1])
    a = oracle.final_state(n, np.array(prep + raw, dtype=W.GATE_DTYPE), th)
    b = oracle.final_state(n, np.array(prep + merged, dtype=W.GATE_DTYPE), thm)
    np.testing.assert_allclose(a, b, atol=1e-13)


def test_mean_energy_gradients_agree():
    """Mean-energy gradient over the CIS states (upstream 1/S): adjoint = parameter-shift (1e-12) and central
    finite differences (1e-7 of the summed coefficient magnitudes)."""
    wl = W.mcvqe(5)
    up = np.full(wl.B, 1.0 / wl.B)
    ga = oracle.grad_adjoint(wl, up)
    gp = oracle.grad_param_shift(wl, up)
    gf = oracle.grad_fd(wl, 1e-4, up)
    np.testing.assert_allclose(ga, gp, atol=1e-12)
    np.testing.assert_allclose(gf, gp, atol=1e-7 * np.abs(wl.coeff).sum())
