"""CPU checks of the pass planner (host logic of the library, no device): every gate is scheduled once,
gates that share a qubit keep their program order, every pass's gates are local to its tile, and running
the circuit in the planned order gives the same state as program order (oracle, complex128)."""
import numpy as np
import pytest

import oracle
from paper_2406_03466_amd import qvpu
from paper_2406_03466_amd import workloads as W


def _check_plan(n, gates, passes, order):
    G = len(gates)
    assert sorted(order.tolist()) == list(range(G))
    assert sum(p["n_ops"] for p in passes) == G
    # per-qubit program order is preserved
    last = {}
    for g in order:
        r = gates[g]
        qs = [int(r["q0"])] + ([int(r["q1"])] if int(r["kind"]) in (W.CNOT, W.CZ) else [])
        for q in qs:
            assert last.get(q, -1) < g, f"gate {g} on qubit {q} runs after a later gate"
            last[q] = g
    # every pass's gates act on its tile's qubits only
    k = 0
    for p in passes:
        for g in order[k:k + p["n_ops"]]:
            r = gates[g]
            m = (1 << int(r["q0"])) | ((1 << int(r["q1"])) if int(r["kind"]) in (W.CNOT, W.CZ) else 0)
            assert m & ~p["local_mask"] == 0
        k += p["n_ops"]
        assert bin(p["local_mask"]).count("1") == p["qubits"]


@pytest.mark.parametrize("engine", [0, 1, 2])
@pytest.mark.parametrize("tile", [6, 8, 13])
def test_random_circuits_planned_order(engine, tile):
    rng = np.random.default_rng(tile * 10 + engine)
    wl = W.random_batch(12, 2, 16, 0, 120, 1, seed_index=60 + tile)
    for b in range(wl.B):
        n = int(wl.n_qubits[b])
        gates = wl.circuit(b)
        passes, order = qvpu.plan_circuit(n, gates, tile, qvpu.QV_C64, engine, with_order=True)
        _check_plan(n, gates, passes, order)
        if n <= 12 and len(gates):
            th = wl.theta_of(b)
            a = oracle.final_state(n, gates, th)
            bst = oracle.final_state(n, gates[order], th)
            np.testing.assert_allclose(a, bst, atol=1e-13)
    del rng


def test_hea_pass_counts_and_tiles():
    """20-qubit circuit learning, 8 layers: the planner packs the 492 gates into a handful of tile passes,
    every register-tiled pass holds 13 qubits with qubits 0..3 contiguous."""
    wl = W.config3(8)
    passes, order = qvpu.plan_circuit(20, wl.circuit(0), 13, qvpu.QV_C64, 0, with_order=True)
    _check_plan(20, wl.circuit(0), passes, order)
    assert len(passes) <= 8
    for p in passes:
        assert p["qubits"] == 13 and p["contiguous_low"] >= 4 and p["n_segments"] >= 1
    stride = qvpu.plan_circuit(20, wl.circuit(0), 13, qvpu.QV_C64, 2)
    assert len(stride) == 492


def test_small_circuits_are_one_pass():
    wl = W.config1()
    passes = qvpu.plan_circuit(10, wl.circuit(0), 13, qvpu.QV_C128, 0)
    assert len(passes) == 1 and passes[0]["qubits"] == 10 and passes[0]["n_ops"] == 116


def test_trainable_cap_per_pass():
    """A pass holds at most 256 trainable gates (their adjoint partial sums live in LDS)."""
    g = [W.gate(W.RY, i % 6, -1, i) for i in range(1300)]
    arr = np.array(g, W.GATE_DTYPE)
    passes = qvpu.plan_circuit(6, arr, 13, qvpu.QV_C64, 0)
    assert [p["n_trainable"] for p in passes] == [256] * 5 + [20]


def test_plan_rejects_bad_input():
    arr = np.array([W.gate(W.CNOT, 0, 0)], W.GATE_DTYPE)
    with pytest.raises(qvpu.QvError):
        qvpu.plan_circuit(4, arr, 13, qvpu.QV_C64, 0)
    with pytest.raises(qvpu.QvError):
        qvpu.plan_circuit(4, np.array([W.gate(W.H, 0)], W.GATE_DTYPE), 3, qvpu.QV_C64, 0)


@pytest.mark.parametrize("fuse_min", [1, 2, 4, 6])
def test_fused_plans_keep_every_gate(fuse_min):
    """Fused-block markers do not change the schedule: every gate appears once, in a valid order, and the
    blocks are counted per pass."""
    wl = W.config3(8)
    gates = wl.circuit(0)
    passes, order = qvpu.plan_circuit(20, gates, 13, qvpu.QV_C64, 0, with_order=True, fuse_min=fuse_min)
    _check_plan(20, gates, passes, order)
    nf = sum(p["n_fused"] for p in passes)
    assert nf > 0
    plain = qvpu.plan_circuit(20, gates, 13, qvpu.QV_C64, 0)
    assert [p["local_mask"] for p in plain] == [p["local_mask"] for p in passes]
    # the stride engine never fuses
    assert sum(p["n_fused"] for p in qvpu.plan_circuit(20, gates, 13, qvpu.QV_C64, 2, fuse_min=fuse_min)) == 0


def test_boundary_cnots_are_folded():
    """CNOT runs at register-segment ends are folded into the segments' addressing: the circuit-learning
    ansatz (CNOT ladders after every rotation layer) has some in every plan, every gate is still scheduled
    once in a valid order, and the LDS and stride engines (no register segments) fold none."""
    wl = W.config3(8)
    gates = wl.circuit(0)
    for fuse_min in (0, 8):
        passes, order = qvpu.plan_circuit(20, gates, 13, qvpu.QV_C64, 0, with_order=True, fuse_min=fuse_min)
        _check_plan(20, gates, passes, order)
        folded = sum(p["n_folded"] for p in passes)
        n_cnot = int(np.sum(gates["kind"] == W.CNOT))
        assert 0 < folded <= n_cnot
    for engine in (1, 2):
        assert sum(p["n_folded"] for p in qvpu.plan_circuit(20, gates, 13, qvpu.QV_C64, engine)) == 0


def test_folded_order_matches_state():
    """Running a CNOT-heavy circuit in the planned order (folded CNOTs at their segment ends) gives the
    program-order state (oracle, complex128)."""
    rng = np.random.default_rng(11)
    n = 9
    circ = []
    for layer in range(6):
        for q in range(n):
            circ.append(W.gate(W.RY, q, -1, len(circ), 0.0))
        for q in range(n - 1):
            circ.append(W.gate(W.CNOT, q, q + 1))
        for _ in range(4):
            a, b = rng.choice(n, size=2, replace=False)
            circ.append(W.gate(W.CNOT, int(a), int(b)))
    gates = np.array(circ, W.GATE_DTYPE)
    theta = rng.uniform(0, 2 * np.pi, size=len(circ))
    passes, order = qvpu.plan_circuit(n, gates, 6, qvpu.QV_C64, 0, with_order=True)
    _check_plan(n, gates, passes, order)
    assert sum(p["n_folded"] for p in passes) > 0
    s0 = oracle.final_state(n, gates, theta)
    s1 = oracle.final_state(n, gates[order], theta)
    assert np.max(np.abs(s0 - s1)) < 1e-12


@pytest.mark.parametrize("case", ["hea", "ddcl", "random"])
def test_zero_masks(case):
    """A pass's zero mask holds the qubits outside its tile that no gate of an earlier pass acts on
    (recomputed here from the planned gate order and the passes' tiles). Before the pass those qubits are
    still |0>, so the state is exactly zero wherever one of them is 1 (oracle state, complex128, after the
    earlier passes' gates in planned order)."""
    rng = np.random.default_rng(5)
    n = 11
    if case == "hea":
        gates = np.array(W.hea_layers(n, 3)[0], W.GATE_DTYPE)
    elif case == "ddcl":
        gates = np.array(W.ddcl_layers(n, 2)[0], W.GATE_DTYPE)
    else:
        gates = W.random_batch(1, n, n, 60, 60, 1, seed_index=51).circuit(0).copy()
    n_par = int(gates["param"].max()) + 1 if (gates["param"] >= 0).any() else 0
    theta = rng.uniform(0, 2 * np.pi, size=max(1, n_par))
    passes, order = qvpu.plan_circuit(n, gates, 6, qvpu.QV_C64, 0, with_order=True)
    assert len(passes) > 1
    full = (1 << n) - 1
    touched, pos, seen_zero = 0, 0, False
    for p in passes:
        expect = full & ~p["local_mask"] & ~touched
        assert p["zero_mask"] == expect, (p["zero_mask"], expect)
        state = oracle.final_state(n, gates[order[:pos]], theta)
        idx = np.arange(1 << n)
        if expect:
            seen_zero = True
            assert np.all(state[(idx & expect) != 0] == 0)
        for gi in order[pos:pos + p["n_ops"]]:
            g = gates[gi]
            touched |= 1 << int(g["q0"])
            if int(g["q1"]) >= 0 and int(g["kind"]) in (W.CNOT, W.CZ):
                touched |= 1 << int(g["q1"])
        pos += p["n_ops"]
    assert pos == len(gates)
    assert seen_zero
