"""GPU test of qv_batch_expectations_static, the expectation call that allocates no device memory (its
partial sums live in the library's static scratch array): called through the C interface, it must give
what qv_batch_expectations gives, on two calls in a row, the second with a smaller batch, with host and
device outputs; a batch needing more partial sums than the array holds, and a batch whose autotuner has
still to choose its tiles, are refused before anything runs.
"""
import ctypes
import json
import sys

import numpy as np
import pytest

import oracle
from paper_2406_03466_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qv():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_03466_amd import qvpu
    qvpu.load()
    return qvpu


def ctx_for(qv, **opts):
    import torch
    return qv.Context(0, torch.cuda.current_stream().cuda_stream, json.dumps(opts) if opts else None)


def static_call(qv, b):
    """qv_batch_expectations_static through the C interface, host outputs."""
    lib = qv.load()
    e = np.zeros(b.B)
    tv = np.zeros(max(1, b.n_tv))
    st = lib.qv_batch_expectations_static(b.h, e.ctypes.data, tv.ctypes.data, 0)
    assert st == qv.QV_OK, qv.last_error()
    return e, tv[: b.n_tv]


def bound(prec, ref, scale):
    return 1e-12 if prec == 1 else 1e-5 * np.maximum(np.abs(ref), scale)


@pytest.mark.parametrize("prec", [1, 0])
def test_static_matches_allocating_call_twice(qv, prec):
    """A 24-circuit uneven batch (2..16 qubits), then a smaller one (6 circuits of 3..8 qubits): the static
    call equals the allocating call bit for bit (same kernels, same order) and the oracle to the bound."""
    for k, wl in enumerate([W.random_batch(24, 2, 16, 0, 80, 5, seed_index=81),
                            W.random_batch(6, 3, 8, 5, 30, 3, seed_index=82)]):
        say(f"static call {k} prec={prec} B={wl.B}")
        b = qv.Batch(ctx_for(qv, autotune="off"), wl, prec)
        e_s, tv_s = static_call(qv, b)
        e_a, tv_a = b.expectations()
        assert np.array_equal(e_s, e_a) and np.array_equal(tv_s, tv_a)
        e_s2, tv_s2 = static_call(qv, b)   # again, after the allocating call
        assert np.array_equal(e_s2, e_a) and np.array_equal(tv_s2, tv_a)
        e_ref, tv_ref, _, _ = oracle.expectations(wl)
        scale = max(float(np.sum(np.abs(wl.terms(c)[2]))) for c in range(wl.B))
        assert (np.abs(e_s - e_ref) <= bound(prec, e_ref, scale)).all()
        assert (np.abs(tv_s - tv_ref) <= bound(prec, tv_ref, 1.0)).all()
        b.close()


def test_static_device_outputs_and_new_parameters(qv):
    """Device outputs, and parameters changed between calls: the 20-qubit circuit-learning batch (64
    samples, 2 layers, complex64) at its parameters and at shifted ones."""
    import torch
    say("static device outputs")
    wl = W.config3(2)
    b = qv.Batch(ctx_for(qv, autotune="off"), wl, 0)
    lib = qv.load()
    e = torch.empty(wl.B, dtype=torch.float64, device="cuda")
    tv = torch.empty(wl.B, dtype=torch.float64, device="cuda")
    for shift in (0.0, 0.3):
        b.set_params(wl.theta + shift)
        assert lib.qv_batch_expectations_static(b.h, ctypes.c_void_p(e.data_ptr()), ctypes.c_void_p(tv.data_ptr()),
                                                1) == qv.QV_OK, qv.last_error()
        torch.cuda.synchronize()
        e_a, _ = b.expectations(want_terms=False)
        assert np.array_equal(e.cpu().numpy(), e_a)
        assert np.array_equal(tv.cpu().numpy(), e_a)   # one unit-weight term: term value = energy
    e_ref, _, _, _ = oracle.expectations(W.with_theta(wl, wl.theta + 0.3))
    assert (np.abs(e.cpu().numpy() - e_ref) <= 1e-5).all()


def test_static_refusals(qv, tmp_path, monkeypatch):
    """Refused before anything runs: a 30-qubit state with 24 diagonal terms needs 3 x 2^16 x 8 partial
    sums (more than the 2^20 of the array); a 16-qubit batch under "autotune": "search" has still to time
    its tile candidates."""
    monkeypatch.setenv("QV_TUNE_CACHE", str(tmp_path / "tune.txt"))
    say("static refusals")
    n = 30
    gates = [W.gate(W.RY, q, -1, q) for q in range(4)]
    zm = np.array([(1 << i) | (1 << (i + 1)) for i in range(24)], np.uint64)
    wl = W.single("big", n, gates, np.full(4, 0.4), (np.zeros(24, np.uint64), zm, np.ones(24)))
    b = qv.Batch(ctx_for(qv, autotune="off"), wl, 0)
    lib = qv.load()
    e = np.zeros(1)
    assert lib.qv_batch_expectations_static(b.h, e.ctypes.data, None, 0) == qv.QV_E_INVALID
    assert "partial sums" in qv.last_error()
    b.close()
    wl2 = W.qcl(n=16, layers=2, samples=4, seed_index=83)
    b2 = qv.Batch(ctx_for(qv, autotune="search"), wl2, 0)
    e = np.zeros(wl2.B)
    assert lib.qv_batch_expectations_static(b2.h, e.ctypes.data, None, 0) == qv.QV_E_STATE
    assert "autotuner" in qv.last_error()
    e_a, _ = b2.expectations(want_terms=False)
    e_s, _ = static_call(qv, b2)
    assert np.array_equal(e_s, e_a)
