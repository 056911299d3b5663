"""GPU parity on the MC-VQE-shaped batch (Section 4.1): one circuit per CIS state, shared entangler
parameters and the shared AIEM Hamiltonian; mean energy over the states (upstream weights 1/S).
Tolerances as in the other parity tests: 1e-12 absolute in complex128; in complex64 1e-5 of
max(|x_ref|, sum_t |c_t|) for energies and of sum_t |c_t| * sum_b |w_b| for gradients."""
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


def check(x, ref, prec, scale, what):
    x, ref = np.asarray(x), np.asarray(ref)
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    err = np.abs(x - ref)
    bad = err > (1e-12 if prec == 1 else 1e-5 * np.maximum(np.abs(ref), scale))
    assert not bad.any(), f"{what}: max err {err.max():.3e} at {int(np.argmax(err))}"


def _run(qv, wl, prec, opts, param_shift=True):
    up = np.full(wl.B, 1.0 / wl.B)
    e_ref, tv_ref, mi, _ = oracle.expectations(wl)
    assert mi < 1e-13
    g_ref = oracle.grad_adjoint(wl, up)
    s = float(np.abs(wl.coeff).sum())
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    check(e, e_ref, prec, s, "energies")
    check(tv, tv_ref, prec, 1.0, "term values")
    g, e2 = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g, g_ref, prec, s, "adjoint mean-energy gradient")
    check(e2, e_ref, prec, s, "energies (gradient call)")
    if param_shift:
        g2, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
        check(g2, g_ref, prec, s, "parameter-shift mean-energy gradient")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"fusion": "on"}, {"tile_qubits": 7}, {"engine": "stride"},
                                  {"engine": "lds", "tile_qubits": 8}, {"fold_cnots": "off"}])
def test_mcvqe10(qv, prec, opts):
    say(f"mcvqe n=10 prec={prec} opts={opts}")
    _run(qv, W.mcvqe(10), prec, opts)


@pytest.mark.parametrize("prec", [1, 0])
def test_mcvqe16_table1_size(qv, prec):
    """Table 1's smallest size: 16 qubits, 92 terms + constant, 76 parameters, 16 CIS states."""
    say(f"mcvqe n=16 prec={prec}")
    wl = W.mcvqe(16)
    assert wl.n_grad() == 76 and wl.extra["n_hamiltonian_terms"] == 92
    _run(qv, wl, prec, {})


def test_mcvqe_zero_angles_give_cis_energies(qv):
    """All entangler angles zero: every state's energy is its CIS energy (checked against the oracle,
    which the CPU tests pin to the closed form)."""
    say("mcvqe zero angles")
    wl = W.with_theta(W.mcvqe(12), np.zeros(5 * 12 - 4))
    e_ref, _, _, _ = oracle.expectations(wl)
    b = qv.Batch(ctx_for(qv), wl, 1)
    e, _ = b.expectations(want_terms=False)
    check(e, e_ref, 1, 1.0, "CIS energies")


@pytest.mark.parametrize("prec", [1, 0])
def test_mcvqe22_table1_largest(qv, prec):
    """Table 1's largest size (22 CIS states of 22 qubits, 106 parameters, 128 terms and a constant)
    against the oracle's stored energies and mean-energy gradient."""
    import os
    say(f"mcvqe n=22 prec={prec}")
    with open(os.path.join(os.path.dirname(__file__), "golden", "mcvqe22.json")) as f:
        gold = json.load(f)
    wl = W.mcvqe(22)
    s = float(np.abs(wl.coeff).sum())
    b = qv.Batch(ctx_for(qv), wl, prec)
    e, _ = b.expectations(want_terms=False)
    check(e, np.array(gold["energies"]), prec, s, "energies")
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=np.array(gold["upstream"]))
    ref = np.array(gold["grad"])
    check(g, ref, prec, s, "gradient")
    say(f"  max |dE| {np.abs(e - np.array(gold['energies'])).max():.2e}  max |dg| {np.abs(g - ref).max():.2e}")
