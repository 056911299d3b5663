"""GPU parity for the probability path of Section 4.2 (output distributions, the Jensen-Shannon divergence
of Eq. 3 and its gradient by the adjoint sweep and by the parameter-shift rule) against the CPU oracle.

Tolerances: complex128 1e-12 absolute. complex64: a probability
within 1e-5 * max(Q_ref, 2^-n) (FP32 amplitudes carry a relative error of a few 1e-6 of the state's norm,
so a probability's error is at the 2^-n scale) and the distribution within 1e-5 in L1; a divergence
within 1e-5 * max(JS_ref, 1); a gradient component within 1e-5 * max(|g_ref|, sum_b |u_b|) (the loss is at
most log 2 per circuit)."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import ddcl as OD
from paper_2406_03466_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def _offsets(wl):
    off = np.zeros(wl.B + 1, np.int64)
    off[1:] = np.cumsum([1 << int(n) for n in wl.n_qubits])
    return off


def check_probs(q, ref, wl, prec):
    err = np.abs(q - ref)
    if prec == 1:
        assert err.max() <= 1e-12, f"probabilities: max err {err.max():.3e}"
        return
    off = _offsets(wl)
    for b in range(wl.B):
        n = int(wl.n_qubits[b])
        e, r = err[off[b]:off[b + 1]], ref[off[b]:off[b + 1]]
        assert (e <= 1e-5 * np.maximum(r, 2.0 ** -n)).all(), f"circuit {b}: max err {e.max():.3e}"
        assert e.sum() <= 1e-5, f"circuit {b}: L1 err {e.sum():.3e}"


def check(x, ref, prec, scale, what):
    x, ref = np.asarray(x), np.asarray(ref)
    err = np.abs(x - ref)
    say(f"  {what}: max err {err.max():.3e}")
    bad = err > (1e-12 if prec == 1 else 1e-5 * np.maximum(np.abs(ref), scale))
    assert not bad.any(), f"{what}: max err {err.max():.3e} at {int(np.argmax(err))}"


OPTS = [{}, {"tile_qubits": 6}, {"engine": "stride"}, {"fusion": "on"}, {"graph": False}]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", OPTS)
def test_probabilities(qv, prec, opts):
    say(f"ddcl probabilities prec={prec} opts={opts}")
    wl = W.ddcl(10, 3, sizes=[7, 10, 4])
    ref = OD.probabilities(wl)
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    check_probs(b.probabilities(), ref, wl, prec)


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("opts", OPTS)
def test_js_gradient(qv, prec, method, opts):
    say(f"ddcl js gradient prec={prec} method={method} opts={opts}")
    wl = W.ddcl(9, 2, sizes=[6, 9])
    t = wl.extra["target"]
    u = np.array([0.7, -1.3])
    js_ref = OD.js_values(wl, t)
    g_ref = OD.js_grad_param_shift(wl, t, u)
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    js, g = b.js_gradient(t, method, u)
    check(js, js_ref, prec, 1.0, "divergences")
    check(g, g_ref, prec, float(np.abs(u).sum()), "gradient")
    # a second call after a plain expectation call reuses the batch's buffers and graphs
    b.expectations(want_terms=False)
    js2, g2 = b.js_gradient(t, method, u)
    check(js2, js_ref, prec, 1.0, "divergences (second call)")
    check(g2, g_ref, prec, float(np.abs(u).sum()), "gradient (second call)")


def test_js_gradient_device_buffers(qv):
    """Device-pointer form: target, upstream, outputs as torch tensors, complex128."""
    import torch
    say("ddcl js gradient, device buffers")
    wl = W.ddcl(8, 2, sizes=[8, 5])
    t = wl.extra["target"]
    u = np.array([1.5, 0.25])
    g_ref = OD.js_grad_param_shift(wl, t, u)
    b = qv.Batch(ctx_for(qv), wl, 1)
    dev = torch.device("cuda:0")
    td, ud = torch.tensor(t, device=dev), torch.tensor(u, device=dev)
    js, g = torch.zeros(wl.B, dtype=torch.float64, device=dev), torch.zeros(wl.n_grad(), dtype=torch.float64, device=dev)
    b.js_gradient(td, 0, ud, js, g)
    torch.cuda.synchronize()
    check(js.cpu().numpy(), OD.js_values(wl, t), 1, 1.0, "divergences")
    check(g.cpu().numpy(), g_ref, 1, 1.0, "gradient")
    q = torch.zeros(b.n_amplitudes(), dtype=torch.float64, device=dev)
    b.probabilities(q)
    torch.cuda.synchronize()
    check_probs(q.cpu().numpy(), OD.probabilities(wl), wl, 1)


def test_bad_target_is_rejected(qv):
    wl = W.ddcl(4, 1, sizes=[4])
    b = qv.Batch(ctx_for(qv), wl, 1)
    t = wl.extra["target"].copy()
    t[3] = -0.1
    with pytest.raises(qv.QvError):
        b.js_gradient(t, 0)
    t[3] = np.nan
    with pytest.raises(qv.QvError):
        b.js_gradient(t, 1)


@pytest.mark.parametrize("prec,method", [(0, 0), (0, 1), (1, 0)])
def test_ddcl20_table2_size(qv, prec, method):
    """Table 2's smallest size (20 qubits, 10 layers, 1200 parameters): the divergence, 64 sampled
    probabilities and 8 gradient components against the oracle's stored values; the last RZ of the last
    layer (parameter 1199) cannot change the distribution, so its component is 0."""
    say(f"ddcl20 prec={prec} method={method}")
    with open(os.path.join(HERE, "golden", "ddcl20.json")) as f:
        gold = json.load(f)
    wl = W.ddcl(20, 10)
    t = wl.extra["target"]
    b = qv.Batch(ctx_for(qv), wl, prec)
    q = b.probabilities()
    idx = np.array(gold["prob_index"])
    ref = np.array(gold["probs"])
    err = np.abs(q[idx] - ref)
    assert (err <= (1e-12 if prec == 1 else 1e-5 * np.maximum(ref, 2.0 ** -20))).all(), err.max()
    assert abs(q.sum() - 1.0) <= (1e-12 if prec == 1 else 1e-5)
    js, g = b.js_gradient(t, method)
    check(js, [gold["js"]], prec, 1.0, "divergence")
    gi = np.array(gold["grad_index"])
    check(g[gi], np.array(gold["grad"]), prec, 1.0, "gradient components")
    assert abs(g[1199]) <= (1e-12 if prec == 1 else 1e-7)


@pytest.mark.parametrize("prec", [1, 0])
def test_js_autograd(qv, prec):
    """torch.autograd through the divergence: forward computes the divergences only, backward reuses the
    forward states for one adjoint sweep seeded with dL/dJS_b."""
    import torch
    from paper_2406_03466_amd.autograd import js_divergence
    say(f"ddcl autograd prec={prec}")
    wl = W.ddcl(8, 2, sizes=[8, 6])
    t = wl.extra["target"]
    u = np.array([0.4, 2.0])
    b = qv.Batch(ctx_for(qv), wl, prec)
    dev = torch.device("cuda:0")
    theta = torch.tensor(wl.theta, device=dev, requires_grad=True)
    js = js_divergence(theta, b, torch.tensor(t, device=dev))
    (js * torch.tensor(u, device=dev)).sum().backward()
    torch.cuda.synchronize()
    check(js.detach().cpu().numpy(), OD.js_values(wl, t), prec, 1.0, "divergences")
    check(theta.grad.cpu().numpy(), OD.js_grad_param_shift(wl, t, u), prec, float(np.abs(u).sum()), "gradient")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("theta,target_index", [(0.0, 2), (0.0, 3), (np.pi / 2, 2), (np.pi, 2)])
def test_degenerate_distributions(qv, prec, method, theta, target_index):
    """Point-mass targets and output distributions with zeros (0 log 0, zero weights): X on qubit 1 then
    RY(theta) on qubit 0, against the oracle (pinned to the closed form on the CPU)."""
    say(f"ddcl degenerate prec={prec} method={method} theta={theta} target={target_index}")
    wl = W.single("deg", 2, [W.gate(W.X, 1), W.gate(W.RY, 0, -1, 0)], [theta])
    t = np.zeros(4)
    t[target_index] = 1.0
    b = qv.Batch(ctx_for(qv), wl, prec)
    js, g = b.js_gradient(t, method)
    check(js, OD.js_values(wl, t), prec, 1.0, "divergence")
    check(g, OD.js_grad_param_shift(wl, t), prec, 1.0, "gradient")
    assert np.isfinite(js).all() and np.isfinite(g).all()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("method", [0, 1])
def test_js_gradient_shared_parameters(qv, prec, method):
    """Circuits sharing one parameter vector (data-fed copies): the divergence gradients of all circuits
    add into one vector."""
    say(f"js shared params prec={prec} method={method}")
    wl = W.qcl(n=7, layers=2, samples=3, seed_index=9)
    rng = np.random.default_rng(5)
    t = rng.exponential(size=wl.B << 7) * (rng.random(wl.B << 7) < 0.6)
    for b in range(wl.B):
        t[b << 7:(b + 1) << 7] /= t[b << 7:(b + 1) << 7].sum()
    u = np.array([1.0, -0.5, 0.25])
    bt = qv.Batch(ctx_for(qv), wl, prec)
    js, g = bt.js_gradient(t, method, u)
    check(js, OD.js_values(wl, t), prec, 1.0, "divergences")
    check(g, OD.js_grad_param_shift(wl, t, u), prec, float(np.abs(u).sum()), "gradient")


@pytest.mark.parametrize("prec", [0, 1])
def test_ddcl26_table2_largest(qv, prec):
    """Table 2's largest size (26 qubits, 10 layers, 1560 parameters), adjoint: the divergence, 64 sampled
    probabilities and 2 gradient components against the oracle's stored values."""
    say(f"ddcl26 prec={prec}")
    with open(os.path.join(HERE, "golden", "ddcl26.json")) as f:
        gold = json.load(f)
    wl = W.ddcl(26, 10)
    t = wl.extra["target"]
    b = qv.Batch(ctx_for(qv), wl, prec)
    q = b.probabilities()
    idx = np.array(gold["prob_index"])
    ref = np.array(gold["probs"])
    err = np.abs(q[idx] - ref)
    assert (err <= (1e-12 if prec == 1 else 1e-5 * np.maximum(ref, 2.0 ** -26))).all(), err.max()
    del q
    js, g = b.js_gradient(t, 0)
    check(js, [gold["js"]], prec, 1.0, "divergence")
    gi = np.array(gold["grad_index"])
    check(g[gi], np.array(gold["grad"]), prec, 1.0, "gradient components")
