"""GPU parity: the HIP library through its C interface against the CPU oracle on the same seeded inputs.

Tolerances (the accuracy targets of the build):
  * complex128 path: |x - x_ref| <= 1e-12 for every energy, term value and gradient component;
  * complex64 path:  |x - x_ref| <= 1e-5 * max(|x_ref|, S), S = sum_t |c_t| for expectations and
    S = sum_t |c_t| * sum_b |w_b| for gradients (random-string expectations are ~2^{-n/2}, so a purely
    relative bound is meaningless near zero).
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
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
    js = json.dumps(opts) if opts else None
    return qv.Context(0, torch.cuda.current_stream().cuda_stream, js)


def c64_tol(ref, scale):
    return 1e-5 * np.maximum(np.abs(ref), scale)


def check(x, ref, prec, scale, what):
    x, ref = np.asarray(x), np.asarray(ref)
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    err = np.abs(x - ref)
    if prec == 1:
        bad = err > 1e-12
    else:
        bad = err > c64_tol(ref, scale)
    assert not bad.any(), f"{what}: max err {err.max():.3e} at {int(np.argmax(err))}"
    return float(err.max()) if err.size else 0.0


def obs_scale(wl):
    if wl.obs_shared:
        return float(np.sum(np.abs(wl.coeff)))
    return max(float(np.sum(np.abs(wl.terms(b)[2]))) for b in range(wl.B))


# --------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"tile_qubits": 6}, {"engine": "stride"}, {"engine": "lds"},
                                  {"engine": "lds", "tile_qubits": 7}, {"graph": False}, {"fusion": "on"},
                                  {"fusion": 2, "tile_qubits": 7}])
def test_c1_expectations(qv, prec, opts):
    say(f"c1 expectations prec={prec} opts={opts}")
    wl = W.config1()
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    check(e, e_ref, prec, obs_scale(wl), "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    st = b.stats()
    assert st["norm_err_max"] < (1e-13 if prec == 1 else 1e-5)


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"tile_qubits": 6}, {"engine": "stride"}, {"engine": "lds"},
                                  {"engine": "lds", "tile_qubits": 7},
                                  {"fusion": 2}, {"fusion": 3, "tile_qubits": 8}])
def test_c1_gradients(qv, prec, opts):
    say(f"c1 gradients prec={prec} opts={opts}")
    wl = W.config1()
    g_ref = oracle.grad_param_shift(wl)
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    g_ad, e_ad = b.gradient(qv.QV_ADJOINT)
    g_ps, e_ps = b.gradient(qv.QV_PARAM_SHIFT)
    s = obs_scale(wl)
    check(g_ad, g_ref, prec, s, "adjoint grad")
    check(g_ps, g_ref, prec, s, "param-shift grad")
    e_ref, _, _, _ = oracle.expectations(wl)
    check(e_ad, e_ref, prec, s, "energy (adjoint call)")
    check(e_ps, e_ref, prec, s, "energy (param-shift call)")


@pytest.mark.parametrize("prec", [1, 0])
def test_c2_full(qv, prec):
    """16 qubits, 8 layers, 100 terms: every energy/term value; adjoint and the 513-circuit parameter-shift
    batch against the oracle gradient."""
    say(f"c2 prec={prec}")
    wl = W.config2()
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    g_ref = oracle.grad_adjoint(wl)
    b = qv.Batch(ctx_for(qv), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    g_ad, _ = b.gradient(qv.QV_ADJOINT)
    check(g_ad, g_ref, prec, s, "adjoint grad")
    g_ps, _ = b.gradient(qv.QV_PARAM_SHIFT)
    check(g_ps, g_ref, prec, s, "param-shift grad")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("tile,engine", [(6, "tiled"), (9, "tiled"), (None, "tiled"), (8, "lds"), (None, "lds"),
                                         (None, "fused"), (8, "fused"), (None, "stride")])
def test_uneven_batch(qv, prec, tile, engine):
    """Circuits of 2..16 qubits and 0..80 gates in one batch: per-circuit energies, terms, states and
    adjoint gradients (own parameters per circuit) with upstream weights."""
    say(f"uneven prec={prec} tile={tile} engine={engine}")
    wl = W.random_batch(24, 2, 16, 0, 80, 5, seed_index=41)
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    up = np.linspace(-1.0, 1.5, wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    opts = {"fusion": 2} if engine == "fused" else {"engine": engine}
    if tile is not None:
        opts["tile_qubits"] = tile
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    for c in [0, 5, 11, 23]:
        n = int(wl.n_qubits[c])
        psi_ref = oracle.final_state(n, wl.circuit(c), wl.theta_of(c))
        psi = b.state(c)
        err = np.max(np.abs(psi - psi_ref))
        assert err < (1e-13 if prec == 1 else 1e-5), (c, err)
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g, g_ref, prec, s * np.sum(np.abs(up)), "adjoint grad")
    g2, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
    check(g2, g_ref, prec, s * np.sum(np.abs(up)), "param-shift grad")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("engine", ["tiled", "lds", "stride"])
def test_one_to_three_qubit_circuits(qv, prec, engine):
    """The degenerate sizes: circuits of 1, 2 and 3 qubits (a complex64 state of 1 qubit is one 16-byte
    vector, so most lanes of a stride pass lie past its end), every one-qubit gate kind: energies, terms
    and adjoint and parameter-shift gradients against the oracle."""
    say(f"1-3 qubits prec={prec} engine={engine}")
    wl = W.random_batch(18, 1, 3, 1, 24, 3, seed_index=43,
                        kinds=[W.H, W.X, W.Y, W.Z, W.S, W.T, W.RX, W.RY, W.RZ])
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    up = np.linspace(1.0, -0.5, wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    b = qv.Batch(ctx_for(qv, engine=engine), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g, g_ref, prec, s * np.sum(np.abs(up)), "adjoint grad")
    g2, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
    check(g2, g_ref, prec, s * np.sum(np.abs(up)), "param-shift grad")


def _degenerate_batch():
    """Four circuits, own parameters and own observables: 5 qubits with no gates; 6 qubits whose parameter 0
    drives three gates (RY, RX, RZ on different qubits) and parameter 1 one; 4 qubits with gates and no
    terms; 3 qubits with fixed angles only (no parameters)."""
    rng = np.random.default_rng(4411)
    g = W.gate
    c0 = []
    c1 = [g(W.H, 1), g(W.RY, 0, -1, 0), g(W.CNOT, 0, 3), g(W.RX, 2, -1, 0), g(W.RY, 5, -1, 1), g(W.CNOT, 2, 5),
          g(W.RZ, 4, -1, 0), g(W.H, 4), g(W.CZ, 4, 1), g(W.RY, 3, -1, 1)]
    c2 = [g(W.H, 0), g(W.RY, 1, -1, 0), g(W.CNOT, 0, 2), g(W.RZ, 3, -1, 1)]
    c3 = [g(W.RX, 0, -1, -1, 0.3), g(W.CNOT, 0, 1), g(W.RY, 2, -1, -1, 1.1), g(W.T, 2)]
    t0 = (np.array([0, 2], np.uint64), np.array([1, 4 | 8], np.uint64), np.array([0.7, -1.3]))
    t1 = W.random_paulis(rng, 6, 6)
    t2 = (np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0))
    t3 = W.random_paulis(rng, 4, 3)
    theta = rng.uniform(0, 2 * np.pi, 4)
    return W._pack("degenerate", [c0, c1, c2, c3], [5, 6, 4, 3], [0, 2, 2, 0], False, theta,
                   [t0, t1, t2, t3], False)


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("engine", ["tiled", "stride"])
def test_degenerate_circuits_and_shared_parameter(qv, prec, engine):
    """A circuit without gates (|0...0>: Z strings give their coefficient, X strings 0), one without terms
    (energy and gradient 0), one without parameters, and a parameter driving three gates (its gradient sums
    the three, by the adjoint and by per-gate shifts): energies, terms and both gradients against the
    oracle, whose chain rule is pinned against finite differences on the CPU."""
    say(f"degenerate prec={prec} engine={engine}")
    wl = _degenerate_batch()
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    assert abs(e_ref[0] - 0.7) < 1e-15 and e_ref[2] == 0.0
    up = np.array([1.0, -0.5, 2.0, 0.25])
    g_ref = oracle.grad_param_shift(wl, up)
    b = qv.Batch(ctx_for(qv, engine=engine), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    g_ad, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g_ad, g_ref, prec, s * np.sum(np.abs(up)), "adjoint grad")
    g_ps, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
    check(g_ps, g_ref, prec, s * np.sum(np.abs(up)), "param-shift grad")
    b.close()


def test_waves_and_engines_bitwise(qv):
    """Results do not depend on how many circuits are in flight (n-virtual-qpus): bitwise equal."""
    say("waves")
    wl = W.random_batch(40, 3, 15, 10, 60, 4, seed_index=42)
    outs = []
    for nv in [1, 4, 40]:
        b = qv.Batch(ctx_for(qv, **{"n-virtual-qpus": nv}), wl, 0)
        e, tv = b.expectations()
        g, _ = b.gradient(qv.QV_ADJOINT)
        outs.append((e, tv, g))
    for o in outs[1:]:
        for a, r in zip(o, outs[0]):
            assert np.array_equal(a, r)


def test_shuffled_batch_permutes_output(qv):
    say("shuffle")
    wl = W.random_batch(20, 3, 14, 5, 40, 3, seed_index=43)
    perm = np.random.default_rng(1).permutation(wl.B)
    e0, _ = qv.Batch(ctx_for(qv), wl, 0).expectations()
    e1, _ = qv.Batch(ctx_for(qv), wl.subset(perm), 0).expectations()
    assert np.array_equal(e0[perm], e1)


def test_graph_replays_with_new_params(qv):
    """The captured graph is replayed with new parameters and eager work in between; each replay matches
    the oracle for its parameters."""
    import torch
    say("graph replays")
    wl = W.qcl(n=12, layers=2, samples=6, seed_index=44)
    b = qv.Batch(ctx_for(qv), wl, 1)
    rng = np.random.default_rng(3)
    for r in range(4):
        th = rng.uniform(0, 2 * np.pi, wl.n_grad())
        b.set_params(th)
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        e, _ = b.expectations()
        e_ref, _, _, _ = oracle.expectations(W.with_theta(wl, th))
        check(e, e_ref, 1, 1.0, f"replay {r}")
        assert torch.isfinite(x)


@pytest.mark.parametrize("prec", [0, 1])
def test_qcl_autograd_small(qv, prec):
    """ExpectationFn forward/backward on a 12-qubit circuit-learning batch against the oracle's adjoint
    gradient and central finite differences of the MSE loss."""
    import torch
    from paper_2406_03466_amd.autograd import expectation
    say(f"qcl autograd prec={prec}")
    wl = W.qcl(n=12, layers=2, samples=8, seed_index=3)
    b = qv.Batch(ctx_for(qv), wl, prec)
    theta = torch.tensor(wl.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    y = torch.tensor(wl.extra["y"], dtype=torch.float64, device="cuda")
    f = expectation(theta, b)
    loss = torch.mean((f - y) ** 2)
    loss.backward()
    e_ref, _, _, _ = oracle.expectations(wl)
    up = 2.0 * (e_ref - wl.extra["y"]) / wl.B
    g_ref = oracle.grad_adjoint(wl, up)
    g_fd = oracle.grad_fd(wl, 1e-4, up)
    assert np.max(np.abs(g_ref - g_fd)) < 1e-7 * np.sum(np.abs(up))
    check(f.detach().cpu().numpy(), e_ref, prec, 1.0, "energies")
    check(theta.grad.cpu().numpy(), g_ref, prec, float(np.sum(np.abs(up))), "grad")


@pytest.mark.parametrize("prec", [0, 1])
def test_autograd_same_batch_two_points(qv, prec):
    """One batch evaluated at two parameter vectors before a single backward (as in a loss that compares
    two points): each backward runs at its own forward's parameters, not at the ones the batch received
    last. Checked against the oracle's adjoint gradient at each point."""
    import torch
    from paper_2406_03466_amd.autograd import expectation
    say(f"autograd two points prec={prec}")
    wl = W.qcl(n=10, layers=2, samples=6, seed_index=8)
    b = qv.Batch(ctx_for(qv), wl, prec)
    th1 = torch.tensor(wl.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    th2_host = np.random.default_rng(3).uniform(0, 2 * np.pi, wl.theta.shape)
    th2 = torch.tensor(th2_host, dtype=torch.float64, device="cuda", requires_grad=True)
    u1 = np.linspace(-1.0, 1.0, wl.B)
    u2 = np.linspace(0.5, -0.25, wl.B)
    f1 = expectation(th1, b)
    f2 = expectation(th2, b)
    loss = (f1 * torch.tensor(u1, device="cuda")).sum() + (f2 * torch.tensor(u2, device="cuda")).sum()
    loss.backward()
    for th, th_host, u, f in ((th1, wl.theta, u1, f1), (th2, th2_host, u2, f2)):
        wl_at = W.with_theta(wl, th_host)
        e_ref, _, _, _ = oracle.expectations(wl_at)
        check(f.detach().cpu().numpy(), e_ref, prec, 1.0, "energies")
        check(th.grad.cpu().numpy(), oracle.grad_adjoint(wl_at, u), prec, float(np.sum(np.abs(u))), "grad")


def test_context_destroyed_before_its_batch(qv):
    """A batch keeps its context alive: destroying the context first (as a garbage collector may do with
    objects in a reference cycle) leaves the batch usable, and destroying the batch afterwards frees both."""
    say("context destroyed first")
    wl = W.config1()
    e_ref, _, _, _ = oracle.expectations(wl)
    ctx = ctx_for(qv)
    b = qv.Batch(ctx, wl, 1)
    ctx.close()
    e, _ = b.expectations()
    check(e, e_ref, 1, 1.0, "energies after the context was destroyed")
    b.close()
    b2 = qv.Batch(ctx_for(qv), wl, 1)
    check(b2.expectations()[0], e_ref, 1, 1.0, "energies on a new context")


def test_earlier_runtime_error_not_reported(qv):
    """A failed HIP call made by someone else on this thread (here hipSetDevice with a device that does
    not exist) leaves the runtime's last-error slot set; the library's next call clears it on entry and
    succeeds instead of reporting that error as its own launch failure."""
    import ctypes
    say("stale runtime error")
    lib = qv.load()
    set_device = lib.hipSetDevice      # the HIP runtime the library itself uses (found through its handle)
    set_device.argtypes = [ctypes.c_int]
    set_device.restype = ctypes.c_int
    wl = W.config1()
    e_ref, _, _, _ = oracle.expectations(wl)
    for graph in (True, False):
        b = qv.Batch(ctx_for(qv, graph=graph), wl, 1)
        assert set_device(4096) != 0
        e, _ = b.expectations()
        check(e, e_ref, 1, 1.0, f"energies (graph {graph})")
        b.close()


def _golden(name):
    p = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(p):
        pytest.skip(f"golden file {name}.json not generated")
    return json.load(open(p))


# the launch configuration bench.py times (tile size, contiguous run and fused-block minimum run chosen by
# the autotuner, eager launches, adjoint levels on generated passes where they time faster)
BENCH_OPTS = {"fusion": "auto", "autotune": "search", "graph": False, "launch_events": True, "specialize": "auto"}


@pytest.mark.parametrize("layers,opts", [(2, {}), (4, {}), (8, {}), (2, BENCH_OPTS), (4, BENCH_OPTS),
                                         (8, BENCH_OPTS), (8, dict(BENCH_OPTS, launch="persistent"))])
def test_qcl20_full_size(qv, layers, opts, tmp_path, monkeypatch):
    """20 qubits, 64 samples, complex64: every energy and every gradient component of the MSE loss against
    the oracle's stored values, with default options and in the launch configuration the benchmark times."""
    monkeypatch.setenv("QV_TUNE_CACHE", str(tmp_path / "tune.txt"))
    say(f"qcl20 L={layers} opts={opts}")
    gold = _golden(f"qcl20_L{layers}")
    wl = W.config3(layers)
    b = qv.Batch(ctx_for(qv, **opts), wl, 0)
    e, _ = b.expectations(want_terms=False)
    ee = check(e, np.array(gold["energies"]), 0, 1.0, "energies")
    up = 2.0 * (e - wl.extra["y"]) / wl.B
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=np.array(gold["upstream"]))
    ge = check(g, np.array(gold["grad"]), 0, float(np.sum(np.abs(gold["upstream"]))), "grad")
    assert np.max(np.abs(up - np.array(gold["upstream"]))) < 1e-5
    say(f"  max |dE| {ee:.2e}  max |dg| {ge:.2e}  stats {b.stats()}")


def test_random1024_full_size(qv):
    """1024 random circuits of 8..22 qubits, complex64: every energy and term value."""
    say("random1024")
    gold = _golden("random1024")
    wl = W.config4()
    b = qv.Batch(ctx_for(qv), wl, 0)
    e, tv = b.expectations()
    check(e, np.array(gold["energies"]), 0, obs_scale(wl), "energies")
    check(tv, np.array(gold["term_values"]), 0, 1.0, "terms")


@pytest.mark.parametrize("n,opts", [(26, {}), (32, {}), (33, {}), (26, {"engine": "stride"})])
def test_large_state_closed_form(qv, n, opts):
    """One HEA layer on n qubits (32: a 32 GiB complex64 state; 33: 64 GiB, amplitude indices past 2^32,
    128 GiB with lambda) with the ZZ chain: the CNOT ladder is a prefix-XOR permutation, so
    E = sum_{i>=1} cos(theta_RY[i]) and dE/dtheta_RY[i] = -sin(theta_RY[i]) (0 for i = 0); checks 64-bit
    indexing at full size, and on the stride engine the non-temporal passes taken for states larger than
    the caches."""
    say(f"large n={n} opts={opts}")
    wl = W.large_hea(n, 1, seed_index=5)
    b = qv.Batch(ctx_for(qv, **opts), wl, 0)
    e, tv = b.expectations()
    ry = wl.theta[:n]
    check(tv, np.cos(ry[1:]), 0, 1.0, "ZZ terms")
    check(e, [np.sum(np.cos(ry[1:]))], 0, n - 1.0, "energy")
    g, _ = b.gradient(qv.QV_ADJOINT)
    want = np.concatenate([[0.0], -np.sin(ry[1:])])
    check(g, want, 0, n - 1.0, "grad")
    st = b.stats()
    assert st["norm_err_max"] < 1e-5
    b.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_stride_engine_full_size(qv, prec):
    """The stride engine on one 22-qubit circuit (RY, RX, RZ and H on every qubit, a CNOT ladder, CZs, a
    second RY layer): every one-qubit access pattern of its global-memory passes (both amplitudes of a pair
    in one 16-byte vector, the partner vector in another lane of the wave, the partner 2^p vectors on), at
    full size; energy, term values and the adjoint gradient against the oracle."""
    say(f"stride engine full size prec={prec}")
    n = 22
    rng = np.random.default_rng(2211)
    gates, k = [], 0
    for q in range(n):
        gates.append(W.gate(W.RY, q, -1, k)); k += 1
        gates.append(W.gate(W.RX, q, -1, k)); k += 1
    gates += [W.gate(W.H, q, -1, -1) for q in range(0, n, 3)]
    for q in range(n):
        gates.append(W.gate(W.RZ, q, -1, k)); k += 1
    gates += [W.gate(W.CNOT, q, q + 1, -1) for q in range(n - 1)]
    gates += [W.gate(W.CZ, q, (q + 7) % n, -1) for q in range(0, n, 5)]
    for q in range(n):
        gates.append(W.gate(W.RY, q, -1, k)); k += 1
    theta = rng.uniform(0, 2 * np.pi, k)
    # terms with values of order one (random 22-qubit Pauli strings have values near zero)
    strings = [{0: "Z"}, {0: "Z", 1: "Z"}, {0: "X"}, {5: "Z", 6: "Z"}, {20: "Z", 21: "Z"}, {21: "X"},
               {10: "Y", 11: "Y"}, {0: "Z", 1: "X"}]
    masks = [W.parse_pauli("".join(d.get(q, "I") for q in range(n))) for d in strings]
    xm = np.array([m[0] for m in masks], np.uint64)
    zm = np.array([m[1] for m in masks], np.uint64)
    co = rng.normal(0.0, 1.0, len(strings))
    wl = W.single(f"stride{n}", n, gates, theta, (xm, zm, co))
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    g_ref = oracle.grad_adjoint(wl)
    b = qv.Batch(ctx_for(qv, engine="stride"), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    g, _ = b.gradient(qv.QV_ADJOINT)
    check(g, g_ref, prec, s, "adjoint grad")
    b.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_neighbour_and_long_range_terms(qv, prec):
    """A many-term observable on a 20-qubit circuit: neighbour XX, YY and XZ terms, single-qubit Z and X,
    and long-range strings (X0 X19, Y2 Z9 X17, X5 X19, Y6 Z9 X13 Y19), 88 terms, several sharing an x-mask
    (XX with YY, X with XZ): term values, energy and adjoint gradient against the oracle."""
    say(f"neighbour and long-range terms prec={prec}")
    n = 20
    rng = np.random.default_rng(7720)
    wl0 = W.large_hea(n, 2, seed_index=9)
    strings = []
    for i in range(n - 1):
        strings.append({i: "X", i + 1: "X"})
        strings.append({i: "Y", i + 1: "Y"})
        strings.append({i: "X", i + 1: "Z"})
    strings += [{i: "Z"} for i in range(n)] + [{i: "X"} for i in range(0, n, 3)]
    strings += [{0: "X", 19: "X"}, {2: "Y", 9: "Z", 17: "X"}, {5: "X", 19: "X"}, {6: "Y", 9: "Z", 13: "X", 19: "Y"}]
    masks = [W.parse_pauli("".join(d.get(q, "I") for q in range(n))) for d in strings]
    xm = np.array([m[0] for m in masks], np.uint64)
    zm = np.array([m[1] for m in masks], np.uint64)
    co = rng.normal(0.0, 1.0, len(strings))
    wl = W.single("tiles20", n, [tuple(g) for g in wl0.circuit(0)], wl0.theta_of(0), (xm, zm, co))
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    g_ref = oracle.grad_adjoint(wl)
    b = qv.Batch(ctx_for(qv), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(tv, tv_ref, prec, 1.0, "terms")
    check(e, e_ref, prec, s, "energy")
    g, _ = b.gradient(qv.QV_ADJOINT)
    check(g, g_ref, prec, s, "adjoint grad")
    b.close()


def test_error_paths_on_device(qv):
    import ctypes
    say("error paths")
    lib = qv.load()
    ctx = ctx_for(qv)
    wl = W.config1()
    a = qv._Arrays(wl)
    h = ctypes.c_void_p()
    assert lib.qv_batch_create(ctx.h, *a.args(), 0, ctypes.byref(h)) == 0
    e = np.zeros(1)
    assert lib.qv_batch_expectations(h, e.ctypes.data, None, 0) == qv.QV_E_STATE
    assert "set_params" in qv.last_error()
    bad = np.full(80, np.nan)
    assert lib.qv_batch_set_params(h, bad.ctypes.data, 0) == qv.QV_E_INVALID
    out = np.zeros(1 << 10, np.complex64)
    assert lib.qv_batch_state(h, 0, out.ctypes.data, 0) == qv.QV_E_STATE
    assert lib.qv_batch_state(h, 5, out.ctypes.data, 0) == qv.QV_E_INVALID
    assert lib.qv_batch_destroy(h) == 0
    assert qv.Context.__init__ is not None
    with pytest.raises(qv.QvError):
        qv.Context(0, None, '{"engine": "warp"}')
    with pytest.raises(qv.QvError):
        qv.Context(0, None, '{"tile_qubits": 20}')
    with pytest.raises(qv.QvError):
        qv.Context(7, None, None)


@pytest.mark.parametrize("prec,contig", [(0, 1), (0, 2), (0, 3), (1, 2)])
def test_contig_qubits(qv, prec, contig):
    """Tiles whose contiguous low runs are short (contig_qubits 1..3) need a longer run-offset table in
    LDS; energies, terms and adjoint gradients stay at parity."""
    say(f"contig prec={prec} contig={contig}")
    wl = W.random_batch(10, 12, 16, 20, 90, 4, seed_index=45)
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    up = np.linspace(0.5, -1.0, wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    b = qv.Batch(ctx_for(qv, contig_qubits=contig, tile_qubits=10), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g, g_ref, prec, s * np.sum(np.abs(up)), "adjoint grad")


def test_autotune_chooses_fused_block_run(qv, tmp_path, monkeypatch):
    """Under "fusion": "auto" the search times fused-block minimum runs as well; the stored choice (tile,
    contiguous run, block width 4, minimum run) is reused by a cached batch; results at parity."""
    monkeypatch.setenv("QV_TUNE_CACHE", str(tmp_path / "tune.txt"))
    say("autotune fusion")
    wl = W.qcl(n=16, layers=3, samples=6, seed_index=47)
    e_ref, _, _, _ = oracle.expectations(wl)
    b = qv.Batch(ctx_for(qv, autotune="search", fusion="auto"), wl, 0)
    e, _ = b.expectations()
    check(e, e_ref, 0, 1.0, "energies (search)")
    st = b.stats()
    assert st["fuse_min_run"] in (0, 4, 6, 8)
    line = [x for x in (tmp_path / "tune.txt").read_text().split("\n") if x.strip()]
    assert len(line) == 1 and line[0].split()[1:5] == [str(st["tile_qubits"]), str(st["contig_qubits"]), "4",
                                                        str(st["fuse_min_run"])]
    b2 = qv.Batch(ctx_for(qv, autotune="cached", fusion="auto"), wl, 0)
    e2, _ = b2.expectations()
    assert np.array_equal(e, e2)
    assert b2.stats()["fuse_min_run"] == st["fuse_min_run"]
    g_ref = oracle.grad_adjoint(wl)
    check(b2.gradient(qv.QV_ADJOINT)[0], g_ref, 0, float(wl.B), "adjoint grad")


def test_autotune_search_and_cache(qv, tmp_path, monkeypatch):
    """The autotuner times its candidates on the device, keeps the fastest, stores it, and a second batch
    of the same shape reuses the stored choice; results stay at parity either way."""
    monkeypatch.setenv("QV_TUNE_CACHE", str(tmp_path / "tune.txt"))
    say("autotune")
    wl = W.qcl(n=16, layers=2, samples=6, seed_index=46)
    e_ref, _, _, _ = oracle.expectations(wl)
    b = qv.Batch(ctx_for(qv, autotune="search"), wl, 0)
    e, _ = b.expectations()
    check(e, e_ref, 0, 1.0, "energies (search)")
    st = b.stats()
    assert 11 <= st["tile_qubits"] <= 13 and 3 <= st["contig_qubits"] <= 4
    lines = (tmp_path / "tune.txt").read_text().split("\n")
    assert len([x for x in lines if x.strip()]) == 1
    b2 = qv.Batch(ctx_for(qv, autotune="cached"), wl, 0)
    e2, _ = b2.expectations()
    assert np.array_equal(e, e2)
    st2 = b2.stats()
    assert (st2["tile_qubits"], st2["contig_qubits"]) == (st["tile_qubits"], st["contig_qubits"])


@pytest.mark.parametrize("layers", [2, 8])
def test_qcl20_fused_blocks(qv, layers):
    """Fused 4-qubit blocks on MFMA (forward passes) at full size: energies and adjoint gradients against the
    oracle's stored values to the complex64 bound, and the plan really holds fused blocks."""
    say(f"qcl20 fused L={layers}")
    gold = _golden(f"qcl20_L{layers}")
    wl = W.config3(layers)
    b = qv.Batch(ctx_for(qv, fusion=4, tile_qubits=13, graph=False, launch_events=True), wl, 0)
    e, _ = b.expectations(want_terms=False)
    check(e, np.array(gold["energies"]), 0, 1.0, "energies")
    assert any(r["kernel"] == "fuse" for r in b.launch_log())
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=np.array(gold["upstream"]))
    check(g, np.array(gold["grad"]), 0, float(np.sum(np.abs(gold["upstream"]))), "grad")
    passes = qv.plan_circuit(20, wl.circuit(0), 13, qv.QV_C64, 0, fuse_min=4)
    assert sum(p["n_fused"] for p in passes) > 0


ALL_KINDS = [W.H, W.X, W.Y, W.Z, W.S, W.T, W.RX, W.RY, W.RZ, W.CNOT, W.CZ]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"fusion": 2}, {"tile_qubits": 7}, {"fold_cnots": "off"}, {"engine": "lds"},
                                  {"engine": "stride"}])
def test_all_gate_kinds(qv, prec, opts):
    """Random circuits over all eleven gate kinds (every op code of the register segments: dense, real and
    diagonal one-qubit gates on register and thread qubits, CNOT with register or thread control, CZ):
    energies, term values and adjoint and parameter-shift gradients against the oracle."""
    say(f"all kinds prec={prec} opts={opts}")
    wl = W.random_batch(12, 3, 13, 20, 120, 4, seed_index=77, kinds=ALL_KINDS)
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    up = np.linspace(0.5, -1.0, wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    g_ad, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g_ad, g_ref, prec, s * float(np.sum(np.abs(up))), "adjoint grad")
    g_ps, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
    check(g_ps, g_ref, prec, s * float(np.sum(np.abs(up))), "param-shift grad")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"fold_cnots": "off"}, {"fusion": 4}, {"tile_qubits": 8}])
def test_cnot_runs_folded(qv, prec, opts):
    """Hardware-efficient circuits (a CNOT ladder after every rotation layer) and CNOT-heavy random circuits:
    the CNOT runs at register-segment ends fold into the LDS addressing by default. Energies and adjoint
    and parameter-shift gradients against the oracle, with folding on and off."""
    say(f"cnot runs prec={prec} opts={opts}")
    for wl in (W.hea_vqe(12, 5, 6, seed_index=21), W.hea_vqe(14, 3, 6, seed_index=22),
               W.random_batch(8, 9, 13, 40, 160, 4, seed_index=23, kinds=[W.RY, W.RZ, W.CNOT, W.CNOT, W.CNOT])):
        e_ref, _, _, _ = oracle.expectations(wl)
        up = np.linspace(1.0, -0.5, wl.B)
        g_ref = oracle.grad_adjoint(wl, up)
        b = qv.Batch(ctx_for(qv, **opts), wl, prec)
        e, _ = b.expectations(want_terms=False)
        s = obs_scale(wl)
        check(e, e_ref, prec, s, "energy")
        g_ad, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
        check(g_ad, g_ref, prec, s * float(np.sum(np.abs(up))), "adjoint grad")
        g_ps, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
        check(g_ps, g_ref, prec, s * float(np.sum(np.abs(up))), "param-shift grad")


@pytest.mark.parametrize("prec", [1, 0])
def test_adjoint_stops_at_first_trainable_gate(qv, prec):
    """The reverse sweep over a circuit's first pass stops at its first trainable gate. Circuits whose first
    passes start with long runs of fixed gates (and, with small tiles, first passes with no trainable gate at
    all, which skip their segment work and the next-tile prefetch): adjoint gradients against the oracle."""
    say(f"adjoint early stop prec={prec}")
    rng = np.random.default_rng(31)
    circuits = []
    for n in (11, 12, 14):
        g = []
        for _ in range(3 * n):   # fixed prefix: H, CNOT ladders, fixed rotations
            q = int(rng.integers(0, n))
            k = int(rng.integers(0, 3))
            if k == 0:
                g.append(W.gate(W.H, q))
            elif k == 1:
                g.append(W.gate(W.CNOT, q, (q + 1) % n))
            else:
                g.append(W.gate(W.RY, q, -1, -1, float(rng.uniform(0, 6.28))))
        p = 0
        for _ in range(4 * n):
            q = int(rng.integers(0, n))
            kind = [W.RY, W.RZ, W.RX][int(rng.integers(0, 3))]
            g.append(W.gate(kind, q, -1, p, 0.0))
            p += 1
            if rng.random() < 0.3:
                a, b2 = rng.choice(n, size=2, replace=False)
                g.append(W.gate(W.CNOT, int(a), int(b2)))
        circuits.append((n, g, p))
    # a first pass with no trainable gate at all: a fixed block on qubits 0..5 fills a 6-qubit tile
    n, g, p = 12, [], 0
    for i in range(30):
        q = i % 6
        g.append(W.gate(W.H, q) if i % 3 == 0 else
                 (W.gate(W.CNOT, q, (q + 1) % 6) if i % 3 == 1 else W.gate(W.RY, q, -1, -1, 0.1 * i)))
    for i in range(24):
        g.append(W.gate([W.RY, W.RZ][i % 2], 6 + i % 6, -1, p, 0.0))
        p += 1
        if i % 5 == 4:
            g.append(W.gate(W.CNOT, 5, 6 + i % 6))
    gates6 = np.array(g, W.GATE_DTYPE)
    assert qv.plan_circuit(n, gates6, 6, prec, 0)[0]["n_trainable"] == 0
    circuits6 = [(n, g, p)]
    for tile, circs in ((8, circuits), (0, circuits), (6, circuits6)):
        for n, g, p in circs:
            theta = rng.uniform(0, 2 * np.pi, size=p)
            xm, zm, cf = W.random_paulis(rng, 5, n)
            wl = W.single(f"prefix{n}", n, g, theta, (xm, zm, cf))
            g_ref = oracle.grad_adjoint(wl)
            opts = {"tile_qubits": tile} if tile else {}
            b = qv.Batch(ctx_for(qv, **opts), wl, prec)
            g_ad, _ = b.gradient(qv.QV_ADJOINT)
            check(g_ad, g_ref, prec, obs_scale(wl), f"adjoint grad n={n} tile={tile}")


def test_qcl20_full_size_complex128(qv):
    """20 qubits, 64 samples, 2 layers in complex128 (register tiles of 2^12 amplitudes, 8 per thread):
    every energy and every gradient component to 1e-12 against the oracle's stored values."""
    say("qcl20 L=2 c128")
    gold = _golden("qcl20_L2")
    wl = W.config3(2)
    b = qv.Batch(ctx_for(qv), wl, 1)
    e, _ = b.expectations(want_terms=False)
    ee = check(e, np.array(gold["energies"]), 1, 1.0, "energies")
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=np.array(gold["upstream"]))
    ge = check(g, np.array(gold["grad"]), 1, 1.0, "grad")
    say(f"  max |dE| {ee:.2e}  max |dg| {ge:.2e}")


@pytest.mark.parametrize("n", [20, 22, 24])
@pytest.mark.parametrize("prec", [0, 1])
def test_hea_ladder_full_depth(qv, n, prec):
    """The 32-qubit workload's shape (10 hardware-efficient layers, trainable RY, fixed RZ, open ZZ chain)
    at 20, 22 and 24 qubits against the oracle's stored energy, term values and full gradient; complex64
    with fused blocks of >= 8 gates (the option the 32-qubit figures use), complex128 unfused."""
    say(f"hea ladder n={n} prec={prec}")
    gold = _golden(f"hea{n}_L10")
    wl = W.large_hea(n, 10)
    opts = {"fusion": "8", "tile_qubits": 13} if prec == 0 else {}
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    s = float(n - 1)
    ee = check(e, np.array(gold["energies"]), prec, s, "energy")
    te = check(tv, np.array(gold["term_values"]), prec, 1.0, "ZZ terms")
    g, _ = b.gradient(qv.QV_ADJOINT)
    ge = check(g, np.array(gold["grad"]), prec, s, "grad")
    if prec == 0:
        assert sum(p["n_fused"] for p in qv.plan_circuit(n, wl.circuit(0), 13, 0, 0, fuse_min=8)) > 0
    say(f"  max |dE| {ee:.2e}  max |dterm| {te:.2e}  max |dg| {ge:.2e}")
    b.close()


def test_hea32_L10_fused_matches_unfused(qv):
    """32 qubits (a 32 GiB complex64 state), 10 layers: the energy, the 31 ZZ terms and the 320-component
    gradient with fused MFMA blocks of >= 8 gates agree with the unfused path to the complex64 bound (the
    oracle cannot hold this state; the 20-24-qubit ladder pins the same circuit shape against it)."""
    say("hea32 L10 fused vs unfused")
    wl = W.config5()
    out = {}
    for fusion in ("off", "8"):
        b = qv.Batch(ctx_for(qv, fusion=fusion, tile_qubits=13), wl, 0)
        e, tv = b.expectations()
        g, _ = b.gradient(qv.QV_ADJOINT)
        out[fusion] = (e, tv, g)
        say(f"  fusion {fusion}: E {e[0]:.9f}")
        b.close()
    (e0, tv0, g0), (e1, tv1, g1) = out["off"], out["8"]
    # both sides carry complex64 rounding, so each is held to the bound against the other
    ee = check(e1, e0, 0, 31.0, "energy")
    te = check(tv1, tv0, 0, 1.0, "ZZ terms")
    ge = check(g1, g0, 0, 31.0, "grad")
    say(f"  max |dE| {ee:.2e}  max |dterm| {te:.2e}  max |dg| {ge:.2e}")
