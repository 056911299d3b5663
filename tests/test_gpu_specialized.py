"""GPU parity of the tile passes generated at run time (context option "specialize"): the same workloads as
the general kernels, against the oracle to the same bounds, and against the general kernels themselves.
The launch log shows the generated kernels ran.
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
GEN = ("rtile_gen", "rtile_adj_gen")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qv(tmp_path_factory):
    import torch
    assert torch.cuda.is_available()
    os.environ["QV_GEN_CACHE"] = str(tmp_path_factory.mktemp("gen_cache"))
    from paper_2406_03466_amd import qvpu
    qvpu.load()
    return qvpu


def ctx_for(qv, **opts):
    import torch
    return qv.Context(0, torch.cuda.current_stream().cuda_stream, json.dumps(opts) if opts else None)


def check(x, ref, prec, scale, what):
    x, ref = np.asarray(x), np.asarray(ref)
    err = np.abs(x - ref)
    bad = err > (1e-12 if prec == 1 else 1e-5 * np.maximum(np.abs(ref), scale))
    assert not bad.any(), f"{what}: max err {err.max():.3e} at {int(np.argmax(err))}"
    return float(err.max()) if err.size else 0.0


def gen_launches(b):
    return [r for r in b.launch_log() if r["kernel"] in GEN]


def obs_scale(wl):
    if wl.obs_shared:
        return float(np.sum(np.abs(wl.coeff)))
    return max(float(np.sum(np.abs(wl.terms(b)[2]))) for b in range(wl.B))


def _golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        return json.load(f)


@pytest.mark.parametrize("layers,spec,inner", [(2, "on", "f32"), (8, "on", "f32"), (8, "adjoint", "f32"),
                                               (8, "auto", "f32"), (2, "adjoint", "f64"), (8, "adjoint", "f64")])
def test_qcl20_generated_vs_general_and_oracle(qv, layers, spec, inner):
    """20 qubits, 64 samples, complex64 in the benchmark's configuration (fused blocks of >= 8 gates, tile
    13), generated passes in both sweeps or in the adjoint only, adjoint inner products in FP32 or FP64:
    energies and the MSE-loss gradient against the stored oracle values, and against the general kernels
    (equal up to floating-point contraction and the inner products' precision)."""
    say(f"qcl20 L={layers} specialize={spec} inner={inner}")
    gold = _golden(f"qcl20_L{layers}")
    wl = W.config3(layers)
    up = np.array(gold["upstream"])
    out = {}
    for mode, inn in (("off", "f32"), (spec, inner)):
        b = qv.Batch(ctx_for(qv, fusion="8", tile_qubits=13, graph=False, launch_events=True, specialize=mode,
                             adjoint_inner=inn), wl, 0)
        e, _ = b.expectations(want_terms=False)
        g, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
        kinds = {r["kernel"] for r in gen_launches(b)}
        want = {"off": set(), "adjoint": {"rtile_adj_gen"}, "on": {"rtile_gen", "rtile_adj_gen"}}.get(mode)
        if want is not None:
            assert kinds == want, kinds
        else:   # auto: generated kernels only in the levels where they timed faster
            assert kinds <= {"rtile_gen", "rtile_adj_gen"}, kinds
        out[mode] = (e, g)
        b.close()
    ee = check(out[spec][0], gold["energies"], 0, 1.0, "energies")
    ge = check(out[spec][1], gold["grad"], 0, float(np.sum(np.abs(up))), "grad")
    d_e = float(np.max(np.abs(out[spec][0] - out["off"][0])))
    d_g = float(np.max(np.abs(out[spec][1] - out["off"][1])))
    say(f"  vs oracle |dE| {ee:.2e} |dg| {ge:.2e}; vs general kernels |dE| {d_e:.2e} |dg| {d_g:.2e}")
    assert d_e <= 1e-6 and d_g <= 1e-6 * float(np.sum(np.abs(up)))


def test_qcl20_c128_generated(qv):
    """The same in complex128 (2 layers, 8 amplitudes per thread): every value to 1e-12."""
    say("qcl20 c128 generated")
    gold = _golden("qcl20_L2")
    wl = W.config3(2)
    b = qv.Batch(ctx_for(qv, specialize="on", graph=False, launch_events=True), wl, 1)
    e, _ = b.expectations(want_terms=False)
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=np.array(gold["upstream"]))
    assert gen_launches(b)
    ee = check(e, gold["energies"], 1, 1.0, "energies")
    ge = check(g, gold["grad"], 1, 1.0, "grad")
    say(f"  |dE| {ee:.2e} |dg| {ge:.2e}")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"tile_qubits": 6}, {"fusion": 2}, {"fusion": 3, "tile_qubits": 8}])
def test_c1_generated(qv, prec, opts):
    """10 qubits, 4 layers, 20 random Pauli strings: energies, terms, and adjoint and parameter-shift
    gradients (the shifted variants run the same generated passes with a moved gate)."""
    say(f"c1 generated prec={prec} opts={opts}")
    wl = W.config1()
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    g_ref = oracle.grad_param_shift(wl)
    b = qv.Batch(ctx_for(qv, specialize="on", **opts), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energies")
    check(tv, tv_ref, prec, 1.0, "terms")
    check(b.gradient(qv.QV_ADJOINT)[0], g_ref, prec, s, "adjoint grad")
    check(b.gradient(qv.QV_PARAM_SHIFT)[0], g_ref, prec, s, "param-shift grad")


@pytest.mark.parametrize("prec", [1, 0])
def test_c1_auto_timed_levels(qv, prec):
    """"specialize": "auto": the forward levels of the base circuits and of every chunk of parameter-shift
    variants, and the reverse levels, are each timed with both kinds of kernel on their first call, then keep
    the faster. Energies, terms and both gradients against the oracle, twice (the second call runs the
    kernels chosen by the first)."""
    say(f"c1 auto prec={prec}")
    wl = W.config1()
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    g_ref = oracle.grad_param_shift(wl)
    b = qv.Batch(ctx_for(qv, specialize="auto", fusion=2), wl, prec)
    s = obs_scale(wl)
    for _ in range(2):
        e, tv = b.expectations()
        check(e, e_ref, prec, s, "energies")
        check(tv, tv_ref, prec, 1.0, "terms")
        check(b.gradient(qv.QV_PARAM_SHIFT)[0], g_ref, prec, s, "param-shift grad")
        check(b.gradient(qv.QV_ADJOINT)[0], g_ref, prec, s, "adjoint grad")
    b.close()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("tile", [None, 8])
def test_uneven_batch_generated(qv, prec, tile):
    """Circuits of 2..16 qubits and 0..80 gates, every one with its own structure: levels of several passes
    keep the general kernels, levels of one pass run generated ones; all gate kinds."""
    say(f"uneven generated prec={prec} tile={tile}")
    wl = W.random_batch(24, 2, 16, 0, 80, 5, seed_index=41, kinds=list(range(11)))
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    up = np.linspace(-1.0, 1.5, wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    opts = {"specialize": "on"}
    if tile:
        opts["tile_qubits"] = tile
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energies")
    check(tv, tv_ref, prec, 1.0, "terms")
    check(b.gradient(qv.QV_ADJOINT, upstream=up)[0], g_ref, prec, s * np.sum(np.abs(up)), "adjoint grad")
    check(b.gradient(qv.QV_PARAM_SHIFT, upstream=up)[0], g_ref, prec, s * np.sum(np.abs(up)), "param-shift grad")


@pytest.mark.parametrize("n", [20, 24])
@pytest.mark.parametrize("prec", [0, 1])
def test_hea_ladder_generated(qv, n, prec):
    """The 32-qubit workload's shape at 20 and 24 qubits, 10 layers, against the stored oracle values."""
    say(f"hea ladder generated n={n} prec={prec}")
    gold = _golden(f"hea{n}_L10")
    wl = W.large_hea(n, 10)
    opts = {"fusion": "8", "tile_qubits": 13} if prec == 0 else {}
    b = qv.Batch(ctx_for(qv, specialize="on", **opts), wl, prec)
    e, tv = b.expectations()
    check(e, gold["energies"], prec, n - 1.0, "energy")
    check(tv, gold["term_values"], prec, 1.0, "terms")
    check(b.gradient(qv.QV_ADJOINT)[0], gold["grad"], prec, n - 1.0, "grad")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("spec", ["on", "auto"])
def test_mcvqe_and_ddcl_generated(qv, prec, spec):
    """MC-VQE at 16 qubits (CIS preparation, merged entanglers, 92 terms; adjoint and parameter-shift mean
    energy gradients) and the DDCL circuit at 12 qubits (Jensen-Shannon gradient by both rules), with
    generated passes everywhere or where they timed faster (the divergence calls time their own levels)."""
    from oracle import ddcl as OD
    say(f"mcvqe/ddcl generated prec={prec} specialize={spec}")
    wl = W.mcvqe(16)
    up = np.full(wl.B, 1.0 / wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    b = qv.Batch(ctx_for(qv, specialize=spec), wl, prec)
    s = float(np.abs(wl.coeff).sum())
    check(b.gradient(qv.QV_ADJOINT, upstream=up)[0], g_ref, prec, s, "mcvqe adjoint")
    check(b.gradient(qv.QV_PARAM_SHIFT, upstream=up)[0], g_ref, prec, s, "mcvqe param-shift")
    wl2 = W.ddcl(12, 3)
    t = wl2.extra["target"]
    g2 = OD.js_grad_param_shift(wl2, t)
    b2 = qv.Batch(ctx_for(qv, specialize=spec), wl2, prec)
    for method in (qv.QV_ADJOINT, qv.QV_PARAM_SHIFT):
        js, g = b2.js_gradient(t, method)
        check(js, OD.js_values(wl2, t), prec, 1.0, "divergence")
        check(g, g2, prec, 1.0, f"js gradient method {method}")
