"""GPU tests of the persistent launch mode: every register-tiled pass of a sweep in one launch, resident
workgroups taking tiles from a queue in level order with bounded per-circuit waits (the batch schedule of
Section 3.2 and Section 4.1, where each virtual QPU works through its segment of the circuit vector, as one
GPU's share).

Results are checked against the oracle to the same bounds as the per-level launches, and bitwise against
the per-level launches where both run the same kernels in the same summation order.
"""
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
    err = np.abs(x - ref)
    bad = err > (1e-12 if prec == 1 else 1e-5 * np.maximum(np.abs(ref), scale))
    assert not bad.any(), f"{what}: max err {err.max():.3e} at {int(np.argmax(err))}"


def obs_scale(wl):
    if wl.obs_shared:
        return float(np.sum(np.abs(wl.coeff)))
    return max(float(np.sum(np.abs(wl.terms(b)[2]))) for b in range(wl.B))


def persistent_launches(b):
    return [r for r in b.launch_log() if r["kernel"] in ("rtile_persist", "rtile_adj_persist")]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("tile", [None, 6])
def test_c1_gradients_persistent(qv, prec, tile):
    """10 qubits, 4 layers: one whole-state pass (default tile) or many levels with waits (tile 6); adjoint
    and parameter-shift gradients and energies against the oracle."""
    say(f"c1 persistent prec={prec} tile={tile}")
    wl = W.config1()
    g_ref = oracle.grad_param_shift(wl)
    e_ref, _, _, _ = oracle.expectations(wl)
    opts = {"launch": "persistent"}
    if tile:
        opts["tile_qubits"] = tile
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    g_ad, e_ad = b.gradient(qv.QV_ADJOINT)
    g_ps, e_ps = b.gradient(qv.QV_PARAM_SHIFT)
    s = obs_scale(wl)
    check(g_ad, g_ref, prec, s, "adjoint grad")
    check(g_ps, g_ref, prec, s, "param-shift grad")
    check(e_ad, e_ref, prec, s, "energy (adjoint call)")
    check(e_ps, e_ref, prec, s, "energy (param-shift call)")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("tile", [9, None])
def test_uneven_batch_persistent(qv, prec, tile):
    """Circuits of 2..16 qubits and 0..80 gates, own parameters, upstream weights: energies, terms, states
    and both gradient rules."""
    say(f"uneven persistent prec={prec} tile={tile}")
    wl = W.random_batch(24, 2, 16, 0, 80, 5, seed_index=41)
    e_ref, tv_ref, _, _ = oracle.expectations(wl)
    up = np.linspace(-1.0, 1.5, wl.B)
    g_ref = oracle.grad_adjoint(wl, up)
    opts = {"launch": "persistent"}
    if tile is not None:
        opts["tile_qubits"] = tile
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    e, tv = b.expectations()
    s = obs_scale(wl)
    check(e, e_ref, prec, s, "energy")
    check(tv, tv_ref, prec, 1.0, "terms")
    for c in [0, 5, 11, 23]:
        n = int(wl.n_qubits[c])
        err = np.max(np.abs(b.state(c) - oracle.final_state(n, wl.circuit(c), wl.theta_of(c))))
        assert err < (1e-13 if prec == 1 else 1e-5), (c, err)
    g, _ = b.gradient(qv.QV_ADJOINT, upstream=up)
    check(g, g_ref, prec, s * np.sum(np.abs(up)), "adjoint grad")
    g2, _ = b.gradient(qv.QV_PARAM_SHIFT, upstream=up)
    check(g2, g_ref, prec, s * np.sum(np.abs(up)), "param-shift grad")


def _levels_vs_persistent(qv, wl, prec, opts, calls):
    out = []
    for launch in ["levels", "persistent"]:
        b = qv.Batch(ctx_for(qv, launch=launch, graph=False, launch_events=True, **opts), wl, prec)
        res = [f(b) for f in calls]
        if launch == "persistent":
            assert persistent_launches(b), "no persistent launch was recorded"
        out.append(res)
        b.close()
    for a, r in zip(out[1], out[0]):
        assert np.array_equal(a, r)
    return out[0]


@pytest.mark.parametrize("layers", [2, 8])
def test_qcl20_persistent_matches_levels_bitwise(qv, layers):
    """20 qubits, 64 samples: every forward and reverse sweep in one launch gives bit-identical energies and
    adjoint gradients to one launch per level (the same tile kernels in the same order per tile)."""
    say(f"qcl20 persistent vs levels L={layers}")
    wl = W.config3(layers)
    up = np.linspace(-0.02, 0.03, wl.B)
    _levels_vs_persistent(qv, wl, 0, {"tile_qubits": 13},
                          [lambda b: b.expectations(want_terms=False)[0],
                           lambda b: b.gradient(qv.QV_ADJOINT, upstream=up)[0]])


@pytest.mark.parametrize("prec", [0, 1])
def test_c2_persistent(qv, prec):
    """16 qubits, 8 layers, 100 terms: the 513-circuit parameter-shift gradient with each sweep of a chunk
    in one launch; bitwise equal to per-level launches and within the bound of the oracle."""
    say(f"c2 persistent prec={prec}")
    wl = W.config2()
    g_ref = oracle.grad_adjoint(wl)
    g_lv, = _levels_vs_persistent(qv, wl, prec, {"tile_qubits": 12 if prec else 13},
                                  [lambda b: b.gradient(qv.QV_PARAM_SHIFT)[0]])
    check(g_lv, g_ref, prec, obs_scale(wl), "param-shift grad")


def test_random1024_persistent(qv):
    """1024 random circuits of 8..22 qubits and 10..200 gates (complex64): one forward launch for the whole
    uneven batch, bitwise equal to per-level launches."""
    say("random1024 persistent")
    wl = W.config4()
    _levels_vs_persistent(qv, wl, 0, {}, [lambda b: b.expectations()[0], lambda b: b.expectations()[1]])


def test_wait_time_out_reports_error(qv):
    """A dependency count that can never be met (forced from the host with wait_extra) makes the waits run
    out after wait_ms; the launch skips the remaining work and ends, the call reports QV_E_DEVICE, and a
    following call on a normal context is correct again."""
    say("persistent time-out")
    wl = W.qcl(n=14, layers=2, samples=4, seed_index=45)
    b = qv.Batch(ctx_for(qv, launch="persistent", tile_qubits=8, wait_ms=2, wait_extra=1), wl, 0)
    with pytest.raises(qv.QvError) as ei:
        b.expectations()
    assert "gave up waiting" in str(ei.value)
    b.close()
    b2 = qv.Batch(ctx_for(qv, launch="persistent", tile_qubits=8), wl, 0)
    e, _ = b2.expectations()
    e_ref, _, _, _ = oracle.expectations(wl)
    check(e, e_ref, 0, 1.0, "energies after a time-out")
