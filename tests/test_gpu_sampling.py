"""GPU parity of shots and bit-string counts (qv_batch_sample; Section 3.1: a circuit's result is the table
of observed bit strings and their counts; Section 4.2) against the CPU oracle's inverse transform sampling
(oracle/sampling.py) on the same uniforms.

Both sides take shot j of circuit b as the first bit string x with C(x) > u C(last), C the running sum of
|psi|^2 in bit-string order. Their running sums differ by rounding (complex128) or by the complex64
amplitudes' error (a distribution within 1e-5 in L1), so a shot whose u C(last) lies within that band of a
bin edge may land in the neighbouring bin: every shot must lie in the bin whose oracle bounds, widened by
the band, hold u C(last); shots farther than the band from both edges of the oracle's bin must agree
exactly; the counts must be those of the library's own shots, in increasing bit-string order, and differ
from the oracle's by at most two per shot inside the band. A chi-square test checks a million shots
against the exact distribution.
"""
import json
import sys

import numpy as np
import pytest
from scipy import stats

from oracle import sampling as OS
from paper_2406_03466_amd import workloads as W

pytestmark = pytest.mark.gpu

BAND = {1: 1e-12, 0: 2e-5}


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


def check_against_oracle(wl, shots, u, smp, per, prec):
    """The banded bin test per shot, exact agreement outside the band, and the counts."""
    band = BAND[prec]
    in_band = 0
    for b in range(wl.B):
        q = OS.distribution(int(wl.n_qubits[b]), np.ascontiguousarray(wl.circuit(b)),
                            np.asarray(wl.theta_of(b), np.float64))
        c = OS.cumulative(q)
        lo_edge = np.concatenate([[0.0], c[:-1]])
        target = u[b * shots:(b + 1) * shots] * c[-1]
        xo = OS.sample_from(q, u[b * shots:(b + 1) * shots])
        xg = smp[b * shots:(b + 1) * shots]
        assert ((xg >= 0) & (xg < q.size)).all()
        assert ((lo_edge[xg] - band <= target) & (target < c[xg] + band)).all(), f"circuit {b}: shot outside its bin"
        near = (np.abs(target - lo_edge[xo]) <= band) | (np.abs(target - c[xo]) <= band)
        assert np.array_equal(xg[~near], xo[~near]), f"circuit {b}: {int(np.sum(xg[~near] != xo[~near]))} shots differ"
        in_band += int(near.sum())
        bits, cnt = per[b]
        ub, uc = np.unique(xg, return_counts=True)
        assert np.array_equal(bits.astype(np.int64), ub) and np.array_equal(cnt, uc), f"circuit {b}: counts"
        ob, oc = OS.counts_of(xo)
        full_o = np.zeros(q.size, np.int64)
        full_o[ob.astype(np.int64)] = oc
        full_g = np.zeros(q.size, np.int64)
        full_g[ub] = uc
        assert np.abs(full_o - full_g).sum() <= 2 * int(near.sum())
    return in_band


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("opts", [{}, {"engine": "stride"}, {"tile_qubits": 8}])
def test_sample_uneven_batch(qv, prec, opts):
    """Circuits of 3..14 qubits and 5..60 gates with their own parameters: every shot and every count."""
    say(f"sample uneven prec={prec} opts={opts}")
    wl = W.random_batch(8, 3, 14, 5, 60, 1, seed_index=61)
    shots = 20000
    u = np.random.default_rng(62).random(wl.B * shots)
    b = qv.Batch(ctx_for(qv, **opts), wl, prec)
    smp, per = b.sample(shots, u)
    nb = check_against_oracle(wl, shots, u, smp, per, prec)
    say(f"  shots within the band: {nb} of {wl.B * shots}")


@pytest.mark.parametrize("prec", [1, 0])
def test_sample_closed_forms(qv, prec):
    """H on all 20 qubits: the shot is the integer part of 2^20 u (uniforms kept off the bin edges); a
    point mass (X on qubits 1, 4, 19) draws only its bit string."""
    say(f"sample closed forms prec={prec}")
    n = 20
    rng = np.random.default_rng(63)
    k = rng.integers(0, 1 << n, 50000)
    u = (k + rng.uniform(0.05, 0.95, k.size)) / (1 << n)
    wl = W.single("hall", n, [W.gate(W.H, q) for q in range(n)])
    smp, per = qv.Batch(ctx_for(qv), wl, prec).sample(k.size, u)
    np.testing.assert_array_equal(smp, k)
    wl2 = W.single("point", n, [W.gate(W.X, 1), W.gate(W.X, 4), W.gate(W.X, 19)])
    smp2, per2 = qv.Batch(ctx_for(qv), wl2, prec).sample(k.size, rng.random(k.size))
    x = (1 << 1) | (1 << 4) | (1 << 19)
    assert (smp2 == x).all() and per2[0][0].tolist() == [x] and per2[0][1].tolist() == [k.size]


@pytest.mark.parametrize("prec", [0, 1])
def test_sample_ddcl20_chi_square(qv, prec):
    """Table 2's smallest DDCL circuit (20 qubits, 10 layers): a million shots against the oracle shot by
    shot, and their counts against the exact distribution by a chi-square test."""
    say(f"sample ddcl20 prec={prec}")
    wl = W.ddcl(20, 10)
    shots = 1 << 20
    u = np.random.default_rng(64).random(shots)
    b = qv.Batch(ctx_for(qv), wl, prec)
    smp, per = b.sample(shots, u)
    nb = check_against_oracle(wl, shots, u, smp, per, prec)
    q = OS.distribution(20, np.ascontiguousarray(wl.circuit(0)), wl.theta)
    full = np.zeros(q.size)
    bits, cnt = per[0]
    full[bits.astype(np.int64)] = cnt
    exp = shots * q / q.sum()
    keep = exp >= 5
    # pool the bins with small expectations into one
    obs_k = np.append(full[keep], full[~keep].sum())
    exp_k = np.append(exp[keep], exp[~keep].sum())
    chi2 = float(np.sum((obs_k - exp_k) ** 2 / exp_k))
    p = stats.chi2.sf(chi2, obs_k.size - 1)
    say(f"  within band {nb}, chi2 {chi2:.1f} on {obs_k.size - 1} dof, p {p:.3g}")
    assert p > 1e-4


def test_sample_device_pointers_match_host(qv):
    import torch
    say("sample device pointers")
    wl = W.random_batch(4, 5, 12, 10, 40, 1, seed_index=65)
    shots = 4096
    u = np.random.default_rng(66).random(wl.B * shots)
    b = qv.Batch(ctx_for(qv), wl, 0)
    smp, per = b.sample(shots, u)
    dev = torch.device("cuda")
    tu = torch.tensor(u, dtype=torch.float64, device=dev)
    ts = torch.empty(wl.B * shots, dtype=torch.int64, device=dev)
    tb = torch.empty(wl.B * shots, dtype=torch.int64, device=dev)
    tc = torch.empty(wl.B * shots, dtype=torch.int64, device=dev)
    tn = torch.empty(wl.B, dtype=torch.int64, device=dev)
    b.sample(shots, tu, ts, tb, tc, tn)
    torch.cuda.synchronize()
    assert np.array_equal(ts.cpu().numpy(), smp)
    nd = tn.cpu().numpy()
    bits, cnt = tb.cpu().numpy(), tc.cpu().numpy()
    for c in range(wl.B):
        assert np.array_equal(bits[c * shots:c * shots + nd[c]].astype(np.uint64), per[c][0])
        assert np.array_equal(cnt[c * shots:c * shots + nd[c]], per[c][1])


def test_sample_rejects_bad_arguments(qv):
    say("sample errors")
    wl = W.random_batch(2, 4, 6, 5, 10, 1, seed_index=67)
    b = qv.Batch(ctx_for(qv), wl, 0)
    u = np.full(2 * 10, 0.5)
    u[7] = 1.0
    with pytest.raises(qv.QvError):
        b.sample(10, u)
    u[7] = -0.1
    with pytest.raises(qv.QvError):
        b.sample(10, u)
    lib = qv.load()
    ok = np.full(2 * 10, 0.25)
    bits = np.zeros(20, np.uint64)
    assert lib.qv_batch_sample(b.h, 10, ok.ctypes.data, None, bits.ctypes.data, None, None, 0) == qv.QV_E_INVALID
    assert lib.qv_batch_sample(b.h, 0, ok.ctypes.data, None, None, None, None, 0) == qv.QV_E_INVALID
    smp, per = b.sample(10, ok)
    assert len(per) == 2 and all(int(c.sum()) == 10 for _, c in per)
