"""The probability path of Section 4.2 on the CPU: the DDCL-shaped workload's sizes against Table 2, the
oracle's Jensen-Shannon divergence (Eq. 3) against scipy and closed forms, its output distributions on the
Bell-pair preparation, and its parameter-shift gradient against central finite differences."""
import json
import os

import numpy as np
import pytest
from scipy.spatial import distance

import oracle
from oracle import ddcl as OD
from paper_2406_03466_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ddcl_table2.json")


@pytest.mark.parametrize("row", json.load(open(GOLDEN))["rows"])
def test_sizes_match_table2(row):
    """N_theta = 60 N_q at 10 layers and 2 N_theta circuits per parameter update, as printed in Table 2."""
    nq, nth, circ = row
    g, P = W.ddcl_layers(nq, json.load(open(GOLDEN))["layers"])
    assert P == nth and 2 * P == circ
    assert sum(1 for x in g if x[3] >= 0) == nth


def _dists(rng, n, zeros=0.3):
    p = rng.exponential(size=n) * (rng.random(n) >= zeros)
    q = rng.exponential(size=n) * (rng.random(n) >= zeros)
    return p / p.sum(), q / q.sum()


@pytest.mark.parametrize("seed", range(6))
def test_js_matches_scipy(seed):
    """scipy's Jensen-Shannon distance (natural log) squared is the divergence of Eq. 3; zeros on either
    side included. Catches a wrong mixture M, a missing factor 1/2 or a dropped term."""
    rng = np.random.default_rng(seed)
    p, q = _dists(rng, 64 + 37 * seed)
    assert OD.js_divergence(p, q) == pytest.approx(distance.jensenshannon(p, q) ** 2, rel=1e-12, abs=1e-15)


def test_js_closed_forms():
    rng = np.random.default_rng(3)
    p, q = _dists(rng, 50)
    assert OD.js_divergence(p, p) == 0.0
    assert OD.js_divergence(p, q) == pytest.approx(OD.js_divergence(q, p), rel=1e-14)
    assert 0.0 < OD.js_divergence(p, q) < np.log(2.0)
    a = np.array([0.5, 0.5, 0.0, 0.0])
    b = np.array([0.0, 0.0, 0.25, 0.75])
    assert OD.js_divergence(a, b) == pytest.approx(np.log(2.0), rel=1e-15)   # disjoint supports
    # two-point distributions: JS of (1, 0) against (t, 1 - t) in closed form
    t = 0.3
    want = 0.5 * (np.log(2 / (1 + t)) + t * np.log(2 * t / (1 + t)) + (1 - t) * np.log(2.0))
    assert OD.js_divergence([1.0, 0.0], [t, 1 - t]) == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("n", [2, 6, 9])
def test_bell_pair_distribution(n):
    """No layers: Bell pairs on (0,1), (2,3), ...; every pair's two bits agree with probability 1/2 each
    value, an unpaired last qubit stays 0."""
    g, P = W.ddcl_layers(n, 0)
    assert P == 0
    wl = W.single("bell", n, g)
    q = OD.probabilities(wl)
    want = np.zeros(1 << n)
    for x in range(1 << n):
        ok = all(((x >> i) & 1) == ((x >> (i + 1)) & 1) for i in range(0, n - 1, 2))
        if n % 2 and (x >> (n - 1)) & 1:
            ok = False
        want[x] = 0.5 ** (n // 2) if ok else 0.0
    np.testing.assert_allclose(q, want, atol=1e-15)


def test_probabilities_are_the_squared_state():
    wl = W.ddcl(5, 2, sizes=[3, 5])
    q = OD.probabilities(wl)
    psi = np.concatenate([oracle.final_state(int(wl.n_qubits[b]), np.ascontiguousarray(wl.circuit(b)),
                                             wl.theta_of(b)) for b in range(wl.B)])
    np.testing.assert_allclose(q, np.abs(psi) ** 2, atol=1e-15)
    np.testing.assert_allclose([q[:8].sum(), q[8:].sum()], [1.0, 1.0], atol=1e-13)


def test_js_gradient_matches_finite_differences():
    """Chain rule through the parameter-shifted probabilities against central differences of the loss
    sum_b u_b JS_b (h = 1e-4; truncation ~1e-9). Catches a wrong derivative of the divergence, a wrong
    sign of the shift or a wrong parameter slice."""
    wl = W.ddcl(4, 1, sizes=[3, 4])
    t = wl.extra["target"]
    u = np.array([0.7, -1.3])
    g = OD.js_grad_param_shift(wl, t, u)
    h = 1e-4
    fd = np.zeros_like(g)
    for j in range(len(g)):
        th = wl.theta.copy()
        vals = []
        for s in (1, -1):
            th2 = th.copy()
            th2[j] += s * h
            vals.append(float(np.dot(u, OD.js_values(W.with_theta(wl, th2), t))))
        fd[j] = (vals[0] - vals[1]) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=2e-8)
    sub = OD.js_grad_param_shift(wl, t, u, only={1, 30})
    assert sub[1] == g[1] and sub[30] == g[30] and np.count_nonzero(sub) <= 2


@pytest.mark.parametrize("theta,target_index,want_js,want_g", [
    (0.0, 2, 0.0, 0.0),                    # target reached exactly: JS = 0, flat
    (0.0, 3, np.log(2.0), 0.0),            # disjoint supports: JS = log 2, flat at theta = 0
    (np.pi / 2, 2, None, None),            # general point: closed form below
])
def test_degenerate_distributions(theta, target_index, want_js, want_g):
    """X on qubit 1, then RY(theta) on qubit 0: Q(2) = cos^2(theta/2), Q(3) = sin^2(theta/2), zero
    elsewhere; target a point mass. JS and its derivative in closed form (0 log 0 = 0)."""
    wl = W.single("deg", 2, [W.gate(W.X, 1), W.gate(W.RY, 0, -1, 0)], [theta])
    t = np.zeros(4)
    t[target_index] = 1.0
    c, s = np.cos(theta / 2) ** 2, np.sin(theta / 2) ** 2
    q = np.array([0.0, 0.0, c, s])
    if want_js is None:
        # P = delta_2: JS = 1/2 [log(2/(1+c)) + c log(2c/(1+c)) + s log 2]
        want_js = 0.5 * (np.log(2 / (1 + c)) + c * np.log(2 * c / (1 + c)) + s * np.log(2.0))
        # d/dtheta with dc = -sin(theta)/2, ds = +sin(theta)/2 (the c/(1+c) terms cancel)
        dc, ds = -np.sin(theta) / 2, np.sin(theta) / 2
        want_g = 0.5 * (dc * np.log(2 * c / (1 + c)) + ds * np.log(2.0))
    np.testing.assert_allclose(OD.probabilities(wl), q, atol=1e-15)
    assert OD.js_values(wl, t)[0] == pytest.approx(want_js, abs=1e-15)
    assert OD.js_grad_param_shift(wl, t)[0] == pytest.approx(want_g, abs=1e-15)
