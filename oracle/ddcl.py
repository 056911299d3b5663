"""ORACLE (test infrastructure only; only the test suite, the smoke check and the benchmark's CPU leg may
use it): the probability path of the data-driven circuit-learning application (Section 4.2), by the plain
definitions, in float64 / complex128 on the CPU.

* output distribution of a circuit: P_theta(b) = |<b|U(theta)|0>|^2 for every bit string b, from the
  oracle's state vector (Section 4.2: running a circuit yields the distribution over all 2^n bit strings);
* Jensen-Shannon divergence, Eq. 3: JS = 1/2 sum_b [P(b) log(P(b)/M(b)) + Q(b) log(Q(b)/M(b))],
  M = (P + Q)/2, natural logarithm, 0 log 0 = 0;
* its gradient the way the paper obtains it, by the parameter-shift rule (2 N_theta circuits per gradient,
  Table 2): every probability is the expectation of a projector, so dQ(b)/dtheta_j = [Q_+(b) - Q_-(b)]/2
  exactly, and dJS/dtheta_j = sum_b dJS/dQ(b) dQ(b)/dtheta_j with dJS/dQ(b) = log(Q(b)/M(b))/2 (the
  terms in dM/dQ cancel); where Q(b) = 0 the product is 0, since dQ(b)/dtheta = 0 at a minimum of Q(b).
"""
from __future__ import annotations

import numpy as np

from . import final_state


def _circuit(wl, b):
    return np.ascontiguousarray(wl.circuit(b)), np.asarray(wl.theta_of(b), np.float64)


def probabilities(wl) -> np.ndarray:
    """Output distributions of every circuit of the batch, concatenated in circuit order."""
    out = []
    for b in range(wl.B):
        g, th = _circuit(wl, b)
        psi = final_state(int(wl.n_qubits[b]), g, th)
        out.append(np.abs(psi) ** 2)
    return np.concatenate(out) if out else np.zeros(0)


def js_divergence(p, q) -> float:
    """Eq. 3 for two distributions over the same bit strings."""
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    m = 0.5 * (p + q)
    s = 0.0
    for v in (p, q):
        nz = v > 0
        s += float(np.sum(v[nz] * np.log(v[nz] / m[nz])))
    return 0.5 * s


def _offsets(wl):
    off = np.zeros(wl.B + 1, np.int64)
    off[1:] = np.cumsum([1 << int(n) for n in wl.n_qubits])
    return off


def js_values(wl, target) -> np.ndarray:
    """JS divergence of every circuit's output distribution against its slice of target."""
    q = probabilities(wl)
    off = _offsets(wl)
    return np.array([js_divergence(target[off[b]:off[b + 1]], q[off[b]:off[b + 1]]) for b in range(wl.B)])


def js_grad_param_shift(wl, target, upstream=None, only=None) -> np.ndarray:
    """Gradient of sum_b u_b JS_b: for every trainable gate occurrence, the circuit with that angle at
    +pi/2 and -pi/2 (the other angles unchanged), chain rule through every probability. Output layout as
    the library's: per-circuit parameter slices, or one vector when parameters are shared. With `only`
    (output indices), the other components are left at 0 and their circuits are not run."""
    off = _offsets(wl)
    u = np.ones(wl.B) if upstream is None else np.asarray(upstream, np.float64)
    grad = np.zeros(wl.n_grad())
    pbase = 0
    for b in range(wl.B):
        n = int(wl.n_qubits[b])
        g, th = _circuit(wl, b)
        p = np.asarray(target[off[b]:off[b + 1]], np.float64)
        q = np.abs(final_state(n, g, th)) ** 2
        m = 0.5 * (p + q)
        w = np.zeros_like(q)
        nz = q > 0
        w[nz] = 0.5 * np.log(q[nz] / m[nz])
        for k in range(len(g)):
            j = int(g["param"][k])
            if j < 0:
                continue
            out = j if wl.params_shared else pbase + j
            if only is not None and out not in only:
                continue
            dq = np.zeros_like(q)
            for sign in (1.0, -1.0):
                gs = g.copy()
                gs["param"][k] = -1
                gs["angle"][k] = th[j] + sign * np.pi / 2
                dq += sign * 0.5 * np.abs(final_state(n, gs, th)) ** 2
            grad[out] += u[b] * float(np.dot(w, dq))
        pbase += int(wl.n_params[b])
    return grad
