"""Writes the stored expected values used by the full-size GPU parity tests. Calls only the CPU oracle
(oracle/) on the seeded workloads; nothing here touches the GPU library.

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_03466_amd import workloads as W  # noqa: E402


def qcl_case(layers):
    wl = W.config3(layers)
    t0 = time.time()
    e, _, mi, used = oracle.expectations(wl)
    y = wl.extra["y"]
    up = 2.0 * (e - y) / wl.B          # d/dE_b of the MSE loss (1/B) sum_b (E_b - y_b)^2
    g = oracle.grad_adjoint(wl, up)
    return {"workload": wl.name, "what": "energies <Z_0> per sample, MSE-loss gradient by oracle adjoint",
            "energies": e.tolist(), "upstream": up.tolist(), "grad": g.tolist(), "max_imag": mi,
            "threads": used, "seconds": time.time() - t0}


def random_case():
    wl = W.config4()
    t0 = time.time()
    e, tv, mi, used = oracle.expectations(wl)
    return {"workload": wl.name, "what": "energies and term values of every circuit",
            "energies": e.tolist(), "term_values": tv.tolist(), "max_imag": mi, "threads": used,
            "seconds": time.time() - t0}


DDCL20_PARAMS = [0, 1, 2, 119, 600, 601, 1197, 1199]


def ddcl20_case():
    """Table 2's smallest DDCL size: 20 qubits, 10 layers, 1200 parameters. The divergence, 64 sampled
    output probabilities and 8 gradient components by the parameter-shift rule (17 oracle circuits)."""
    from oracle import ddcl as OD
    wl = W.ddcl(20, 10)
    t0 = time.time()
    t = wl.extra["target"]
    q = OD.probabilities(wl)
    idx = np.random.default_rng(20).choice(len(q), size=64, replace=False)
    g = OD.js_grad_param_shift(wl, t, None, only=set(DDCL20_PARAMS))
    return {"workload": wl.name, "what": "JS divergence, sampled probabilities, gradient components (param-shift)",
            "js": OD.js_divergence(t, q), "prob_index": idx.tolist(), "probs": q[idx].tolist(),
            "grad_index": DDCL20_PARAMS, "grad": [float(g[j]) for j in DDCL20_PARAMS],
            "seconds": time.time() - t0}


DDCL26_PARAMS = [0, 1559]


def ddcl26_case():
    """Table 2's largest DDCL size: 26 qubits, 10 layers, 1560 parameters. The divergence, 64 sampled
    probabilities and 2 gradient components (the first angle and the last, which cannot change the
    distribution) by the parameter-shift rule: 5 oracle circuits of 2^26 amplitudes."""
    from oracle import ddcl as OD
    wl = W.ddcl(26, 10)
    t0 = time.time()
    t = wl.extra["target"]
    q = OD.probabilities(wl)
    idx = np.random.default_rng(26).choice(len(q), size=64, replace=False)
    js = OD.js_divergence(t, q)
    del q
    g = OD.js_grad_param_shift(wl, t, None, only=set(DDCL26_PARAMS))
    return {"workload": wl.name, "what": "JS divergence, sampled probabilities, gradient components (param-shift)",
            "js": js, "prob_index": idx.tolist(), "probs": [float(v) for v in OD.probabilities(wl)[idx]],
            "grad_index": DDCL26_PARAMS, "grad": [float(g[j]) for j in DDCL26_PARAMS],
            "seconds": time.time() - t0}


def mcvqe22_case():
    """Table 1's largest MC-VQE size: 22 CIS states of 22 qubits, 106 shared parameters, 128 terms and a
    constant. Energies and the mean-energy gradient (upstream 1/22) by the oracle's adjoint."""
    wl = W.mcvqe(22)
    t0 = time.time()
    e, _, mi, used = oracle.expectations(wl)
    up = np.full(wl.B, 1.0 / wl.B)
    g = oracle.grad_adjoint(wl, up)
    return {"workload": wl.name, "what": "energies, mean-energy gradient by oracle adjoint",
            "energies": e.tolist(), "upstream": up.tolist(), "grad": g.tolist(), "max_imag": mi,
            "threads": used, "seconds": time.time() - t0}


def hea_ladder_case(n):
    """The 32-qubit workload's shape (10 hardware-efficient layers, trainable RY, fixed RZ, the open ZZ
    chain) at a size the oracle runs: energy, term values and the gradient of all 10 n RY angles by the
    oracle's adjoint."""
    wl = W.large_hea(n, 10)
    t0 = time.time()
    e, tv, mi, used = oracle.expectations(wl)
    g = oracle.grad_adjoint(wl)
    return {"workload": wl.name, "what": "energy, ZZ term values, gradient by oracle adjoint",
            "energies": e.tolist(), "term_values": tv.tolist(), "grad": g.tolist(), "max_imag": mi,
            "threads": used, "seconds": time.time() - t0}


CASES = {
    "qcl20_L2": lambda: qcl_case(2),
    "qcl20_L4": lambda: qcl_case(4),
    "hea20_L10": lambda: hea_ladder_case(20),
    "hea22_L10": lambda: hea_ladder_case(22),
    "hea24_L10": lambda: hea_ladder_case(24),
    "qcl20_L8": lambda: qcl_case(8),
    "random1024": random_case,
    "ddcl20": ddcl20_case,
    "mcvqe22": mcvqe22_case,
    "ddcl26": ddcl26_case,
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for name in names:
        out = CASES[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f)
        print(name, f"{out['seconds']:.1f}s", flush=True)
