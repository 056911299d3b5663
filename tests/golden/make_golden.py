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


CASES = {
    "qcl20_L2": lambda: qcl_case(2),
    "qcl20_L8": lambda: qcl_case(8),
    "random1024": random_case,
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for name in names:
        out = CASES[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f)
        print(name, f"{out['seconds']:.1f}s", flush=True)
