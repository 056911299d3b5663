"""ORACLE: a plain complex128 CPU state-vector simulator (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this package.
It computes, by the plain definitions, what the GPU library computes:

* expectation values <0|U(theta)^dagger P U(theta)|0> of Pauli strings and their weighted sum
  (the energy of Eq. 1; the Hamiltonian written as a weighted sum of Pauli strings whose expectations
  a simulator evaluates directly, Section 4.1);
* gradients by the parameter-shift rule (Section 4.1 and 4.2 name it as the gradient method),
  by central finite differences, and by the adjoint method (Jones and Gacon, 2020; not in the paper).

The arithmetic lives in ``qv_oracle.c`` (plain C, complex128, OpenMP only across independent circuits
or independent amplitude pairs). This module only builds and calls it. The probability path of Section
4.2 (output distributions, the Jensen-Shannon divergence of Eq. 3 and its parameter-shift gradient) is in
``oracle/ddcl.py``, and shots drawn from the output distributions with their bit-string counts (Section
3.1) in ``oracle/sampling.py``, both in numpy on top of this module's final states.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("param", "<i4"), ("angle", "<f8")])

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        lib.orc_batch_expectations.argtypes = [i32, P, P, P, P, i32, P, P, P, P, P, i32, P, P, P, i32]
        lib.orc_batch_expectations.restype = ctypes.c_int
        lib.orc_batch_grad_param_shift.argtypes = [i32, P, P, P, P, i32, P, P, P, P, P, i32, P, P, i32]
        lib.orc_batch_grad_param_shift.restype = ctypes.c_int
        lib.orc_batch_grad_fd.argtypes = [i32, P, P, P, P, i32, P, P, P, P, P, i32, P, ctypes.c_double, P, i32]
        lib.orc_batch_grad_fd.restype = ctypes.c_int
        lib.orc_batch_grad_adjoint.argtypes = [i32, P, P, P, P, i32, P, P, P, P, P, i32, P, P, i32]
        lib.orc_batch_grad_adjoint.restype = ctypes.c_int
        lib.orc_final_state.argtypes = [i32, P, ctypes.c_int64, P, P]
        lib.orc_final_state.restype = ctypes.c_int
        lib.orc_max_threads.argtypes = [i32]
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Args:
    """Contiguous, correctly typed copies of a batch description."""

    def __init__(self, n_qubits, gate_offsets, gates, n_params, params_shared, theta, term_offsets,
                 xmask, zmask, coeff, obs_shared):
        self.B = int(len(n_qubits))
        self.nq = np.ascontiguousarray(n_qubits, dtype=np.int32)
        self.goff = np.ascontiguousarray(gate_offsets, dtype=np.int64)
        self.gates = np.ascontiguousarray(gates).astype(GATE_DTYPE, copy=False)
        self.np_ = np.ascontiguousarray(n_params, dtype=np.int32)
        self.shared = int(bool(params_shared))
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.toff = np.ascontiguousarray(term_offsets, dtype=np.int64)
        self.xm = np.ascontiguousarray(xmask, dtype=np.uint64)
        self.zm = np.ascontiguousarray(zmask, dtype=np.uint64)
        self.cf = np.ascontiguousarray(coeff, dtype=np.float64)
        self.obs_shared = int(bool(obs_shared))
        if self.theta.size == 0:
            self.theta = np.zeros(1)
        if self.xm.size == 0:
            self.xm = np.zeros(1, np.uint64)
            self.zm = np.zeros(1, np.uint64)
            self.cf = np.zeros(1)

    def head(self):
        return (self.B, _ptr(self.nq), _ptr(self.goff), _ptr(self.gates), _ptr(self.np_), self.shared,
                _ptr(self.theta), _ptr(self.toff), _ptr(self.xm), _ptr(self.zm), _ptr(self.cf), self.obs_shared)

    def n_grad(self):
        return int(self.np_[0]) if self.shared else int(self.np_.sum())

    def n_term_values(self):
        if self.obs_shared:
            return self.B * int(self.toff[1] - self.toff[0])
        return int(self.toff[-1] - self.toff[0])


def _args(wl):
    return _Args(wl.n_qubits, wl.gate_offsets, wl.gates, wl.n_params, wl.params_shared, wl.theta,
                 wl.term_offsets, wl.xmask, wl.zmask, wl.coeff, wl.obs_shared)


def expectations(wl, nthreads: int = 0):
    """Returns (energies[B], term_values[sum T_b], max |Im <P>|, threads used)."""
    a = _args(wl)
    e = np.zeros(a.B)
    tv = np.zeros(max(1, a.n_term_values()))
    mi = np.zeros(1)
    used = _load().orc_batch_expectations(*a.head(), _ptr(e), _ptr(tv), _ptr(mi), int(nthreads))
    return e, tv[: a.n_term_values()], float(mi[0]), used


def grad_param_shift(wl, upstream=None, nthreads: int = 0):
    a = _args(wl)
    g = np.zeros(max(1, a.n_grad()))
    up = None if upstream is None else np.ascontiguousarray(upstream, dtype=np.float64)
    _load().orc_batch_grad_param_shift(*a.head(), _ptr(up), _ptr(g), int(nthreads))
    return g[: a.n_grad()]


def grad_fd(wl, h: float = 1e-4, upstream=None, nthreads: int = 0):
    a = _args(wl)
    g = np.zeros(max(1, a.n_grad()))
    up = None if upstream is None else np.ascontiguousarray(upstream, dtype=np.float64)
    _load().orc_batch_grad_fd(*a.head(), _ptr(up), float(h), _ptr(g), int(nthreads))
    return g[: a.n_grad()]


def grad_adjoint(wl, upstream=None, nthreads: int = 0):
    a = _args(wl)
    g = np.zeros(max(1, a.n_grad()))
    up = None if upstream is None else np.ascontiguousarray(upstream, dtype=np.float64)
    _load().orc_batch_grad_adjoint(*a.head(), _ptr(up), _ptr(g), int(nthreads))
    return g[: a.n_grad()]


def final_state(n: int, gates, theta) -> np.ndarray:
    """Final complex128 state of one circuit started from |0...0>."""
    g = np.ascontiguousarray(gates).astype(GATE_DTYPE, copy=False)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size == 0:
        th = np.zeros(1)
    out = np.zeros(1 << n, dtype=np.complex128)
    _load().orc_final_state(int(n), _ptr(g), int(len(g)), _ptr(th), _ptr(out))
    return out


def max_threads(nthreads: int = 0) -> int:
    return int(_load().orc_max_threads(int(nthreads)))
