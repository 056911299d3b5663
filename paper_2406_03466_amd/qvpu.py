"""ctypes binding of the qvpu C interface (include/qvpu.h), with the same names.

Argument marshalling only: every step of the computation runs in the HIP library. Device buffers and
streams come from PyTorch (tensor.data_ptr(), torch.cuda.current_stream().cuda_stream). If the built
library is missing the binding raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqvpu.so")

QV_OK, QV_E_INVALID, QV_E_OOM, QV_E_DEVICE, QV_E_UNSUPPORTED, QV_E_STATE = 0, -1, -2, -3, -4, -5
QV_C64, QV_C128 = 0, 1
QV_ADJOINT, QV_PARAM_SHIFT = 0, 1
STATUS_NAMES = {0: "QV_OK", -1: "QV_E_INVALID", -2: "QV_E_OOM", -3: "QV_E_DEVICE", -4: "QV_E_UNSUPPORTED",
                -5: "QV_E_STATE"}


class QvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.msg = msg


class qv_stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int64), ("launches", ctypes.c_int64), ("algorithmic_bytes", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("norm_err_max", ctypes.c_double), ("tile_qubits", ctypes.c_int32),
                ("contig_qubits", ctypes.c_int32), ("passes_per_circuit_max", ctypes.c_int32),
                ("fuse_min_run", ctypes.c_int32)]


class qv_launch_rec(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("level", ctypes.c_int32), ("bytes", ctypes.c_int64),
                ("ms", ctypes.c_double), ("flops", ctypes.c_double)]


KERNEL_NAMES = ["init", "tile", "tile_adj", "stride", "stride_adj", "expect", "finalize", "lambda",
                "grad_reduce", "shift_combine", "rtile", "rtile_adj", "matrices", "rtile_persist",
                "rtile_adj_persist", "fuse", "probs", "diag_seed", "diag_expect", "segment_sum", "sample", "rtile_gen", "rtile_adj_gen",
                "rtile_lam"]

class qv_pass_info(ctypes.Structure):
    _fields_ = [("local_mask", ctypes.c_uint64), ("qubits", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("n_trainable", ctypes.c_int32), ("n_segments", ctypes.c_int32), ("first_gate", ctypes.c_int32),
                ("contiguous_low", ctypes.c_int32), ("n_fused", ctypes.c_int32), ("n_folded", ctypes.c_int32),
                ("zero_mask", ctypes.c_uint64)]


_lib = None

EXPORTS = ["qv_ctx_create", "qv_ctx_set_stream", "qv_ctx_destroy", "qv_batch_create", "qv_validate_batch",
           "qv_batch_set_params", "qv_batch_expectations", "qv_batch_expectations_static", "qv_batch_gradient", "qv_batch_probabilities",
           "qv_batch_js_gradient", "qv_batch_sample", "qv_batch_state", "qv_batch_stats", "qv_batch_destroy",
           "qv_batch_launch_log", "qv_plan_circuit", "qv_last_error", "qv_version"]


def load():
    """Loads libqvpu.so (built by `python -m paper_2406_03466_amd.build`)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2406_03466_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    lib.qv_ctx_create.argtypes = [i32, P, ctypes.c_char_p, ctypes.POINTER(P)]
    lib.qv_ctx_set_stream.argtypes = [P, P]
    lib.qv_ctx_destroy.argtypes = [P]
    lib.qv_batch_create.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, i32, i32, ctypes.POINTER(P)]
    lib.qv_validate_batch.argtypes = [i32, P, P, P, P, i32, P, P, P, P, i32, i32]
    lib.qv_batch_set_params.argtypes = [P, P, i32]
    lib.qv_batch_expectations.argtypes = [P, P, P, i32]
    lib.qv_batch_expectations_static.argtypes = [P, P, P, i32]
    lib.qv_batch_gradient.argtypes = [P, i32, P, P, P, i32]
    lib.qv_batch_probabilities.argtypes = [P, P, i32]
    lib.qv_batch_js_gradient.argtypes = [P, i32, P, P, P, P, i32]
    lib.qv_batch_sample.argtypes = [P, ctypes.c_int64, P, P, P, P, P, i32]
    lib.qv_batch_state.argtypes = [P, i32, P, i32]
    lib.qv_batch_stats.argtypes = [P, ctypes.POINTER(qv_stats)]
    lib.qv_batch_destroy.argtypes = [P]
    lib.qv_batch_launch_log.argtypes = [P, ctypes.POINTER(qv_launch_rec), i32, ctypes.POINTER(i32)]
    lib.qv_plan_circuit.argtypes = [i32, ctypes.c_int64, P, i32, i32, i32, i32, i32,
                                    ctypes.POINTER(qv_pass_info), ctypes.POINTER(i32), P]
    for f in ["qv_ctx_create", "qv_ctx_set_stream", "qv_ctx_destroy", "qv_batch_create", "qv_validate_batch",
              "qv_batch_set_params", "qv_batch_expectations", "qv_batch_expectations_static", "qv_batch_gradient", "qv_batch_probabilities",
              "qv_batch_js_gradient", "qv_batch_sample", "qv_batch_state", "qv_batch_stats", "qv_batch_destroy",
              "qv_batch_launch_log", "qv_plan_circuit"]:
        getattr(lib, f).restype = st
    lib.qv_last_error.restype = ctypes.c_char_p
    lib.qv_last_error.argtypes = []
    lib.qv_version.restype = ctypes.c_char_p
    lib.qv_version.argtypes = []
    _lib = lib
    return lib


def last_error() -> str:
    return load().qv_last_error().decode()


def _check(status: int):
    if status != QV_OK:
        raise QvError(status, last_error())


def _ptr(a) -> Optional[int]:
    """Host numpy array or torch tensor -> address (None for None)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class _Arrays:
    """Contiguous, typed host copies of a batch description, kept alive for the call."""

    def __init__(self, wl: W.Workload):
        self.nq = np.ascontiguousarray(wl.n_qubits, np.int32)
        self.goff = np.ascontiguousarray(wl.gate_offsets, np.int64)
        self.gates = np.ascontiguousarray(wl.gates).astype(W.GATE_DTYPE, copy=False)
        if self.gates.size == 0:
            self.gates = np.zeros(1, W.GATE_DTYPE)
        self.np_ = np.ascontiguousarray(wl.n_params, np.int32)
        self.toff = np.ascontiguousarray(wl.term_offsets, np.int64)
        self.xm = np.ascontiguousarray(wl.xmask, np.uint64)
        self.zm = np.ascontiguousarray(wl.zmask, np.uint64)
        self.cf = np.ascontiguousarray(wl.coeff, np.float64)
        if self.xm.size == 0:
            self.xm, self.zm, self.cf = np.zeros(1, np.uint64), np.zeros(1, np.uint64), np.zeros(1)
        self.B = int(len(self.nq))
        self.shared = int(bool(wl.params_shared))
        self.obs_shared = int(bool(wl.obs_shared))

    def args(self):
        return (self.B, _ptr(self.nq), _ptr(self.goff), _ptr(self.gates), _ptr(self.np_), self.shared,
                _ptr(self.toff), _ptr(self.xm), _ptr(self.zm), _ptr(self.cf), self.obs_shared)


def plan_circuit(n: int, gates, tile_qubits: int = 0, precision: int = QV_C64, engine: int = 0,
                 with_order: bool = False, fuse_min: int = 0):
    """qv_plan_circuit: the passes the planner makes for one circuit (host only, no device); with
    with_order, also the gate indices in execution order."""
    g = np.ascontiguousarray(gates).astype(W.GATE_DTYPE, copy=False)
    if g.size == 0:
        g = np.zeros(1, W.GATE_DTYPE)
        ng = 0
    else:
        ng = len(g)
    cnt = ctypes.c_int32(0)
    _check(load().qv_plan_circuit(int(n), ng, _ptr(g), int(tile_qubits), int(precision), int(engine),
                                  int(fuse_min), 0, None, ctypes.byref(cnt), None))
    arr = (qv_pass_info * max(1, cnt.value))()
    order = np.zeros(max(1, ng), np.int32)
    _check(load().qv_plan_circuit(int(n), ng, _ptr(g), int(tile_qubits), int(precision), int(engine),
                                  int(fuse_min), cnt.value, arr, ctypes.byref(cnt), _ptr(order)))
    passes = [{k: getattr(arr[i], k) for k, _ in qv_pass_info._fields_} for i in range(cnt.value)]
    return (passes, order[:ng]) if with_order else passes


def validate_batch(wl: W.Workload, precision: int = QV_C64) -> tuple:
    """qv_validate_batch: runs the checks of qv_batch_create without a device. Returns (status, message)."""
    a = _Arrays(wl)
    st = load().qv_validate_batch(*a.args(), int(precision))
    return st, last_error()


class Context:
    """qv_ctx: one device, one stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, options: Optional[str] = None):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.qv_ctx_create(int(device), stream, options.encode() if options else None, ctypes.byref(h)))
        self.h = h
        self.device = device

    def set_stream(self, stream: Optional[int]):
        _check(load().qv_ctx_set_stream(self.h, stream))

    def close(self):
        if self.h:
            _check(load().qv_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """qv_batch: a submitted batch of circuits with its observable."""

    def __init__(self, ctx: Context, wl: W.Workload, precision: int = QV_C64):
        lib = load()
        self.ctx = ctx
        self.wl = wl
        self.precision = precision
        a = _Arrays(wl)
        h = ctypes.c_void_p()
        _check(lib.qv_batch_create(ctx.h, *a.args(), int(precision), ctypes.byref(h)))
        self.h = h
        self.B = wl.B
        self.n_grad = wl.n_grad()
        self.n_tv = wl.B * int(wl.term_offsets[1] - wl.term_offsets[0]) if wl.obs_shared else \
            int(wl.term_offsets[-1] - wl.term_offsets[0])
        self.param_version = 0
        if len(wl.theta) or self.n_grad == 0:
            self.set_params(np.asarray(wl.theta, np.float64))

    def set_params(self, theta):
        """theta: host float64 array or a float64 device tensor. Every call advances param_version, so a
        caller holding an earlier version knows the batch has moved to other parameters."""
        self.param_version += 1
        if isinstance(theta, np.ndarray):
            th = np.ascontiguousarray(theta, np.float64)
            if th.size == 0:
                th = np.zeros(1)
            _check(load().qv_batch_set_params(self.h, _ptr(th), 0))
        else:
            _check(load().qv_batch_set_params(self.h, _ptr(theta), 1))

    def expectations(self, energies=None, term_values=None, want_terms: bool = True):
        """Host mode (no outputs given): returns (energies[B], term_values[...]) as numpy arrays.
        Device mode: pass float64 device tensors; they are filled in stream order."""
        lib = load()
        if energies is None:
            e = np.zeros(self.B)
            tv = np.zeros(max(1, self.n_tv)) if want_terms else None
            _check(lib.qv_batch_expectations(self.h, _ptr(e), _ptr(tv), 0))
            return e, (tv[: self.n_tv] if tv is not None else None)
        _check(lib.qv_batch_expectations(self.h, _ptr(energies), _ptr(term_values), 1))
        return energies, term_values

    def expectations_static(self, energies=None, term_values=None, want_terms: bool = True):
        """qv_batch_expectations_static (no device allocation; see the header); as expectations()."""
        lib = load()
        if energies is None:
            e = np.zeros(self.B)
            tv = np.zeros(max(1, self.n_tv)) if want_terms else None
            _check(lib.qv_batch_expectations_static(self.h, _ptr(e), _ptr(tv), 0))
            return e, (tv[: self.n_tv] if tv is not None else None)
        _check(lib.qv_batch_expectations_static(self.h, _ptr(energies), _ptr(term_values), 1))
        return energies, term_values

    def gradient(self, method: int = QV_ADJOINT, upstream=None, grad=None, energies=None):
        lib = load()
        if grad is None:
            up = None if upstream is None else np.ascontiguousarray(upstream, np.float64)
            g = np.zeros(max(1, self.n_grad))
            e = np.zeros(self.B)
            _check(lib.qv_batch_gradient(self.h, int(method), _ptr(up), _ptr(g), _ptr(e), 0))
            return g[: self.n_grad], e
        _check(lib.qv_batch_gradient(self.h, int(method), _ptr(upstream), _ptr(grad), _ptr(energies), 1))
        return grad, energies

    def n_amplitudes(self) -> int:
        return int(sum(1 << int(n) for n in self.wl.n_qubits))

    def probabilities(self, probs=None):
        """Output distributions of every circuit, concatenated (circuit b's 2^n_b values in order). Host
        mode returns a numpy array; device mode fills a float64 device tensor of n_amplitudes() values."""
        if probs is None:
            out = np.zeros(self.n_amplitudes())
            _check(load().qv_batch_probabilities(self.h, _ptr(out), 0))
            return out
        _check(load().qv_batch_probabilities(self.h, _ptr(probs), 1))
        return probs

    def js_gradient(self, target, method: int = QV_ADJOINT, upstream=None, js=None, grad=None):
        """Jensen-Shannon divergences against target distributions (layout of probabilities()) and the
        gradient of sum_b upstream_b JS_b. Host mode returns (js[B], grad); device mode takes float64
        device tensors for target, upstream (or None), js and grad (grad None: divergences only)."""
        lib = load()
        if grad is None and js is None:
            t = np.ascontiguousarray(target, np.float64)
            if t.shape != (self.n_amplitudes(),):
                raise ValueError(f"target must hold {self.n_amplitudes()} values, got shape {t.shape}")
            up = None if upstream is None else np.ascontiguousarray(upstream, np.float64)
            g = np.zeros(max(1, self.n_grad))
            j = np.zeros(self.B)
            _check(lib.qv_batch_js_gradient(self.h, int(method), _ptr(t), _ptr(up), _ptr(j), _ptr(g), 0))
            return j, g[: self.n_grad]
        _check(lib.qv_batch_js_gradient(self.h, int(method), _ptr(target), _ptr(upstream), _ptr(js), _ptr(grad), 1))
        return js, grad

    def sample(self, shots: int, uniforms, samples=None, bitstrings=None, counts=None, n_distinct=None,
               want_samples: bool = True):
        """qv_batch_sample. Host mode (uniforms a numpy array of B * shots values in [0, 1)): returns
        (samples[B * shots] or None, [(bitstrings, counts) per circuit]). Device mode: uniforms and the
        outputs are device tensors (int64 samples or None, uint64-as-int64 bitstrings, int64 counts and
        n_distinct), filled in stream order."""
        lib = load()
        if isinstance(uniforms, np.ndarray):
            u = np.ascontiguousarray(uniforms, np.float64)
            if u.shape != (self.B * shots,):
                raise ValueError(f"uniforms must hold {self.B * shots} values, got shape {u.shape}")
            smp = np.zeros(self.B * shots, np.int64) if want_samples else None
            bits = np.zeros(self.B * shots, np.uint64)
            cnt = np.zeros(self.B * shots, np.int64)
            nd = np.zeros(self.B, np.int64)
            _check(lib.qv_batch_sample(self.h, int(shots), _ptr(u), _ptr(smp), _ptr(bits), _ptr(cnt), _ptr(nd), 0))
            per = [(bits[b * shots: b * shots + nd[b]].copy(), cnt[b * shots: b * shots + nd[b]].copy())
                   for b in range(self.B)]
            return smp, per
        _check(lib.qv_batch_sample(self.h, int(shots), _ptr(uniforms), _ptr(samples), _ptr(bitstrings),
                                   _ptr(counts), _ptr(n_distinct), 1))
        return samples, bitstrings, counts, n_distinct

    def state(self, circuit: int) -> np.ndarray:
        n = int(self.wl.n_qubits[circuit])
        dt = np.complex64 if self.precision == QV_C64 else np.complex128
        out = np.zeros(1 << n, dt)
        _check(load().qv_batch_state(self.h, int(circuit), _ptr(out), 0))
        return out

    def stats(self) -> dict:
        s = qv_stats()
        _check(load().qv_batch_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in qv_stats._fields_}

    def launch_log(self) -> list:
        """Per-launch records of the last call (context option "launch_events")."""
        n = ctypes.c_int32(0)
        _check(load().qv_batch_launch_log(self.h, None, 0, ctypes.byref(n)))
        if n.value == 0:
            return []
        arr = (qv_launch_rec * n.value)()
        _check(load().qv_batch_launch_log(self.h, arr, n.value, ctypes.byref(n)))
        return [{"kernel": KERNEL_NAMES[r.kernel], "level": r.level, "bytes": r.bytes, "ms": r.ms,
                 "flops": r.flops} for r in arr]

    def close(self):
        if getattr(self, "h", None):
            _check(load().qv_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
