"""CPU-only checks of the C interface: the library loads, exports every function include/qvpu.h declares,
and the validation layer rejects malformed batches with the documented status and a message, without a
device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_03466_amd import qvpu
from paper_2406_03466_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qvpu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qv_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = qvpu.load()
    names = _declared()
    assert "qv_batch_create" in names and "qv_batch_gradient" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(qvpu.EXPORTS)


def test_version_string():
    assert b"gfx950" in qvpu.load().qv_version()


def _ok():
    return W.config1()


def test_valid_batch_passes():
    st, msg = qvpu.validate_batch(_ok(), qvpu.QV_C64)
    assert st == qvpu.QV_OK and msg == ""
    st, _ = qvpu.validate_batch(W.config4(), qvpu.QV_C128)
    assert st == qvpu.QV_OK


def _mutate(field, idx, value):
    wl = _ok()
    g = wl.gates.copy()
    g[field][idx] = value
    wl.gates = g
    return wl


@pytest.mark.parametrize("wl,needle", [
    (_mutate("q0", 0, 10), "out of range"),
    (_mutate("q0", 0, -1), "out of range"),
    (_mutate("kind", 3, 42), "unknown kind"),
    (_mutate("param", 0, 80), "param 80 out of range"),
    (_mutate("param", 0, -2), "out of range"),
])
def test_bad_gates(wl, needle):
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID
    assert needle in msg


def test_control_equals_target():
    wl = _ok()
    g = wl.gates.copy()
    k = int(np.nonzero(g["kind"] == W.CNOT)[0][0])
    g["q1"][k] = g["q0"][k]
    wl.gates = g
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID and "both qubits" in msg


def test_fixed_angle_must_be_finite_and_param_only_on_rotations():
    wl = W.single("x", 2, [W.gate(W.RY, 0, -1, -1, float("nan"))])
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID and "non-finite angle" in msg
    wl = W.single("x", 2, [W.gate(W.H, 0, -1, -1)])
    g = wl.gates.copy()
    g["param"][0] = 0
    wl.gates = g
    wl.n_params = np.array([1], np.int32)
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID and "only RX/RY/RZ" in msg


def test_qubit_counts_and_offsets():
    wl = _ok()
    wl.n_qubits = np.array([35], np.int32)
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID and "[1, 34]" in msg
    wl = _ok()
    wl.gate_offsets = np.array([0, 200], np.int64)
    wl2 = W.random_batch(3, 3, 5, 2, 5, 2, seed_index=7)
    wl2.gate_offsets = wl2.gate_offsets[[0, 2, 1, 3]]
    st, msg = qvpu.validate_batch(wl2)
    assert st == qvpu.QV_E_INVALID and "non-decreasing" in msg


def test_mask_outside_register_and_bad_coeff():
    wl = _ok()
    wl.xmask = wl.xmask.copy()
    wl.xmask[3] = np.uint64(1 << 10)
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID and "outside circuit" in msg
    wl = _ok()
    wl.coeff = wl.coeff.copy()
    wl.coeff[0] = np.inf
    st, msg = qvpu.validate_batch(wl)
    assert st == qvpu.QV_E_INVALID and "non-finite coefficient" in msg


def test_shared_params_need_equal_counts_and_precision_checked():
    wl = W.random_batch(3, 3, 5, 5, 10, 2, seed_index=8)
    wl.params_shared = True
    st, msg = qvpu.validate_batch(wl)
    if len(set(wl.n_params.tolist())) > 1:
        assert st == qvpu.QV_E_INVALID and "equal n_params" in msg
    st, msg = qvpu.validate_batch(_ok(), 7)
    assert st == qvpu.QV_E_INVALID and "precision" in msg


def test_null_pointers_rejected():
    lib = qvpu.load()
    st = lib.qv_validate_batch(1, None, None, None, None, 0, None, None, None, None, 1, 0)
    assert st == qvpu.QV_E_INVALID
    assert "must not be NULL" in qvpu.last_error()
    h = ctypes.c_void_p()
    st = lib.qv_batch_create(None, 1, None, None, None, None, 0, None, None, None, None, 1, 0, ctypes.byref(h))
    assert st == qvpu.QV_E_INVALID and "ctx must not be NULL" in qvpu.last_error()
    assert lib.qv_batch_destroy(None) == qvpu.QV_E_INVALID
    assert lib.qv_ctx_destroy(None) == qvpu.QV_E_INVALID


@pytest.mark.parametrize("opts,code", [('{"launch": "sometimes"}', "QV_E_INVALID"),
                                       ('{"specialize": "sometimes"}', "QV_E_INVALID"),
                                       ('{"adjoint_inner": "f16"}', "QV_E_INVALID"),
                                       ('{"adjoint_inner": "f64"}', "QV_E_INVALID"),
                                       ('{"adjoint_inner": "f64", "specialize": "off"}', "QV_E_INVALID"),
                                       ('{"wait_ms": -1}', "QV_E_INVALID"),
                                       ('{"persist_chunk": 65}', "QV_E_INVALID"),
                                       ('{"wait_extra": -2}', "QV_E_INVALID"),
                                       ('{"fusion": 99}', "QV_E_INVALID"),
                                       ('{"fusion": "sometimes"}', "QV_E_INVALID"),
                                       ('{"tile_qubits": 20}', "QV_E_INVALID"),
                                       ('{"no_such_key": 1}', "QV_E_INVALID")])
def test_context_options_checked_before_device(opts, code):
    """Context options are parsed before any device call, so a bad option is reported as such even on a
    host without a GPU."""
    with pytest.raises(qvpu.QvError) as ei:
        qvpu.Context(0, None, opts)
    assert code in str(ei.value)
