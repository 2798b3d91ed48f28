"""The C ABI: libqs.so loads and exports every symbol include/qs.h declares,
and argument errors come back as status codes (host-side checks only; no
device work is started here)."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

from paper_2406_14084_amd import qs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "qs.h")).read()
    return sorted(set(re.findall(r"^QS_API\s+[\w\s\*]+?\b(qs_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_core_calls():
    syms = declared_symbols()
    for name in ("qs_create", "qs_apply_gate", "qs_fuse", "qs_apply_plan", "qs_probs", "qs_expect"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = qs.lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_symbols()) == set(qs.SIGNATURES)


def test_version():
    assert qs.lib().qs_version().decode().startswith("libqs")


def test_create_rejects_bad_n_and_dtype():
    h = C.c_void_p()
    assert qs.lib().qs_create(0, 0, C.byref(h)) == -1
    assert qs.lib().qs_create(35, 0, C.byref(h)) == -1
    assert qs.lib().qs_create(10, 7, C.byref(h)) == -1
    assert "dtype" in qs.lib().qs_last_error().decode()


def test_unattached_handle_is_state_error():
    L = qs.lib()
    h = C.c_void_p()
    assert L.qs_create(8, 0, C.byref(h)) == 0
    assert L.qs_init_zero(h) == -5
    assert "attached" in L.qs_last_error().decode()
    t = (C.c_int * 1)(0)
    m = (C.c_double * 8)()
    assert L.qs_apply_gate(h, 1, t, m) == -5
    assert L.qs_destroy(h) == 0


def test_null_arguments():
    L = qs.lib()
    assert L.qs_init_zero(None) == -1
    assert L.qs_apply_plan(None, None) == -1
    assert L.qs_fuse(None, 3, None, None) == -1


def test_workspace_size_query():
    L = qs.lib()
    nb = C.c_size_t()
    assert L.qs_workspace_size(30, 0, C.byref(nb)) == 0 and nb.value >= 1 << 20
    assert L.qs_workspace_size(0, 0, C.byref(nb)) == -1
    assert L.qs_workspace_size(10, 5, C.byref(nb)) == -1
    assert L.qs_workspace_size(10, 0, None) == -1


def test_attach_rejects_host_memory_and_bad_workspace():
    L = qs.lib()
    h = C.c_void_p()
    assert L.qs_create(4, 0, C.byref(h)) == 0
    buf = C.create_string_buffer(16 * 16 + 256)
    p = (C.addressof(buf) + 255) & ~255
    # wrong size first (checked before any HIP call), then host memory
    assert L.qs_attach(h, C.c_void_p(p), 100, None, None, 0) == -1
    assert "expected 256 bytes" in L.qs_last_error().decode()
    assert L.qs_attach(h, C.c_void_p(p + 16), 256, None, None, 0) == -1
    assert "aligned" in L.qs_last_error().decode()
    assert L.qs_attach(h, C.c_void_p(p), 256, None, None, 0) == -1
    assert "device memory" in L.qs_last_error().decode()
    assert L.qs_get_amplitudes(h, 0, 1, C.c_void_p(p)) == -5
    assert L.qs_destroy(h) == 0


def test_batch_workspace_size():
    """States of instances above the smaller of the two LDS chunk sizes the
    autotuner may pick (12 qubits for complex64) go to the workspace: 2^n
    amplitudes plus one cut-value byte each."""
    import numpy as np
    edges = np.array([0, 1, 1, 2, 2, 0], dtype=np.int32)
    g = np.array([0.3], dtype=np.float64)
    b = np.array([0.2], dtype=np.float64)
    L = qs.lib()

    def inst(n):
        return qs.QaoaInst_C(n, 3, 1, edges.ctypes.data_as(C.POINTER(C.c_int)),
                             g.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)))
    arr = (qs.QaoaInst_C * 3)(inst(10), inst(14), inst(16))
    nb = C.c_size_t()
    assert L.qs_batch_qaoa_workspace_size(3, arr, 1, C.byref(nb)) == 0
    amps = (1 << 14) + (1 << 16)
    assert nb.value == amps * 8 + amps
    assert L.qs_batch_qaoa_workspace_size(1, arr, 1, C.byref(nb)) == 0 and nb.value == 0
    at13 = (qs.QaoaInst_C * 1)(inst(13))
    assert L.qs_batch_qaoa_workspace_size(1, at13, 1, C.byref(nb)) == 0 and nb.value == (1 << 13) * 9
    bad = (qs.QaoaInst_C * 1)(inst(21))
    assert L.qs_batch_qaoa_workspace_size(1, bad, 1, C.byref(nb)) == -1
    assert L.qs_batch_qaoa_create(1, bad, 1, None, None, 0, None) == -1
