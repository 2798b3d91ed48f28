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
