"""qs_expect_noalloc (the entry point for callers that cannot allocate: its
scratch is a fixed array in the library) against qs_expect on the same
states, called through the C ABI: two calls in a row, the second on a
smaller state with fewer terms, each checked against qs_expect and the
oracle."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _terms(rng, n, count):
    return [(int(rng.integers(1 << n)), int(rng.integers(1 << n)), float(rng.standard_normal())) for _ in range(count)]


def _call(fn, st, terms):
    arr = (qs.Pauli_C * max(1, len(terms)))()
    for i, (x, z, c) in enumerate(terms):
        arr[i] = qs.Pauli_C(x, z, c)
    out = C.c_double()
    qs.check(fn(st.h, len(terms), arr, C.byref(out)))
    return out.value


def test_noalloc_matches_expect_twice():
    need_gpu()
    L = qs.lib()
    rng = np.random.default_rng(77)
    for n, count, seed in ((18, 64, 1), (11, 5, 2)):
        c = I.random_dense(n, 50, seed=seed, kmax=3)
        say("noalloc expect", n, count)
        st = qs.State(n, "c128")
        st.init_zero()
        st.apply_plan(qs.Plan(c, kmax=4))
        terms = _terms(rng, n, count)
        got = _call(L.qs_expect_noalloc, st, terms)
        ref = _call(L.qs_expect, st, terms)
        want = sim.expect(sim.run(c), terms)
        say("noalloc %.17g  expect %.17g  oracle %.17g" % (got, ref, want))
        assert got == ref
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_noalloc_rejects_too_many_terms():
    need_gpu()
    L = qs.lib()
    st = qs.State(8, "c128")
    st.init_zero()
    arr = (qs.Pauli_C * 65)()
    out = C.c_double()
    assert L.qs_expect_noalloc(st.h, 65, arr, C.byref(out)) == -1
    assert "64" in L.qs_last_error().decode()
