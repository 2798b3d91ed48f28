"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that the pins catch every one of them.

Each mutant is a text substitution applied to oracle.c, compiled into a
temporary directory; the original file is never modified.
"""
from __future__ import annotations

import os

import pytest

from oracle import build, sim
from tests import test_oracle_pins as pins

MUTANTS = {
    "transposed_matrix": [("U[2 * (r * d + c)], ui = U[2 * (r * d + c) + 1]",
                           "U[2 * (c * d + r)], ui = U[2 * (c * d + r) + 1]")],
    "wrong_sign_real": [("sr += ur * vr[c] - ui * vi[c];", "sr += ur * vr[c] + ui * vi[c];")],
    "dropped_imag_term": [("si += ur * vi[c] + ui * vr[c];", "si += ur * vi[c];")],
    "reversed_local_bits": [("if ((r >> (k - 1 - j)) & 1)", "if ((r >> j) & 1)")],
    "swap_identity": [("m |= (bb << a[j]) | (ba << b[j]);", "m |= (ba << a[j]) | (bb << b[j]);")],
    "y_phase_sign": [("double pim = (ny == 1) ? 1.0", "double pim = (ny == 1) ? -1.0")],
    "missing_conjugate": [("double br = psi[2 * j], bi = -psi[2 * j + 1];",
                           "double br = psi[2 * j], bi = psi[2 * j + 1];")],
    "probs_dropped_imag": [("p[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];",
                            "p[i] = psi[2 * i] * psi[2 * i];")],
    "probs_index_shift": [("for (i64 i = 0; i < N; ++i) p[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];",
                           "for (i64 i = 0; i < N; ++i) p[i] = psi[2 * (i ^ 1)] * psi[2 * (i ^ 1)] + psi[2 * (i ^ 1) + 1] * psi[2 * (i ^ 1) + 1];")],
    "probs_cross_term": [("p[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];",
                          "p[i] = psi[2 * i] * psi[2 * i] + psi[2 * i] * psi[2 * i + 1];")],
    "qaoa_phase_sign": [("double th = -gamma", "double th = gamma")],
    "cut_and_not_xor": [("(((z >> edges[2 * e]) ^ (z >> edges[2 * e + 1])) & 1)",
                         "(((z >> edges[2 * e]) & (z >> edges[2 * e + 1])) & 1)")],
    "off_by_one_target_mask": [("if (base & tmask) continue;", "if (base & (tmask >> 1)) continue;")],
    "z_sign_dropped": [("double sign = (__builtin_popcountll((unsigned long long)i & z) & 1) ? -1.0 : 1.0;",
                        "double sign = 1.0;")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    with open(build.SRC) as f:
        src = f.read()
    for old, new in MUTANTS[name]:
        assert old in src, "mutation site vanished: %r" % old
        src = src.replace(old, new)
    msrc = os.path.join(tmp_path, "oracle_mutant.c")
    with open(msrc, "w") as f:
        f.write(src)
    out = build.build(force=True, src=msrc, out=os.path.join(tmp_path, "libmut.so"))
    L = sim.lib(out)
    failed = []
    for chk in pins.ALL_CHECKS:
        try:
            chk(L)
        except (AssertionError, ValueError):
            failed.append(chk.__name__)
    assert failed, "mutant %s passed every pin" % name
