"""How the gate-by-gate path classifies gates (host logic, no GPU): controls
are peeled off, the rest is diagonal, a permutation with phases, or dense."""
from __future__ import annotations

import numpy as np

from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs


def controlled(u, nctrl):
    """Block matrix with the controls as the leading (most significant) bits."""
    d = u.shape[0]
    m = np.eye(d << nctrl, dtype=np.complex128)
    m[-d:, -d:] = u
    return m


def test_textbook_gates():
    rng = np.random.default_rng(3)
    cases = [
        ("H", (4,), I.g_h(), (0, [], 1)),
        ("X", (2,), I.g_x(), (2, [], 1)),
        ("Y", (2,), I.g_y(), (2, [], 1)),
        ("Z", (2,), I.g_z(), (1, [], 1)),
        ("RZ", (5,), I.g_rz(0.3), (1, [], 1)),
        ("CX", (3, 7), I.g_cx(), (2, [3], 1)),
        ("CZ", (3, 7), I.g_cz(), (1, [3], 1)),
        ("CP", (6, 1), I.g_cp(0.9), (1, [6], 1)),
        ("SWAP", (0, 9), I.g_swap(), (2, [], 2)),
        ("RZZ", (0, 9), I.g_rzz(0.4), (1, [], 2)),
        ("CCX", (5, 2, 8), controlled(I.g_x(), 2), (2, [2, 5], 1)),
        ("CU", (1, 4), controlled(I.g_haar(rng, 2), 1), (0, [1], 1)),
        ("C2U", (9, 0, 3, 6), controlled(I.g_haar(rng, 4), 2), (0, [0, 9], 2)),
        ("CU4", (11, 0, 3, 6, 2), controlled(I.g_haar(rng, 16), 1), (0, [11], 4)),
        ("SU4", (2, 3), I.g_haar(rng, 4), (0, [], 2)),
    ]
    for name, tg, m, want in cases:
        assert qs.gate_class(tg, m) == want, (name, qs.gate_class(tg, m), want)


def test_control_on_the_low_local_bit():
    """A control that is the second-listed target (the least significant
    local bit): CX with the control listed last."""
    m = np.zeros((4, 4), dtype=np.complex128)
    # |t c>: flip t when c = 1; local index = 2 t + c
    for t in range(2):
        for c in range(2):
            m[2 * (t ^ c) + c, 2 * t + c] = 1
    assert qs.gate_class((4, 1), m) == (2, [1], 1)


def test_identity_keeps_one_target():
    """The identity is never all-controls: one target stays (a diagonal of
    ones, which the kernel then skips)."""
    kind, ctrl, act = qs.gate_class((1, 2, 3), np.eye(8))
    assert act >= 1 and kind == 1
