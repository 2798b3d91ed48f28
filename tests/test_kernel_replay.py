"""CPU replay of the blocked kernel's program (host only, no GPU).

The encoded program of a plan is interpreted here with exactly the index
arithmetic of the HIP kernel (chunk base from the workgroup index, thread
and register bits of each layout, XOR-swizzled LDS slots, P_in / P_out
addresses, register masks of dense ops, bit lists of diagonal ops).  The
replay asserts that every global and LDS index stays in bounds, that each
load, exchange and store is a bijection, and that the result equals the CPU
oracle.  This checks the kernel's indexing before it ever runs on a GPU.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs

PROG_HDR, PHASE_HDR, OP_WORDS = 8, 4, 4
MAP_WORDS = 44   # words of the load/store map before a block's table


def _pdep(v, mask):
    r, i = 0, 0
    for b in range(8):
        if (mask >> b) & 1:
            r |= ((v >> i) & 1) << b
            i += 1
    return r


def _pext(v, mask):
    r = np.zeros_like(v)
    i = 0
    for b in range(16):
        if (mask >> b) & 1:
            r |= ((v >> b) & 1) << i
            i += 1
    return r


def _thread_local(tid, T, tb):
    l = np.zeros_like(tid)
    for j in range(tb):
        l |= ((tid >> j) & 1) << T[j]
    return l


def _local_to_phys(l, P, C):
    o = np.zeros(l.shape, dtype=np.int64)
    for b in range(C):
        o |= ((l >> b) & 1).astype(np.int64) << int(P[b])
    return o


def _swz(l, swlo, swhi):
    f = np.zeros_like(l)
    h = l >> 4
    for b in range(8):
        f ^= np.where((h >> b) & 1, (swlo >> (4 * b)) & 15, 0)
    for b in range(2):
        f ^= np.where((h >> (8 + b)) & 1, (swhi >> (4 * b)) & 15, 0)
    f ^= np.where((l >> 3) & 1, (swhi >> 28) & 7, 0)
    return l ^ f


def _replay_mfma(v, mask, k, A, R, tb):
    """The wave algorithm of the matrix-core op: registers -> the wave's LDS
    region S[element][vector] -> B operands -> 32x32x2 products with the
    documented operand layouts (A[i][k], B[k][j] in lane i|j + 32 k; D[i][j] in
    lane j + 32 ((i / 4) % 2), accumulator 4 (i / 8) + i % 4) -> S -> registers."""
    assert R == 5 and k in (4, 5) and bin(mask).count("1") == k and mask < 32
    nth = 1 << tb
    assert nth % 64 == 0
    D, NV, NMB = 1 << k, 64 << (5 - k), (1 << k) // 16
    A = np.asarray(A[:NMB * D * 64], dtype=np.float64).reshape(NMB, D, 64)
    nw = v.shape[0]
    vw = v.reshape(nw, nth // 64, 64, 32)
    S = np.zeros((nw, nth // 64, D, NV), dtype=np.complex128)
    rest = 31 & ~mask
    for m in range(32):
        c, e = _pext(m, mask), _pext(m, rest)
        S[:, :, c, 64 * e:64 * e + 64] = vw[:, :, :, m]
    for t in range(NV // 32):
        # B operand of step s, lane (n, h): part s % 2 of element 2 (s // 2) + h of vector 32 t + n
        B = np.zeros((nw, nth // 64, D, 64))
        for s in range(D):
            for h in (0, 1):
                x = S[:, :, 2 * (s // 2) + h, 32 * t:32 * t + 32]
                B[:, :, s, 32 * h:32 * h + 32] = x.real if s % 2 == 0 else x.imag
        for mb in range(NMB):
            acc = np.zeros((nw, nth // 64, 32, 32))
            for s in range(D):
                Aop = np.stack([A[mb, s, 0:32], A[mb, s, 32:64]], axis=1)                 # A[i][kk]
                Bop = np.stack([B[:, :, s, 0:32], B[:, :, s, 32:64]], axis=2)             # B[kk][j]
                acc += np.einsum("ik,wvkj->wvij", Aop, Bop)
            # D in lanes/accumulators, then as the kernel stores it: accumulators g, g + 1 of
            # lane (n, h) -> element 16 mb + 4 (g / 4) + 2 h + (g % 4) / 2 of vector 32 t + n
            lanes = np.zeros((nw, nth // 64, 64, 16))
            for i in range(32):
                for j in range(32):
                    lanes[:, :, j + 32 * ((i // 4) % 2), 4 * (i // 8) + i % 4] = acc[:, :, i, j]
            for lane in range(64):
                n_, h = lane % 32, lane // 32
                for g in range(0, 16, 2):
                    row = 16 * mb + 4 * (g // 4) + 2 * h + (g % 4) // 2
                    S[:, :, row, 32 * t + n_] = lanes[:, :, lane, g] + 1j * lanes[:, :, lane, g + 1]
    out = np.empty_like(vw)
    for m in range(32):
        c, e = _pext(m, mask), _pext(m, rest)
        out[:, :, :, m] = S[:, :, c, 64 * e:64 * e + 64]
    return out.reshape(v.shape)


def replay_block(psi, w, n, R, mats, c64=False):
    nph, C = int(w[0]), int(w[1])
    assert int(w[2]) == R
    tb = C - R
    NR = 1 << R
    Pin = [int(x) for x in w[PROG_HDR:PROG_HDR + C]]
    Pout = [int(x) for x in w[PROG_HDR + C:PROG_HDR + 2 * C]]
    assert sorted(Pin) == sorted(Pout) and len(set(Pin)) == C and max(Pin) < n
    comp = [q for q in range(n) if q not in Pin]
    nwg = 1 << (n - C)
    wg = np.arange(nwg, dtype=np.int64)
    base = np.zeros(nwg, dtype=np.int64)
    for bi, q in enumerate(comp):
        base |= ((wg >> bi) & 1) << q
    tid = np.arange(1 << tb, dtype=np.int64)
    ph = PROG_HDR + 2 * C
    tab_off, tab_words = int(w[4]), int(w[5])
    # the kernel stages the table in 16-byte words from a 16-byte aligned block program
    assert tab_off % 4 == 0 and tab_words % 4 == 0 and (tab_words == 0 or tab_off >= ph)
    # the table plus the exchange buffer (half the chunk in half-buffer blocks) must fit 160 KiB
    half = (int(w[3]) & 4) != 0
    assert ((8 if c64 else 16) << (C - 1 if half else C)) + 4 * tab_words <= 160 * 1024

    def layout(at):
        Rb = [int(x) for x in w[at + PHASE_HDR:at + PHASE_HDR + R]]
        T = [int(x) for x in w[at + PHASE_HDR + R:at + PHASE_HDR + C]]
        assert sorted(Rb + T) == list(range(C)), (Rb, T)
        return Rb, T

    def gidx(Rb, T, P):
        g = base[:, None] | _local_to_phys(_thread_local(tid, T, tb), P, C)[None, :]
        o = np.array([sum(1 << P[Rb[j]] for j in range(R) if (m >> j) & 1) for m in range(NR)], dtype=np.int64)
        return g[:, :, None] | o[None, None, :]

    # the load/store map right before the table: the kernel takes its global addresses from
    # it; it must agree with the first and last phases' layouts
    mp = [int(x) for x in w[tab_off - MAP_WORDS:tab_off]]
    assert (mp[26] & 0xffffffff) | ((mp[27] & 0xffffffff) << 32) == sum(1 << q for q in Pin)
    assert all(x == 0 for x in mp[tb:16] + mp[16 + R:21] + mp[21 + R:26] + mp[28 + tb:44])

    def midx(tcol, rcol):
        g = np.zeros_like(tid)
        for j in range(tb):
            g |= ((tid >> j) & 1) << mp[tcol + j]
        o = np.array([sum(1 << mp[rcol + j] for j in range(R) if (m >> j) & 1) for m in range(NR)], dtype=np.int64)
        return (base[:, None] | g[None, :])[:, :, None] | o[None, None, :]

    Rb, T = layout(ph)
    li = midx(0, 16)
    assert np.array_equal(li, gidx(Rb, T, Pin)), "load map disagrees with the first layout"
    assert li.min() >= 0 and li.max() < (1 << n)
    assert np.unique(li).size == li.size == (1 << n), "load is not a bijection"
    v = psi[li]
    prev = None
    for p in range(nph):
        nops = int(w[ph])
        Rb, T = layout(ph)
        if p > 0:
            swlo, swhi = int(np.uint32(w[ph + 1])), int(np.uint32(w[ph + 2]))
            pR, pT = layout(prev)
            wt = _swz(_thread_local(tid, pT, tb), swlo, swhi)
            rt = _swz(_thread_local(tid, T, tb), swlo, swhi)
            wl = np.array([int(_swz(np.array([sum(1 << pR[j] for j in range(R) if (m >> j) & 1)]), swlo, swhi)[0])
                           for m in range(NR)])
            rl = np.array([int(_swz(np.array([sum(1 << Rb[j] for j in range(R) if (m >> j) & 1)]), swlo, swhi)[0])
                           for m in range(NR)])
            ws = wt[:, None] ^ wl[None, :]
            rs = rt[:, None] ^ rl[None, :]
            # the kernel forms the same slots from the program's exchange block
            X = ph + PHASE_HDR + C
            ab = 8 if c64 else 16
            xw = [int(x) for x in w[X:X + tb]]
            xr = [int(x) for x in w[X + tb:X + 2 * tb]]
            wo = np.array([int(x) for x in w[X + 2 * tb:X + 2 * tb + NR]])
            ro = np.array([int(x) for x in w[X + 2 * tb + NR:X + 2 * tb + 2 * NR]])
            kw = np.zeros_like(tid)
            kr = np.zeros_like(tid)
            for j in range(tb):
                kw ^= np.where((tid >> j) & 1, xw[j], 0)
                kr ^= np.where((tid >> j) & 1, xr[j], 0)
            hx = int(np.uint32(w[ph + 3])) >> 24
            hjw, hjr = (hx & 15) - 1, (hx >> 4) - 1
            assert (hjw >= 0) == half == (hjr >= 0)
            if hjw >= 0:
                # split bit: a thread bit in both layouts (positions hjw, hjr), dropped from the addresses
                assert pT[hjw] == T[hjr] and T[hjr] >= 4
                bb = T[hjr] + (3 if c64 else 4)
                drop = lambda x: (x & ((1 << bb) - 1)) | ((x >> (bb + 1)) << bb)
                assert np.array_equal(kw[:, None] ^ wo[None, :], drop(ws * ab))
                assert np.array_equal(kr[:, None] ^ ro[None, :], drop(rs * ab))
            else:
                assert np.array_equal(kw[:, None] ^ wo[None, :], ws * ab)
                assert np.array_equal(kr[:, None] ^ ro[None, :], rs * ab)
            xt = int(w[ph + 3]) & 0xffffff
            if xt > 0:   # the kernel forms kw, kr from per-nibble XOR tables in the LDS table
                a = xt - 1
                NIB = 34
                assert a + 2 * NIB <= tab_words and tb <= 9
                tabv = np.array([int(x) for x in w[tab_off + a:tab_off + a + 2 * NIB]], dtype=np.int64)
                for side, want in ((0, kw), (1, kr)):
                    t0 = tabv[side * NIB:side * NIB + 16]
                    t1 = tabv[side * NIB + 16:side * NIB + 32]
                    t2 = tabv[side * NIB + 32:side * NIB + 34]
                    got = t0[tid & 15] ^ t1[(tid >> 4) & 15] ^ t2[(tid >> 8) & 1]
                    assert np.array_equal(got, want)
            for s in (ws, rs):
                assert s.min() >= 0 and s.max() < (1 << C)
                assert np.unique(s).size == s.size == (1 << C), "exchange is not a bijection"
            if hjw < 0:
                lds = np.zeros((nwg, 1 << C), dtype=np.complex128)
                lds[:, ws.reshape(-1)] = v.reshape(nwg, -1)
                v = lds[:, rs.reshape(-1)].reshape(nwg, 1 << tb, NR)
            else:
                # two rounds through half the buffer, as the kernel runs them
                cw = (kw[:, None] ^ wo[None, :]) // ab
                cr = (kr[:, None] ^ ro[None, :]) // ab
                v = v.copy()
                # registers are updated in place, round by round, as in the kernel
                v = v.copy()
                for h in (0, 1):
                    sw_, sr_ = ((tid >> hjw) & 1) == h, ((tid >> hjr) & 1) == h
                    for s in (cw[sw_], cr[sr_]):
                        assert s.min() >= 0 and s.max() < (1 << (C - 1))
                        assert np.unique(s).size == s.size == (1 << (C - 1)), "half round is not a bijection"
                    lds = np.full((nwg, 1 << (C - 1)), np.nan, dtype=np.complex128)
                    lds[:, cw[sw_].reshape(-1)] = v[:, sw_, :].reshape(nwg, -1)
                    v[:, sr_, :] = lds[:, cr[sr_].reshape(-1)].reshape(nwg, -1, NR)
        op = ph + PHASE_HDR + C + 2 * tb + 2 * NR
        for _ in range(nops):
            w0 = int(w[op])
            kind, variant, k = w0 & 0xff, (w0 >> 8) & 0xff, (w0 >> 16) & 0xff
            moff = int(np.uint32(w[op + 1])) | (int(w[op + 2]) << 32)
            if kind == 12:        # padding no-op
                pass
            elif kind == 0:
                assert bin(variant).count("1") == k and variant < NR
                D = 1 << k
                M = mats[moff:moff + 2 * D * D].view(np.complex128).reshape(D, D)
                out = v.copy()
                for b0 in range(NR):
                    if b0 & variant:
                        continue
                    cols = [b0 | _pdep(c, variant) for c in range(D)]
                    vin = v[:, :, cols]
                    res = np.einsum("rc,wtc->wtr", M, vin)
                    out[:, :, cols] = res
                v = out
            elif kind == 9:       # multi-controlled X: flip register bit t where the controls hold cval
                t, ctrl = variant & 7, variant >> 3
                cval = int(w[op + 3])
                assert t < R and ctrl < NR and not (ctrl >> t) & 1 and (cval & ~ctrl) == 0
                src = np.array([m ^ (1 << t) if (m & ctrl) == cval else m for m in range(NR)])
                v = v[:, :, src]
            elif kind == 10:      # SWAP of register bits a < b
                a, b = variant & 7, variant >> 3
                assert a < b < R
                src = np.array([(m & ~((1 << a) | (1 << b))) | (((m >> a) & 1) << b) | (((m >> b) & 1) << a)
                                for m in range(NR)])
                v = v[:, :, src]
            elif kind == 6:       # one 2x2 gate per register bit of the mask, ascending
                idx = 0
                for j in range(R):
                    if not (variant >> j) & 1:
                        continue
                    M = mats[moff + 8 * idx:moff + 8 * idx + 8].view(np.complex128).reshape(2, 2)
                    out = v.copy()
                    for b0 in range(NR):
                        if (b0 >> j) & 1:
                            continue
                        cols = [b0, b0 | (1 << j)]
                        out[:, :, cols] = np.einsum("rc,wtc->wtr", M, v[:, :, cols])
                    v = out
                    idx += 1
            elif kind == 8 or kind == 11:  # two shears per register bit, ascending;
                # kind 11: then a diagonal on the registers (2^R entries after the coefficients)
                idx = 0
                for j in range(R):
                    if not (variant >> j) & 1:
                        continue
                    beta, alpha = float(mats[moff + 2 * idx]), float(mats[moff + 2 * idx + 1])
                    assert abs(beta) <= 0.5 + 1e-15 and abs(alpha) <= 1 + 1e-15
                    lo = [m for m in range(NR) if not (m >> j) & 1]
                    hi = [m | (1 << j) for m in lo]
                    x0, x1 = v[:, :, lo].copy(), v[:, :, hi].copy()
                    x0 = x0 + beta * x1
                    x1 = x1 + alpha * x0
                    v = v.copy()
                    v[:, :, lo], v[:, :, hi] = x0, x1
                    idx += 1
                if kind == 11:
                    E = mats[moff + 2 * idx:moff + 2 * idx + 2 * NR].view(np.complex128)
                    v = v * E[None, None, :]
            elif kind == 2:       # register diagonal: uniform entry per register
                E = mats[moff:moff + 2 * NR].view(np.complex128)
                v = v * E[None, None, :]
            elif kind == 3:       # per-row diagonal: row = pext(tid, tmask)
                tmask = int(w[op + 1])
                row = _pext(tid, tmask)
                kt = bin(tmask).count("1")
                rm = variant >> 1  # register positions of the op: 2^kr entries per row
                assert rm < NR and variant < 64
                ne = 1 << bin(rm).count("1")
                ent = np.array([_pext(m, rm) for m in range(NR)])
                if variant & 1:   # rows in device memory (table too large for LDS)
                    goff = int(np.uint32(w[op + 2])) | (int(w[op + 3]) << 32)
                    E = mats[goff:goff + 2 * ne * (1 << kt)].view(np.complex128).reshape(1 << kt, ne)
                else:             # rows in the LDS table
                    wpe = 2 if c64 else 4
                    a = tab_off + int(w[op + 3])
                    assert a % 4 == 0 and int(w[op + 3]) + wpe * ne * (1 << kt) <= tab_words
                    raw = np.ascontiguousarray(w[a:a + wpe * ne * (1 << kt)])
                    E = (raw.view(np.complex64).astype(np.complex128) if c64 else raw.view(np.complex128))
                    E = E.reshape(1 << kt, ne)
                v = v * E[row][:, ent][None, :, :]
            elif kind == 7:       # complex64 dense op on matrix cores, emulated lane by lane
                v = _replay_mfma(v, variant, k, mats[moff:], R, tb)
            elif kind == 4:       # +-1 on registers
                s = int(np.uint32(w[op + 3]))
                sg = np.array([-1.0 if (s >> m) & 1 else 1.0 for m in range(NR)])
                v = v * sg[None, None, :]
            elif kind == 5:       # +-1 per row, masks in the LDS table
                tmask = int(w[op + 1])
                row = _pext(tid, tmask)
                kt = bin(tmask).count("1")
                a = tab_off + int(w[op + 3])
                assert int(w[op + 3]) + (1 << kt) <= tab_words
                masks = np.array([int(np.uint32(x)) for x in w[a:a + (1 << kt)]], dtype=np.int64)
                s = masks[row]
                sg = np.where(((s[:, None] >> np.arange(NR)[None, :]) & 1) == 1, -1.0, 1.0)
                v = v * sg[None, :, :]
            else:
                raise AssertionError("unknown op kind %d" % kind)
            op += OP_WORDS
        prev = ph
        ph = op
    Rb, T = layout(prev)
    assert (int(np.uint32(w[3])) >> 8) == prev, "flags word must locate the last phase (store layout)"
    # pending X gates: the store inverts these physical bits of every address
    inv = (int(np.uint32(w[6])) | (int(np.uint32(w[7])) << 32))
    assert inv & ~sum(1 << q for q in Pout) == 0
    assert tab_off - MAP_WORDS >= ph, "load/store map overlaps the phases"
    so = midx(28, 21) ^ inv
    assert np.array_equal(so, gidx(Rb, T, Pout) ^ inv), "store map disagrees with the last layout"
    assert so.min() >= 0 and so.max() < (1 << n)
    assert np.unique(so).size == so.size == (1 << n), "store is not a bijection"
    for i in range(nwg):   # each workgroup writes exactly what it read
        assert np.array_equal(np.sort(so[i].reshape(-1)), np.sort(li[i].reshape(-1)))
    # Without an exchange there is no barrier between loads and stores: then a
    # thread may only overwrite positions it loaded itself, unless the program
    # asks the kernel for a barrier (flag bit 1).
    if nph == 1 and not (int(w[3]) & 2):
        assert np.array_equal(np.sort(so, axis=2), np.sort(li, axis=2)), "store/load race between threads"
    if Pin != Pout or inv:
        assert int(w[3]) & 2
    out = psi.copy()
    out[so] = v
    return out


def replay_plan(plan, n, psi0=None):
    w, offs, R, C, mats = plan.program()
    if psi0 is None:
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1
    else:
        psi = np.array(psi0, dtype=np.complex128)
    c64 = plan.stats()["dtype"] == 1
    assert all(int(o) % 4 == 0 for o in offs)
    for o in offs:
        psi = replay_block(psi, w[o:], n, R, mats, c64)
    return psi


@pytest.mark.parametrize("cfg", [
    dict(n=6, seed=1, kmax=3), dict(n=10, seed=2, kmax=4), dict(n=12, seed=3, kmax=5),
    dict(n=12, seed=4, kmax=4, chunk_qubits=9, low_qubits=3),
    dict(n=13, seed=5, kmax=4, swaps=False), dict(n=13, seed=6, kmax=2, fusion=False),
    dict(n=12, seed=7, kmax=5, reg_qubits=5), dict(n=11, seed=8, kmax=3, chunk_qubits=7, reg_qubits=3),
    dict(n=3, seed=9, kmax=3), dict(n=1, seed=10, kmax=1), dict(n=12, seed=11, kmax=3, planner=2),
    dict(n=14, seed=12, kmax=4, chunk_qubits=8), dict(n=15, seed=13, kmax=2, chunk_qubits=9, low_qubits=2),
    dict(n=14, seed=14, kmax=3, chunk_qubits=12, reg_qubits=3),
])
def test_replay_matches_oracle(cfg):
    cfg = dict(cfg)
    n, seed = cfg.pop("n"), cfg.pop("seed")
    c = I.random_dense(n, 80, seed, kmax=min(3, n))
    p = qs.Plan(c, **cfg)
    got = replay_plan(p, n)
    want = sim.run(c)
    assert np.max(np.abs(got - want)) <= 1e-12


def test_replay_u3_cz_and_layered():
    """Includes blocks whose exchanges run in two rounds through half the LDS
    buffer (U3 + CZ: rotations and diagonals only)."""
    halves = 0
    for c in (I.random_u3_2q(n=14, depth=12, seed=3), I.layered_rotations(n=13, layers=8, seed=4),
              I.random_u3_2q(n=16, depth=10, seed=1)):
        p = qs.Plan(c, kmax=5)
        w, offs, R, C, mats = p.program()
        halves += sum(1 for o in offs if int(w[o + 3]) & 4)
        assert np.max(np.abs(replay_plan(p, c.n) - sim.run(c))) <= 1e-12
    assert halves > 0
    # complex64 (8-byte amplitudes: the split bit sits one position lower in the byte address)
    c = I.random_u3_2q(n=15, depth=10, seed=15)
    p = qs.Plan(c, kmax=5, dtype="c64")
    w, offs, R, C, mats = p.program()
    assert sum(1 for o in offs if int(w[o + 3]) & 4) > 0
    assert np.max(np.abs(replay_plan(p, c.n) - sim.run(c))) <= 1e-6


def test_replay_swap_plan_is_bit_permutation():
    """A plan with only swap passes moves amplitudes exactly as Eq. 4."""
    # qs_swap_qubits builds its program inside the library; the same passes
    # appear in plans whose final layout needs restoring, covered above.  Here:
    # a circuit of SWAP gates only, planned with swaps on.
    n = 12
    c = I.Circuit(n)
    rng = np.random.default_rng(3)
    for _ in range(10):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        c.add("SWAP", (a, b), I.g_swap())
    p = qs.Plan(c, kmax=2)
    got = replay_plan(p, n)
    assert np.max(np.abs(got - sim.run(c))) <= 1e-15


def test_replay_covers_folded_swaps_and_swap_passes():
    """The configurations above include blocks whose write-back permutes
    qubits and standalone swap passes (so the race check above is exercised)."""
    c = I.random_dense(14, 80, 12, kmax=3)
    p = qs.Plan(c, kmax=4, chunk_qubits=8)
    w, offs, R, C, mats = p.program()
    flags = [int(w[o + 3]) for o in offs]
    assert any(f & 1 for f in flags) and any(f & 2 for f in flags)


def test_replay_uses_every_diagonal_encoding():
    """Circuits with general and +-1 diagonals exercise the register, row and
    sign encodings of diagonal ops; with single-qubit gates split (phase,
    rotation, phase) and kept whole, also the rotation and grouped
    single-qubit encodings, and rotations fused with the diagonal after them."""
    n = 13
    kinds = set()
    for seed in range(4):
        c = I.random_u3_2q(n=n, depth=6, seed=seed)
        rng = np.random.default_rng(seed)
        for _ in range(20):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            c.add("RZZ", (a, b), I.g_rzz(float(rng.uniform(0, 6))))
        c2 = I.random_dense(9, 60, 50 + seed, kmax=3, kinds=("dense", "diag"))
        for cc in (c, c2):
            for split in (True, False):
                p = qs.Plan(cc, kmax=4, split=split)
                kinds |= _op_kinds(p)
                assert np.max(np.abs(replay_plan(p, cc.n) - sim.run(cc))) <= 1e-12
    assert {0, 2, 3, 4, 5, 6, 8, 11} <= kinds, kinds


def test_split_needs_a_unitary_gate():
    """Only gates that the phase * rotation * phase factorisation reproduces
    are split: a non-unitary single-qubit matrix stays a dense op, and the
    replayed state (unitary and non-unitary gates mixed) equals the oracle's."""
    n = 9
    c = I.random_u3_2q(n=n, depth=4, seed=41)
    c.add("M", (3,), np.array([[1.0, 0.0], [0.5, 1.0]], dtype=np.complex128))
    c.add("M", (5,), np.array([[0.6, 0.8j], [0.8j, 0.6]], dtype=np.complex128))   # unitary
    p = qs.Plan(c, kmax=3)
    s = p.stats()
    assert s["ops_dense"][1] == 1 and s["ops_rot"] >= 1 + n * 4
    assert np.max(np.abs(replay_plan(p, n) - sim.run(c))) <= 1e-12


def _op_kinds(p):
    kinds = set()
    w, offs, R, C, mats = p.program()
    for o in offs:
            nph = int(w[o]); ph = o + PROG_HDR + 2 * C
            for _ in range(nph):
                nops = int(w[ph]); op = ph + PHASE_HDR + C + 2 * (C - R) + 2 * (1 << R)
                for _ in range(nops):
                    kinds.add(int(w[op]) & 0xff); op += OP_WORDS
                ph = op
    return kinds


def test_exchange_swizzle_spreads_lanes():
    """For every exchange of the 30-qubit benchmark plan, lanes 0-7 of a
    wavefront hit 8 distinct 16-byte LDS slots mod 128 B and lanes 0-15 hit 16
    distinct slots mod 256 B, on both the write and the read side."""
    c = I.random_u3_2q(n=30, depth=40, seed=30002)
    p = qs.Plan(c, kmax=5)
    w, offs, R, C, mats = p.program()
    lanes = np.arange(64, dtype=np.int64)
    bad = 0
    total = 0
    for o in offs:
        nph = int(w[o]); ph = o + PROG_HDR + 2 * C; pT = None
        for i in range(nph):
            T = [int(x) for x in w[ph + PHASE_HDR + R:ph + PHASE_HDR + C]]
            if i > 0:
                swlo, swhi = int(np.uint32(w[ph + 1])), int(np.uint32(w[ph + 2]))
                for TT in (pT, T):
                    s = _swz(_thread_local(lanes, TT, C - R), swlo, swhi)
                    total += 1
                    if len(set((s[:8] & 7).tolist())) < 8 or len(set((s[:16] & 15).tolist())) < 16:
                        bad += 1
            pT = T
            ph = ph + PHASE_HDR + C + 2 * (C - R) + 2 * (1 << R) + OP_WORDS * int(w[ph])
    assert total > 0 and bad == 0, (bad, total)


def _diag_row_variants(p):
    out = set()
    w, offs, R, C, mats = p.program()
    for o in offs:
        nph = int(w[o]); ph = o + PROG_HDR + 2 * C
        for _ in range(nph):
            nops = int(w[ph]); op = ph + PHASE_HDR + C + 2 * (C - R) + 2 * (1 << R)
            for _ in range(nops):
                if int(w[op]) & 0xff == 3:
                    out.add((int(w[op]) >> 8) & 1)
                op += OP_WORDS
            ph = op
    return out


def _five_qubit_circuit(n, seed, count=10):
    rng = np.random.default_rng(seed)
    c = I.random_dense(n, 60, seed, kmax=3)
    for _ in range(count):
        tg = tuple(int(x) for x in rng.choice(n, 5, replace=False))
        c.add("U5", tg, I.g_haar(rng, 32))
    return c


@pytest.mark.parametrize("cfg", [
    dict(n=13, seed=1), dict(n=14, seed=2, chunk_qubits=11), dict(n=15, seed=3, chunk_qubits=12),
    dict(n=16, seed=4, swaps=False),
])
def test_replay_complex64_matrix_core_ops(cfg):
    """Complex64 plans encode dense ops of 4-5 qubits for the matrix cores;
    the lane-by-lane emulation of the kernel's algorithm (with the program's
    FP64 copy of the operands) reproduces the oracle; an index mistake in the
    operand or result layouts would show as O(1) errors."""
    cfg = dict(cfg)
    n, seed = cfg.pop("n"), cfg.pop("seed")
    c = _five_qubit_circuit(n, seed)
    p = qs.Plan(c, kmax=5, dtype="c64", **cfg)
    s = p.stats()
    assert s["ops_mfma"] > 0 and 7 in _op_kinds(p)
    assert s["ops_mfma"] <= s["ops_dense"][4] + s["ops_dense"][5]
    # complex64 LDS tables of diagonals hold FP32 entries (rounded once): ~1e-9 here
    assert np.max(np.abs(replay_plan(p, n) - sim.run(c))) <= 1e-7
    q = qs.Plan(c, kmax=5, dtype="c64", mfma=False, **cfg)
    assert q.stats()["ops_mfma"] == 0 and 7 not in _op_kinds(q)


def test_matrix_core_ops_need_full_waves():
    """No matrix-core op where a workgroup has less than a wavefront of threads
    or the plan is complex128."""
    c = _five_qubit_circuit(12, 5)
    assert qs.Plan(c, kmax=5, dtype="c64", chunk_qubits=10).stats()["ops_mfma"] == 0
    assert qs.Plan(c, kmax=5, dtype="c128").stats()["ops_mfma"] == 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_replay_large_diagonal_tables_spill(dtype):
    """Diagonals merged over many thread bits make row tables larger than the
    16 KiB the LDS keeps for tables; those tables are read from device memory
    (DIAG_ROW variant bit 0) and the replay still matches the oracle."""
    n = 13        # one block: every diagonal of the circuit lands in one table
    rng = np.random.default_rng(7)
    c = I.Circuit(n)
    for _ in range(40):
        tg = tuple(int(x) for x in rng.choice(n, 5, replace=False))
        c.add("D5", tg, np.diag(np.exp(1j * rng.uniform(0, 6.3, 32))))
        c.add("H", (int(rng.integers(n)),), I.g_h())
    p = qs.Plan(c, kmax=5, chunk_qubits=13, reg_qubits=3, dtype=dtype)
    assert _diag_row_variants(p) == {0, 1}
    tol = 1e-7 if dtype == "c64" else 1e-12
    assert np.max(np.abs(replay_plan(p, n) - sim.run(c))) <= tol


def _perm_circuit(n, ngates, seed, with_rot=True):
    """X, CX (both orientations), CCX and SWAP on random qubits, optionally
    interleaved with U3 gates."""
    rng = np.random.default_rng(seed)
    c = I.Circuit(n)
    for _ in range(ngates):
        kind = int(rng.integers(0, 5 if with_rot else 4))
        if kind == 0:
            c.add("X", (int(rng.integers(n)),), I.g_x())
        elif kind == 1:
            c.add("CX", tuple(int(x) for x in rng.choice(n, 2, replace=False)), I.g_cx())
        elif kind == 2:
            m = np.eye(8, dtype=np.complex128)
            m[[6, 7]] = m[[7, 6]]
            c.add("CCX", tuple(int(x) for x in rng.choice(n, 3, replace=False)), m)
        elif kind == 3:
            c.add("SWAP", tuple(int(x) for x in rng.choice(n, 2, replace=False)), I.g_swap())
        else:
            c.add("U3", (int(rng.integers(n)),), I.g_u3(*rng.uniform(0, 6.3, 3)))
    return c


@pytest.mark.parametrize("dtype,reg", [("c128", 0), ("c128", 3), ("c64", 0)])
def test_replay_permutation_ops(dtype, reg):
    """X, CX, CCX and SWAP become permutation ops (register moves, no
    arithmetic): a pure permutation circuit replays bit for bit, and one mixed
    with U3 gates matches the oracle; U3 + CX plans no longer fuse the CXs
    into dense two-qubit ops."""
    n = 14
    c = _perm_circuit(n, 200, 5, with_rot=False)
    p = qs.Plan(c, kmax=5, dtype=dtype, reg_qubits=reg)
    s = p.stats()
    assert s["ops_perm"] > 0 and s["flops_per_amp"] == 0 and 9 in _op_kinds(p) and 10 not in _op_kinds(p)
    rng = np.random.default_rng(1)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    got = replay_plan(p, n, psi0=psi0)
    want = psi0.copy()
    sim.apply_circuit(want, c)
    assert np.array_equal(got, want)
    c = _perm_circuit(n, 200, 6, with_rot=True)
    p = qs.Plan(c, kmax=5, dtype=dtype, reg_qubits=reg)
    assert p.stats()["ops_perm"] > 0
    tol = 1e-6 if dtype == "c64" else 1e-12
    assert np.max(np.abs(replay_plan(p, n) - sim.run(c))) <= tol
    c = I.random_u3_2q(n=20, depth=8, seed=3, two="CX")
    s = qs.Plan(c, kmax=5, dtype=dtype).stats()
    assert s["ops_perm"] > 0 and s["ops_dense"][2] + s["ops_dense"][3] < s["ops_perm"], s


def _flip_masks(p):
    w, offs, R, C, mats = p.program()
    return [(int(np.uint32(w[o + 6])) | (int(np.uint32(w[o + 7])) << 32), int(w[o + 3])) for o in offs]


def test_pending_x_store_mask():
    """A single-qubit gate with a rotation angle above pi/4 is run as X U' (U' well
    conditioned) with the X left pending: later gates of the block on that qubit are
    conjugated (a CX controlled by it becomes a CX on 0), X gates only toggle the
    pending set (no op at all), and the block's store inverts the pending bits
    (header words 6-7, with the load/store barrier flag).  The replay must match
    the oracle, and the rotations' shear coefficients stay within |beta| <= 1/2,
    |alpha| <= 1 (asserted by the replay)."""
    n = 12
    c = I.Circuit(n)
    c.add("RY", (3,), I.g_ry(2.6))                  # theta/2 = 1.3 > pi/4: pending X on qubit 3
    c.add("CX", (3, 7), I.g_cx())                    # control carries the pending X
    c.add("X", (10,), I.g_x())                       # a bare X: no op
    c.add("RY", (5,), I.g_ry(0.4))                   # small angle: no X
    c.add("CZ", (3, 10), I.g_cz())                   # diagonal on two pending bits
    c.add("U3", (7,), I.g_u3(2.9, 0.3, -1.1))
    p = qs.Plan(c, kmax=5)
    masks = _flip_masks(p)
    assert any(m for m, _ in masks)
    for m, flags in masks:
        if m:
            assert flags & 2                          # loads before stores
    got = replay_plan(p, n)
    assert np.max(np.abs(got - sim.run(c))) <= 1e-12
    # X gates alone: no op and no arithmetic, the state permuted by the store only
    cx = I.Circuit(n)
    for q in (0, 4, 9, 11, 4):
        cx.add("X", (q,), I.g_x())
    px = qs.Plan(cx, kmax=5)
    s = px.stats()
    assert s["flops_per_amp"] == 0 and s["ops_perm"] == 0
    rng = np.random.default_rng(3)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    want = psi0.copy()
    sim.apply_circuit(want, cx)
    assert np.array_equal(replay_plan(px, n, psi0=psi0), want)


def test_negative_control_mcx_encoding():
    """An X pending on a CX's control turns it into a CX on 0: the op word carries the
    control values (word 3) within the control mask, and the kernel path exists."""
    n = 10
    c = I.Circuit(n)
    c.add("RY", (1,), I.g_ry(2.8))
    c.add("CX", (1, 2), I.g_cx())
    c.add("RY", (2,), I.g_ry(0.3))
    p = qs.Plan(c, kmax=5)
    w, offs, R, C, mats = p.program()
    found = []
    for o in offs:
        nph = int(w[o]); ph = o + PROG_HDR + 2 * C
        for _ in range(nph):
            nops = int(w[ph]); op = ph + PHASE_HDR + C + 2 * (C - R) + 2 * (1 << R)
            for _ in range(nops):
                if int(w[op]) & 0xff == 9:
                    var = (int(w[op]) >> 8) & 0xff
                    found.append((var >> 3, int(w[op + 3])))
                op += OP_WORDS
            ph = op
    assert found and all(cv & ~ctrl == 0 for ctrl, cv in found)
    assert any(cv != ctrl for ctrl, cv in found)      # at least one control on 0
    assert np.max(np.abs(replay_plan(p, n) - sim.run(c))) <= 1e-12


def test_replay_rejects_a_wrong_load_store_map():
    """The kernel takes every global address from the load/store map before the table;
    the replay checks it against the layouts, so a map with two thread-bit positions
    exchanged, a register-bit position changed or a wrong chunk mask must be caught
    (mistakes planted in a host copy of the encoded program)."""
    n = 14
    c = I.random_u3_2q(n=n, depth=6, seed=21)
    p = qs.Plan(c, kmax=5)
    w, offs, R, C, mats = p.program()
    o = int(offs[0])
    blk = np.array(w[o:], copy=True)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    replay_block(psi, blk, n, R, mats)            # the encoded map passes
    mp0 = int(blk[4]) - MAP_WORDS
    for plant in ("swap_thread_bits", "register_bit", "mask"):
        bad = blk.copy()
        if plant == "swap_thread_bits":
            bad[mp0], bad[mp0 + 1] = blk[mp0 + 1], blk[mp0]
        elif plant == "register_bit":
            bad[mp0 + 21] = blk[mp0 + 22]
        else:
            bad[mp0 + 26] = int(blk[mp0 + 26]) ^ 1
        with pytest.raises(AssertionError):
            replay_block(psi, bad, n, R, mats)
