"""HBM calibration: a plain device copy of known size, and the library's own
permutation pass, timed with events.

Two uses:
  * the bandwidth ceilings the blocked pass is compared against (a copy and
    an in-place gathered pass over a 16 GiB complex128 state);
  * the reference for hardware counters: under `rocprofv3 --pmc FETCH_SIZE`
    (then WRITE_SIZE) the copy kernel moves exactly --gib GiB each way, so
    the counter's reading for it turns counter units into bytes.

    python -m paper_2406_14084_amd.calib_copy [--gib 16] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=int, default=16)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-swap", action="store_true", help="copy only")
    a = ap.parse_args(argv)
    import torch
    from . import qs
    nbytes = a.gib << 30
    src = torch.ones(nbytes // 16, dtype=torch.complex128, device="cuda")
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {"bytes_each_way": nbytes}
    dst.copy_(src)
    ms = []
    for _ in range(a.reps):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        ev[1].synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    out["copy_ms_best"] = min(ms)
    out["copy_gbs"] = 2 * nbytes / (min(ms) * 1e-3) / 1e9
    print("copy: %d GiB each way, best %.2f ms, %.0f GB/s" % (a.gib, min(ms), out["copy_gbs"]), flush=True)
    del dst
    if not a.no_swap:
        n = (nbytes // 16).bit_length() - 1
        st = qs.State(n, "c128", tensor=src)
        for name, aa, bb in (("4 low + 8 high qubits", (4, 5, 6, 7), (n - 1, n - 2, n - 3, n - 4)),
                             ("2 low qubits exchanged with 2 high", (0, 1), (n - 1, n - 2))):
            st.swap_qubits(aa, bb)
            ms = []
            for _ in range(a.reps):
                ev[0].record()
                st.swap_qubits(aa, bb)
                ev[1].record()
                ev[1].synchronize()
                ms.append(ev[0].elapsed_time(ev[1]))
            gbs = 2 * nbytes / (min(ms) * 1e-3) / 1e9
            out["swap_pass_" + name] = gbs
            print("in-place permutation pass (%s): best %.2f ms, %.0f GB/s" % (name, min(ms), gbs), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
