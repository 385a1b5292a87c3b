"""Autotuner for libpfresample's launch parameters (pfr_tuning in the C header).

Times the candidate values of every parameter on the current GPU with HIP
events (median of --reps launches, the 256 MB Infinity Cache flushed before
each), checks that every candidate produces the same bits as the defaults
(the parameters only change how work is split), and writes the winners as a
flat JSON object, which the binding loads at start-up from
paper_1301_4019_amd/tuning.json (or $PFR_TUNING).

    python -m paper_1301_4019_amd.autotune [--out PATH] [--reps 15]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def _b_star(y, eps=0.01):
    from .inputs import expected_weight
    return math.ceil(math.log(eps) / math.log(1.0 - expected_weight(y)))


class Timer:
    def __init__(self, torch, reps):
        self.torch = torch
        self.reps = reps
        self.flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")

    def __call__(self, fn):
        torch = self.torch
        fn()  # warm-up (and first-touch of cached workspaces)
        times = []
        for _ in range(self.reps):
            self.flush.fill_(1)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times))


def tune(reps=15, log=print):
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs

    torch.cuda.set_device(0)
    timer = Timer(torch, reps)
    default = pfr.default_tuning()
    pfr.set_tuning(**default)
    chosen = dict(default)
    meas = {}

    def with_tuning(fields, fn):
        pfr.set_tuning(**{**chosen, **fields})
        try:
            return fn()
        finally:
            pfr.set_tuning(**chosen)

    def same(a, b, what):
        if not torch.equal(a, b):
            raise RuntimeError(f"autotune: {what} changed the result")

    W = {}

    def weights(n, y):
        key = (n, y)
        if key not in W:
            W[key] = torch.from_numpy(inputs.weights(n, y, seed=1000 + n)).cuda()
        return W[key]

    # ---- single_wg_max: one workgroup versus the multi-kernel scan, per length
    rows = {}
    best = 0
    for n in (1024, 2048, 4096, 8192, 16384, 32768):
        w = weights(n, 2.0)
        out = torch.empty(n, dtype=torch.int32, device="cuda")

        def run():
            for s in ("stratified", "systematic", "multinomial"):
                getattr(pfr, "resample_" + s)(w, seed=1, out=out)

        t_one = with_tuning({"single_wg_max": n}, lambda: timer(run))
        ref = out.clone()
        t_multi = with_tuning({"single_wg_max": n - 1}, lambda: timer(run))
        same(out, ref, "single_wg_max")
        rows[n] = {"one_workgroup_ms": t_one, "multi_kernel_ms": t_multi}
        if t_one <= t_multi:
            best = n
        log(f"single_wg_max n={n}: one {t_one:.4f} ms, multi {t_multi:.4f} ms")
    chosen["single_wg_max"] = best
    meas["single_wg_max"] = rows

    # ---- direct_max_blocks: emit workgroups form their own carries, or a carry kernel
    rows = {}
    best = 0
    for lg in (14, 16, 18, 19, 20, 21):
        n = 1 << lg
        nb = n // 1024
        w = weights(n, 2.0)
        out = torch.empty(n, dtype=torch.int32, device="cuda")

        def run():
            pfr.resample_stratified(w, seed=1, out=out)
            pfr.resample_systematic(w, seed=1, out=out)

        t_direct = with_tuning({"direct_max_blocks": min(nb, 2048)}, lambda: timer(run))
        ref = out.clone()
        t_carry = with_tuning({"direct_max_blocks": 0}, lambda: timer(run))
        same(out, ref, "direct_max_blocks")
        rows[n] = {"direct_ms": t_direct, "carry_kernel_ms": t_carry}
        if t_direct <= t_carry and nb <= 2048:
            best = nb
        log(f"direct_max_blocks n=2^{lg}: direct {t_direct:.4f} ms, carries {t_carry:.4f} ms")
    chosen["direct_max_blocks"] = best
    meas["direct_max_blocks"] = rows

    # ---- metropolis_chunk (global-memory kernel), n = 2^20, B = 16
    n = 1 << 20
    w = weights(n, 2.0)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    rows = {}
    ref = None
    for chunk in (256, 512, 1024, 2048, 4096):
        t = with_tuning({"metropolis_chunk": chunk, "metropolis_table_min_B": 0},
                        lambda: timer(lambda: pfr.resample_metropolis(w, 16, seed=1, out=out)))
        if ref is None:
            ref = out.clone()
        same(out, ref, "metropolis_chunk")
        rows[chunk] = t
        log(f"metropolis_chunk {chunk}: {t:.4f} ms")
    chosen["metropolis_chunk"] = min(rows, key=rows.get)
    meas["metropolis_chunk"] = rows

    # ---- metropolis_table_min_B: bound table or not, per y (B from the bias bound)
    rows = {}
    wins = []
    for y in (0.0, 1.0, 2.0, 3.0, 4.0):
        B = _b_star(y)
        w = weights(n, y)
        run = lambda: pfr.resample_metropolis(w, B, seed=1, out=out)  # noqa: E731
        t_tab = with_tuning({"metropolis_table_min_B": 1}, lambda: timer(run))
        ref = out.clone()
        t_plain = with_tuning({"metropolis_table_min_B": 0}, lambda: timer(run))
        same(out, ref, "metropolis_table_min_B")
        rows[B] = {"table_ms": t_tab, "plain_ms": t_plain}
        if t_tab < t_plain:
            wins.append(B)
        log(f"metropolis table y={y} B={B}: table {t_tab:.4f} ms, plain {t_plain:.4f} ms")
    # smallest B from which the table wins at every larger measured B
    Bs = sorted(rows)
    thr = 0
    for b in reversed(Bs):
        if rows[b]["table_ms"] < rows[b]["plain_ms"]:
            thr = b
        else:
            break
    chosen["metropolis_table_min_B"] = thr
    meas["metropolis_table_min_B"] = rows

    # ---- rejection_per_wave and rejection_table, n = 2^20, y = 2..4
    rows = {}
    ref = {}
    for table in (1, 0):
        for pw in (64, 128, 256, 512, 1024):
            tot = 0.0
            for y in (2.0, 3.0, 4.0):
                w = weights(n, y)
                t = with_tuning({"rejection_per_wave": pw, "rejection_table": table},
                                lambda: timer(lambda: pfr.resample_rejection(w, 1.0, seed=1,
                                                                             out=out)))
                if y not in ref:
                    ref[y] = out.clone()
                same(out, ref[y], "rejection schedule")
                tot += t
            rows[f"table={table},per_wave={pw}"] = tot
            log(f"rejection table={table} per_wave={pw}: {tot:.4f} ms (y = 2, 3, 4)")
    best = min(rows, key=rows.get)
    chosen["rejection_table"] = int(best.split(",")[0].split("=")[1])
    chosen["rejection_per_wave"] = int(best.split(",")[1].split("=")[1])
    meas["rejection"] = rows

    pfr.set_tuning(**chosen)
    return chosen, meas


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--out", default=os.path.join(here, "tuning.json"))
    ap.add_argument("--reps", type=int, default=15)
    args = ap.parse_args()
    import torch
    t0 = time.time()
    chosen, meas = tune(args.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
    doc = {"version": 1, **chosen,
           "device": torch.cuda.get_device_name(0),
           "tuned_seconds": round(time.time() - t0, 1),
           "measured_ms": meas}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps({"version": 1, **chosen}), flush=True)


if __name__ == "__main__":
    main()
