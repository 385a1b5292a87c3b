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

    # ---- ragged batches (config 4): 4096 float32 vectors, N_f = 2^(8+8v)
    batch_tune(torch, pfr, inputs, timer, chosen, meas, with_tuning, same, log)

    pfr.set_tuning(**chosen)
    return chosen, meas


def batch_tune(torch, pfr, inputs, timer, chosen, meas, with_tuning, same, log):
    """Launch shapes of the ragged-batch kernels, each checked bit for bit
    against the first candidate.  The collective threshold is measured per
    bucket of the longest segment (batches of 4096 vectors with lengths
    log-uniform up to 2^10 .. 2^16), the others on the full 4096-vector batch;
    the Metropolis chunk also on the filter step's shape (1024 vectors of 2^14
    particles, short chains), since one value serves both."""
    from . import _lib

    def batch(hi_log2, seed=0):
        w_np, off_np, ys = inputs.ragged_batch(n_filters=4096, seed=seed)
        if hi_log2 < 16:  # the same vectors, cut to at most 2^hi_log2 particles
            lens = np.minimum(np.diff(off_np), 1 << hi_log2)
            parts = [w_np[off_np[f]:off_np[f] + lens[f]] for f in range(lens.size)]
            w_np = np.concatenate(parts)
            off_np = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        B = np.array([_b_star(float(y)) for y in ys], dtype=np.int32)
        return (torch.from_numpy(w_np).cuda(), torch.from_numpy(off_np).cuda(),
                int(np.diff(off_np).max()), torch.from_numpy(B).cuda())

    # batch_scan_wg_max_len: one workgroup per segment up to this longest segment
    rows = {}
    thr = 0
    for lg in (10, 12, 14, 16):
        w, off, max_len, B = batch(lg)
        out = torch.empty(w.numel(), dtype=torch.int32, device="cuda")
        ws = pfr.new_workspace(pfr.workspace_bytes(_lib.OP_MULTINOMIAL, w.numel(), off, max_len))

        def run():
            for s in ("stratified", "systematic", "multinomial"):
                getattr(pfr, "resample_" + s)(w, seed=1, offsets=off, max_len=max_len, out=out,
                                              workspace=ws)

        t_wg = with_tuning({"batch_scan_wg_max_len": _lib.MAX_BATCH_SEGMENT}, lambda: timer(run))
        ref = out.clone()
        t_blk = with_tuning({"batch_scan_wg_max_len": 0}, lambda: timer(run))
        same(out, ref, "batch_scan_wg_max_len")
        rows[f"max_len<=2^{lg}"] = {"one_workgroup_per_segment_ms": t_wg,
                                    "block_parallel_ms": t_blk}
        log(f"batch collective max_len 2^{lg}: one workgroup per segment {t_wg:.4f} ms, "
            f"block-parallel {t_blk:.4f} ms")
    # the largest bucket up to which one workgroup per segment wins at every bucket
    for lg in (10, 12, 14, 16):
        r = rows[f"max_len<=2^{lg}"]
        if r["one_workgroup_per_segment_ms"] < r["block_parallel_ms"]:
            thr = 1 << lg
        else:
            break
    chosen["batch_scan_wg_max_len"] = min(thr, _lib.MAX_BATCH_SEGMENT)
    meas["batch_scan_wg_max_len"] = rows

    w, off, max_len, B = batch(16)
    both = torch.empty(2 * w.numel(), dtype=torch.int32, device="cuda")
    out_m, out = both[:w.numel()], both[w.numel():]
    perm = torch.empty_like(out)

    def pick(name, cands, fn, result):
        rows, ref = {}, None
        for c in cands:
            t = with_tuning({name: c}, lambda: timer(fn))
            if ref is None:
                ref = result.clone()
            same(result, ref, name)
            rows[c] = t
            log(f"{name} {c}: {t:.4f} ms")
        chosen[name] = min(rows, key=rows.get)
        meas[name] = rows

    def metro():
        pfr.resample_metropolis(w, 0, seed=1, B_per_filter=B, offsets=off, max_len=max_len,
                                out=out_m)

    def rej():
        pfr.resample_rejection(w, 1.0, seed=1, offsets=off, max_len=max_len, out=out)

    def alt_both():
        metro()
        rej()

    # the filter step's shape: 1024 vectors of 2^14 particles with the short
    # chains of moderate weight sets (y_f ~ U[0, 1.5), B of eq. (B))
    g = np.random.default_rng(1)
    fy = g.uniform(0.0, 1.5, 1024)
    fw = torch.from_numpy(np.concatenate(
        [inputs.weights(1 << 14, float(y), seed=f + 1) for f, y in enumerate(fy)])).cuda()
    foff = torch.arange(0, 1025, dtype=torch.int64, device="cuda") * (1 << 14)
    fB = torch.tensor([_b_star(float(y)) for y in fy], dtype=torch.int32, device="cuda")
    both_f = torch.empty(fw.numel() + w.numel(), dtype=torch.int32, device="cuda")

    def metro_filter():
        pfr.resample_metropolis(fw, 0, seed=1, B_per_filter=fB, offsets=foff, max_len=1 << 14,
                                out=both_f[:fw.numel()])

    def pick_shared(name, cands, fns, result):
        """One value for several workloads: the smallest sum over the
        workloads of the time relative to that workload's best candidate."""
        rows, ref = {}, None
        for c in cands:
            ts = [with_tuning({name: c}, lambda: timer(fn)) for fn in fns]
            if ref is None:
                ref = result.clone()
            same(result, ref, name)
            rows[c] = ts
            log(f"{name} {c}: " + ", ".join(f"{t:.4f} ms" for t in ts))
        best = [min(r[i] for r in rows.values()) for i in range(len(fns))]
        score = {c: sum(t / b for t, b in zip(ts, best)) for c, ts in rows.items()}
        chosen[name] = min(score, key=score.get)
        meas[name] = {c: {"ms": ts, "score": score[c]} for c, ts in rows.items()}

    def metro_ragged():
        pfr.resample_metropolis(w, 0, seed=1, B_per_filter=B, offsets=off, max_len=max_len,
                                out=both_f[fw.numel():])

    pick("batch_stage_max_kb", (128, 64, 16), alt_both, both)
    pick_shared("batch_metropolis_chunk", (1024, 2048, 4096, 8192, 16384),
                (metro_ragged, metro_filter), both_f)
    def rej_ragged():
        pfr.resample_rejection(w, 1.0, seed=1, offsets=off, max_len=max_len,
                               out=both_f[fw.numel():])

    def rej_filter():
        pfr.resample_rejection(fw, 1.0, seed=1, offsets=foff, max_len=1 << 14,
                               out=both_f[:fw.numel()])

    # like the Metropolis chunk, the rejection schedule serves both batch shapes
    pick_shared("batch_rejection_per_wave", (64, 128, 256, 512, 1024), (rej_ragged, rej_filter),
                both_f)

    a_unsorted = torch.empty_like(out)
    pfr.resample_metropolis(w, 0, seed=1, B_per_filter=B, offsets=off, max_len=max_len,
                            out=a_unsorted)
    a_sorted = pfr.resample_systematic(w, seed=1, offsets=off, max_len=max_len)

    def permute_both():
        pfr.permute_ancestors(a_unsorted, offsets=off, max_len=max_len, out=perm)
        pfr.permute_ancestors(a_sorted, sorted_hint=True, offsets=off, max_len=max_len, out=perm)

    pick("batch_permute_lds_max", (16384, 8192, 4096), permute_both, perm)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--out", default=os.path.join(here, "tuning.json"))
    ap.add_argument("--reps", type=int, default=15)
    args = ap.parse_args()
    import torch
    t0 = time.time()
    chosen, meas = tune(args.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
    from . import _lib
    doc = {"version": _lib.TUNING_VERSION, **chosen,
           "arch": device_arch(),
           "device": torch.cuda.get_device_name(0),
           "tuned_seconds": round(time.time() - t0, 1),
           "measured_ms": meas}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps({"version": _lib.TUNING_VERSION, "arch": doc["arch"], **chosen}), flush=True)


def device_arch():
    """The GPU's ISA name (gfx950 on MI355X), which keys the tuning file."""
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


if __name__ == "__main__":
    main()
