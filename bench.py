"""Benchmark of the resampling step on one MI355X.

Workload (one step): n = 2^20 float32 weights w_i = exp(-(x_i - y)^2 / 2),
x_i ~ N(0,1), for each y in {0, 1, 2, 3, 4}; each weight set is resampled by
all five resamplers -- multinomial, stratified, systematic (exact prefix sums),
Metropolis with B from the bias bound (eps = 1/100, beta = E[w]/w_max, giving
B = 4, 6, 16, 60, 354), rejection with w_max = 1 -- and every ancestry is then
permuted for in-place propagation (for the three collective schemes the
claim pass of the permutation is fused into the emission: resample_permuted).
That is 25 resamples of 2^20 particles per step; inputs are resident in HBM
before the timed region.

Prints one JSON line: whole-step particles/s, the roofline of the dominant
kernel measured with HIP events inside the timed steps, the HBM fraction of
each scheme at n = 2^20, batched filters/s on the ragged 4096-vector batch
(the metric's second part), a per-scheme breakdown, the CPU oracle timed on
a bounded sample of the same workload, and ('concurrent') the same steps with
the five weight sets spread over three HIP streams.  The timed steps run on
one stream (--streams) so that the dominant kernel's events time it alone.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--streams S] [--concurrent-streams C]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 1 << 20
YS = (0.0, 1.0, 2.0, 3.0, 4.0)
SCHEMES = ("multinomial", "stratified", "systematic", "metropolis", "rejection")
# schemes whose claim pass of the permutation is fused into the resampler
# (resample_permuted); the others run resample_<scheme> then permute_ancestors
FUSED = ("multinomial", "stratified", "systematic")
HBM_PEAK_GBS = 8000.0
# Philox4x32-10 per call: 20 32x32->64-bit products (one v_mad_u64_u32 each)
# and 20 three-input xors (one v_bitop3_b32 each) = 40 VALU instructions per
# lane; 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-instructions/s,
# i.e. 9.83e11 calls/s.  (A Philox-only kernel measures 8.55e11 calls/s.)
PHILOX_PEAK_PER_S = 256 * 4 * 16 * 2.4e9 / 40.0
# Random 4-byte loads from a 1-4 MB table, measured with a plain gather kernel
# (one line per lane from L2): the rate Metropolis' weight loads run into.
GATHER_CEILING_PER_S = 2.65e11


# HBM bytes per launch of the dominant kernel (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 from
# two rocprofv3 --pmc passes, scaled by a 256 MiB copy; profiles/metropolis_table_n2p20_pmc.md).
# Set to None when the kernel changes until the counters are taken again.
DOMINANT_TRAFFIC_BYTES = (42.5 + 4.0) * (1 << 20)
# VALU instructions per lane and Metropolis step of the dominant kernel (SQ_INSTS_VALU x 64 /
# steps, same profile; None when the kernel changes), against the lane-instruction rate of
# 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz.
DOMINANT_VALU_PER_STEP = 44.5
LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9


def metropolis_calls_per_lane(B):
    """Philox calls of a B-step chain: four steps per three calls."""
    return 3 * (B // 4) + (3 * (B % 4) + 3) // 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def b_star(y, eps=0.01):
    from paper_1301_4019_amd.inputs import expected_weight
    return math.ceil(math.log(eps) / math.log(1.0 - expected_weight(y)))


def cpu_model():
    """Host CPU model name and logical core count (from /proc/cpuinfo)."""
    name, count = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    count += 1
                    name = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return name, count or (os.cpu_count() or 0)


def cpu_baseline(n_sample: int, budget_s: float = 30.0, max_runs: int = 5):
    """The oracle on the benchmark step: every (weight set, resampler) cell at
    n_sample particles plus its permutation (Code 10), Metropolis and
    rejection on every host core (their lanes are independent; the all-cores
    legs give the serial oracle's bits), the collective schemes and the
    permutation single-threaded (binary128 sums in order).  Each cell's time
    is the median of up to max_runs runs: every cell runs once, then the
    cheapest cells run again while the time budget lasts."""
    import oracle
    from paper_1301_4019_amd import inputs
    threads = oracle.default_threads()

    def run(w, y, s):
        if s == "metropolis":
            a = oracle.metropolis_mt(w, b_star(y), seed=1, nthreads=threads)
        elif s == "rejection":
            a = oracle.rejection_mt(w, 1.0, seed=1, nthreads=threads)[0]
        else:
            a = getattr(oracle, s)(w, seed=1)[0]
        oracle.permute(a)

    ws = {y: inputs.weights(n_sample, y, seed=100 + int(y)) for y in YS}
    times = {(y, s): [] for y in YS for s in SCHEMES}
    t_start = time.perf_counter()
    for _ in range(max_runs):
        order = sorted(times, key=lambda c: float(np.median(times[c])) if times[c] else 0.0)
        for c in order:
            if times[c] and len(times[c]) >= max_runs:
                continue
            if times[c] and time.perf_counter() - t_start > budget_s:
                break
            t0 = time.perf_counter()
            run(ws[c[0]], c[0], c[1])
            times[c].append(time.perf_counter() - t0)
    step_s = sum(float(np.median(v)) for v in times.values())
    runs = [len(v) for v in times.values()]
    name, logical = cpu_model()
    return {"value": len(YS) * len(SCHEMES) * n_sample / step_s, "unit": "particles/s",
            "cores": threads, "kind": "oracle",
            "cpu": {"model": name, "logical_cores": logical},
            "step_s": step_s,
            "sample": (f"the full step (5 weight sets x 5 resamplers + permutation) at n = "
                       f"{n_sample}; Metropolis and rejection on {threads} threads, the "
                       f"collective schemes and the permutation on one; per cell the median of "
                       f"{min(runs)}-{max(runs)} runs; "
                       f"{time.perf_counter() - t_start:.1f} s of host time")}


def implied_bias(torch, pfr, w, precision, e=None, workspace=None):
    """Deterministic bias of a precision mode for one weight vector: with r the
    scaled prefix the mode computes (pfr_scaled_prefix), the stratified and
    systematic schemes give particle i r_i - r_{i-1} offspring in expectation
    (the multinomial scheme too, up to its cap), against n w_i / W exactly.
    Returns sum_i (dr_i - n w_i / W)^2 and max_i |dr_i - n w_i / W|; the
    reference uses the binary64 weights and a binary64 total."""
    n = w.numel()
    if e is None:
        wd = w.double()
        e = n * wd / wd.sum()
    r = pfr.scaled_prefix(w, precision=precision, workspace=workspace)
    dr = torch.diff(r, prepend=torch.zeros(1, dtype=torch.float64, device=r.device))
    d = dr - e
    return float((d * d).sum()), float(d.abs().max())


def batch_implied_bias(torch, pfr, w32, off_np):
    """Deterministic bias (as implied_bias) over the vectors of a ragged batch,
    for the batched exact and compensated-binary32 forms (float32 weights; a
    batched call forms each vector's prefix bit for bit as a call on it alone)
    and the plain per-filter binary64 form (float64 weights): the sum over the
    vectors and the largest single-vector value."""
    out = {}
    w64 = w32.double()
    # one workspace of the largest vector's size serves every call
    from paper_1301_4019_amd import _lib
    max_len = int(np.diff(off_np).max())
    ws = pfr.new_workspace(pfr.workspace_bytes(_lib.OP_SCALED_PREFIX, max_len), w32.device)
    for name, ww, prec in (("exact_batched", w32, pfr.SCAN_EXACT),
                           ("comp_f32_batched", w32, pfr.SCAN_COMP_F32),
                           ("f64_per_filter", w64, pfr.SCAN_F64)):
        tot, worst, dmax = 0.0, 0.0, 0.0
        for f in range(off_np.size - 1):
            seg = ww[int(off_np[f]):int(off_np[f + 1])]
            if seg.numel() == 0:
                continue
            b2, mx = implied_bias(torch, pfr, seg, prec, workspace=ws)
            tot += b2
            worst = max(worst, b2)
            dmax = max(dmax, mx)
        out[name] = {"sum_bias2": tot, "max_bias2_per_vector": worst, "max_abs_dev": dmax}
    return out


def precision_sweep(args):
    """Bias of the collective resamplers per prefix-sum precision mode.

    For each n, one weight vector (y = 3, data seed 0) is resampled K times
    (Philox seeds 1..K) by every collective scheme in every precision mode,
    with Metropolis (B = 60) and rejection (w_max = 1) as controls.  Offspring
    are counted on the GPU and accumulated in binary64.  Reported, as in the
    paper's section 3: ||Bias||^2 = sum_i (mean o_i - n w_i / W)^2, the MSE,
    their ratio (about 1 / (K + 1) for an unbiased scheme) and MSE / n, plus
    the noise-corrected excess ||Bias||^2 - tr(Var) / K with an approximate
    standard error (particles treated as independent), and per mode the
    deterministic bias implied by the scaled prefix the mode computes
    (implied_bias).  The ragged batch of 4096 vectors adds the deterministic
    bias of its batched compensated-binary32 form and of the per-filter
    binary64 form.
    """
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K = args.replicates
    y = 3.0
    modes = {"exact": pfr.SCAN_EXACT, "f64": pfr.SCAN_F64, "comp_f32": pfr.SCAN_COMP_F32,
             "naive_f32": pfr.SCAN_NAIVE_F32}
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    rows, implied = [], []
    t_start = time.perf_counter()
    for lg in args.sweep_log2n:
        n = 1 << lg
        w = torch.from_numpy(inputs.weights(n, y, seed=0)).to(dev)
        wd = w.double()
        e = n * wd / wd.sum()
        for mode, prec in modes.items():
            b2, mx = implied_bias(torch, pfr, w, prec, e)
            implied.append({"n": n, "precision": mode, "bias2": b2, "max_abs_dev": mx})
        a = torch.empty(n, dtype=torch.int32, device=dev)
        cases = [(s, m) for s in ("multinomial", "stratified", "systematic") for m in modes]
        cases += [("metropolis", "-"), ("rejection", "-")]
        for scheme, mode in cases:
            S1 = torch.zeros(n, dtype=torch.float64, device=dev)
            S2 = torch.zeros(n, dtype=torch.float64, device=dev)
            for k in range(K):
                if scheme == "metropolis":
                    pfr.resample_metropolis(w, 60, seed=1 + k, out=a)
                elif scheme == "rejection":
                    pfr.resample_rejection(w, 1.0, seed=1 + k, out=a, flags=flags)
                else:
                    getattr(pfr, "resample_" + scheme)(w, seed=1 + k, precision=modes[mode],
                                                      out=a, flags=flags)
                o = torch.bincount(a, minlength=n).double()
                S1 += o
                S2 += o * o
            mean = S1 / K
            d = mean - e
            bias2 = float((d * d).sum())
            mse = float((S2 / K - 2.0 * e * mean + e * e).sum())
            v = (S2 - K * mean * mean) / (K - 1)
            var_tr = float(v.sum())
            se = math.sqrt(float((4.0 * d * d * v / K + 2.0 * v * v / (K * K)).sum()))
            rows.append({"n": n, "scheme": scheme, "precision": mode, "bias2": bias2, "mse": mse,
                         "bias2_over_mse": bias2 / mse, "mse_over_n": mse / n,
                         "bias2_excess": bias2 - var_tr / K, "bias2_excess_se": se})
        log(f"n = 2^{lg} done ({time.perf_counter() - t_start:.0f} s)")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised during the sweep: {int(flags.cpu()[0])}")
    w_np, off_np, _ = inputs.ragged_batch(n_filters=4096, seed=0)
    batch = batch_implied_bias(torch, pfr, torch.from_numpy(w_np).to(dev), off_np)
    result = {"metric": "bias contribution to the MSE per prefix-sum precision",
              "unit": "ratio", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
              "config": {"workload": "precision sweep: y = 3 weights (data seed 0), "
                                     f"{K} Philox seeds per case, n = 2^" +
                                     ",".join(str(v) for v in args.sweep_log2n),
                         "replicates": K, "y": y, "unbiased_ratio": 1.0 / (K + 1)},
              "rows": rows, "implied": implied, "batch_implied": batch}
    print(json.dumps(result), flush=True)


def _time_ms(fn, reps, torch):
    """Mean milliseconds per call of fn over reps calls (wall clock, synchronised)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


class StepWorkload:
    """The benchmark step: its inputs, outputs, workspaces and calls.

    Weight set y (n = 2^20 float32, data seed 100 + y) is resampled by every
    scheme with Philox seed 1 and every ancestry is permuted, exactly as timed;
    the GPU parity tests run this same object."""

    DOMINANT = (4.0, "metropolis")

    def __init__(self, torch, pfr, dev, n_streams=1):
        from paper_1301_4019_amd import inputs, _lib
        self.torch, self.pfr, self._lib = torch, pfr, _lib
        self.w = [torch.from_numpy(inputs.weights(N, y, seed=100 + int(y))).to(dev) for y in YS]
        self.Bs = [b_star(y) for y in YS]
        self.out = {(y, s): torch.empty(N, dtype=torch.int32, device=dev)
                    for y in YS for s in SCHEMES}
        self.perm = {(y, s): torch.empty(N, dtype=torch.int32, device=dev)
                     for y in YS for s in SCHEMES}
        # one stream per group of weight sets (the resamples of different
        # weight sets are independent); workspaces are per stream.  Stream 0
        # is the current stream.
        self.streams = [torch.cuda.current_stream()] + [torch.cuda.Stream(device=dev)
                                                        for _ in range(n_streams - 1)]
        self.wsp = {}
        for k, st in enumerate(self.streams):
            with torch.cuda.stream(st):
                for op in (_lib.OP_MULTINOMIAL, _lib.OP_STRATIFIED, _lib.OP_SYSTEMATIC,
                           _lib.OP_PERMUTE):
                    self.wsp[(k, op)] = pfr.new_workspace(max(256, pfr.workspace_bytes(op, N)),
                                                          dev)
        torch.cuda.synchronize()
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ev = []

    def resample(self, yi, y, s, k):
        pfr, _lib = self.pfr, self._lib
        w = self.w[yi]
        a = self.out[(y, s)]
        if s == "metropolis":
            pfr.resample_metropolis(w, self.Bs[yi], seed=1, out=a)
        elif s == "rejection":
            pfr.resample_rejection(w, 1.0, seed=1, out=a, flags=self.flags)
        else:
            op = {"multinomial": _lib.OP_MULTINOMIAL, "stratified": _lib.OP_STRATIFIED,
                  "systematic": _lib.OP_SYSTEMATIC}[s]
            getattr(pfr, "resample_" + s)(w, seed=1, out=a, flags=self.flags,
                                          workspace=self.wsp[(k, op)])
        return a

    def permute(self, y, s, k):
        self.pfr.permute_ancestors(self.out[(y, s)],
                                   sorted_hint=s not in ("metropolis", "rejection"),
                                   out=self.perm[(y, s)], flags=self.flags,
                                   workspace=self.wsp[(k, self._lib.OP_PERMUTE)])

    def step(self, record=False, n_st=1):
        torch, pfr = self.torch, self.pfr
        for yi, y in enumerate(YS):
            k = yi % n_st
            stream = self.streams[k]
            with torch.cuda.stream(stream):
                for s in SCHEMES:
                    if s in FUSED:
                        # the emission writes the claim vector and marks itself
                        pfr.resample_permuted(s, self.w[yi], seed=1, out=self.out[(y, s)],
                                              permuted=self.perm[(y, s)], flags=self.flags)
                        continue
                    if record and (y, s) == self.DOMINANT:
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        self.resample(yi, y, s, k)
                        e1.record(stream)
                        self.ev.append((e0, e1))
                    else:
                        self.resample(yi, y, s, k)
                    self.permute(y, s, k)


def batch_calls(pfr, w, offsets, max_len, B, a, flags):
    """The ragged-batch calls the benchmark times, one per (scheme, mode)."""
    calls = {}
    for s in ("multinomial", "stratified", "systematic"):
        fn = getattr(pfr, "resample_" + s)
        for mode, prec in (("exact", pfr.SCAN_EXACT), ("comp_f32", pfr.SCAN_COMP_F32)):
            calls[f"{s}_{mode}"] = (lambda fn=fn, prec=prec: fn(
                w, seed=1, precision=prec, offsets=offsets, max_len=max_len, out=a, flags=flags))
    calls["metropolis"] = lambda: pfr.resample_metropolis(
        w, 0, seed=1, B_per_filter=B, offsets=offsets, max_len=max_len, out=a)
    calls["rejection"] = lambda: pfr.resample_rejection(
        w, 1.0, seed=1, offsets=offsets, max_len=max_len, out=a, flags=flags)
    return calls


def batched_summary(torch, pfr, inputs, dev, stream, reps=5):
    """Filters/s of each resampler on the ragged batch (4096 float32 vectors,
    N_f = 2^(8+8v), y_f ~ U[0,4], seed 0), one launch sequence per call, HIP
    events around `reps` calls; plus the per-filter binary64 systematic form
    replayed from a captured graph."""
    F = 4096
    w_np, off_np, ys = inputs.ragged_batch(n_filters=F, seed=0)
    total = int(off_np[-1])
    max_len = int(np.diff(off_np).max())
    w = torch.from_numpy(w_np).to(dev)
    offsets = torch.from_numpy(off_np).to(dev)
    B = torch.tensor([b_star(float(y)) for y in ys], dtype=torch.int32, device=dev)
    a = torch.empty(total, dtype=torch.int32, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)

    def timed(fn):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {name: F / (1e-3 * timed(fn))
           for name, fn in batch_calls(pfr, w, offsets, max_len, B, a, flags).items()}
    w64 = w.double()
    views = [(w64[off_np[f]:off_np[f + 1]], a[off_np[f]:off_np[f + 1]]) for f in range(F)]

    def per_filter():
        for f, (wf, af) in enumerate(views):
            pfr.resample_systematic(wf, seed=1, filter_base=f, precision=pfr.SCAN_F64, out=af,
                                    flags=flags)

    per_filter()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        per_filter()
    out["systematic_f64_per_filter_graph"] = F / (1e-3 * timed(g.replay))
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised in the batch: {int(flags.cpu()[0])}")
    stated_bias = batch_implied_bias(torch, pfr, w, off_np)
    return {"unit": "filters/s", "filters": F, "particles": total, "max_len": max_len,
            "stated_bias": stated_bias,
            "workload": "ragged batch: 4096 float32 weight vectors, N_f = 2^(8+8v), v ~ U[0,1), "
                        "y_f ~ U[0,4] (seed 0); one launch sequence per resampler",
            "filters_per_s": out}


def batch_workload(args):
    """Ragged batch: 4096 weight vectors, N_f log-uniform in [2^8, 2^16], y_f ~ U[0,4],
    float32.  Every resampler runs once over the whole batch (one launch), the
    collective ones with exact and with compensated binary32 prefix sums;
    Metropolis takes B_f from the bias bound for y_f, rejection w_max = 1.  The
    per-filter form runs the systematic resampler filter by filter on float64
    weights with binary64 prefix sums (4096 calls), eagerly and replayed from a
    captured graph."""
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    F = args.filters
    w_np, off_np, ys = inputs.ragged_batch(n_filters=F, seed=0)
    total = int(off_np[-1])
    sizes = np.diff(off_np)
    max_len = int(sizes.max())
    w = torch.from_numpy(w_np).to(dev)
    w64 = w.double()
    offsets = torch.from_numpy(off_np).to(dev)
    B = torch.tensor([b_star(float(y)) for y in ys], dtype=torch.int32, device=dev)
    a = torch.empty(total, dtype=torch.int32, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    log(f"batch: {F} filters, {total} particles, max N_f {max_len}")

    def run(scheme, precision=pfr.SCAN_EXACT):
        if scheme == "metropolis":
            return lambda: pfr.resample_metropolis(w, 0, seed=1, B_per_filter=B, offsets=offsets,
                                                   max_len=max_len, out=a)
        if scheme == "rejection":
            return lambda: pfr.resample_rejection(w, 1.0, seed=1, offsets=offsets,
                                                  max_len=max_len, out=a, flags=flags)
        fn = getattr(pfr, "resample_" + scheme)
        return lambda: fn(w, seed=1, precision=precision, offsets=offsets, max_len=max_len,
                          out=a, flags=flags)

    rows = []
    cases = [(s, "exact") for s in ("multinomial", "stratified", "systematic")]
    cases += [(s, "comp_f32") for s in ("multinomial", "stratified", "systematic")]
    cases += [("metropolis", "-"), ("rejection", "-")]
    prec = {"exact": pfr.SCAN_EXACT, "comp_f32": pfr.SCAN_COMP_F32, "-": pfr.SCAN_EXACT}
    for scheme, mode in cases:
        fn = run(scheme, prec[mode])
        fn()
        ms = _time_ms(fn, args.steps, torch)
        rows.append({"scheme": scheme, "precision": mode, "form": "batched, one launch",
                     "ms": ms, "filters_per_s": F / (ms * 1e-3),
                     "particles_per_s": total / (ms * 1e-3),
                     "hbm_frac_8B_per_particle": 8.0 * total / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)})
        log(f"  {scheme:12s} {mode:9s} {ms:8.3f} ms")

    # per-filter form: one call per filter, float64 weights, binary64 prefix sums
    views = [(w64[off_np[f]:off_np[f + 1]], a[off_np[f]:off_np[f + 1]]) for f in range(F)]

    def per_filter():
        for f, (wf, af) in enumerate(views):
            pfr.resample_systematic(wf, seed=1, filter_base=f, precision=pfr.SCAN_F64, out=af,
                                    flags=flags)

    per_filter()
    ms_eager = _time_ms(per_filter, max(1, args.steps // 4), torch)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        per_filter()
    g.replay()
    ms_graph = _time_ms(g.replay, max(1, args.steps // 4), torch)
    for form, ms in (("per-filter calls", ms_eager), ("per-filter calls, captured graph",
                                                      ms_graph)):
        rows.append({"scheme": "systematic", "precision": "f64", "form": form, "ms": ms,
                     "filters_per_s": F / (ms * 1e-3), "particles_per_s": total / (ms * 1e-3)})
        log(f"  systematic   f64 {form}: {ms:8.3f} ms")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised: {int(flags.cpu()[0])}")
    print(json.dumps({"metric": "batched filters/sec", "unit": "filters/s",
                      "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "ragged batch: 4096 float32 weight vectors, N_f = "
                                             "2^(8+8v), v ~ U[0,1), y_f ~ U[0,4] (seed 0)",
                                 "filters": F, "particles": total, "max_len": max_len},
                      "rows": rows}), flush=True)


def decision_workload(args):
    """Fastest resampler per (N, y), and the Metropolis bias / time trade-off.

    Decision matrix (section 3.4): for N = 2^4 .. 2^22 and y = 0, 1/2, .., 4,
    float32 weights w = exp(-(x - y)^2 / 2), x ~ N(0, 1) (data seed 0), every
    resampler is timed until it has delivered an ancestry satisfying the
    in-place predicate -- the resample followed by permute_ancestors -- with
    HIP events around --decision-reps back-to-back calls; the cell takes the
    scheme of least mean time.  Metropolis takes B = B* from the bias bound
    with beta = mean(w) / w_max of the weight vector itself, rejection w_max = 1
    (the bound of these weights).

    Metropolis trade-off (section 3.3): y = 4, B = ceil(B* / C) for C = 1, 2,
    4, 8, with multinomial as the unbiased reference: ||Bias||^2 / MSE and
    MSE / N over --replicates Philox seeds, and the time per resample.

    Multinomial forms: Code 5 as printed (one independent uniform and one
    search per particle, unsorted output) against the sorted-uniform merge,
    y = 2, device time with and without the permutation.
    """
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    reps = args.decision_reps
    lgs = list(range(args.decision_log2n[0], args.decision_log2n[1] + 1))
    ys = [0.5 * k for k in range(9)]
    nmax = 1 << lgs[-1]
    a = torch.empty(nmax, dtype=torch.int32, device=dev)
    c = torch.empty(nmax, dtype=torch.int32, device=dev)

    def b_of(wn):
        beta = float(np.mean(wn, dtype=np.float64)) / float(wn.max())
        if beta >= 1.0:
            return 1
        return max(1, math.ceil(math.log(0.01) / math.log(1.0 - beta)))

    def call(scheme, w, n, B):
        out, perm = a[:n], c[:n]
        if scheme == "metropolis":
            pfr.resample_metropolis(w, B, seed=1, out=out)
        elif scheme == "rejection":
            pfr.resample_rejection(w, 1.0, seed=1, out=out, flags=flags)
        else:
            getattr(pfr, "resample_" + scheme)(w, seed=1, out=out, flags=flags)
        pfr.permute_ancestors(out, sorted_hint=scheme not in ("metropolis", "rejection",
                                                               "multinomial_iid"),
                              out=perm, flags=flags)

    def device_us(fn):
        fn()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        e1.synchronize()
        return 1e3 * e0.elapsed_time(e1) / reps

    cells = []
    t_start = time.perf_counter()
    for lg in lgs:
        n = 1 << lg
        for y in ys:
            wn = inputs.weights(n, y, seed=0)
            w = torch.from_numpy(wn).to(dev)
            B = b_of(wn)
            times, eager = {}, {}
            for scheme in SCHEMES:
                call(scheme, w, n, B)  # warm-up, workspaces
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    call(scheme, w, n, B)
                e1.record(stream)
                e1.synchronize()
                eager[scheme] = 1e3 * e0.elapsed_time(e1) / reps
                # device time alone: the same calls replayed from a captured graph
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    for _ in range(reps):
                        call(scheme, w, n, B)
                g.replay()
                e0.record(stream)
                g.replay()
                e1.record(stream)
                e1.synchronize()
                times[scheme] = 1e3 * e0.elapsed_time(e1) / reps
                del g
            best = min(times, key=times.get)
            cells.append({"log2n": lg, "y": y, "B": B, "us": times, "eager_us": eager,
                          "fastest": best, "fastest_eager": min(eager, key=eager.get)})
        log(f"decision n = 2^{lg} done ({time.perf_counter() - t_start:.0f} s)")

    # Metropolis B = B*/C against multinomial, y = 4
    K = args.replicates
    y = 4.0
    trade = []
    for lg in args.tradeoff_log2n:
        n = 1 << lg
        wn = inputs.weights(n, y, seed=0)
        w = torch.from_numpy(wn).to(dev)
        wd = w.double()
        e = n * wd / wd.sum()
        Bs = b_of(wn)
        out = a[:n]
        cases = [("multinomial", None)] + [("metropolis", C) for C in (1, 2, 4, 8)]
        for scheme, C in cases:
            B = None if C is None else max(1, math.ceil(Bs / C))
            S1 = torch.zeros(n, dtype=torch.float64, device=dev)
            S2 = torch.zeros(n, dtype=torch.float64, device=dev)
            t_ms = 0.0
            for k in range(K):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                if scheme == "metropolis":
                    pfr.resample_metropolis(w, B, seed=1 + k, out=out)
                else:
                    pfr.resample_multinomial(w, seed=1 + k, out=out, flags=flags)
                e1.record(stream)
                o = torch.bincount(out, minlength=n).double()
                S1 += o
                S2 += o * o
                e1.synchronize()
                t_ms += e0.elapsed_time(e1)
            mean = S1 / K
            bias2 = float(((mean - e) ** 2).sum())
            mse = float((S2 / K - 2.0 * e * mean + e * e).sum())
            trade.append({"log2n": lg, "scheme": scheme, "C": C, "B": B,
                          "bias2_over_mse": bias2 / mse, "mse_over_n": mse / n,
                          "resample_us": 1e3 * t_ms / K})
        log(f"trade-off n = 2^{lg} done ({time.perf_counter() - t_start:.0f} s)")
    # the two multinomial forms: Code 5 as printed (independent uniforms, a
    # search per particle, unsorted output) against the sorted-uniform merge
    forms = []
    for lg in args.forms_log2n:
        n = 1 << lg
        if n > nmax:
            a = torch.empty(n, dtype=torch.int32, device=dev)
            c = torch.empty(n, dtype=torch.int32, device=dev)
            nmax = n
        w = torch.from_numpy(inputs.weights(n, 2.0, seed=0)).to(dev)
        out, perm = a[:n], c[:n]
        row = {"log2n": lg}
        for scheme in ("multinomial", "multinomial_iid"):
            fn = getattr(pfr, "resample_" + scheme)
            row[scheme + "_us"] = device_us(lambda: fn(w, seed=1, out=out, flags=flags))
            row[scheme + "_with_permute_us"] = device_us(lambda: call(scheme, w, n, 0))
        forms.append(row)
        log(f"multinomial forms n = 2^{lg}: sorted {row['multinomial_us']:.1f} us, "
            f"independent {row['multinomial_iid_us']:.1f} us")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised: {int(flags.cpu()[0])}")

    letters = {"multinomial": "M", "stratified": "S", "systematic": "Y", "metropolis": "P",
               "rejection": "R"}
    grid, grid_eager = [], []
    for lg in lgs:
        row = "".join(letters[cl["fastest"]] for cl in cells if cl["log2n"] == lg)
        grid.append(f"2^{lg:<2d} {row}")
        row = "".join(letters[cl["fastest_eager"]] for cl in cells if cl["log2n"] == lg)
        grid_eager.append(f"2^{lg:<2d} {row}")
    print(json.dumps({"metric": "fastest resampler per (N, y) incl. permutation; Metropolis "
                                "bias/time at B = B*/C",
                      "unit": "us", "higher_is_better": False, "n_gpus": 1,
                      "data": "synthetic",
                      "config": {"workload": "decision matrix: N = 2^" + str(lgs[0]) + "..2^" +
                                             str(lgs[-1]) + ", y = 0..4 step 1/2, float32 "
                                             "weights (data seed 0); trade-off at y = 4",
                                 "reps": reps, "replicates": K,
                                 "legend": "M multinomial, S stratified, Y systematic, "
                                           "P Metropolis, R rejection; columns y = 0..4"},
                      "matrix": grid, "matrix_eager": grid_eager, "cells": cells,
                      "tradeoff": trade, "multinomial_forms": forms}), flush=True)


def aux_workload(args):
    """Auxiliary exports on float32 / int32 data resident in HBM, HIP-event timed
    (mean over --steps calls after a warm-up), against their algorithmic bytes:
      ancestors_to_offspring  read a, write o                 8 B / particle
      effective_sample_size   read w                           4 B / particle
      copy_particles          read c, read + write the copied state rows
    for a single vector of 2^20 and 2^24 particles (systematic ancestry of
    y = 2 weights; Metropolis ancestry for the unsorted count) and the
    4096-vector ragged batch."""
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    rows = []

    def timed(fn):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / args.steps

    def add(case, what, ms, n, nbytes):
        rows.append({"case": case, "op": what, "us": 1e3 * ms, "particles_per_s": n / (ms * 1e-3),
                     "algorithmic_bytes": nbytes, "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)})
        log(f"  {case:22s} {what:30s} {1e3 * ms:9.1f} us  {nbytes / (ms * 1e-3) / 1e9:7.0f} GB/s")

    cases = []
    for lg in (20, 24):
        n = 1 << lg
        w = torch.from_numpy(inputs.weights(n, 2.0, seed=lg)).to(dev)
        cases.append((f"single n=2^{lg}", w, None, n))
    wb, offb, _ = inputs.ragged_batch(n_filters=4096, seed=0)
    cases.append(("batch 4096 ragged", torch.from_numpy(wb).to(dev),
                  torch.from_numpy(offb).to(dev), int(np.diff(offb).max())))
    for case, w, off, ml in cases:
        n = w.numel()
        kw = {} if off is None else {"offsets": off, "max_len": ml}
        a = pfr.resample_systematic(w, seed=1, flags=flags, **kw)
        am = pfr.resample_metropolis(w, 16, seed=1, **kw)
        cperm = pfr.permute_ancestors(a, sorted_hint=True, flags=flags, **kw)
        o = torch.empty(n, dtype=torch.int32, device=dev)
        copied = int((cperm != torch.arange(n, device=dev, dtype=torch.int32)).sum()) \
            if off is None else None
        add(case, "a2o sorted", timed(lambda: pfr.ancestors_to_offspring(
            a, sorted_hint=True, out=o, flags=flags, **kw)), n, 8 * n)
        add(case, "a2o unsorted (Metropolis)", timed(lambda: pfr.ancestors_to_offspring(
            am, out=o, flags=flags, **kw)), n, 8 * n)
        e = pfr.effective_sample_size(w, flags=flags, **kw)
        add(case, "ess", timed(lambda: pfr.effective_sample_size(w, out=e, flags=flags, **kw)),
            n, 4 * n)
        if off is None:
            for D, layout in ((1, "rows"), (4, "rows"), (4, "columns")):
                x = torch.zeros(n, D, dtype=torch.float32, device=dev)
                if layout == "columns":
                    x = torch.zeros(D, n, dtype=torch.float32, device=dev).t()
                add(case, f"copy D={D} {layout} ({copied} moved)",
                    timed(lambda: pfr.copy_particles(cperm, x, flags=flags)), n,
                    4 * n + 8 * D * copied)
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised: {int(flags.cpu()[0])}")
    print(json.dumps({"metric": "auxiliary exports: time and HBM fraction of algorithmic bytes",
                      "unit": "us", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "ancestors_to_offspring, effective_sample_size, "
                                             "copy_particles; n = 2^20, 2^24 and the 4096-vector "
                                             "ragged batch", "steps": args.steps},
                      "rows": rows}), flush=True)


def philox_workload(args):
    """Philox round-count study: the product build (Philox4x32-10) against the
    study build with 7 rounds (libpfresample_philox7.so), same kernels
    otherwise.  Speed: device time of each resampler at n = 2^20 for
    y = 0, 2, 4 (captured graph, mean of --decision-reps calls).  Quality: the
    bias share ||Bias||^2 / MSE and MSE / n at n = 2^16, y = 3 over
    --replicates Philox seeds (about 1 / (K + 1) when unbiased)."""
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs, build as pbuild

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    reps = args.decision_reps
    K = args.replicates
    n = 1 << 20
    ws = {y: torch.from_numpy(inputs.weights(n, y, seed=100 + int(y))).to(dev) for y in (0.0, 2.0, 4.0)}
    out = torch.empty(n, dtype=torch.int32, device=dev)

    def resample(scheme, w, y, seed=1, a=out):
        if scheme == "metropolis":
            pfr.resample_metropolis(w, b_star(y), seed=seed, out=a)
        elif scheme == "rejection":
            pfr.resample_rejection(w, 1.0, seed=seed, out=a, flags=flags)
        else:
            getattr(pfr, "resample_" + scheme)(w, seed=seed, out=a, flags=flags)

    def device_us(fn):
        fn()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        e1.synchronize()
        return 1e3 * e0.elapsed_time(e1) / reps

    def measure(rounds):
        speed = []
        for y, w in ws.items():
            for scheme in SCHEMES:
                speed.append({"rounds": rounds, "y": y, "scheme": scheme,
                              "us": device_us(lambda: resample(scheme, w, y))})
        nq = 1 << 16
        wq = torch.from_numpy(inputs.weights(nq, 3.0, seed=0)).to(dev)
        wd = wq.double()
        e = nq * wd / wd.sum()
        aq = torch.empty(nq, dtype=torch.int32, device=dev)
        quality = []
        for scheme in ("multinomial", "systematic", "metropolis", "rejection"):
            S1 = torch.zeros(nq, dtype=torch.float64, device=dev)
            S2 = torch.zeros(nq, dtype=torch.float64, device=dev)
            for k in range(K):
                resample(scheme, wq, 3.0, seed=1 + k, a=aq)
                o = torch.bincount(aq, minlength=nq).double()
                S1 += o
                S2 += o * o
            mean = S1 / K
            bias2 = float(((mean - e) ** 2).sum())
            mse = float((S2 / K - 2.0 * e * mean + e * e).sum())
            quality.append({"rounds": rounds, "scheme": scheme, "bias2_over_mse": bias2 / mse,
                            "mse_over_n": mse / nq})
        return speed, quality

    assert pfr._lib.load().pfr_philox_rounds() == 10
    sp10, q10 = measure(10)
    log("10 rounds measured")
    with pfr._lib.use_library(pbuild.variant_path(7)) as lib7:
        assert lib7.pfr_philox_rounds() == 7
        sp7, q7 = measure(7)
    log("7 rounds measured")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised: {int(flags.cpu()[0])}")
    for a, b in zip(sp10, sp7):
        log(f"  y={a['y']:.0f} {a['scheme']:12s} 10 rounds {a['us']:8.1f} us   7 rounds "
            f"{b['us']:8.1f} us   ratio {a['us'] / b['us']:.2f}")
    for a, b in zip(q10, q7):
        log(f"  quality {a['scheme']:12s} bias2/mse {a['bias2_over_mse']:.4f} / "
            f"{b['bias2_over_mse']:.4f}   mse/n {a['mse_over_n']:.4f} / {b['mse_over_n']:.4f}")
    print(json.dumps({"metric": "resampler time and bias with Philox4x32-10 vs 7 rounds",
                      "unit": "us", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "n = 2^20, y = 0, 2, 4 (speed); n = 2^16, y = 3, "
                                             f"{K} seeds (quality)", "reps": reps},
                      "speed": sp10 + sp7, "quality": q10 + q7}), flush=True)


def scaling_workload(args):
    """The collective resamplers on one long vector, n = 2^20 .. 2^26 float32
    weights (uniform on [0.01, 1.01), seed 0): device time of one call (median
    of 5, the Infinity Cache flushed before each), particles/s and the HBM
    fraction of the 8 algorithmic bytes per particle (read w, write a)."""
    import torch
    import paper_1301_4019_amd as pfr

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    g = torch.Generator(device=dev)
    rows = []
    for lg in args.scaling_log2n:
        n = 1 << lg
        g.manual_seed(0)
        w = torch.rand(n, device=dev, dtype=torch.float32, generator=g) + 0.01
        a = torch.empty(n, dtype=torch.int32, device=dev)
        for s in ("multinomial", "stratified", "systematic"):
            fn = getattr(pfr, "resample_" + s)
            fn(w, seed=1, out=a, flags=flags)
            ts = []
            for r in range(5):
                flush.fill_(r)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn(w, seed=1, out=a, flags=flags)
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            t = sorted(ts)[2]
            rows.append({"log2n": lg, "scheme": s, "us": t * 1e6, "particles_per_s": n / t,
                         "hbm_frac_8B_per_particle": 8.0 * n / t / (HBM_PEAK_GBS * 1e9)})
            log(f"  n=2^{lg} {s:12s} {t * 1e6:9.1f} us  {n / t:.3e} particles/s  "
                f"{100 * 8.0 * n / t / (HBM_PEAK_GBS * 1e9):.1f} % HBM")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised: {int(flags.cpu()[0])}")
    print(json.dumps({"metric": "collective resamplers on one long vector", "unit": "particles/s",
                      "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "single vector, float32 weights U[0.01, 1.01), "
                                             "n = 2^" + ",".join(map(str, args.scaling_log2n))},
                      "rows": rows}), flush=True)


def permute_workload(args):
    """The ancestor permutation (Code 10) on one vector, n = 2^20 .. 2^24: the
    Metropolis ancestry (B = 60) of the bench weights for y = 0 and 4, with the
    bucketed claim (the workspace pfr_workspace_bytes reports) and with the
    atomic claim (a workspace of 8 bytes per particle), and the systematic
    ancestry through the sorted claim.  Device time per call (HIP events, median
    of 9, the Infinity Cache flushed before each) and the HBM fraction of the 8
    algorithmic bytes per particle (read a, write c)."""
    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs, _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    rows = []

    def timed(fn):
        fn()
        ts = []
        for r in range(9):
            flush.fill_(r)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return sorted(ts)[4]

    for lg in args.permute_log2n:
        n = 1 << lg
        out = torch.empty(n, dtype=torch.int32, device=dev)
        full = pfr.workspace_bytes(_lib.OP_PERMUTE, n)
        small = 2 * ((4 * n + 255) // 256 * 256)
        ws_full, ws_small = pfr.new_workspace(full, dev), pfr.new_workspace(small, dev)
        for y in (0.0, 4.0):
            w = torch.from_numpy(inputs.weights(n, y, seed=100 + int(y))).to(dev)
            a = pfr.resample_metropolis(w, 60, seed=1)
            s = pfr.resample_systematic(w, seed=1)
            cases = {"unsorted_bucketed": lambda: pfr.permute_ancestors(a, out=out, workspace=ws_full),
                     "unsorted_atomic": lambda: pfr.permute_ancestors(a, out=out, workspace=ws_small),
                     "sorted": lambda: pfr.permute_ancestors(s, sorted_hint=True, out=out,
                                                             workspace=ws_full)}
            for name, fn in cases.items():
                t = timed(fn)
                rows.append({"log2n": lg, "y": y, "case": name, "us": t * 1e6,
                             "hbm_frac_8B_per_particle": 8.0 * n / t / (HBM_PEAK_GBS * 1e9)})
                log(f"  n=2^{lg} y={y:.0f} {name:18s} {t * 1e6:9.1f} us  "
                    f"{100 * 8.0 * n / t / (HBM_PEAK_GBS * 1e9):.1f} % HBM")
    print(json.dumps({"metric": "ancestor permutation on one vector", "unit": "us",
                      "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "Metropolis (B = 60) and systematic ancestries of "
                                             "the bench weights, n = 2^" +
                                             ",".join(map(str, args.permute_log2n))},
                      "rows": rows}), flush=True)


def filter_workload(args):
    """Bootstrap filter on x_t = 0.9 x_{t-1} + N(0,1), y_t = x_t + N(0, 0.5^2):
    1024 filters of 2^14 particles, T = 200 synthetic observations (seed 0); one
    captured graph of a step (resample, permute, copy, propagate, weight) is
    replayed T times.  filters/s = 1024 / wall time of the T steps; log Z-hat
    is compared with the Kalman value."""
    import torch
    import oracle
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    F, n, T = args.filters_ssm, 1 << 14, 200
    phi, q, r = 0.9, 1.0, 0.5
    s0 = q / math.sqrt(1 - phi * phi)
    y = inputs.ssm_data(T, phi=phi, q=q, r=r, seed=0)[1]
    logZ = oracle.kalman_loglik(y, phi, q, r, s0)
    rows = []
    for scheme in SCHEMES:
        flt = pfr.LGSSMFilter(y, F, n, phi=phi, q=q, r=r, scheme=scheme, seed=1, device=dev)
        flt.run()  # capture and warm up
        times = []
        for _ in range(args.filter_reps):
            flt.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(T):
                flt.graph.replay()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        lz = flt.log_z.cpu().numpy()
        if int(flt.flags.cpu()[0]) != 0:
            raise RuntimeError(f"data flags raised: {int(flt.flags.cpu()[0])}")
        ratio = np.exp(lz - logZ)
        sec = float(np.median(times))
        rows.append({"scheme": scheme, "seconds_T_steps": sec, "filters_per_s": F / sec,
                     "us_per_step": 1e6 * sec / T,
                     "particles_per_s": F * n * T / sec,
                     "mean_logZhat_minus_logZ": float(lz.mean() - logZ),
                     "sd_logZhat": float(lz.std(ddof=1)),
                     "mean_Zhat_over_Z": float(ratio.mean()),
                     "se_Zhat_over_Z": float(ratio.std(ddof=1) / math.sqrt(F))})
        log(f"  {scheme:12s} {1e6 * sec / T:8.1f} us/step  {F / sec:10.1f} filters/s  "
            f"Zhat/Z {ratio.mean():.4f} +- {ratio.std(ddof=1) / math.sqrt(F):.4f}")
        del flt
    print(json.dumps({"metric": "batched filters/sec (full bootstrap filter, hipGraph step)",
                      "unit": "filters/s", "higher_is_better": True, "n_gpus": 1,
                      "data": "synthetic",
                      "config": {"workload": "bootstrap filter, 1-D linear-Gaussian SSM "
                                             "phi=0.9 q=1 r=0.5, y from seed 0",
                                 "filters": F, "n": n, "T": T, "logZ_kalman": logZ},
                      "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched filters/s summary of the default workload")
    ap.add_argument("--streams", type=int, default=1,
                    help="HIP streams the independent resamples of a step are spread over "
                         "(weight set y on stream y mod S)")
    ap.add_argument("--concurrent-streams", type=int, default=3,
                    help="also time the step with the weight sets on this many streams "
                         "(reported as 'concurrent'; 1 = off)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB, a kernel of "
                         "known traffic for scaling hardware byte counters")
    ap.add_argument("--cpu-sample", type=int, default=N)
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="host seconds for repeated oracle runs (each cell runs at least once)")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-cache variant of the step")
    ap.add_argument("--workload", choices=("step", "precision", "batch", "filter", "decision",
                                              "aux", "philox", "scaling", "permute"),
                    default="step",
                    help="step: the timed resampling step (default); precision: the bias "
                         "sweep over prefix-sum precision modes; batch: ragged batch of "
                         "4096 filters; filter: full bootstrap filter, 1024 x 2^14 x 200; "
                         "decision: fastest scheme per (N, y) and the Metropolis B*/C "
                         "trade-off; aux: the auxiliary exports; philox: 10 vs 7 Philox "
                         "rounds; scaling: collective schemes at n = 2^20..2^26; permute: "
                         "the ancestor permutation at n = 2^20..2^24")
    ap.add_argument("--filters", type=int, default=4096)
    ap.add_argument("--filters-ssm", type=int, default=1024)
    ap.add_argument("--filter-reps", type=int, default=3)
    ap.add_argument("--replicates", type=int, default=1000)
    ap.add_argument("--sweep-log2n", type=int, nargs="+", default=[16, 18, 20, 22, 24])
    ap.add_argument("--decision-log2n", type=int, nargs=2, default=[4, 22])
    ap.add_argument("--decision-reps", type=int, default=20)
    ap.add_argument("--tradeoff-log2n", type=int, nargs="+", default=[12, 16, 20])
    ap.add_argument("--forms-log2n", type=int, nargs="+", default=[10, 14, 18, 20, 22, 24])
    ap.add_argument("--scaling-log2n", type=int, nargs="+", default=[20, 22, 24, 26])
    ap.add_argument("--permute-log2n", type=int, nargs="+", default=[20, 22, 24])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the resampling step here runs on a single MI355X "
              "and has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "precision":
        precision_sweep(args)
        return
    if args.workload == "batch":
        batch_workload(args)
        return
    if args.workload == "filter":
        filter_workload(args)
        return
    if args.workload == "decision":
        decision_workload(args)
        return
    if args.workload == "aux":
        aux_workload(args)
        return
    if args.workload == "philox":
        philox_workload(args)
        return
    if args.workload == "scaling":
        scaling_workload(args)
        return
    if args.workload == "permute":
        permute_workload(args)
        return

    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs, _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"libpfresample {pfr.version()} on {torch.cuda.get_device_name(0)}")

    if args.copy_calibration_mb > 0:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    n_streams = max(1, min(args.streams, len(YS)))
    n_conc = max(1, min(args.concurrent_streams, len(YS)))
    wl = StepWorkload(torch, pfr, dev, max(n_streams, n_conc))
    Bs, flags, ev, dominant = wl.Bs, wl.flags, wl.ev, wl.DOMINANT
    out, perm, wsp, ws_ = wl.out, wl.perm, wl.wsp, wl.w
    resample = wl.resample

    def step(record=False, n_st=n_streams):
        wl.step(record, n_st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised during the benchmark: {int(flags.cpu()[0])}")

    # the same steps with the weight sets spread over several streams, so that
    # the short launches of one set overlap the long kernels of another
    concurrent = None
    if n_conc > 1 and n_conc != n_streams:
        for _ in range(args.warmup):
            step(n_st=n_conc)
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        for _ in range(args.steps):
            step(n_st=n_conc)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc0
        concurrent = {"streams": n_conc, "ms_per_step": 1e3 * tc / args.steps,
                      "value": len(YS) * len(SCHEMES) * N * args.steps / tc,
                      "unit": "particles/s"}
        log(f"timed {args.steps} steps on {n_conc} streams in {tc:.3f} s")
        if int(flags.cpu()[0]) != 0:
            raise RuntimeError(f"data flags raised during the benchmark: {int(flags.cpu()[0])}")

    ms_step = 1e3 * elapsed / args.steps
    particles = len(YS) * len(SCHEMES) * N
    value = particles * args.steps / elapsed

    # the same step with cold caches: a 512 MiB write (twice the Infinity
    # Cache) before each step, HIP events around the step alone
    cold = None
    if not args.no_cold:
        flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        cur = torch.cuda.current_stream()
        t_cold = []
        for r in range(args.steps):
            flush.fill_(r & 0xFF)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(cur)
            step()
            e1.record(cur)
            e1.synchronize()
            t_cold.append(e0.elapsed_time(e1))
        del flush
        ms_cold = float(np.median(t_cold))
        cold = {"ms_per_step": ms_cold, "value": particles / (1e-3 * ms_cold),
                "unit": "particles/s", "flush_bytes": 512 << 20,
                "timing": f"HIP events around each step, a 512 MiB write before it, median of "
                          f"{args.steps}"}
        log(f"cold-cache step: {ms_cold:.3f} ms")
        if int(flags.cpu()[0]) != 0:
            raise RuntimeError(f"data flags raised during the benchmark: {int(flags.cpu()[0])}")

    dom_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    B_dom = Bs[YS.index(dominant[0])]
    dom_calls = N * metropolis_calls_per_lane(B_dom)
    achieved = dom_calls / (dom_ms * 1e-3)
    gathers = N * B_dom / (dom_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": f"Metropolis resample (y=4, B={B_dom})",
                "achieved": achieved / 1e9, "peak": PHILOX_PEAK_PER_S / 1e9,
                "unit": "G Philox4x32-10 calls/s", "frac": achieved / PHILOX_PEAK_PER_S,
                "limiter": (f"VALU instruction count: {gathers / 1e9:.0f} G steps/s x "
                            f"{DOMINANT_VALU_PER_STEP} VALU per step = "
                            f"{gathers * DOMINANT_VALU_PER_STEP / LANE_INSTR_PER_S:.2f} of the "
                            f"lane-instruction rate at 2.4 GHz (24 of the {DOMINANT_VALU_PER_STEP} "
                            f"are Philox); the steps run at "
                            f"{gathers / GATHER_CEILING_PER_S:.2f} x the "
                            f"{GATHER_CEILING_PER_S / 1e9:.0f} G/s of a plain gather kernel, "
                            f"the bound table skipping two thirds of the weight loads")
                           if DOMINANT_VALU_PER_STEP else None,
                "traffic": DOMINANT_TRAFFIC_BYTES, "traffic_unit": "bytes per launch",
                "algorithmic_bytes": 8.0 * N, "avg_launch_ms": dom_ms}

    # per-scheme breakdown (untimed pass, events around each call, one stream;
    # the timed steps have been synchronised, so stream 0's workspaces are free)
    stream = torch.cuda.current_stream()
    breakdown = {}
    for s in SCHEMES:
        rows = []
        for yi, y in enumerate(YS):
            reps = 5
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                resample(yi, y, s, 0)
            e1.record(stream)
            for _ in range(reps):
                pfr.permute_ancestors(out[(y, s)],
                                      sorted_hint=s not in ("metropolis", "rejection"),
                                      out=perm[(y, s)], flags=flags,
                                      workspace=wsp[(0, _lib.OP_PERMUTE)])
            e2.record(stream)
            torch.cuda.synchronize()
            t_res = e0.elapsed_time(e1) / reps
            t_perm = e1.elapsed_time(e2) / reps
            fused = {}
            if s in FUSED:
                e3 = torch.cuda.Event(enable_timing=True)
                e2.synchronize()
                e2.record(stream)
                for _ in range(reps):
                    pfr.resample_permuted(s, ws_[yi], seed=1, out=out[(y, s)],
                                          permuted=perm[(y, s)], flags=flags)
                e3.record(stream)
                e3.synchronize()
                fused = {"fused_us": 1e3 * e2.elapsed_time(e3) / reps}
            rows.append({"y": y, "resample_us": 1e3 * t_res, "permute_us": 1e3 * t_perm, **fused,
                         "particles_per_s": N / (t_res * 1e-3),
                         "hbm_frac_8B_per_particle": 8.0 * N / (t_res * 1e-3) / (HBM_PEAK_GBS * 1e9)})
        breakdown[s] = rows
    log("breakdown done")

    # the metric's second part: batched filters/s on the ragged batch of
    # 4096 vectors (one launch per resampler; per-filter binary64 form beside)
    batched = None
    if not args.no_batched:
        batched = batched_summary(torch, pfr, inputs, dev, stream, reps=5)
        log("batched summary done")
    hbm_2p20 = {s: max(r["hbm_frac_8B_per_particle"] for r in rows) for s, rows in breakdown.items()}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(args.cpu_sample, args.cpu_budget)

    result = {
        "metric": "resampled particles/sec and % HBM roofline at N=2^20 FP32; batched filters/sec",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single resample, n=2^20 float32 weights, y in {0,1,2,3,4}, "
                               "five resamplers (Metropolis B from the bias bound, rejection "
                               "w_max=1) + permute_ancestors on each output",
                   "n": N, "y": list(YS), "B": Bs, "resamples_per_step": len(YS) * len(SCHEMES),
                   "streams": n_streams},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "concurrent": concurrent,
        "cold": cold,
        "hbm_frac_8B_per_particle_at_2p20": hbm_2p20,
        "batched": batched,
        "breakdown": breakdown,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
