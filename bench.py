"""Benchmark of the resampling step on one MI355X.

Workload (one step): n = 2^20 float32 weights w_i = exp(-(x_i - y)^2 / 2),
x_i ~ N(0,1), for each y in {0, 1, 2, 3, 4}; each weight set is resampled by
all five resamplers -- multinomial, stratified, systematic (exact prefix sums),
Metropolis with B from the bias bound (eps = 1/100, beta = E[w]/w_max, giving
B = 4, 6, 16, 60, 354), rejection with w_max = 1 -- and every ancestry is then
permuted for in-place propagation.  That is 25 resamples of 2^20 particles
per step; inputs are resident in HBM before the timed region.

Prints one JSON line: whole-step particles/s, the roofline of the dominant
kernel measured with HIP events inside the timed steps, a per-scheme
breakdown, and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
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
HBM_PEAK_GBS = 8000.0
# Philox4x32-10 per call: 20 32x32->64-bit products (one v_mad_u64_u32 each,
# quarter rate: 4 lane-cycles) and 20 three-input xors (1 lane-cycle each) =
# 100 lane-cycles; 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-cycles/s.
PHILOX_PEAK_PER_S = 256 * 4 * 16 * 2.4e9 / 100.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def b_star(y, eps=0.01):
    from paper_1301_4019_amd.inputs import expected_weight
    return math.ceil(math.log(eps) / math.log(1.0 - expected_weight(y)))


def cpu_baseline(n_sample: int):
    """The oracle (single-threaded C, binary128 sums) on the same step at n_sample."""
    import oracle
    from paper_1301_4019_amd import inputs
    t0 = time.perf_counter()
    done = 0
    for y in YS:
        w = inputs.weights(n_sample, y, seed=100 + int(y))
        for s in SCHEMES:
            if s == "metropolis":
                a = oracle.metropolis(w, b_star(y), seed=1)
            elif s == "rejection":
                a = oracle.rejection(w, 1.0, seed=1)[0]
            else:
                a = getattr(oracle, s)(w, seed=1)[0]
            oracle.permute(a)
            done += n_sample
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"the full step (5 weight sets x 5 resamplers + permutation) at n = "
                      f"{n_sample} instead of 2^20; {dt:.1f} s on one host core"}


def precision_sweep(args):
    """Bias of the collective resamplers per prefix-sum precision mode.

    For each n, one weight vector (y = 3, data seed 0) is resampled K times
    (Philox seeds 1..K) by every collective scheme in every precision mode,
    with Metropolis (B = 60) and rejection (w_max = 1) as controls.  Offspring
    are counted on the GPU and accumulated in binary64.  Reported, as in the
    paper's section 3: ||Bias||^2 = sum_i (mean o_i - n w_i / W)^2, the MSE,
    their ratio (about 1 / (K + 1) for an unbiased scheme) and MSE / n, plus
    the noise-corrected excess ||Bias||^2 - tr(Var) / K.
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
    rows = []
    t_start = time.perf_counter()
    for lg in args.sweep_log2n:
        n = 1 << lg
        w = torch.from_numpy(inputs.weights(n, y, seed=0)).to(dev)
        wd = w.double()
        e = n * wd / wd.sum()
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
            bias2 = float(((mean - e) ** 2).sum())
            mse = float((S2 / K - 2.0 * e * mean + e * e).sum())
            var_tr = float(((S2 - K * mean * mean) / (K - 1)).sum())
            rows.append({"n": n, "scheme": scheme, "precision": mode, "bias2": bias2, "mse": mse,
                         "bias2_over_mse": bias2 / mse, "mse_over_n": mse / n,
                         "bias2_excess": bias2 - var_tr / K})
        log(f"n = 2^{lg} done ({time.perf_counter() - t_start:.0f} s)")
    if int(flags.cpu()[0]) != 0:
        raise RuntimeError(f"data flags raised during the sweep: {int(flags.cpu()[0])}")
    result = {"metric": "bias contribution to the MSE per prefix-sum precision",
              "unit": "ratio", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
              "config": {"workload": "precision sweep: y = 3 weights (data seed 0), "
                                     f"{K} Philox seeds per case, n = 2^" +
                                     ",".join(str(v) for v in args.sweep_log2n),
                         "replicates": K, "y": y, "unbiased_ratio": 1.0 / (K + 1)},
              "rows": rows}
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 18)
    ap.add_argument("--workload", choices=("step", "precision"), default="step",
                    help="step: the timed resampling step (default); precision: the bias "
                         "sweep over prefix-sum precision modes")
    ap.add_argument("--replicates", type=int, default=256)
    ap.add_argument("--sweep-log2n", type=int, nargs="+", default=[16, 18, 20, 22, 24])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the resampling step here runs on a single MI355X "
              "and has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "precision":
        precision_sweep(args)
        return

    import torch
    import paper_1301_4019_amd as pfr
    from paper_1301_4019_amd import inputs, _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"libpfresample {pfr.version()} on {torch.cuda.get_device_name(0)}")

    ws_ = [torch.from_numpy(inputs.weights(N, y, seed=100 + int(y))).to(dev) for y in YS]
    Bs = [b_star(y) for y in YS]
    out = {(y, s): torch.empty(N, dtype=torch.int32, device=dev) for y in YS for s in SCHEMES}
    perm = {(y, s): torch.empty(N, dtype=torch.int32, device=dev) for y in YS for s in SCHEMES}
    wsp = {op: pfr.new_workspace(max(256, pfr.workspace_bytes(op, N)), dev)
           for op in (_lib.OP_MULTINOMIAL, _lib.OP_STRATIFIED, _lib.OP_SYSTEMATIC,
                      _lib.OP_PERMUTE)}
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    dominant = (4.0, "metropolis")
    ev = []

    def resample(yi, y, s):
        w = ws_[yi]
        a = out[(y, s)]
        if s == "metropolis":
            pfr.resample_metropolis(w, Bs[yi], seed=1, out=a)
        elif s == "rejection":
            pfr.resample_rejection(w, 1.0, seed=1, out=a, flags=flags)
        else:
            op = {"multinomial": _lib.OP_MULTINOMIAL, "stratified": _lib.OP_STRATIFIED,
                  "systematic": _lib.OP_SYSTEMATIC}[s]
            getattr(pfr, "resample_" + s)(w, seed=1, out=a, flags=flags, workspace=wsp[op])
        return a

    def step(record=False):
        for yi, y in enumerate(YS):
            for s in SCHEMES:
                if record and (y, s) == dominant:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    a = resample(yi, y, s)
                    e1.record(stream)
                    ev.append((e0, e1))
                else:
                    a = resample(yi, y, s)
                pfr.permute_ancestors(a, sorted_hint=s not in ("metropolis", "rejection"),
                                      out=perm[(y, s)], flags=flags,
                                      workspace=wsp[_lib.OP_PERMUTE])

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

    ms_step = 1e3 * elapsed / args.steps
    particles = len(YS) * len(SCHEMES) * N
    value = particles * args.steps / elapsed

    dom_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    dom_calls = N * Bs[YS.index(dominant[0])]
    achieved = dom_calls / (dom_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": "k_metropolis<float> (y=4, B=354)",
                "achieved": achieved / 1e9, "peak": PHILOX_PEAK_PER_S / 1e9,
                "unit": "G Philox4x32-10 calls/s", "frac": achieved / PHILOX_PEAK_PER_S,
                "traffic": None, "avg_launch_ms": dom_ms}

    # per-scheme breakdown (untimed pass, events around each call)
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
                resample(yi, y, s)
            e1.record(stream)
            for _ in range(reps):
                pfr.permute_ancestors(out[(y, s)],
                                      sorted_hint=s not in ("metropolis", "rejection"),
                                      out=perm[(y, s)], flags=flags,
                                      workspace=wsp[_lib.OP_PERMUTE])
            e2.record(stream)
            torch.cuda.synchronize()
            t_res = e0.elapsed_time(e1) / reps
            t_perm = e1.elapsed_time(e2) / reps
            rows.append({"y": y, "resample_us": 1e3 * t_res, "permute_us": 1e3 * t_perm,
                         "particles_per_s": N / (t_res * 1e-3),
                         "hbm_frac_8B_per_particle": 8.0 * N / (t_res * 1e-3) / (HBM_PEAK_GBS * 1e9)})
        breakdown[s] = rows
    log("breakdown done")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(args.cpu_sample)

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
                   "n": N, "y": list(YS), "B": Bs, "resamples_per_step": len(YS) * len(SCHEMES)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "breakdown": breakdown,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
