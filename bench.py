#!/usr/bin/env python3
"""Benchmark of the ordering-ICA hot path on one MI355X.

One step = the whole path on one batch of device-resident synthetic input:
whitening (FP64) -> batched kurtosis fixed point with removal of converged rows
-> FP64 kurtosis -> clustering up to sign, ordering and the Gaussianity test.

Default workload: the precision form at N=128, T=1e6, K=16,384 random starts
(48 Laplace, 32 Student-t nu=5, 24 uniform, 16 sines, 8 Gaussian sources):
BF16 data and BF16 MFMA with FP32 sums, then FP32 passes until the FP32
threshold; its roofline entry is the BF16 fused kernel against the BF16 MFMA
peak.  The same workload then runs in the plain FP32 form (time to the same
unique components), and the timed run's unique set is compared with the stored
FP64 oracle run of this workload when it is present.

Prints one JSON line.  ``value`` is thread-iterations per second over the whole
step (a thread-iteration is one update of one start vector: 2 N T MACs);
``ms_per_step`` is the time from raw data in HBM to the unique list on the host.

``--workload eeg_shaped_n64`` times the plain FP32 form on the EEG-shaped
mixture (N=64, T=2e5, K=4096) and compares the mixed-precision form;
``--workload pruner_n64`` times the learned-pruner workload (N=64, T=2e5,
K=65536, held-out seed 5300) against the plain FP32 and unpruned BF16 runs;
``--workload batched_n16_128`` times 64 datasets in one batched call.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
HBM_PROFILES = {
    "eeg_shaped_n64": os.path.join(ROOT, "profiles", "fused_update_eeg_shaped_n64_hbm_counters.txt"),
    "precision_n128": os.path.join(ROOT, "profiles", "fused_update_bf16_precision_n128_hbm_counters.txt"),
    "batched_n16_128": os.path.join(ROOT, "profiles", "batched_n16_128_hbm_counters.txt"),
}
GOLDEN = os.path.join(ROOT, "tests", "golden", "{}_oracle.json")


def counted_traffic(workload):
    """HBM bytes per launch of the fused update from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel's sources (the
    listed files, hashed in order as one byte string) have changed since those
    counters were taken."""
    import hashlib
    try:
        fields = {}
        for line in open(HBM_PROFILES[workload]):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for name in fields["source_files"].split(","):
            h.update(open(os.path.join(ROOT, name.strip()), "rb").read())
        if h.hexdigest() != fields["source_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="precision_n128",
                    choices=["eeg_shaped_n64", "precision_n128", "pruner_n64", "batched_n16_128"])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=None,
                    help="start rows in the CPU-oracle sample (default 256 at N=128, else 4096)")
    ap.add_argument("--cpu-passes", type=int, default=None,
                    help="passes in the CPU-oracle sample (default 4 at N=128, else 5)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison runs of the other precision forms (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--plain-coop-launch", action="store_true",
                    help="launch the all-rounds clustering without the cooperative-launch API "
                         "(profiling runs: the same kernel, a launch the profiler follows)")
    return ap.parse_args()


def copy_calibration(dev):
    """One plain 256 MiB device copy: the reference for the HBM counters."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(prob, rows: int, passes: int):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    whitening of the full data, then `passes` passes of the batched fixed point
    for the first `rows` start vectors (max_iter = passes, no early exit at
    this threshold)."""
    import threadpoolctl

    from oracle import ica
    info = threadpoolctl.threadpool_info()
    threads = max([d.get("num_threads", 1) for d in info] or [1])
    t0 = time.perf_counter()
    Xw, *_ = ica.whiten(prob.X)
    t1 = time.perf_counter()
    _, _, _, _, ti = ica.fixed_point(Xw, prob.W0[:rows], tol=1e-300, max_iter=passes)
    t2 = time.perf_counter()
    return {
        "value": ti / (t2 - t1),
        "unit": "thread-iterations/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{rows} of {prob.K} start rows x {passes} passes of the FP64 fixed point on "
                   f"the full N={prob.N}, T={prob.T} data (whitening {t1 - t0:.2f} s not counted); "
                   f"{os.cpu_count()} host CPUs ({cpu_model()}), BLAS threads {threads}"),
        "whiten_s": t1 - t0,
        "fixed_point_s": t2 - t1,
    }


def vs_oracle(workload, res):
    """Errors of a timed run's unique set against the stored FP64 oracle run of
    the same workload (tests/golden), in raw-data space; None if not stored."""
    path = GOLDEN.format(workload)
    if not os.path.exists(path):
        return None
    ref = json.load(open(path))
    n = ref["n_accepted"]
    V = res["V"].cpu().numpy()
    na = res["n_accepted"]
    U = res["U"].cpu().numpy()[:na] @ V
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    Ur = np.array(ref["U_raw"])[:n]
    cos = np.abs(U @ Ur.T) if na and n else np.zeros((na, n))
    best = cos.max(axis=1) if n else np.zeros(na)
    match = cos.argmax(axis=1) if n else np.zeros(na, int)
    ar = np.array(ref["alpha"])
    a = res["alpha"].cpu().numpy()[:na]
    rel = np.abs(a - ar[match]) / np.maximum(np.abs(ar[match]), 0.1) if na and n else np.zeros(0)
    return {"oracle": os.path.relpath(path, ROOT), "same_n_unique": res["n_unique"] == ref["n_unique"],
            "same_n_accepted": na == n, "one_to_one": len(set(match.tolist())) == na,
            "max_1_minus_abs_cos": float(np.max(1 - best)) if na else None,
            "max_kurtosis_rel_err": float(rel.max()) if rel.size else None}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path would "
              "shard by start rows across GPUs, which this program does not run.",
              file=sys.stderr)
        return 2
    import torch

    from paper_2408_17118_amd import oica, synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.plain_coop_launch:
        oica.set_option(oica.OPT_COOP_LAUNCH_API, 0)
    if args.workload == "batched_n16_128":
        return bench_batched(args)
    dev = torch.device("cuda", 0)
    bf16 = args.workload in ("precision_n128", "pruner_n64")
    if args.workload == "precision_n128":
        prob = synth.precision_workload()
    elif args.workload == "pruner_n64":
        prob = synth.pruner_workload(5300)
    else:
        prob = synth.eeg_shaped()
    N, T, K = prob.N, prob.T, prob.K
    precision = "bf16" if bf16 else "f32"
    X = torch.from_numpy(prob.X).to(dev)
    W0 = torch.from_numpy(prob.W0.astype(np.float32)).to(dev)
    ctx = oica.Context(0)
    pruner = None
    if args.workload == "pruner_n64":
        m = json.load(open(os.path.join(ROOT, "paper_2408_17118_amd", "pruner_model.json")))
        pruner = oica.Pruner(ctx, np.array(m["weights"], np.float32), m["feat_mean"], m["feat_std"])
        pruner.set_threshold(m["theta"])
    if args.copy_calibration:
        copy_calibration(dev)

    def step(profile=False):
        return oica.ordering_ica(ctx, X, W0, tol=1e-6, max_iter=1000, tau=1e-3, profile=profile,
                                 precision=precision, tol_bf16=1e-3, refine_iters=5, pruner=pruner)

    for i in range(args.warmup):
        r = step()
        print(f"warmup {i}: {r['fp']['passes']} passes, {r['n_accepted']} accepted", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(step(profile=True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    ti = sum(r["fp"]["thread_iters"] for r in runs)
    ti_refine = sum(r["fp"]["refine_thread_iters"] for r in runs)
    value = (ti + ti_refine) / (t1 - t0)
    # dominant kernel: the fused update.  Algorithmic work per launch = 4 N T
    # flops per active row (2 N T MACs); average active rows per launch =
    # thread_iters / launches (launches issued after the last row stopped, before
    # the host's next poll, count with zero rows, exactly as a profiler sees them).
    upd_ms = sum(r["fp"]["update_ms"] for r in runs)
    launches = sum(r["fp"]["update_launches"] for r in runs)
    flops = 4.0 * N * T * ti
    achieved_tflops = flops / (upd_ms * 1e-3) / 1e12 if upd_ms > 0 else None
    peak = PEAK_BF16_MFMA_TFLOPS if bf16 else PEAK_FP32_MFMA_TFLOPS
    np_ = ((N + 31) // 32) * 32
    wk_ = 2 if np_ <= 64 else 1
    if bf16:
        tail = f"; <{np_},1> in passes with <= 128 active rows" if wk_ == 2 else ""
        kname = f"k_fused_bf16<{np_},{wk_},2> (GEMM1 on bf16 hi+lo rows + cube + GEMM2, BF16 MFMA{tail})"
    else:
        kname = (f"k_fused_f32<{np_},{wk_}> (GEMM1 + cube + GEMM2, FP32 MFMA; "
                 f"k_fused_f32_thin<{np_}> in passes with <= 256 active rows)")
    last = runs[-1]
    out = {
        "metric": "thread-iterations/sec (K*N*T MACs) + time-to-unique-components vs plain FP32",
        "value": value,
        "unit": "thread-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if bf16 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "T": T, "K": K, "tol": 1e-6,
                   "max_iter": 1000, "precision": precision,
                   "tol_bf16": 1e-3 if bf16 else None,
                   "seed": {"eeg_shaped_n64": 1, "precision_n128": 3, "pruner_n64": 5300}[args.workload],
                   "passes": last["fp"]["passes"], "thread_iters_per_step": last["fp"]["thread_iters"],
                   "fp32_thread_iters_per_step": last["fp"]["refine_thread_iters"],
                   "n_unique": last["n_unique"], "n_accepted": last["n_accepted"],
                   "time_to_unique_ms": ms_per_step},
        "roofline": {
            "bound": "mfma",
            "kernel": kname,
            "achieved": achieved_tflops,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": (achieved_tflops / peak) if achieved_tflops else None,
            "traffic": counted_traffic(args.workload),
            "traffic_unit": "bytes/launch (HBM FETCH+WRITE, calibrated)",
            "avg_launch_ms": upd_ms / launches if launches else None,
            "avg_rows_per_launch": ti / launches if launches else None,
            "update_share_of_step": (upd_ms / args.steps) / ms_per_step if ms_per_step else None,
        },
    }
    # the comparison runs (outside the timed region): the same workload in the
    # other form(s), same data and start vectors
    def compare(name, **kw):
        oica.ordering_ica(ctx, X, W0, tol=1e-6, max_iter=1000, **kw)   # warm-up
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            r = oica.ordering_ica(ctx, X, W0, tol=1e-6, max_iter=1000, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - c0) * 1e3 / reps
        n = min(r["n_accepted"], last["n_accepted"])
        Ua = last["U"].cpu().numpy()[:n] @ last["V"].cpu().numpy()
        Ub = r["U"].cpu().numpy()[:n] @ r["V"].cpu().numpy()
        Ua /= np.linalg.norm(Ua, axis=1, keepdims=True)
        Ub /= np.linalg.norm(Ub, axis=1, keepdims=True)
        cos = np.abs(Ua @ Ub.T).max(axis=1) if n else np.zeros(0)
        return {"form": name, "time_to_unique_ms": ms, "thread_iters": r["fp"]["thread_iters"],
                "fp32_thread_iters": r["fp"]["refine_thread_iters"], "n_accepted": r["n_accepted"],
                "same_accepted_count": r["n_accepted"] == last["n_accepted"],
                "min_abs_cos_vs_timed": float(cos.min()) if n else None,
                "pruned": r["fp"].get("pruned", 0)}
    if args.no_compare:
        pass
    elif args.workload == "precision_n128":
        pf = compare("plain fp32", precision="f32")
        out["plain_fp32"] = pf
        out["speedup_vs_plain_fp32"] = pf["time_to_unique_ms"] / ms_per_step
    elif args.workload == "eeg_shaped_n64":
        mp = compare("bf16 + fp32 finish (mixed precision)", precision="bf16", tol_bf16=1e-3)
        mp["speedup_vs_plain_fp32"] = ms_per_step / mp["time_to_unique_ms"]
        out["mixed_precision"] = mp
    elif args.workload == "pruner_n64":
        pf = compare("plain fp32", precision="f32")
        ub = compare("bf16 without pruner", precision="bf16", tol_bf16=1e-3)
        out["plain_fp32"] = pf
        out["bf16_unpruned"] = ub
        out["speedup_vs_plain_fp32"] = pf["time_to_unique_ms"] / ms_per_step
        out["pruner_thread_iter_saving"] = 1.0 - (ti / args.steps) / ub["thread_iters"]
    vo = vs_oracle(args.workload, last)
    if vo is not None:
        out["vs_oracle"] = vo
    if not args.no_cpu_baseline:
        rows = args.cpu_rows or (256 if N == 128 else 4096)
        passes = args.cpu_passes or (4 if N == 128 else 5)
        cb = cpu_baseline(prob, rows, passes)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    ctx.close()
    print(json.dumps(out))
    return 0


def bench_batched(args):
    """Many-dataset workload: 64 datasets (N uniform over 16..128 in steps of 8,
    T log-uniform in [2e4, 5e5], K = 1024 each), raw data resident on the GPU.
    A step is whitening of every dataset, one batched fixed point (BF16 data,
    FP32 finish) and the unique set of every dataset.  Compared with the same
    datasets run one call at a time, and with the batched FP32 form."""
    import torch

    from paper_2408_17118_amd import oica, synth
    dev = torch.device("cuda", 0)
    Xs, W0s, NT = [], [], []
    for N, T, rng in synth.batched_shapes():
        p = synth.batched_problem(N, T, rng)
        Xs.append(torch.from_numpy(p.X).to(dev))
        W0s.append(torch.from_numpy(p.W0.astype(np.float32)).to(dev))
        NT.append((N, T))
        del p
        if len(Xs) % 16 == 0:
            print(f"generated {len(Xs)} datasets", file=sys.stderr, flush=True)
    if args.copy_calibration:
        copy_calibration(dev)
    ctx = oica.Context(0)
    kw = dict(tol=1e-6, max_iter=1000, tau=1e-3, precision="bf16", tol_bf16=1e-3, refine_iters=5)

    def step(profile=False, **over):
        return oica.ordering_ica_batched(ctx, Xs, W0s, profile=profile, **{**kw, **over})

    for i in range(args.warmup):
        res, st = step()
        print(f"warmup {i}: {st}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(profile=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    ti = sum(st["thread_iters"] + st["refine_thread_iters"] for _, st in runs)
    upd_ms = sum(st["update_ms"] for _, st in runs)
    flops = sum(st["update_flops"] for _, st in runs)
    launches = sum(st["update_launches"] for _, st in runs)
    achieved = flops / (upd_ms * 1e-3) / 1e12 if upd_ms > 0 else None
    last, lst = runs[-1]
    accepted = [r["n_accepted"] for r in last]

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - c0) * 1e3 / reps, out

    def seq():
        return [oica.ordering_ica(ctx, X, W0, **kw) for X, W0 in zip(Xs, W0s)]
    if not args.no_compare:
        seq_ms, seq_res = timed(seq)
        f32_ms, (f32_res, f32_st) = timed(lambda: step(precision="f32"))
    out = {
        "metric": "thread-iterations/sec (K*N*T MACs) + time-to-unique-components vs plain FP32",
        "value": ti / (t1 - t0),
        "unit": "thread-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "batched_n16_128", "datasets": len(Xs), "K_each": 1024,
                   "sum_NT": int(sum(n * t for n, t in NT)), "tol": 1e-6, "max_iter": 1000,
                   "precision": "bf16", "tol_bf16": 1e-3, "seed": 4, "passes": lst["passes"],
                   "thread_iters_per_step": lst["thread_iters"],
                   "fp32_thread_iters_per_step": lst["refine_thread_iters"],
                   "grid": lst["grid"], "wk32": lst["wk32"], "wk64": lst["wk64"],
                   "n_accepted_total": int(sum(accepted)), "time_to_unique_ms": ms_per_step},
        "roofline": {
            "bound": "mfma",
            "kernel": "k_fused_batched<bf16> (persistent; GEMM1 on bf16 hi+lo rows + cube + GEMM2, BF16 MFMA)",
            "achieved": achieved,
            "peak": PEAK_BF16_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_MFMA_TFLOPS if achieved else None,
            "traffic": counted_traffic("batched_n16_128"),
            "avg_launch_ms": upd_ms / launches if launches else None,
            "update_share_of_step": (upd_ms / args.steps) / ms_per_step,
        },
    }
    if not args.no_compare:
        out["one_call_per_dataset"] = {
            "form": "bf16 + fp32 finish, one ordering_ica call per dataset",
            "time_to_unique_ms": seq_ms,
            "speedup_of_batched": seq_ms / ms_per_step,
            "n_accepted_total": int(sum(r["n_accepted"] for r in seq_res)),
        }
        out["batched_fp32"] = {
            "form": "batched, fp32 data",
            "time_to_unique_ms": f32_ms,
            "thread_iters": f32_st["thread_iters"],
            "n_accepted_total": int(sum(r["n_accepted"] for r in f32_res)),
            "speedup_of_bf16": f32_ms / ms_per_step,
        }
    ctx.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
