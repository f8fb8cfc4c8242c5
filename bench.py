"""Throughput benchmark: trajectories/s of pruned vs full evolution of
amplitude-damped bucket-brigade QRAM queries on one MI355X.

Workload (one step): the n = 10, k = 4, gamma = 1e-3 data-loading query in
both encodings, 1e5 trajectories each (seeded synthetic memory and noise),
run in pruned mode; the full mode is timed the same way as the comparator.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K, GAMMA = 10, 4, 1e-3
CFG_ID = 3
PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes per clock x 2.4 GHz
COUNTER_FILE = os.path.join(ROOT, "profiles", "evolve_qubit_n10k4_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2609_34935_amd", "csrc", "qram_kernels.hip")


def ops_per_component_slice(n, k):
    """Algorithmic work of one explicit component through one slice: about
    6 FP64 operations (K0 weight, |A|^2, accumulation) and 2n + 3k integer
    operations (site moves and mask merge)."""
    return 6 + 2 * n + 3 * k


def traffic_from_profile():
    """HBM bytes per launch of the qubit evolution kernel from the committed
    rocprofv3 counter summary, or None if the kernel changed since."""
    try:
        prof = json.load(open(COUNTER_FILE))
    except (OSError, ValueError):
        return None
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if prof.get("kernel_sha256") != src:
        return None
    return prof.get("hbm_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(mem, ntraj_sample):
    from oracle import oracle as O
    threads = min(16, os.cpu_count() or 1)
    t_enc = {}
    for enc in (1, 0):
        t0 = time.perf_counter()
        _, _, _, used = O.run_batch(N, K, enc, GAMMA, mem, 880000 + CFG_ID, 0, ntraj_sample, nthreads=threads)
        t_enc[enc] = time.perf_counter() - t0
    total = 2 * ntraj_sample
    return {"value": total / (t_enc[0] + t_enc[1]), "unit": "trajectories/s", "cores": used, "kind": "oracle",
            "sample": f"first {ntraj_sample} trajectories of each encoding (qubit {t_enc[1]:.2f} s, "
                      f"qutrit {t_enc[0]:.2f} s wall), full evolution of every branch on the host"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ntraj", type=int, default=100000)
    ap.add_argument("--cpu-sample", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--launch-cache", default=None,
                    help="JSON file of tuned launch shapes: read if present, else written")
    ap.add_argument("--modes", default="pruned,full")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(trajectories shard by index range across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_34935_amd as P
    from paper_2609_34935_amd.inputs import memory_words

    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del x, y
    mem = memory_words(N, K, 1000 + CFG_ID)
    seed = 880000 + CFG_ID
    nt = args.ntraj
    T = 6 * N + 2 * K
    ctxs = {enc: P.QramContext(N, K, enc, GAMMA, mem) for enc in (P.QRAM_QUBIT, P.QRAM_QUTRIT)}
    tuned = {}
    cache = None
    if args.launch_cache and os.path.exists(args.launch_cache):
        cache = json.load(open(args.launch_cache))
    for enc, ctx in ctxs.items():
        for mode in (P.QRAM_MODE_PRUNED, P.QRAM_MODE_FULL):
            key = f"{enc}:{mode}"
            if cache and key in cache:
                ctx.set_launch(mode, *cache[key])
            elif not args.no_tune:
                ms = ctx.autotune(mode, seed, 0, min(nt, 16384))
                log(f"autotune enc={enc} mode={mode}: {ctx.get_launch(mode)} {ms:.3f} ms")
            tuned[(enc, mode)] = ctx.get_launch(mode)
    if args.launch_cache and cache is None:
        json.dump({f"{e}:{m}": list(v) for (e, m), v in tuned.items()}, open(args.launch_cache, "w"))
    modes = [P.QRAM_MODE_PRUNED] + ([P.QRAM_MODE_FULL] if "full" in args.modes.split(",") else [])
    stream = torch.cuda.current_stream()
    d_fid = {enc: torch.empty(nt, dtype=torch.float64, device="cuda") for enc in ctxs}
    d_st = {enc: torch.empty(nt * 32, dtype=torch.uint8, device="cuda") for enc in ctxs}

    def step(mode):
        for enc, ctx in ctxs.items():
            fn = ctx.run_pruned_async if mode == P.QRAM_MODE_PRUNED else ctx.run_full_async
            fn(seed, 0, nt, d_fid[enc], d_st[enc], stream=stream)

    results = {}
    for mode in modes:
        for _ in range(args.warmup):
            step(mode)
        torch.cuda.synchronize()
        for ctx in ctxs.values():
            ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stage = {}
        for enc, ctx in ctxs.items():
            stage[enc] = ctx.stage_times()
            ctx.set_timing(False)
        st = {enc: np.frombuffer(d_st[enc].cpu().numpy().tobytes(), dtype=P.STATS_DTYPE) for enc in ctxs}
        fids = {enc: d_fid[enc].cpu().numpy() for enc in ctxs}
        results[mode] = dict(dt=dt, stage=stage, st=st, fid=fids)
        log(f"mode={mode}: {args.steps} steps in {dt:.3f} s")

    pr, fu = results[P.QRAM_MODE_PRUNED], results.get(P.QRAM_MODE_FULL)
    total = 2 * nt * args.steps
    value = total / pr["dt"]
    full_value = total / fu["dt"] if fu else None
    if fu:
        for enc in ctxs:  # the two modes must agree trajectory by trajectory
            a, b = pr["fid"][enc], fu["fid"][enc]
            assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(np.abs(b), 1e-3)), "pruned and full disagree"

    # roofline of the dominant kernel: the qubit evolution launch
    (ms_stage, nb) = pr["stage"][P.QRAM_QUBIT]
    evolve_ms = ms_stage[2] / max(nb, 1)
    units = float(pr["st"][P.QRAM_QUBIT]["n_explicit"].astype(np.float64).sum()) * (T - 1)
    achieved = units * ops_per_component_slice(N, K) / (evolve_ms * 1e-3) / 1e12
    per_enc = {}
    for enc, name in ((P.QRAM_QUBIT, "qubit"), (P.QRAM_QUTRIT, "qutrit")):
        s = pr["st"][enc]
        ms_p, nbp = pr["stage"][enc]
        ms_f, nbf = fu["stage"][enc] if fu else (np.full(3, np.nan), 1)
        per_enc[name] = {
            "pruned_evolve_ms": round(ms_p[2] / max(nbp, 1), 3),
            "full_evolve_ms": None if not fu else round(ms_f[2] / max(nbf, 1), 3),
            "sample_classify_ms": round((ms_p[0] + ms_p[1]) / max(nbp, 1), 3),
            "pruned_traj_per_s_kernels": round(nt / (ms_p.sum() / max(nbp, 1) * 1e-3), 1),
            "full_traj_per_s_kernels": None if not fu else round(nt / (ms_f.sum() / max(nbf, 1) * 1e-3), 1),
            "evolved_fraction": round(float(s["n_explicit"].mean()) / (2**N * (2**K if enc == P.QRAM_QUBIT else 1)), 4),
            "mean_fidelity": round(float(pr["fid"][enc].mean()), 6),
            "launch_pruned": tuned[(enc, P.QRAM_MODE_PRUNED)],
            "launch_full": tuned[(enc, P.QRAM_MODE_FULL)],
        }
    line = {
        "metric": "trajectories/sec pruned vs full at n=10, gamma=1e-3 (1 GPU); p50/p99 req latency",
        "value": round(value, 1),
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(pr["dt"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bucket-brigade QRAM query n=10 k=4 gamma=1e-3, qubit and qutrit "
                               "encodings, 1e5 trajectories each, pruned evolution",
                   "n": N, "k": K, "gamma": GAMMA, "trajectories_per_step": 2 * nt,
                   "memory": "seeded Bernoulli(0.5), mem_seed 1003", "seed": seed},
        "full_value": None if full_value is None else round(full_value, 1),
        "speedup_pruned_over_full": None if full_value is None else round(value / full_value, 4),
        "per_encoding": per_enc,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TOPS, 3),
                     "unit": "TOP/s", "frac": round(achieved / PEAK_ALU_TOPS, 4),
                     "traffic": traffic_from_profile(),
                     "kernel": "k_evolve<qubit> pruned", "launch_ms": round(evolve_ms, 3),
                     "units_per_launch": units, "ops_per_unit": ops_per_component_slice(N, K)},
        "latency": None,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(mem, args.cpu_sample)
    print(json.dumps(line), flush=True)
    for ctx in ctxs.values():
        ctx.close()


if __name__ == "__main__":
    main()
