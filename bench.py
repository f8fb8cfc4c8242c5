"""Throughput benchmark: trajectories/s of pruned vs plain full evolution of
amplitude-damped bucket-brigade QRAM queries on one MI355X, plus the serving
mix's p50/p99 request latency.

Headline step: the n = 10, k = 4, gamma = 1e-3 data-loading query in both
encodings, 1e5 trajectories each (seeded synthetic memory and noise), pruned
evolution (Alg. 1), inputs and outputs resident on the device.  Timed beside
it on the same trajectories:
  - the plain full evolution (every component of every branch explicit,
    slice by slice, nothing predicted): full_value, the comparator;
  - the trajectory kernel's full mode (every branch explicit, components
    untouched by jumps implicit): full_engine_value;
  - the pruned step as HIP graphs; the qubit step under the damping-only
    subtree marking;
  - the n = 6, k = 1 qubit query at three gammas (pruned, full, plain) and
    the n = 14, k = 1 qutrit stress case (traj/s and device footprint);
  - the serving mix through the request server (Poisson arrivals);
  - the oracle on the host's cores (cpu_baseline).
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
PEAK_HBM_GBS = 8000.0                    # MI355X HBM3E
PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes per clock x 2.4 GHz
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2609_34935_amd", "csrc")
# committed rocprofv3 counter summaries: (file, kernel sources)
COUNTERS = {
    "evolve_qubit": ("evolve_qubit_n10k4_main_counters.json", ("qram_evolve.hip", "qram_device.h",
                                                               "qram_internal.h", "qram_records.h")),
    "evolve_qutrit": ("evolve_qutrit_n10k4_main_counters.json", ("qram_evolve.hip", "qram_device.h",
                                                                 "qram_internal.h", "qram_records.h")),
    "plain_qubit": ("plain_qubit_n10k4_counters.json", ("qram_plain.hip", "qram_device.h", "qram_internal.h")),
}


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def traffic_from_profile(key):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the
    committed counter summary, or None if the kernel's sources changed since."""
    name, srcs = COUNTERS[key]
    try:
        prof = json.load(open(os.path.join(PROFILES, name)))
    except (OSError, ValueError):
        return None
    if prof.get("kernel_sha256") != sources_sha256(srcs):
        return None
    return prof.get("hbm_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ops_per_component_slice(n, k):
    """The explicit sweep's work per component and slice: about 6 FP64
    operations (K0 scale, |A|^2, accumulation) and 2n + 3k integer operations
    (site moves, mask merge)."""
    return 6 + 2 * n + 3 * k


def bytes_per_component(n, k):
    """Explicit state of one component in the plain sweep: complex FP64
    amplitude (16 B), its site list (2 B per entry, 2n + 3k entries at
    most) and a count (4 B), rounded up to 8 B."""
    b = 16 + 2 * (2 * n + 3 * k) + 4
    return (b + 7) // 8 * 8


def cpu_baseline(mem, n_qubit, n_qutrit):
    """The oracle (full evolution of every branch, plain C, OpenMP over
    trajectories) on the first trajectories of each encoding."""
    from oracle import oracle as O
    host = os.cpu_count() or 1
    threads = min(16, host)  # one GPU's share of a 16-CPU-per-GPU host
    per = {}
    used = threads
    for enc, cnt in ((1, n_qubit), (0, n_qutrit)):
        t0 = time.perf_counter()
        _, _, _, used = O.run_batch(N, K, enc, GAMMA, mem, 880000 + CFG_ID, 0, cnt, nthreads=threads)
        per[enc] = (time.perf_counter() - t0, cnt)
    # one step holds as many qubit as qutrit trajectories
    t_pair = per[1][0] / per[1][1] + per[0][0] / per[0][1]
    one = {}
    for enc, cnt in ((1, max(1, n_qubit // 16)), (0, max(1, n_qutrit // 16))):
        t0 = time.perf_counter()
        O.run_batch(N, K, enc, GAMMA, mem, 880000 + CFG_ID, 0, cnt, nthreads=1)
        one[enc] = (time.perf_counter() - t0, cnt)
    t_one = one[1][0] / one[1][1] + one[0][0] / one[0][1]
    return {"value": round(2.0 / t_pair, 2), "unit": "trajectories/s", "cores": used, "kind": "oracle",
            "host_cpu_count": host,
            "sample": f"first {per[1][1]} qubit and {per[0][1]} qutrit trajectories of the step's workload "
                      f"({per[1][0]:.1f} s and {per[0][0]:.1f} s wall on {used} threads: the host reports "
                      f"{host} CPUs, one GPU's share is 16), full evolution of every branch on the host; "
                      "value = 2 / (mean qubit + mean qutrit time per trajectory)",
            "single_thread": {"value": round(2.0 / t_one, 2), "unit": "trajectories/s",
                              "sample": f"first {one[1][1]} qubit and {one[0][1]} qutrit trajectories on one "
                                        f"thread ({one[1][0]:.1f} s and {one[0][0]:.1f} s)"}}


def _serve_once(P, reqs, mems, arrivals, chunk, max_active, budget_gib, tag):
    with P.QramServer(int(budget_gib * (1 << 30)), max_active=max_active, chunk=chunk) as srv:
        t0 = time.perf_counter()
        tickets = []
        for r, mem, ta in zip(reqs, mems, arrivals):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(r["n"], r["k"], r["enc"], r["gamma"], mem, r["seed"], r["shots"],
                                      P.QRAM_MODE_PRUNED))
        res = []
        for i, t in enumerate(tickets):
            res.append(srv.wait(t))
            if (i + 1) % 250 == 0:
                log(f"serving {tag}: {i + 1}/{len(reqs)} requests done")
        wall = time.perf_counter() - t0
    bad = [x for x in res if x["state"] != "done"]
    if bad:
        raise RuntimeError(f"serving requests failed: {bad[:3]}")
    lat = np.array([x["latency_ms"] for x in res])
    shots = sum(x["shots"] for x in res)
    return {"p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mean_ms": round(float(lat.mean()), 2), "max_ms": round(float(lat.max()), 2),
            "queue_p50_ms": round(float(np.percentile([x["queue_ms"] for x in res], 50)), 2),
            "requests": len(reqs), "trajectories": int(shots),
            "aggregate_traj_per_s": round(shots / wall, 1), "wall_s": round(wall, 3)}


def serving_leg(P, nreq, ncap, seed, chunk, max_active, budget_gib):
    """The serving mix through the request server.  The capacity mu (requests
    per second) is measured on the first ncap requests submitted at once (a
    warm-up too); then nreq requests arrive as a Poisson stream at 0.5 mu and
    at 0.8 mu.  Latency is submission to results on the host."""
    from paper_2609_34935_amd.inputs import memory_words, request_mix
    out = {}
    reqs = request_mix(nreq, seed)
    mems = [memory_words(r["n"], r["k"], r["mem_seed"]) for r in reqs]
    sat = _serve_once(P, reqs[:ncap], mems[:ncap], np.zeros(ncap), chunk, max_active, budget_gib, "saturated")
    mu = ncap / sat["wall_s"]
    out["saturated"] = dict(sat, capacity_req_per_s=round(mu, 2))
    for frac, key in ((0.5, "load_0.5"), (0.8, "load_0.8")):
        rng = np.random.default_rng(seed + 100 + int(frac * 10))
        arrivals = np.cumsum(rng.exponential(1.0 / (frac * mu), size=nreq))
        out[key] = dict(_serve_once(P, reqs, mems, arrivals, chunk, max_active, budget_gib, key),
                        arrival_rate_per_s=round(frac * mu, 2))
    head = out["load_0.8"]
    return {"p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "at": "Poisson arrivals at 0.8 x measured capacity",
            "aggregate_traj_per_s": out["saturated"]["aggregate_traj_per_s"], **out,
            "mix": "n~U{4..12}, k~U{1,2,4}, encoding~U, gamma log-uniform [1e-5,1e-2], "
                   "shots log-uniform [1e3,1e5], seeded Bernoulli(0.5) memory, pruned mode, master seed "
                   f"{seed}; capacity from the first {ncap} requests at once, then {nreq} requests per "
                   f"Poisson phase, arrival times seeded {seed + 105} and {seed + 108}",
            "server": {"max_active": max_active, "chunk": chunk, "hbm_budget_gib": budget_gib}}


def time_mode(ctx, fn, seed, nt, reps, d_fid, d_st, stream):
    import torch
    fn(seed, 0, nt, d_fid, d_st, stream=stream)  # warm-up (buffers, code)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn(seed, 0, nt, d_fid, d_st, stream=stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def stats_of(P, d_st):
    return np.frombuffer(d_st.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)


def config2_leg(P, reps):
    """Qubit n = 6, k = 1 at gamma in {1e-4, 1e-3, 1e-2}, 1e4 trajectories:
    pruned, the kernel's full mode and the plain full evolution."""
    import torch
    from paper_2609_34935_amd.inputs import memory_words
    n, k, nt, seed = 6, 1, 10000, 880002
    mem = memory_words(n, k, 1002)
    stream = torch.cuda.current_stream()
    d_fid = torch.empty(nt, dtype=torch.float64, device="cuda")
    d_st = torch.empty(nt * 32, dtype=torch.uint8, device="cuda")
    out = {}
    for gamma in (1e-4, 1e-3, 1e-2):
        with P.QramContext(n, k, P.QRAM_QUBIT, gamma, mem) as ctx:
            row, fids = {}, {}
            ctx.autotune(P.QRAM_MODE_PLAIN, seed + 1, 0, nt)  # (plain engine: shape by the autotuner)
            row["plain_launch"] = list(ctx.get_launch(P.QRAM_MODE_PLAIN))
            for name, fn in (("pruned", ctx.run_pruned_async), ("full_engine", ctx.run_full_async),
                             ("plain", ctx.run_plain_async)):
                dt = time_mode(ctx, fn, seed, nt, reps, d_fid, d_st, stream)
                row[name] = round(nt / dt, 1)
                fids[name] = d_fid.cpu().numpy()
                if name == "pruned":
                    s = stats_of(P, d_st)
                    row["evolved_fraction"] = round(float(s["n_explicit"].mean()) / 2 ** (n + k), 4)
                    row["mean_bad"] = round(float(s["n_bad"].mean()), 3)
            ctx.errors()
        for name in ("full_engine", "plain"):
            assert np.all(np.abs(fids[name] - fids["pruned"]) <= 1e-12 * np.maximum(np.abs(fids["pruned"]), 1e-3))
        row["speedup_pruned_over_plain"] = round(row["pruned"] / row["plain"], 3)
        row["ideal_speedup"] = round(1.0 / row["evolved_fraction"], 3)
        out[f"gamma={gamma:g}"] = row
        log(f"C2 gamma={gamma:g}: {row}")
    return {"workload": "qubit n=6 k=1, 1e4 trajectories per gamma, seed 880002, mem_seed 1002",
            "unit": "trajectories/s", **out}


def config5_leg(P, nt, nt_plain):
    """Qutrit n = 14, k = 1, gamma = 1e-2: every branch is bad, so pruned
    evolves what full does; traj/s and device footprint of each mode."""
    import torch
    from paper_2609_34935_amd.inputs import memory_words
    n, k, gamma, seed = 14, 1, 1e-2, 880005
    mem = memory_words(n, k, 1005)
    stream = torch.cuda.current_stream()
    out = {"workload": f"qutrit n=14 k=1 gamma=1e-2, seed {seed}, mem_seed 1005", "unit": "trajectories/s"}
    with P.QramContext(n, k, P.QRAM_QUTRIT, gamma, mem) as ctx:
        ctx.autotune(P.QRAM_MODE_PLAIN, seed + 1, 0, min(nt_plain, 8192))  # (plain engine: shape by the autotuner)
        out["plain_launch"] = list(ctx.get_launch(P.QRAM_MODE_PLAIN))
        for name, mode, fn, cnt in (("pruned", P.QRAM_MODE_PRUNED, ctx.run_pruned_async, nt),
                                    ("full_engine", P.QRAM_MODE_FULL, ctx.run_full_async, nt),
                                    ("plain", P.QRAM_MODE_PLAIN, ctx.run_plain_async, nt_plain)):
            d_fid = torch.empty(cnt, dtype=torch.float64, device="cuda")
            d_st = torch.empty(cnt * 32, dtype=torch.uint8, device="cuda")
            dt = time_mode(ctx, fn, seed, cnt, 1, d_fid, d_st, stream)
            f1, f_all = ctx.footprint(mode, 1), ctx.footprint(mode, cnt)
            out[name] = {"traj_per_s": round(cnt / dt, 1), "trajectories": cnt,
                         "footprint_one_in_flight_bytes": int(f1), "footprint_bytes": int(f_all)}
            if name == "pruned":
                s = stats_of(P, d_st)
                out["mean_candidates"] = round(float(s["n_cand"].mean()), 1)
                out["evolved_fraction"] = round(float(s["n_explicit"].mean()) / 2 ** n, 4)
            log(f"C5 {name}: {out[name]}")
            del d_fid, d_st
        ctx.errors()
    out["footprint_note"] = ("footprint_one_in_flight_bytes: device bytes held for runs of one trajectory "
                             "(context tables plus one workgroup's work state); footprint_bytes: for the whole "
                             "run as batched")
    return out


# The paper's full-versus-pruned benchmark (App. D, Table 5): per-query
# milliseconds (t_full, t_pruned) on one CPU thread, qubit encoding, k = 3,
# eps = gamma, data-loading input.  Context for the GPU figures beside them.
PAPER_TABLE5 = {
    (0.0, 4): (0.5731, 0.0307), (0.0, 6): (4.043, 0.0859), (0.0, 8): (21.56, 0.2424),
    (0.0, 10): (124.8, 0.7592), (0.0, 12): (725.1, 2.548),
    (1e-5, 4): (0.7496, 0.0497), (1e-5, 6): (4.815, 0.2348), (1e-5, 8): (29.12, 1.417),
    (1e-5, 10): (173.9, 11.29), (1e-5, 12): (1258.0, 125.4),
    (1e-4, 4): (0.7586, 0.0964), (1e-4, 6): (4.885, 0.8590), (1e-4, 8): (31.26, 8.250),
    (1e-4, 10): (243.0, 95.92), (1e-4, 12): (2750.0, 1655.0),
    (1e-3, 4): (0.7895, 0.3668), (1e-3, 6): (6.251, 4.491), (1e-3, 8): (55.15, 51.81),
    (1e-3, 10): (800.1, 794.1), (1e-3, 12): (11814.0, 11816.0),
}


def table5_leg(P, scale=1.0, points=None):
    """The paper's full-versus-pruned workload (Fig. 3, App. D): qubit, k = 3,
    eps = gamma in {0, 1e-5, 1e-4, 1e-3}, n = 4..12, data-loading input.
    Pruned (Alg. 1) against the plain full evolution of every branch, on the
    GPU, with equal fidelities checked on every trajectory."""
    import torch
    from paper_2609_34935_amd.inputs import memory_words
    k, seed = 3, 880007
    stream = torch.cuda.current_stream()
    rows = []
    for p in (0.0, 1e-5, 1e-4, 1e-3):
        for n in (4, 6, 8, 10, 12):
            if points is not None and (p, n) not in points:
                continue
            # enough trajectories per workgroup that the slowest trajectories
            # do not set the launch time (the paper's figure is a mean)
            nt = {4: 65536, 6: 32768, 8: 16384, 10: 8192, 12: 4096}[n]
            if p >= 1e-3 and n >= 10:
                nt //= 4
            nt = int(max(64, nt * scale))
            mem = memory_words(n, k, 1007 + n)
            d_fid = torch.empty(nt, dtype=torch.float64, device="cuda")
            d_st = torch.empty(nt * 32, dtype=torch.uint8, device="cuda")
            with P.QramContext(n, k, P.QRAM_QUBIT, p, mem, eps=p) as ctx:
                row = {"eps=gamma": p, "n": n, "trajectories": nt}
                fids = {}
                for name, fn in (("pruned", ctx.run_pruned_async), ("full", ctx.run_plain_async)):
                    # plain-engine launch shape: the autotuner's pick where a
                    # trajectory holds at most 4096 components, else the
                    # library's automatic one (recorded after the runs: a
                    # split run's choice depends on the batch)
                    mode = P.QRAM_MODE_PRUNED if name == "pruned" else P.QRAM_MODE_PLAIN
                    if (p > 0 or name == "full") and 2 ** (n + k) <= 4096:
                        ctx.autotune(mode, seed + 1, 0, min(nt, 8192))
                    reps = 3 if name == "pruned" else 1
                    dt = time_mode(ctx, fn, seed, nt, reps, d_fid, d_st, stream)
                    if p > 0 or name == "full":
                        row.setdefault("launch", {})[name] = list(ctx.get_launch(mode))
                    row[f"{name}_traj_per_s"] = round(nt / dt, 1)
                    fids[name] = d_fid.cpu().numpy()
                    if name == "pruned":
                        s = stats_of(P, d_st)
                        row["evolved_pct"] = round(100.0 * float(s["n_explicit"].mean()) / 2 ** (n + k), 2)
                ctx.errors()
            assert np.all(np.abs(fids["full"] - fids["pruned"]) <= 1e-12 * np.maximum(np.abs(fids["pruned"]), 1e-3))
            row["speedup"] = round(row["pruned_traj_per_s"] / row["full_traj_per_s"], 2)
            tf, tp = PAPER_TABLE5[(p, n)]
            row["paper_cpu_1thread"] = {"full_traj_per_s": round(1000.0 / tf, 3),
                                        "pruned_traj_per_s": round(1000.0 / tp, 3), "speedup": round(tf / tp, 2)}
            rows.append(row)
            log(f"Table 5 workload eps=gamma={p:g} n={n}: {row}")
            del d_fid, d_st
    return {"workload": "qubit k=3, eps=gamma, data-loading input (Fig. 3 / Table 5), seed 880007, "
                        "mem_seed 1007+n", "unit": "trajectories/s", "rows": rows,
            "paper": "Table 5: one thread of an i9-13900KF, FP64 (context, not a target)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ntraj", type=int, default=100000)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--cpu-qubit", type=int, default=768)
    ap.add_argument("--cpu-qutrit", type=int, default=6144)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--launch-cache", default=os.path.join(ROOT, "paper_2609_34935_amd", "tuned",
                                                        "launch_n10k4_gamma1e-3.json"),
                    help="JSON file of launch shapes chosen by the autotuner: read if present")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner on the whole step and write its picks to --launch-cache")
    ap.add_argument("--modes", default="pruned,full,plain")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-subtree", action="store_true",
                    help="skip the qubit step under the damping-only subtree marking")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--c5-ntraj", type=int, default=100000)
    ap.add_argument("--c5-plain-ntraj", type=int, default=20000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-table5", action="store_true")
    ap.add_argument("--table5-scale", type=float, default=1.0)
    ap.add_argument("--table5-points", default=None,
                    help="only these points of the Table 5 workload, as eps:n,eps:n (e.g. 1e-5:8)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-capacity-requests", type=int, default=400)
    ap.add_argument("--serve-chunk", type=int, default=16384)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=96.0)
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
    modes_req = args.modes.split(",")
    ctxs = {enc: P.QramContext(N, K, enc, GAMMA, mem) for enc in (P.QRAM_QUBIT, P.QRAM_QUTRIT)}
    all_modes = (P.QRAM_MODE_PRUNED, P.QRAM_MODE_FULL, P.QRAM_MODE_PLAIN)

    # launch shapes: the autotuner's picks on the whole step (cached)
    tuned, tune_ms = {}, {}
    cache = None
    if args.launch_cache and os.path.exists(args.launch_cache) and not args.retune:
        cache = json.load(open(args.launch_cache))
    for enc, ctx in ctxs.items():
        for mode in all_modes:
            key = f"{enc}:{mode}"
            if cache and key in cache:
                ctx.set_launch(mode, *cache[key])
            else:
                tune_ms[key] = round(ctx.autotune(mode, seed, 0, nt), 3)
                log(f"autotune enc={enc} mode={mode}: {ctx.get_launch(mode)} {tune_ms[key]:.3f} ms")
            tuned[(enc, mode)] = ctx.get_launch(mode)
    if args.launch_cache and cache is None:
        json.dump({f"{e}:{m}": list(v) for (e, m), v in tuned.items()}, open(args.launch_cache, "w"))

    stream = torch.cuda.current_stream()
    d_fid = {enc: torch.empty(nt, dtype=torch.float64, device="cuda") for enc in ctxs}
    d_st = {enc: torch.empty(nt * 32, dtype=torch.uint8, device="cuda") for enc in ctxs}

    def step(mode):
        for enc, ctx in ctxs.items():
            fn = {P.QRAM_MODE_PRUNED: ctx.run_pruned_async, P.QRAM_MODE_FULL: ctx.run_full_async,
                  P.QRAM_MODE_PLAIN: ctx.run_plain_async}[mode]
            fn(seed, 0, nt, d_fid[enc], d_st[enc], stream=stream)

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            step(mode)
        torch.cuda.synchronize()
        for ctx in ctxs.values():
            ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stage, buckets = {}, {}
        for enc, ctx in ctxs.items():
            launches = ctx.stage_launches()
            buckets[enc] = ctx.stage_buckets()
            stage[enc] = ctx.stage_times() + (launches,)
            ctx.set_timing(False)
            ctx.errors()
        st = {enc: stats_of(P, d_st[enc]) for enc in ctxs}
        fids = {enc: d_fid[enc].cpu().numpy() for enc in ctxs}
        log(f"mode={mode}: {steps} steps in {dt:.3f} s")
        return dict(dt=dt, steps=steps, stage=stage, buckets=buckets, st=st, fid=fids)

    pr = timed(P.QRAM_MODE_PRUNED, args.steps, args.warmup)
    fe = timed(P.QRAM_MODE_FULL, args.steps, args.warmup) if "full" in modes_req else None
    pl = timed(P.QRAM_MODE_PLAIN, args.plain_steps, 1) if "plain" in modes_req else None
    total = 2 * nt
    value = total * pr["steps"] / pr["dt"]
    full_engine_value = total * fe["steps"] / fe["dt"] if fe else None
    full_value = total * pl["steps"] / pl["dt"] if pl else None
    for other in (fe, pl):  # every mode agrees with the pruned one trajectory by trajectory
        if other:
            for enc in ctxs:
                a, b = pr["fid"][enc], other["fid"][enc]
                assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(np.abs(a), 1e-3)), "modes disagree"

    graph_value = None
    if not args.no_graph:
        for ctx in ctxs.values():
            ctx.set_option(P.qram.QRAM_OPT_GRAPH, 1)
        step(P.QRAM_MODE_PRUNED)  # capture and instantiate once; the timed steps replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(P.QRAM_MODE_PRUNED)
        torch.cuda.synchronize()
        graph_value = total * args.steps / (time.perf_counter() - t0)
        for enc, ctx in ctxs.items():
            ctx.set_option(P.qram.QRAM_OPT_GRAPH, 0)
            assert np.array_equal(d_fid[enc].cpu().numpy(), pr["fid"][enc]), "graph replay differs"
        log(f"graph replay: {graph_value:.1f} trajectories/s")

    # the damping-only subtree marking of the qubit encoding (exact for
    # damping, fewer explicit addresses): the same step and trajectories
    subtree = None
    if not args.no_subtree:
        qctx = ctxs[P.QRAM_QUBIT]
        qctx.set_option(P.qram.QRAM_OPT_SUBTREE_MARKING, 1)
        step(P.QRAM_MODE_PRUNED)
        torch.cuda.synchronize()
        qctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(P.QRAM_MODE_PRUNED)
        torch.cuda.synchronize()
        dt_sub = time.perf_counter() - t0
        ms_s, nbs = qctx.stage_times()
        qctx.set_timing(False)
        qctx.set_option(P.qram.QRAM_OPT_SUBTREE_MARKING, 0)
        qctx.errors()
        fs = d_fid[P.QRAM_QUBIT].cpu().numpy()
        ss = stats_of(P, d_st[P.QRAM_QUBIT])
        ref_f = pr["fid"][P.QRAM_QUBIT]
        assert np.all(np.abs(fs - ref_f) <= 1e-12 * np.maximum(np.abs(ref_f), 1e-3)), \
            "subtree marking changed a fidelity"
        sub_value = total * args.steps / dt_sub
        subtree = {
            "value": round(sub_value, 1),
            "speedup_over_plain_full": None if full_value is None else round(sub_value / full_value, 3),
            "qubit_pruned_evolve_ms": round(ms_s[2] / max(nbs, 1), 3),
            "qubit_evolved_fraction": round(float(ss["n_explicit"].mean()) / 2 ** (N + K), 4),
            "qubit_mean_bad": round(float(ss["n_bad"].mean()), 2),
            "rule": "qubit damping candidates mark their own subtree (Eq. subtree) instead of "
                    "Eq. badrange; qutrit unchanged; fidelities equal the uniform rule's",
        }
        log(f"subtree marking: {sub_value:.1f} trajectories/s")

    # roofline of the dominant kernel: the largest bucket launch of the
    # qubit evolution kernel in the pruned step
    bk = pr["buckets"][P.QRAM_QUBIT]
    dom = max(range(len(bk)), key=lambda i: bk[i]["ms"])
    launch_ms = bk[dom]["ms"] / max(bk[dom]["launches"], 1)
    sq = pr["st"][P.QRAM_QUBIT]
    lo = bk[dom - 1]["emax"] if dom > 0 else 0
    sel = (sq["n_explicit"] > lo) & (sq["n_explicit"] <= bk[dom]["emax"])
    assert int(sel.sum()) == bk[dom]["ntraj_last"], "bucket membership"
    # compulsory bytes of the stage per trajectory: its candidate list in
    # (4 B each), its explicit-address list in (2 B each), fidelity and
    # statistics out (8 + 32 B)
    traj_bytes = 4.0 * sq["n_cand"][sel] + 2.0 * (sq["n_explicit"][sel] >> K) + 40.0
    bytes_launch = float(traj_bytes.sum())
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    sweep_units = float(sq["n_explicit"][sel].astype(np.float64).sum()) * (T - 1)
    sweep_rate = sweep_units * ops_per_component_slice(N, K) / (launch_ms * 1e-3) / 1e12
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": traffic_from_profile("evolve_qubit"),
        "kernel": f"k_evolve<qubit> bucket {dom} (up to {bk[dom]['emax']} components; pruned step)",
        "launch_ms": round(launch_ms, 3), "launches_timed": bk[dom]["launches"],
        "units_per_launch": int(sel.sum()), "unit_of_work": "trajectory",
        "bytes_per_unit": round(bytes_launch / max(int(sel.sum()), 1), 2),
        "bytes_rule": "4 B per candidate in + 2 B per explicit address in + 40 B out (fid, stats)",
        "other_launches": [{"bucket": i, "ms": round(b["ms"] / max(b["launches"], 1), 3),
                            "trajectories": b["ntraj_last"]} for i, b in enumerate(bk) if i != dom],
        "explicit_sweep_equivalent": {
            "unit": "component-slice", "ops_per_unit": ops_per_component_slice(N, K),
            "units_per_launch": sweep_units, "rate_tops": round(sweep_rate, 3),
            "of_alu_peak": round(sweep_rate / PEAK_ALU_TOPS, 3)},
    }

    # the plain comparator's own roofline (the explicit sweep itself)
    roofline_plain = None
    if pl:
        ms_q = pl["stage"][P.QRAM_QUBIT][0][2] / max(pl["stage"][P.QRAM_QUBIT][1], 1)
        E = 2 ** (N + K)
        units = float(nt) * E * (T - 1)
        rate_alu = units * ops_per_component_slice(N, K) / (ms_q * 1e-3) / 1e12
        b_sweep = units * 2 * bytes_per_component(N, K)
        rate_sweep = b_sweep / (ms_q * 1e-3) / 1e9
        # The kernel moves only the record pieces in use and touches an
        # amplitude only where it is needed, so the sweep's byte count is no
        # lower bound for it: its rate is the counted HBM bytes (null when
        # the counters are of other kernel sources) over the launch time.
        traffic = traffic_from_profile("plain_qubit")
        rate_hbm = traffic / (ms_q * 1e-3) / 1e9 if traffic else None
        roofline_plain = {
            "bound": "hbm", "achieved": round(rate_hbm, 2) if rate_hbm else None, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(rate_hbm / PEAK_HBM_GBS, 4) if rate_hbm else None, "traffic": traffic,
            "kernel": "k_plain<qubit> (plain full evolution)", "launch_ms": round(ms_q, 3),
            "units_per_launch": units, "unit_of_work": "component-slice",
            "bytes_per_unit": round(traffic / units, 2) if traffic else None,
            "bytes_rule": "HBM bytes per launch as counted (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "sweep_equivalent": {"bytes_per_unit": 2 * bytes_per_component(N, K),
                                 "rule": "amplitude and longest site list read and written every slice",
                                 "rate_gbs": round(rate_sweep, 2), "of_hbm_peak": round(rate_sweep / PEAK_HBM_GBS, 4)},
            "alu": {"ops_per_unit": ops_per_component_slice(N, K), "rate_tops": round(rate_alu, 3),
                    "peak": round(PEAK_ALU_TOPS, 3), "frac": round(rate_alu / PEAK_ALU_TOPS, 4)}}

    per_enc = {}
    for enc, name in ((P.QRAM_QUBIT, "qubit"), (P.QRAM_QUTRIT, "qutrit")):
        s = pr["st"][enc]
        ms_p, nbp, _ = pr["stage"][enc]
        row = {
            "pruned_evolve_ms": round(ms_p[2] / max(nbp, 1), 3),
            "sample_classify_ms": round((ms_p[0] + ms_p[1]) / max(nbp, 1), 3),
            "pruned_buckets": [{"ms": round(b["ms"] / max(b["launches"], 1), 3), "trajectories": b["ntraj_last"],
                                "emax": b["emax"]} for b in pr["buckets"][enc]],
            "evolved_fraction": round(float(s["n_explicit"].mean()) / (2**N * (2**K if enc == P.QRAM_QUBIT else 1)), 4),
            "mean_fidelity": round(float(pr["fid"][enc].mean()), 6),
            "mean_jumps": round(float(s["n_jumps"].mean()), 4),
            "launch": {m: tuned[(enc, mode)] for m, mode in (("pruned", P.QRAM_MODE_PRUNED),
                                                              ("full_engine", P.QRAM_MODE_FULL),
                                                              ("plain", P.QRAM_MODE_PLAIN))},
        }
        for key, res in (("full_engine", fe), ("plain", pl)):
            if res:
                ms_x, nbx, _ = res["stage"][enc]
                row[f"{key}_evolve_ms"] = round(ms_x[2] / max(nbx, 1), 3)
                row[f"{key}_traj_per_s"] = round(nt * res["steps"] / (ms_x.sum() * 1e-3), 1)
        row["pruned_traj_per_s"] = round(nt / (ms_p.sum() / max(nbp, 1) * 1e-3), 1)
        per_enc[name] = row

    line = {
        "metric": "trajectories/sec pruned vs full at n=10, gamma=1e-3 (1 GPU); p50/p99 req latency",
        "value": round(value, 1),
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(pr["dt"] / pr["steps"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bucket-brigade QRAM query n=10 k=4 gamma=1e-3, qubit and qutrit "
                               "encodings, 1e5 trajectories each, pruned evolution",
                   "n": N, "k": K, "gamma": GAMMA, "trajectories_per_step": total,
                   "memory": "seeded Bernoulli(0.5), mem_seed 1003", "seed": seed},
        "full_value": None if full_value is None else round(full_value, 1),
        "full_kind": "plain full evolution: every component of every branch explicit, slice by slice",
        "speedup_pruned_over_full": None if full_value is None else round(value / full_value, 3),
        "full_engine_value": None if full_engine_value is None else round(full_engine_value, 1),
        "speedup_pruned_over_full_engine": None if full_engine_value is None else round(value / full_engine_value, 4),
        "graph_value": None if graph_value is None else round(graph_value, 1),
        "subtree_marking": subtree,
        "per_encoding": per_enc,
        "launch_shapes": {"source": "autotuner on the whole step" if tune_ms else
                          f"cache {os.path.relpath(args.launch_cache, ROOT)} (written by bench.py --retune)",
                          "tune_ms": tune_ms or None},
        "roofline": roofline,
        "roofline_plain": roofline_plain,
        "config2": None, "config5": None, "table5": None,
        "latency": None,
        "cpu_baseline": None,
    }
    for ctx in ctxs.values():
        ctx.close()
    del d_fid, d_st
    torch.cuda.empty_cache()
    if not args.no_c2:
        line["config2"] = config2_leg(P, reps=5)
    if not args.no_c5:
        line["config5"] = config5_leg(P, args.c5_ntraj, args.c5_plain_ntraj)
    if not args.no_table5:
        pts = None
        if args.table5_points:
            pts = {(float(e), int(n)) for e, n in (x.split(":") for x in args.table5_points.split(","))}
        line["table5"] = table5_leg(P, args.table5_scale, pts)
    torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving mix")
        line["latency"] = serving_leg(P, args.serve_requests, args.serve_capacity_requests, 4242,
                                      args.serve_chunk, args.serve_slots, args.serve_budget_gib)
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(mem, args.cpu_qubit, args.cpu_qutrit)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
