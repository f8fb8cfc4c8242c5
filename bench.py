"""Throughput benchmark: trajectories/s of pruned vs full evolution of
amplitude-damped bucket-brigade QRAM queries on one MI355X, plus the serving
mix's p50/p99 request latency.

Workload of one step: the n = 10, k = 4, gamma = 1e-3 data-loading query in
both encodings, 1e5 trajectories each (seeded synthetic memory and noise),
pruned evolution, inputs and outputs resident on the device.  The full mode is
timed the same way as the comparator, the same pruned step once more as one
HIP graph per batch, and the serving mix (Poisson arrivals, mixed n, k,
encoding, gamma and shots) through the request server.  Prints one JSON line.
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
KERNEL_SRCS = [os.path.join(ROOT, "paper_2609_34935_amd", "csrc", f)
               for f in ("qram_evolve.hip", "qram_device.h", "qram_internal.h")]


def kernel_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


# Algorithmic unit of the dominant kernel: one mask test of the joint damping
# layer (Eq. maskweight), i.e. one (candidate, explicit component) pair: the
# candidate's site and level compared with the component's excited set, and
# the outcome merged into the component's mask (2 integer operations).
OPS_PER_MASK_TEST = 2


def ops_per_component_slice(n, k):
    """Work of one explicit component through one slice when every component
    is carried explicitly slice by slice: about 6 FP64 operations (K0
    weight, |A|^2, accumulation) and 2n + 3k integer operations (site moves
    and mask merge).  Reported for comparison only."""
    return 6 + 2 * n + 3 * k


def traffic_from_profile():
    """HBM bytes per launch of the qubit evolution kernel from the committed
    rocprofv3 counter summary, or None if the kernel changed since."""
    try:
        prof = json.load(open(COUNTER_FILE))
    except (OSError, ValueError):
        return None
    if prof.get("kernel_sha256") != kernel_sha256():
        return None
    return prof.get("hbm_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(mem, n_qubit, n_qutrit):
    """The oracle (full evolution of every branch, plain C, OpenMP over
    trajectories) on the first trajectories of each encoding."""
    from oracle import oracle as O
    threads = min(16, os.cpu_count() or 1)
    per = {}
    used = threads
    for enc, cnt in ((1, n_qubit), (0, n_qutrit)):
        t0 = time.perf_counter()
        _, _, _, used = O.run_batch(N, K, enc, GAMMA, mem, 880000 + CFG_ID, 0, cnt, nthreads=threads)
        per[enc] = (time.perf_counter() - t0, cnt)
    # one step holds as many qubit as qutrit trajectories
    t_pair = per[1][0] / per[1][1] + per[0][0] / per[0][1]
    # the same oracle on one thread (the paper's simulator is single-threaded)
    one = {}
    for enc, cnt in ((1, max(1, n_qubit // 16)), (0, max(1, n_qutrit // 16))):
        t0 = time.perf_counter()
        O.run_batch(N, K, enc, GAMMA, mem, 880000 + CFG_ID, 0, cnt, nthreads=1)
        one[enc] = (time.perf_counter() - t0, cnt)
    t_one = one[1][0] / one[1][1] + one[0][0] / one[0][1]
    return {"value": round(2.0 / t_pair, 2), "unit": "trajectories/s", "cores": used, "kind": "oracle",
            "sample": f"first {per[1][1]} qubit and {per[0][1]} qutrit trajectories of the step's workload "
                      f"({per[1][0]:.1f} s and {per[0][0]:.1f} s wall on {used} threads), full evolution of "
                      "every branch on the host; value = 2 / (mean qubit + mean qutrit time per trajectory)",
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
            if (i + 1) % 64 == 0:
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


def serving_leg(P, nreq, seed, chunk, max_active, budget_gib):
    """The serving mix through the request server.  The capacity mu (requests
    per second) is measured with every request submitted at once; then the
    mix arrives as a Poisson stream at 0.5 mu and 0.8 mu.  Latency is
    submission to results on the host, measured by the server."""
    from paper_2609_34935_amd.inputs import memory_words, request_mix
    out = {}
    reqs = request_mix(nreq, seed)
    mems = [memory_words(r["n"], r["k"], r["mem_seed"]) for r in reqs]
    sat = _serve_once(P, reqs, mems, np.zeros(nreq), chunk, max_active, budget_gib, "saturated")
    mu = nreq / sat["wall_s"]
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
                   f"{seed}; the same requests in every phase, arrival times seeded {seed + 105} and {seed + 108}",
            "server": {"max_active": max_active, "chunk": chunk, "hbm_budget_gib": budget_gib}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ntraj", type=int, default=100000)
    ap.add_argument("--cpu-qubit", type=int, default=768)
    ap.add_argument("--cpu-qutrit", type=int, default=6144)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--launch-cache", default=os.path.join(ROOT, "paper_2609_34935_amd", "tuned",
                                                        "launch_n10k4_gamma1e-3.json"),
                    help="JSON file of tuned launch shapes: read if present, else written "
                         "(default: the shapes shipped for this workload)")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner instead of reading the launch cache")
    ap.add_argument("--modes", default="pruned,full")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-subtree", action="store_true",
                    help="skip the qubit step under the damping-only subtree marking")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
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
    ctxs = {enc: P.QramContext(N, K, enc, GAMMA, mem) for enc in (P.QRAM_QUBIT, P.QRAM_QUTRIT)}
    tuned = {}
    cache = None
    if args.launch_cache and os.path.exists(args.launch_cache) and not args.retune:
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
    if args.launch_cache and cache is None and not os.path.exists(args.launch_cache):
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
            launches = ctx.stage_launches()
            stage[enc] = ctx.stage_times() + (launches,)
            ctx.set_timing(False)
            ctx.errors()
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

    graph_value = None
    if not args.no_graph:
        for ctx in ctxs.values():
            ctx.set_option(P.qram.QRAM_OPT_GRAPH, 1)
        step(P.QRAM_MODE_PRUNED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(P.QRAM_MODE_PRUNED)
        torch.cuda.synchronize()
        graph_value = total / (time.perf_counter() - t0)
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
        ss = np.frombuffer(d_st[P.QRAM_QUBIT].cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
        ref_f = pr["fid"][P.QRAM_QUBIT]
        assert np.all(np.abs(fs - ref_f) <= 1e-12 * np.maximum(np.abs(ref_f), 1e-3)), \
            "subtree marking changed a fidelity"
        sub_value = total / dt_sub
        subtree = {
            "value": round(sub_value, 1),
            "speedup_over_full": None if full_value is None else round(sub_value / full_value, 4),
            "qubit_pruned_evolve_ms": round(ms_s[2] / max(nbs, 1), 3),
            "qubit_evolved_fraction": round(float(ss["n_explicit"].mean()) / 2 ** (N + K), 4),
            "qubit_mean_bad": round(float(ss["n_bad"].mean()), 2),
            "rule": "qubit damping candidates mark their own subtree (Eq. subtree) instead of "
                    "Eq. badrange; qutrit unchanged; fidelities equal the uniform rule's",
        }
        log(f"subtree marking: {sub_value:.1f} trajectories/s")

    # roofline of the dominant kernel: the qubit evolution launches
    ms_stage, nb, nlaunch = pr["stage"][P.QRAM_QUBIT]
    evolve_ms_step = ms_stage[2] / max(nb, 1)
    launch_ms = ms_stage[2] / max(nlaunch, 1)
    sq = pr["st"][P.QRAM_QUBIT]
    units_step = float((sq["n_cand"].astype(np.float64) * sq["n_explicit"].astype(np.float64)).sum())
    achieved = units_step * OPS_PER_MASK_TEST / (evolve_ms_step * 1e-3) / 1e12
    sweep_units = float(sq["n_explicit"].astype(np.float64).sum()) * (T - 1)
    sweep_rate = sweep_units * ops_per_component_slice(N, K) / (evolve_ms_step * 1e-3) / 1e12
    per_enc = {}
    for enc, name in ((P.QRAM_QUBIT, "qubit"), (P.QRAM_QUTRIT, "qutrit")):
        s = pr["st"][enc]
        ms_p, nbp, _ = pr["stage"][enc]
        ms_f, nbf, _ = fu["stage"][enc] if fu else (np.full(3, np.nan), 1, 0)
        per_enc[name] = {
            "pruned_evolve_ms": round(ms_p[2] / max(nbp, 1), 3),
            "full_evolve_ms": None if not fu else round(ms_f[2] / max(nbf, 1), 3),
            "sample_classify_ms": round((ms_p[0] + ms_p[1]) / max(nbp, 1), 3),
            "pruned_traj_per_s_kernels": round(nt / (ms_p.sum() / max(nbp, 1) * 1e-3), 1),
            "full_traj_per_s_kernels": None if not fu else round(nt / (ms_f.sum() / max(nbf, 1) * 1e-3), 1),
            "evolved_fraction": round(float(s["n_explicit"].mean()) / (2**N * (2**K if enc == P.QRAM_QUBIT else 1)), 4),
            "mean_fidelity": round(float(pr["fid"][enc].mean()), 6),
            "mean_jumps": round(float(s["n_jumps"].mean()), 4),
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
        "graph_value": None if graph_value is None else round(graph_value, 1),
        "subtree_marking": subtree,
        "per_encoding": per_enc,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TOPS, 3),
                     "unit": "TOP/s", "frac": round(achieved / PEAK_ALU_TOPS, 4),
                     "traffic": traffic_from_profile(),
                     "kernel": "k_evolve<qubit> (pruned step)", "launch_ms": round(launch_ms, 3),
                     "launches_per_step": round(nlaunch / max(nb, 1), 2),
                     "work_unit": "mask test (candidate x explicit component)",
                     "units_per_launch": units_step / max(nlaunch / max(nb, 1), 1),
                     "ops_per_unit": OPS_PER_MASK_TEST,
                     "explicit_sweep_equivalent": {
                         "unit": "explicit component-slice", "ops_per_unit": ops_per_component_slice(N, K),
                         "rate_tops": round(sweep_rate, 3)}},
        "latency": None,
        "cpu_baseline": None,
    }
    for ctx in ctxs.values():
        ctx.close()
    del d_fid, d_st
    torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving mix")
        line["latency"] = serving_leg(P, args.serve_requests, 4242, args.serve_chunk,
                                      args.serve_slots, args.serve_budget_gib)
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(mem, args.cpu_qubit, args.cpu_qutrit)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
