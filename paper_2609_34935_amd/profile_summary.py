"""Short text summaries of rocprofv3 CSV output (kernel trace, counters).

    python -m paper_2609_34935_amd.profile_summary trace KERNEL_TRACE.csv OUT.txt --command "..."
    python -m paper_2609_34935_amd.profile_summary counters --fetch F.csv --write W.csv [--sq S.csv] \\
        --kernel 'k_evolve<1,' [--wg 512] [--src FILE ...] OUT.json --command "..." [--command "..."]
    python -m paper_2609_34935_amd.profile_summary states S.csv --kernel 'k_evolve<1,' OUT.txt --command "..."
    python -m paper_2609_34935_amd.profile_summary pmc A.csv [B.csv ...] --kernel KERNEL [--wg 512] --out OUT.txt --command "..."

The counter summary scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by
what the same counters read for the largest plain device copy of the run
(a 256 MiB copy: 268435456 bytes read and written) and reports HBM bytes per
launch of the named kernel (only the dispatches of workgroup size --wg when
given: one work bucket's launches).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import OrderedDict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRCS = [os.path.join(HERE, "csrc", f)
               for f in ("qram_evolve.hip", "qram_device.h", "qram_internal.h", "qram_records.h")]
COPY_BYTES = 268435456


def kernel_sha256(srcs=None):
    h = hashlib.sha256()
    for f in srcs or KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def short_name(name):
    for cut in ("(qr::", "(unsigned", "(void"):
        i = name.find(cut)
        if i > 0:
            name = name[:i]
    return name.replace("void ", "").replace("qr::(anonymous namespace)::", "").replace("qr::", "").strip()


def trace_summary(path, out, commands):
    rows = list(csv.DictReader(open(path)))
    agg = OrderedDict()
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        name = short_name(r["Kernel_Name"])
        key = (name, r.get("Workgroup_Size_X", r.get("Workgroup_Size", "")))
        a = agg.setdefault(key, [0, 0.0, 1e30, 0.0])
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
    total = sum(v[1] for v in agg.values())
    lines = ["rocprofv3 kernel trace summary", ""]
    lines += [f"command: {c}" for c in commands]
    lines += ["", f"{'kernel':<44} {'wg':>5} {'calls':>6} {'total ms':>10} {'avg ms':>9} {'min ms':>9} {'max ms':>9} {'%':>6}"]
    for (name, wg), (n, t, lo, hi) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{name[:44]:<44} {wg:>5} {n:>6} {t:>10.3f} {t / n:>9.3f} {lo:>9.3f} {hi:>9.3f} {100 * t / total:>6.2f}")
    byname = OrderedDict()
    for (name, _), (n, t, lo, hi) in agg.items():
        a = byname.setdefault(name, [0, 0.0])
        a[0] += n
        a[1] += t
    lines += ["", "all workgroup sizes together:", f"{'kernel':<44} {'calls':>6} {'total ms':>10} {'avg ms':>9}"]
    for name, (n, t) in sorted(byname.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{name[:44]:<44} {n:>6} {t:>10.3f} {t / n:>9.3f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_dispatch(path):
    d = OrderedDict()
    for r in csv.DictReader(open(path)):
        key = int(r["Dispatch_Id"])
        e = d.setdefault(key, {"name": r["Kernel_Name"], "grid": r.get("Grid_Size"), "wg": r.get("Workgroup_Size")})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return d


def _match(v, kernel, wg):
    return kernel in v["name"] and (wg is None or str(v.get("wg")) == str(wg))


def counter_summary(fetch, write, sq, kernel, out, commands, wg=None, srcs=None):
    srcs = [os.path.abspath(f) for f in srcs] if srcs else KERNEL_SRCS
    res = {"kernel": kernel, "workgroup": wg, "kernel_sha256": kernel_sha256(srcs), "commands": commands,
           "sources": [os.path.relpath(f, os.path.dirname(HERE)) for f in srcs]}
    for path, ctr, tag in ((fetch, "FETCH_SIZE", "fetch"), (write, "WRITE_SIZE", "write")):
        d = _per_dispatch(path)
        copies = [v[ctr] for v in d.values() if "copyBuffer" in v["name"] and ctr in v]
        if not copies:
            raise SystemExit(f"no calibration copy in {path}")
        cal_kib = max(copies)
        factor = COPY_BYTES / (cal_kib * 1024.0)
        ks = [v[ctr] for v in d.values() if _match(v, kernel, wg) and ctr in v]
        if not ks:
            raise SystemExit(f"no dispatch of {kernel} in {path}")
        res[f"copy_{tag}_kib"] = cal_kib
        res[f"copy_factor_{tag}"] = round(factor, 4)
        res[f"launches_{tag}"] = len(ks)
        res[f"{tag}_bytes_per_launch"] = round(sum(ks) * 1024.0 * factor / len(ks), 1)
    res["hbm_bytes_per_launch"] = round(res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"], 1)
    if sq:
        d = _per_dispatch(sq)
        ks = [v for v in d.values() if _match(v, kernel, wg)]
        for c in sorted({c for v in ks for c in v if c.startswith("SQ_")}):
            res[f"{c}_per_launch"] = round(sum(v.get(c, 0.0) for v in ks) / len(ks), 1)
    json.dump(res, open(out, "w"), indent=1)
    txt = os.path.splitext(out)[0] + ".txt"
    lines = ["rocprofv3 counter summary (per launch of the kernel below)", ""]
    lines += [f"command: {c}" for c in commands]
    lines += [""] + [f"{k}: {v}" for k, v in res.items() if k != "commands"]
    open(txt, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def state_summary(sq, kernel, out, commands):
    """Per-launch SQ counters of one run, and each as a fraction of the
    wave-cycles (SQ_WAVE_CYCLES), for the largest launch of the kernel."""
    d = _per_dispatch(sq)
    ks = [v for v in d.values() if kernel in v["name"] and "SQ_WAVE_CYCLES" in v]
    if not ks:
        raise SystemExit(f"no dispatch of {kernel} in {sq}")
    big = max(ks, key=lambda v: v["SQ_WAVE_CYCLES"])
    wc = big["SQ_WAVE_CYCLES"]
    lines = ["rocprofv3 wave-state counters (largest launch of the kernel below)", ""]
    lines += [f"command: {c}" for c in commands]
    lines += ["", f"kernel: {kernel}", f"kernel_sha256: {kernel_sha256()}", f"workgroup: {big['wg']}", ""]
    for c in sorted(k for k in big if k.startswith("SQ_")):
        lines.append(f"{c:<24} {big[c]:>16.4e}   {big[c] / wc:>7.3f} of SQ_WAVE_CYCLES")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def pmc_summary(paths, kernel, out, commands, wg=None, srcs=None):
    """Per-launch means of every counter in the given runs (each run one
    pass of counters) for the named kernel, with the L2 hit rate when both
    TCC_HIT and TCC_MISS were taken."""
    srcs = [os.path.abspath(f) for f in srcs] if srcs else None
    lines = ["rocprofv3 counters, mean per launch of the kernel below", ""]
    lines += [f"command: {c}" for c in commands]
    lines += ["", f"kernel: {kernel}", f"workgroup: {wg}", f"kernel_sha256: {kernel_sha256(srcs)}", ""]
    vals = OrderedDict()
    for path in paths:
        ks = [v for v in _per_dispatch(path).values() if _match(v, kernel, wg)]
        if not ks:
            raise SystemExit(f"no dispatch of {kernel} in {path}")
        for c in sorted({c for v in ks for c in v if c not in ("name", "grid", "wg")}):
            vals[c] = (sum(v.get(c, 0.0) for v in ks) / len(ks), len(ks))
    for c, (v, n) in vals.items():
        lines.append(f"{c:<24} {v:>16.4e}   ({n} launches)")
    hit = next((vals[c][0] for c in vals if c.startswith("TCC_HIT")), None)
    miss = next((vals[c][0] for c in vals if c.startswith("TCC_MISS")), None)
    if hit is not None and miss is not None and hit + miss > 0:
        lines.append(f"{'L2 hit rate':<24} {hit / (hit + miss):>16.4f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--command", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--sq", default=None)
    c.add_argument("--kernel", required=True)
    c.add_argument("--wg", default=None, help="only dispatches of this workgroup size")
    c.add_argument("--src", action="append", default=None, help="kernel source files (for the sha)")
    c.add_argument("out")
    c.add_argument("--command", action="append", default=[])
    w = sub.add_parser("states")
    w.add_argument("csv")
    w.add_argument("--kernel", required=True)
    w.add_argument("out")
    w.add_argument("--command", action="append", default=[])
    m = sub.add_parser("pmc")
    m.add_argument("csv", nargs="+")
    m.add_argument("--kernel", required=True)
    m.add_argument("--wg", default=None)
    m.add_argument("--src", action="append", default=None)
    m.add_argument("--out", required=True)
    m.add_argument("--command", action="append", default=[])
    a = ap.parse_args()
    if a.what == "trace":
        trace_summary(a.csv, a.out, a.command)
    elif a.what == "pmc":
        pmc_summary(a.csv, a.kernel, a.out, a.command, a.wg, a.src)
    elif a.what == "states":
        state_summary(a.csv, a.kernel, a.out, a.command)
    else:
        counter_summary(a.fetch, a.write, a.sq, a.kernel, a.out, a.command, a.wg, a.src)


if __name__ == "__main__":
    main()
