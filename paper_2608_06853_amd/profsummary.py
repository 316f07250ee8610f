"""Condense rocprofv3 CSV output into the short text summaries kept with the
library (per-kernel durations; HBM traffic per dispatch from FETCH_SIZE and
WRITE_SIZE scaled by a plain copy of known size).

    python -m paper_2608_06853_amd.profsummary stats --dir OUT --cmd "..." > FILE
    python -m paper_2608_06853_amd.profsummary traffic --fetch D1 --write D2 \
        --copy-fetch D3 --copy-write D4 --copy-bytes B --cmd "..." > FILE
    python -m paper_2608_06853_amd.profsummary counters --dir OUT --cmd "..." > FILE

The traffic summary records, per kernel family, the SHA-256 of the sources the
kernel is compiled from, so a reader can tell whether the counters still describe
the current kernel.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COMMON = ["af_device.h", "af_internal.h"]

# kernel family -> (symbol pattern, translation unit)
FAMILIES = {
    "table": (r"k_table[<(]", "k_table.hip"),
    "das_fwd": (r"k_das_fwd<", "k_das.hip"),
    "das_adj": (r"k_das_adj<", "k_das.hip"),
    "zero_tx": (r"k_zero_tx\(", "k_das.hip"),
    "das_rx": (r"k_das_rx<", "k_das.hip"),
    "loc": (r"k_loc\(", "k_das.hip"),
    "cmpe": (r"k_cmpe\(", "k_cmpe.hip"),
    "gscale": (r"k_gscale\(", "k_misc.hip"),
    "path_adj": (r"k_path_adj\(", "k_path.hip"),
    "path_chunk": (r"k_path_chunk\(", "k_path.hip"),
    "path_reduce": (r"k_path_reduce\(", "k_path.hip"),
    "prepare_grid": (r"k_prepare_grid\(", "k_misc.hip"),
    "finalize": (r"k_finalize\(", "k_misc.hip"),
    "grad_fold": (r"k_grad_fold\(", "k_misc.hip"),
    "sim_synth": (r"k_sim_synth\(", "k_sim.hip"),
    "sim_times": (r"k_sim_times\(", "k_sim.hip"),
    "conv_fwd": (r"k_conv_fwd\(", "k_cnn.hip"),
    "conv_bwd_data": (r"k_conv_bwd_data(_s2)?\(", "k_cnn.hip"),
    "conv_bwd_weight": (r"k_conv_bwd_weight\(", "k_cnn.hip"),
    "conv_wreduce": (r"k_conv_wreduce\(", "k_cnn.hip"),
    "conv_wsum": (r"k_conv_wsum\(", "k_cnn.hip"),
    "copy": (r"__amd_rocclr_copyBuffer", None),
}


def source_hash(family: str) -> str:
    tu = FAMILIES[family][1]
    if tu is None:
        return "-"
    h = hashlib.sha256()
    for f in [tu] + COMMON:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def family_of(name: str):
    for fam, (pat, _) in FAMILIES.items():
        if re.search(pat, name):
            return fam
    return None


def _csv(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def stats(args):
    rows = _csv(_find(args.dir, "kernel_stats.csv"))
    trace = {}
    try:
        for r in _csv(_find(args.dir, "kernel_trace.csv")):
            trace.setdefault(r["Kernel_Name"], r)
    except FileNotFoundError:
        pass
    print(f"# rocprofv3 --kernel-trace --stats summary: {args.title}")
    print(f"# command: {args.cmd}")
    print("# family        calls   total_ms    avg_us     min_us     max_us    pct   vgpr  kernel")
    for r in rows:
        name = r["Name"]
        fam = family_of(name) or "-"
        t = trace.get(name, {})
        print(f"{fam:14s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
              f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:10.2f} "
              f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f} "
              f"{t.get('VGPR_Count', '-'):>5s}  {name[:90]}")


def _per_dispatch(d):
    """Mean counter value (KiB) per dispatch of each kernel family."""
    rows = _csv(_find(d, "counter_collection.csv"))
    per = {}
    for r in rows:
        fam = family_of(r["Kernel_Name"])
        if fam is None:
            continue
        per.setdefault(fam, {}).setdefault(r["Dispatch_Id"], 0.0)
        per[fam][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {f: (sum(v.values()) / len(v), len(v)) for f, v in per.items()}


def traffic(args):
    fe, wr = _per_dispatch(args.fetch), _per_dispatch(args.write)
    cf, cw = _per_dispatch(args.copy_fetch), _per_dispatch(args.copy_write)
    kib = args.copy_bytes / 1024.0
    sf = kib / cf["copy"][0]
    sw = kib / cw["copy"][0]
    print(f"# HBM traffic per dispatch from rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE in KiB): {args.title}")
    print(f"# command: {args.cmd}")
    print(f"# calibration: a device copy of {args.copy_bytes} B reads FETCH_SIZE {cf['copy'][0]:.1f} KiB "
          f"and WRITE_SIZE {cw['copy'][0]:.1f} KiB -> fetch_scale {sf:.4f} write_scale {sw:.4f}")
    print("# bytes = counter KiB x 1024 x scale; source = SHA-256 (16 hex) of the kernel's sources")
    print(f"fetch_scale {sf:.6f}")
    print(f"write_scale {sw:.6f}")
    print("# family        source            dispatches  fetch_KiB    write_KiB    bytes_per_dispatch")
    for fam in sorted(set(fe) | set(wr)):
        f_k = fe.get(fam, (0.0, 0))
        w_k = wr.get(fam, (0.0, 0))
        b = (f_k[0] * sf + w_k[0] * sw) * 1024.0
        print(f"{fam:14s} {source_hash(fam):17s} {max(f_k[1], w_k[1]):6d} {f_k[0]:12.1f} "
              f"{w_k[0]:12.1f} {b:16.0f}")


def counters(args):
    """Per kernel family: mean SQ counters per dispatch, the dispatch duration from
    the counter run's timestamps, VALU instructions per CU per ns and the share of
    active lanes in VALU instructions."""
    rows = _csv(_find(args.dir, "counter_collection.csv"))
    per, dur = {}, {}
    for r in rows:
        fam = family_of(r["Kernel_Name"])
        if fam is None:
            continue
        d = per.setdefault(fam, {}).setdefault(r["Counter_Name"], {})
        d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        dur.setdefault(fam, {})[r["Dispatch_Id"]] = (float(r["End_Timestamp"]) -
                                                     float(r["Start_Timestamp"]))
    print(f"# rocprofv3 --pmc SQ counters per dispatch: {args.title}")
    print(f"# command: {args.cmd}")
    print(f"# valu_per_cu_ns = SQ_INSTS_VALU / dispatch duration / {args.cus} CUs; "
          "lane_util = SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)")
    names = sorted({c for f in per.values() for c in f})
    print("# family        source            duration_us  valu_per_cu_ns  lane_util  " + "  ".join(names))
    for fam in sorted(per):
        m = {c: sum(v.values()) / len(v) for c, v in per[fam].items()}
        t = sum(dur[fam].values()) / len(dur[fam])
        rate = m.get("SQ_INSTS_VALU", 0.0) / t / args.cus if t > 0 else 0.0
        util = (m.get("SQ_THREAD_CYCLES_VALU", 0.0) / (64.0 * m["SQ_ACTIVE_INST_VALU"])
                if m.get("SQ_ACTIVE_INST_VALU") else 0.0)
        print(f"{fam:14s} {source_hash(fam):17s} {t / 1e3:11.1f} {rate:15.2f} {util:10.3f}  " +
              "  ".join(f"{m.get(c, 0.0):.4g}" for c in names))


def read_counters(path: str) -> dict:
    """{family: (source hash, VALU instructions per CU per ns, lane utilisation)}
    from a counter summary."""
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            out[p[0]] = (p[1], float(p[3]), float(p[4]))
    return out


def read_traffic(path: str) -> dict:
    """{family: (source hash, bytes per dispatch)} from a traffic summary."""
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if len(p) == 6:
                out[p[0]] = (p[1], float(p[5]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--dir", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="")
    b = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        b.add_argument("--" + k.replace("_", "-"), required=True, dest=k)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--cmd", required=True)
    b.add_argument("--title", default="")
    c = sub.add_parser("counters")
    c.add_argument("--dir", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--cus", type=int, default=256)
    args = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "counters": counters}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
