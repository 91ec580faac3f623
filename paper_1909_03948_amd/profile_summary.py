"""Summaries of rocprofv3 output for the timed kernel classes of the solver.

    python -m paper_1909_03948_amd.profile_summary trace <rocprofv3 -d dir> <out.json>
    python -m paper_1909_03948_amd.profile_summary pmc <rocprofv3 -d dir> <out.json>
    python -m paper_1909_03948_amd.profile_summary traffic <fetch.json> <write.json> <workload> <traffic.json>

The classes match the library's sampled timer: mg_down / mg_up are the fused
V-cycle kernels of the finest level only (in dispatch order, the first k_down
and the last k_up of each run of multigrid kernels), mg_bottom, pcg_apply and
pcg_update are single-level, gram is the block product.  The bandwidth-bound
classes are split into two launch populations as the timer splits them:
single right-hand sides (mg_down, ...) and batched solves (mg_down_b, ...).
The split goes by the finest level's precision in the kernel name: in the
default precision mode every solve of fewer than eight columns is an FP64
PCG (its finest-level kernels take double vectors) and every solve of eight
or more an FP32 PCG inside FP64 refinement (float vectors throughout).  `trace` reads the
kernel-trace CSV (per-dispatch durations); `pmc` reads a one-counter
counter-collection CSV (FETCH_SIZE or WRITE_SIZE, KiB per dispatch) and also
reports the counter of the run's last plain device copy (the benchmark ends
with a 256 MiB copy), the reference for scaling the counter to bytes.
`traffic` scales a FETCH_SIZE and a WRITE_SIZE summary of one workload by
their copies (256 MiB read and written) into HBM bytes per launch and merges
them into the traffic file under that workload, with the hash of the kernel
sources they were taken on.
"""
from __future__ import annotations

import collections
import csv
import glob
import json
import os
import sys

CLASSES = (("hinv::k_down<", "mg_down"), ("hinv::k_up<", "mg_up"), ("hinv::k_bottom<", "mg_bottom"),
           ("hinv::k_pcg_apply<", "pcg_apply"), ("hinv::k_pcg_update<", "pcg_update"),
           ("k_gram_bf16", "gram"), ("k_gram_f64", "gram"), ("k_gram_wide", "gram"))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_class(name):
    for key, cls in CLASSES:
        if key in name:
            return cls
    return None


def short(name):
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "").replace("hinv::", "").strip()


SPLIT = ("mg_down", "mg_up", "pcg_apply", "pcg_update")


def population(cls, name):
    """Class of a finest-level dispatch with its launch population: the batched
    (FP32) variants of the bandwidth-bound classes get the suffix _b."""
    if cls in SPLIT and "double" not in short(name):
        return cls + "_b"
    return cls


def finest_mask(classes):
    """Per dispatch (in dispatch order): does it belong to its class's timed population."""
    out = []
    for i, c in enumerate(classes):
        if c == "mg_down":
            out.append(i == 0 or classes[i - 1] != "mg_down")
        elif c == "mg_up":
            out.append(i + 1 == len(classes) or classes[i + 1] != "mg_up")
        else:
            out.append(c is not None)
    return out


def read_csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(files[0])))


def summarize_trace(d):
    rows = read_csv(d, "kernel_trace.csv")
    disp = sorted((int(r["Dispatch_Id"]), r["Kernel_Name"],
                   int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows)
    classes = [kernel_class(n) for _, n, _ in disp]
    mask = finest_mask(classes)
    agg = collections.defaultdict(lambda: [0, 0])
    per_name = collections.defaultdict(lambda: [0, 0])
    total = 0
    for (_, name, dur), c, m in zip(disp, classes, mask):
        total += dur
        per_name[short(name)][0] += 1
        per_name[short(name)][1] += dur
        if c and m:
            c = population(c, name)
            agg[c][0] += 1
            agg[c][1] += dur
    top = sorted(per_name.items(), key=lambda kv: -kv[1][1])[:20]
    return dict(
        dispatches=len(disp), total_ms=total / 1e6,
        classes={c: dict(dispatches=n, avg_us=t / n / 1e3, total_ms=t / 1e6) for c, (n, t) in agg.items()},
        top_kernels=[dict(kernel=k, calls=n, total_ms=t / 1e6, share=t / total, avg_us=t / n / 1e3)
                     for k, (n, t) in top])


def summarize_pmc(d):
    rows = read_csv(d, "counter_collection.csv")
    disp = sorted((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]))
                  for r in rows)
    classes = [kernel_class(n) for _, n, _, _ in disp]
    mask = finest_mask(classes)
    agg = collections.defaultdict(lambda: [0, 0.0, collections.Counter()])
    copy = None
    for (_, name, _, v), c, m in zip(disp, classes, mask):
        if name.startswith(COPY_KERNEL):
            copy = v
        if c and m:
            c = population(c, name)
            agg[c][0] += 1
            agg[c][1] += v
            agg[c][2][short(name)] += 1
    return dict(counter=disp[0][2] if disp else None, copy_kib=copy,
                classes={c: dict(dispatches=n, kib_per_dispatch=s / n, variants=dict(var))
                         for c, (n, s, var) in agg.items()})


COPY_BYTES = 256 * 1024 * 1024


def kernel_source_hash(root):
    """Hash of the V-cycle and PCG kernel sources (the traffic is valid while they are unchanged)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("mgkernels.h", "grid.h"):
        h.update(open(os.path.join(root, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def merge_traffic(fetch_json, write_json, workload, out):
    fe, wr = json.load(open(fetch_json)), json.load(open(write_json))
    ff = COPY_BYTES / (1024.0 * fe["copy_kib"])  # bytes per counted KiB
    wf = COPY_BYTES / (1024.0 * wr["copy_kib"])
    kern = {}
    for c, e in fe["classes"].items():
        w = wr["classes"].get(c)
        if not w:
            continue
        fb, wb = 1024.0 * e["kib_per_dispatch"] * ff, 1024.0 * w["kib_per_dispatch"] * wf
        kern[c] = dict(dispatches=e["dispatches"], fetch_bytes_per_launch=fb, write_bytes_per_launch=wb,
                       hbm_bytes_per_launch=fb + wb, variants=e["variants"])
    root = os.path.dirname(os.path.abspath(__file__))
    doc = json.load(open(out)) if os.path.exists(out) else {}
    doc.setdefault("workloads", {})[workload] = dict(
        source_hash=kernel_source_hash(root),
        calibration=dict(copy_bytes=COPY_BYTES, fetch_kib=fe["copy_kib"], write_kib=wr["copy_kib"],
                         fetch_factor=ff, write_factor=wf),
        kernels=kern)
    json.dump(doc, open(out, "w"), indent=1)
    return doc["workloads"][workload]


def main(argv):
    if len(argv) == 6 and argv[1] == "traffic":
        res = merge_traffic(argv[2], argv[3], argv[4], argv[5])
        print(json.dumps({c: round(v["hbm_bytes_per_launch"]) for c, v in res["kernels"].items()}))
        return
    if len(argv) != 4 or argv[1] not in ("trace", "pmc"):
        raise SystemExit(__doc__)
    res = summarize_trace(argv[2]) if argv[1] == "trace" else summarize_pmc(argv[2])
    json.dump(res, open(argv[3], "w"), indent=1)
    print(json.dumps({c: round(v.get("avg_us", v.get("kib_per_dispatch", 0.0)), 2)
                      for c, v in res["classes"].items()}))


if __name__ == "__main__":
    main(sys.argv)
