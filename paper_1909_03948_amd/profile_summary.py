"""Summaries of rocprofv3 output for the timed kernel classes of the solver.

    python -m paper_1909_03948_amd.profile_summary trace <rocprofv3 -d dir> <out.json>
    python -m paper_1909_03948_amd.profile_summary pmc <rocprofv3 -d dir> <out.json>
    python -m paper_1909_03948_amd.profile_summary traffic <fetch.json> <write.json> <workload> <traffic.json>
    python -m paper_1909_03948_amd.profile_summary markdown <trace.json> <bench.json> <traffic.json> <workload> <profiles dir>
    python -m paper_1909_03948_amd.profile_summary stats-markdown <rocprofv3 -d dir> <bench.json> <out.md>

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
sources they were taken on.  `markdown` writes the two committed summaries of
a workload (kernel_trace_<workload>.md, hbm_traffic.md) from a trace
summary, the benchmark's JSON line of the same workload and the traffic
file; `stats-markdown` writes the top kernels of a rocprofv3 --stats run
(the learned-preconditioner workload) beside its benchmark line.
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


def _bench_line(path):
    return json.loads(open(path).read().strip().splitlines()[-1])


def write_markdown(trace_json, bench_json, traffic_json, workload, outdir):
    """kernel_trace_<workload>.md and hbm_traffic.md from the summaries."""
    t = json.load(open(trace_json))
    b = _bench_line(bench_json)
    doc = json.load(open(traffic_json))
    pm = doc["workloads"][workload]
    cfg = b.get("config", {})
    what = (f"{cfg['N']} x {cfg['N']} mesh: Newton-CG MAP, double pass k = {cfg['k']}, p = {cfg['p']}, "
            f"{cfg.get('posterior_samples', 0)} posterior samples") if "N" in cfg and "k" in cfg else "benchmark workload"
    L = [f"# Kernel trace: {workload} ({what})\n",
         "Command (from the repository root, on the MI355X machine; the run's CSV stays under its output directory):\n",
         "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o run -- "
         "python3 <repo>/bench.py --steps 1 --warmup 1 --no-extras --no-cpu-baseline\n",
         "Summarized with `python -m paper_1909_03948_amd.profile_summary trace <out>/trace <out>/trace.json` and "
         "`python -m paper_1909_03948_amd.profile_summary markdown <out>/trace.json <bench.json> profiles/pmc_traffic.json "
         f"{workload} profiles`.  One warm-up and one timed step.\n",
         f"Total kernel time {t['total_ms']:.1f} ms over {t['dispatches']} dispatches (profiled run, both steps).\n",
         "## Timed classes: trace against the benchmark's live HIP-event samples\n",
         "Live figures: `python bench.py --steps 3 --warmup 1` (same workload, no profiler).  The classes without `_b` "
         "are the finest-level kernels of single-right-hand-side solves (the Newton-CG phase), `_b` the same kernels in "
         "batched solves (eigensolver passes, samples).  The events time the eagerly launched second and third PCG "
         "iterations of every 16th single-column solve and of every batched solve; the trace averages every "
         "finest-level dispatch, graph replays included.\n",
         "| class | trace dispatches | trace avg µs | bench sampled | bench avg µs | algorithmic bytes (or flops) per launch "
         "| bench rate | HBM bytes per launch (counters) |",
         "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for c, v in t["classes"].items():
        k = b.get("kernels", {}).get(c, {})
        unit = "TFLOP/s" if c == "gram" else "GB/s"
        rate = k.get("rate", 0.0) / (1e3 if c == "gram" else 1.0)
        hb = pm["kernels"].get(c, {}).get("hbm_bytes_per_launch")
        L.append(f"| {c} | {v['dispatches']} | {v['avg_us']:.2f} | {k.get('timed', '-')} | {k.get('avg_us', 0.0):.2f} | "
                 f"{k.get('work_per_launch', 0.0):.4g} | {rate:.0f} {unit} | {f'{hb:.4g}' if hb else '-'} |")
    r = b.get("roofline")
    if r:
        L.append(f"\nBench roofline line: dominant bandwidth-bound class `{r['kernel']}` ({r['population']}), "
                 f"{r['avg_us']:.2f} µs per launch (events; trace {t['classes'][r['kernel']]['avg_us']:.2f} µs), "
                 f"achieved {r['achieved']:.0f} GB/s of {r['peak']:.0f} ({100 * r['frac']:.1f}%).\n")
    L += ["## Top kernels (all levels)\n", "| kernel | calls | total ms | share | avg µs |", "|---|---:|---:|---:|---:|"]
    for k in t["top_kernels"][:16]:
        L.append(f"| `{k['kernel']}` | {k['calls']} | {k['total_ms']:.2f} | {100 * k['share']:.1f}% | {k['avg_us']:.2f} |")
    open(os.path.join(outdir, f"kernel_trace_{workload}.md"), "w").write("\n".join(L) + "\n")
    c = pm["calibration"]
    H = ["# HBM traffic of the timed classes (rocprofv3 counters)\n",
         "Commands (one counter per run, on the MI355X machine):\n",
         "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/FETCH_SIZE -o run -- "
         "python3 <repo>/bench.py --steps 1 --warmup 0 --no-extras --no-cpu-baseline --calibration-copy",
         "    (the same with --pmc WRITE_SIZE)",
         "    python -m paper_1909_03948_amd.profile_summary pmc <out>/FETCH_SIZE <out>/FETCH_SIZE.json   (and WRITE_SIZE)",
         f"    python -m paper_1909_03948_amd.profile_summary traffic <out>/FETCH_SIZE.json <out>/WRITE_SIZE.json {workload} "
         "profiles/pmc_traffic.json\n",
         "Each counter is averaged over the finest-level dispatches of a class (single-column and batched populations "
         "apart, by the finest level's precision in the kernel name) and scaled by what it reads for the run's closing "
         "256 MiB device copy.  `bench.py` reports the HBM bytes per launch of each class while the V-cycle kernel "
         "sources hash to `source_hash`.\n",
         f"## {workload}\n",
         f"Calibration: FETCH_SIZE {c['fetch_kib']:.0f} KiB and WRITE_SIZE {c['write_kib']:.0f} KiB for 256 MiB read and "
         f"written: factors {c['fetch_factor']:.4f} and {c['write_factor']:.4f}; kernel sources {pm['source_hash']}.\n",
         "| class | dispatches | fetch bytes / launch | write bytes / launch | HBM bytes / launch | algorithmic bytes / "
         "launch (bench) | HBM / algorithmic |",
         "|---|---:|---:|---:|---:|---:|---:|"]
    for cl, v in pm["kernels"].items():
        alg = b.get("kernels", {}).get(cl, {}).get("work_per_launch")
        ratio = f"{v['hbm_bytes_per_launch'] / alg:.2f}" if alg and cl != "gram" else "-"
        H.append(f"| {cl} | {v['dispatches']} | {v['fetch_bytes_per_launch']:.4g} | {v['write_bytes_per_launch']:.4g} | "
                 f"{v['hbm_bytes_per_launch']:.4g} | {f'{alg:.4g}' if alg else '-'} | {ratio} |")
    if cfg.get("n_params") and cfg.get("k") is not None:
        nn, ss = cfg["n_params"], cfg["k"] + cfg.get("p", 0)
        H.append(f"\nThe gram row's algorithmic figure is flops, not bytes: its compulsory traffic is n (s1 + s2) 8 bytes "
                 f"= {nn * 2 * ss * 8:.3g} at n = {nn}, s = {ss} (X ≠ Y; half of it for YᵀY).")
    open(os.path.join(outdir, "hbm_traffic.md"), "w").write("\n".join(H) + "\n")


def write_stats_markdown(d, bench_json, out):
    """Top kernels of a rocprofv3 --stats run beside the benchmark line (learned workload)."""
    rows = read_csv(d, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    b = _bench_line(bench_json)
    keys = ("value", "unit", "harvest_s", "train_s", "heldout_energy_loss", "solvers")
    L = ["# Kernel trace: learned1024 (harvest 20 000 pairs on the 1024 x 1024 problem, 4 000 Adam steps of the "
         "residual CNN, flexible CG with and without it)\n",
         "Command (from the repository root, on the MI355X machine):\n",
         "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <out>/learned -o run "
         "-- python3 <repo>/bench.py --workload learned1024\n",
         "Summarized with `python -m paper_1909_03948_amd.profile_summary stats-markdown <out>/learned <bench.json> "
         "profiles/kernel_trace_learned1024.md`, the bench line from `python bench.py --workload learned1024`.\n",
         f"Total kernel time {tot / 1e6:.1f} ms.  The convolution kernels multiply BF16 operands on the matrix cores "
         "(gfx950 16x16x32 for the 32-channel layers); their rate counts 2 x pixels x 9 x C_in x C_out flops per layer "
         "and image.\n",
         "Bench line of the same workload (no profiler): " + json.dumps({k: b.get(k) for k in keys}) + "\n",
         "| kernel | calls | total ms | share | avg µs |", "|---|---:|---:|---:|---:|"]
    for r in rows[:20]:
        L.append(f"| `{short(r['Name'])[:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                 f"{100 * float(r['TotalDurationNs']) / tot:.1f}% | {float(r['AverageNs']) / 1e3:.2f} |")
    open(out, "w").write("\n".join(L) + "\n")


def main(argv):
    if len(argv) == 7 and argv[1] == "markdown":
        write_markdown(argv[2], argv[3], argv[4], argv[5], argv[6])
        return
    if len(argv) == 5 and argv[1] == "stats-markdown":
        write_stats_markdown(argv[2], argv[3], argv[4])
        return
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
