"""Host logic of the profile summarizer: the finest-level selection of the
V-cycle classes in dispatch order, per-class averages, and the scaling of
the counters by the closing device copy (synthetic rocprofv3 CSVs)."""
import csv
import json

from paper_1909_03948_amd import profile_summary as ps

COPY = "__amd_rocclr_copyBuffer"


def _cycle():
    # one V-cycle over two levels above the bottom, then the PCG vector kernels
    return ["void hinv::k_down<double, hinv::OpA<double>, 8>(...)",
            "void hinv::k_down<double, hinv::OpA<double>, 8>(...)",
            "void hinv::k_bottom<double, 0>(...)",
            "void hinv::k_up<double, hinv::OpA<double>, 16>(...)",
            "void hinv::k_up<double, hinv::OpA<double>, 16>(...)",
            "void hinv::k_pcg_apply<double, hinv::OpA<double> >(...)",
            "void hinv::k_pcg_update<double>(...)"]


def test_finest_mask_picks_first_down_and_last_up():
    names = _cycle() * 2
    cls = [ps.kernel_class(n) for n in names]
    mask = ps.finest_mask(cls)
    picked = [(c, i % 7) for i, (c, m) in enumerate(zip(cls, mask)) if m]
    assert picked == [("mg_down", 0), ("mg_bottom", 2), ("mg_up", 4), ("pcg_apply", 5), ("pcg_update", 6)] * 2


def test_trace_summary_averages_finest_dispatches(tmp_path):
    names = _cycle() * 3
    # durations: finest down 10, coarse down 4, bottom 8, coarse up 3, finest up 9, apply 6, update 5 (ns x 1000)
    dur = [10, 4, 8, 3, 9, 6, 5] * 3
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 0
        for i, (n, d) in enumerate(zip(names, dur)):
            w.writerow([i + 1, n, t, t + 1000 * d])
            t += 1000 * d + 500
    res = ps.summarize_trace(str(tmp_path))
    assert res["dispatches"] == 21
    c = res["classes"]
    assert c["mg_down"]["dispatches"] == 3 and abs(c["mg_down"]["avg_us"] - 10.0) < 1e-9
    assert c["mg_up"]["dispatches"] == 3 and abs(c["mg_up"]["avg_us"] - 9.0) < 1e-9
    assert abs(c["mg_bottom"]["avg_us"] - 8.0) < 1e-9 and abs(c["pcg_update"]["avg_us"] - 5.0) < 1e-9
    assert abs(res["total_ms"] - sum(dur) * 1e-3) < 1e-9


def _counter_csv(path, counter, values, copy_kib):
    names = _cycle()
    with open(path / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (n, v) in enumerate(zip(names, values)):
            w.writerow([i + 1, n, counter, v])
        w.writerow([len(names) + 1, COPY, counter, 7.0])  # an earlier small copy is ignored
        w.writerow([len(names) + 2, "void hinv::k_pcg_update<double>(...)", counter, 100.0])
        w.writerow([len(names) + 3, COPY, counter, copy_kib])


def test_traffic_scales_by_the_closing_copy(tmp_path):
    fdir, wdir = tmp_path / "f", tmp_path / "w"
    fdir.mkdir()
    wdir.mkdir()
    # FETCH counts half the bytes (as the hardware counter does), WRITE all of them
    _counter_csv(fdir, "FETCH_SIZE", [50, 20, 3, 10, 40, 30, 60], 131072.0)
    _counter_csv(wdir, "WRITE_SIZE", [25, 9, 1, 5, 30, 20, 40], 262144.0)
    fe, wr = ps.summarize_pmc(str(fdir)), ps.summarize_pmc(str(wdir))
    assert fe["copy_kib"] == 131072.0 and wr["copy_kib"] == 262144.0
    assert fe["classes"]["mg_down"]["kib_per_dispatch"] == 50
    assert fe["classes"]["pcg_update"]["kib_per_dispatch"] == 80  # (60 + 100) / 2
    json.dump(fe, open(tmp_path / "fe.json", "w"))
    json.dump(wr, open(tmp_path / "wr.json", "w"))
    out = tmp_path / "traffic.json"
    ent = ps.merge_traffic(str(tmp_path / "fe.json"), str(tmp_path / "wr.json"), "w1", str(out))
    assert abs(ent["calibration"]["fetch_factor"] - 2.0) < 1e-12
    assert abs(ent["calibration"]["write_factor"] - 1.0) < 1e-12
    up = ent["kernels"]["mg_up"]
    assert abs(up["hbm_bytes_per_launch"] - (40 * 2 + 30) * 1024) < 1e-6
    assert json.load(open(out))["workloads"]["w1"]["source_hash"] == ent["source_hash"]


def test_batched_variants_form_their_own_population():
    # a batched FP32 cycle: float vectors on every level
    names = ["void hinv::k_down<float, hinv::OpA<float>, 16, float>(...)",
             "void hinv::k_down<float, hinv::OpA<float>, 16, float>(...)",
             "void hinv::k_bottom<float, 0, 32>(...)",
             "void hinv::k_up<float, hinv::OpA<float>, 32, float, float>(...)",
             "void hinv::k_up<float, hinv::OpA<float>, 32, float, float>(...)",
             "void hinv::k_pcg_apply<float, hinv::OpA<float>, false>(...)",
             "void hinv::k_pcg_update<float>(...)"]
    # a single-column FP64 cycle: double vectors on the finest level only
    single = ["void hinv::k_down<float, hinv::OpA<float>, 8, double>(...)",
              "void hinv::k_down<float, hinv::OpA<float>, 8, float>(...)",
              "void hinv::k_bottom<float, 0, 32>(...)",
              "void hinv::k_up<float, hinv::OpA<float>, 16, float, float>(...)",
              "void hinv::k_up<float, hinv::OpA<float>, 16, double, double>(...)",
              "void hinv::k_pcg_apply<double, hinv::OpA<double>, false>(...)",
              "void hinv::k_pcg_update<double>(...)"]
    seq = names + single
    cls = [ps.kernel_class(n) for n in seq]
    mask = ps.finest_mask(cls)
    picked = [ps.population(c, n) for c, n, m in zip(cls, seq, mask) if m]
    assert picked == ["mg_down_b", "mg_bottom", "mg_up_b", "pcg_apply_b", "pcg_update_b",
                      "mg_down", "mg_bottom", "mg_up", "pcg_apply", "pcg_update"]


def test_short_names_keep_helper_kernels():
    assert ps.short("void hinv::(anonymous namespace)::k_cheb_mass<32>(hinv::OpKA<double>, int)") == "k_cheb_mass<32>"
    assert ps.short("void hinv::k_up<float, hinv::OpA<float>, 16>(hinv::OpA<float>)") == "k_up<float, OpA<float>, 16>"


def test_markdown_summaries_from_the_json_summaries(tmp_path):
    """The committed summaries are written from the trace summary, the bench
    line and the traffic file; every timed class gets a row with its figures."""
    trace = {"total_ms": 12.5, "dispatches": 40,
             "classes": {"mg_down": {"dispatches": 4, "avg_us": 18.0}, "gram": {"dispatches": 1, "avg_us": 2900.0}},
             "top_kernels": [{"kernel": "k_down<float>", "calls": 4, "total_ms": 0.072, "share": 0.5, "avg_us": 18.0}]}
    bench = {"config": {"N": 1024, "k": 200, "p": 20, "posterior_samples": 1000, "n_params": 1050625},
             "kernels": {"mg_down": {"timed": 3, "avg_us": 19.0, "work_per_launch": 2.0e7, "rate": 1052.0},
                         "gram": {"timed": 1, "avg_us": 2950.0, "work_per_launch": 1.0e11, "rate": 35000.0}},
             "roofline": {"kernel": "mg_down", "population": "single right-hand side", "avg_us": 19.0,
                          "achieved": 1052.0, "peak": 8000.0, "frac": 0.1315}}
    traffic = {"workloads": {"poisson1024": {
        "source_hash": "abc", "calibration": {"fetch_kib": 131091, "write_kib": 262144, "fetch_factor": 2.0,
                                              "write_factor": 1.0},
        "kernels": {"mg_down": {"dispatches": 4, "fetch_bytes_per_launch": 1.5e7, "write_bytes_per_launch": 4.5e6,
                                "hbm_bytes_per_launch": 1.95e7}}}}}
    for name, doc in (("trace.json", trace), ("traffic.json", traffic)):
        json.dump(doc, open(tmp_path / name, "w"))
    (tmp_path / "bench.json").write_text("[bench] log line\n" + json.dumps(bench) + "\n")
    ps.write_markdown(str(tmp_path / "trace.json"), str(tmp_path / "bench.json"), str(tmp_path / "traffic.json"),
                      "poisson1024", str(tmp_path))
    kt = (tmp_path / "kernel_trace_poisson1024.md").read_text()
    assert "1024 x 1024 mesh" in kt and "| mg_down | 4 | 18.00 | 3 | 19.00 | 2e+07 | 1052 GB/s | 1.95e+07 |" in kt
    assert "| gram | 1 | 2900.00 | 1 | 2950.00 | 1e+11 | 35 TFLOP/s | - |" in kt
    assert "achieved 1052 GB/s of 8000 (13.2%)" in kt
    hb = (tmp_path / "hbm_traffic.md").read_text()
    assert "| mg_down | 4 | 1.5e+07 | 4.5e+06 | 1.95e+07 | 2e+07 | 0.97 |" in hb
    assert "kernel sources abc" in hb
