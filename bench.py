"""Benchmark: Hessian-vector products/s at a 1e-10 residual and time to MAP +
rank-k posterior, on one MI355X.

One step = the whole hot path on the 256 x 256 Poisson coefficient-inversion
workload (66 049 parameters, 400 observations, bilaplacian prior gamma = 0.1,
delta = 0.5): inexact Newton-CG from the prior mean to |g| <= 1e-6 |g_0|, then
the double-pass randomized eigensolver with k = 50, p = 20 (all 70 probe
vectors in one batched multi-right-hand-side solve per pass).  Every PDE
solve reaches a relative residual of 1e-10 (single right-hand sides: FP64 CG
preconditioned by an FP32 multigrid V-cycle; batches: FP32 multigrid-PCG
inside FP64 refinement); the eigensolver's block product Q^T (A Q) runs on
BF16 matrix cores with FP32 accumulation.

value = Hessian-vector products completed in the timed steps / wall time
(each Newton-CG Hessian action and each eigensolver column counts one).
ms_per_step = time to MAP + rank-k posterior.  Inputs (probe matrix, data) are
resident on the device before timing starts.

``--workload poisson1024`` runs the 1024 x 1024 workload instead (1 050 625
parameters, 2 000 observations, gamma = 0.05, delta = 1, k = 200, p = 20): the
same step followed by 1 000 posterior samples through the low-rank update,
their white noise drawn on the device by the counter-based generator.

``--workload learned1024`` runs the learned correction on the 1024 x 1024
problem: 20 000 training pairs harvested from the incremental solves of 50
seeded true fields, the residual CNN trained on the device, then flexible CG
with and without it against multigrid PCG at a 1e-10 relative residual on a
held-out field (iterations and wall time).

``--workload uneven64`` runs 64 independent inversions with mesh sizes drawn
from {64, 128, 256, 512}, their own prior parameters, observations and true
fields: one step is the double pass (k = 50, p = 20) of every instance at its
true parameter through the batch (one multi-right-hand-side solve per mesh
size), and the same work instance by instance is timed beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

WORKLOAD = "poisson256"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFLOPS = 78.6   # dense FP64 matrix cores
BF16_MFMA_PEAK_TFLOPS = 2500.0
TIMED_CLASSES = ["mg_down", "mg_up", "mg_bottom", "pcg_apply", "pcg_update", "gram"]
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def setup_gpu(cfg, precision, seed=synth.MASTER_SEED):
    import torch
    from paper_1909_03948_amd import hinv as hv
    N, q = cfg["N"], cfg["q"]
    n = (N + 1) ** 2
    ctx = hv.Context(0)
    obs = synth.obs_points(q, seed=seed)
    prob = hv.Problem(ctx, N, cfg["gamma"], cfg["delta"], obs_xy=obs, d_obs=None, sigma=0.01,
                      m_prior=cfg["m_prior"], precision=precision, rtol=1e-10)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    # synthetic truth: a prior draw; data = B u(m_true) + 1% noise (Sec. 5.1)
    m_true = dev(np.zeros(n))
    prob.prior_sample(dev(synth.white_noise(N, seed=seed)), m_true)
    u_true = dev(np.zeros(n))
    prob.forward(m_true, u_true)
    Bu = dev(np.zeros(q))
    prob.observe(u_true, Bu)
    torch.cuda.synchronize()
    sigma = 0.01 * float(u_true.abs().max())
    d = Bu.cpu().numpy() + sigma * synth.obs_noise(q, seed=seed)
    prob.set_data(d, sigma)
    s = cfg["k"] + cfg["p"]
    omega = dev(synth.omega(n, s, seed=seed))
    torch.cuda.synchronize()
    return ctx, prob, omega, dict(n=n, sigma=sigma)


def run_step(prob, omega, cfg, tprod, m_map, V, samples=None):
    """MAP point, rank-k eigenpairs and (if ``samples`` = (count, chunk, eta, out))
    posterior samples drawn with device white noise."""
    import torch
    from paper_1909_03948_amd import hinv as hv
    t0 = time.perf_counter()
    ninfo = prob.map_newton(m_map, rel_tol=1e-6)
    t1 = time.perf_counter()
    lam, einfo = prob.lowrank_eig(omega, cfg["k"], V, mode=hv.HESS_MISFIT, tprod=tprod)
    t2 = time.perf_counter()
    if samples is not None:
        count, chunk, eta, out = samples
        for first in range(0, count, chunk):
            c = min(chunk, count - first)
            prob.white_noise(synth.MASTER_SEED, synth.STREAM_POST, first, eta[:c])
            prob.posterior_sample(m_map, lam, V, eta[:c], out[:c])
        torch.cuda.synchronize()
    t3 = time.perf_counter()
    if not ninfo["converged"]:
        log(f"WARNING: Newton did not reach its tolerance (status {ninfo['status']}, "
            f"{ninfo['iterations']} iterations)")
    s = cfg["k"] + cfg["p"]
    hvps = ninfo["hessian_applies"] + 2 * s
    return dict(hvps=hvps, newton_s=t1 - t0, eig_s=t2 - t1, sample_s=t3 - t2, newton=ninfo,
                eig=einfo, lam=lam)


def roofline(ctx, steps, tprod, workload):
    """Per-class sampled event timings -> roofline of the dominant class."""
    kern = {}
    for name in TIMED_CLASSES:
        r = ctx.kernel_timer_read(name)
        if r["timed"] == 0:
            continue
        avg_ms = r["ms"] / r["timed"]
        kern[name] = dict(launches=r["launches"], timed=r["timed"], avg_us=1e3 * avg_ms,
                          est_total_ms=avg_ms * r["launches"],
                          work_per_launch=r["work"] / r["timed"],
                          rate=r["work"] / (r["ms"] * 1e-3) / 1e9)  # GB/s or GFLOP/s
    if not kern:
        return None, kern
    dom = max(kern, key=lambda k: kern[k]["est_total_ms"])
    k = kern[dom]
    if dom == "gram":
        peak = BF16_MFMA_PEAK_TFLOPS if tprod == "bf16" else FP64_MFMA_PEAK_TFLOPS
        roof = dict(bound="mfma", achieved=k["rate"] / 1e3, peak=peak, unit="TFLOP/s",
                    frac=k["rate"] / 1e3 / peak, traffic=None)
    else:
        roof = dict(bound="hbm", achieved=k["rate"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=k["rate"] / HBM_PEAK_GBS, traffic=None)
    roof["kernel"] = dom
    roof["avg_us"] = k["avg_us"]
    roof["algorithmic_bytes_per_launch" if dom != "gram" else "flops_per_launch"] = k["work_per_launch"]
    # HBM bytes per launch from the committed counter summary of this workload,
    # valid while the kernel sources are those the counters were taken on
    if os.path.exists(PMC_FILE) and dom != "gram":
        from paper_1909_03948_amd.profile_summary import kernel_source_hash
        wl = json.load(open(PMC_FILE)).get("workloads", {}).get(workload, {})
        ent = wl.get("kernels", {}).get(dom)
        src = os.path.join(ROOT, "paper_1909_03948_amd")
        if ent and wl.get("source_hash") == kernel_source_hash(src):
            roof["traffic"] = ent["hbm_bytes_per_launch"]
    return roof, kern


def cpu_baseline(cfg, workload, budget_s=20.0):
    """Oracle HVPs (misfit part) at the true parameter of the same workload,
    factorization reused, until the time budget is spent."""
    from oracle import model
    N, q = cfg["N"], cfg["q"]
    prob, m_true, _ = model.make_instance(dict(N=N, q=q, gamma=cfg["gamma"], delta=cfg["delta"],
                                               m_prior=cfg["m_prior"]), synth.MASTER_SEED,
                                          synth.white_noise(N)[0], synth.obs_points(q),
                                          synth.obs_noise(q))
    u = prob.forward(m_true)
    p = prob.adjoint(m_true, u)
    dirs = synth.test_vectors(prob.n, 160, stream=synth.STREAM_OMEGA)
    prob.hessian_apply(m_true, u, p, dirs[0], model.HESS_MISFIT)  # factorization outside timing
    count, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and count < len(dirs):
        prob.hessian_apply(m_true, u, p, dirs[count], model.HESS_MISFIT)
        count += 1
    dt = time.perf_counter() - t0
    return dict(value=count / dt, unit="HVP/s", cores=1, kind="oracle",
                sample=f"{count} misfit Hessian actions of the {workload} workload at the true "
                       f"parameter, sparse LU of A(m) reused, {dt:.1f} s single-threaded SuperLU")


def run_uneven(a):
    """Uneven batch: 64 instances, double pass k = 50, p = 20 for all of them."""
    import torch
    from paper_1909_03948_amd import hinv as hv
    specs = synth.uneven_batch(64)
    k, p = 50, 20
    s = k + p
    prec = {"auto": hv.PREC_AUTO, "fp32ir": hv.PREC_FP32_IR, "fp64": hv.PREC_FP64}[a.precision]
    tprod = hv.TPROD_BF16 if a.tprod == "bf16" else hv.TPROD_FP64
    ctx = hv.Context(0)
    probs, omegas, Vs = [], [], []
    log("setup: 64 instances, sizes", sorted({sp["N"] for sp in specs}))
    for sp in specs:
        N, q, seed = sp["N"], sp["q"], sp["seed"]
        n = (N + 1) ** 2
        gp = hv.Problem(ctx, N, sp["gamma"], sp["delta"], obs_xy=synth.obs_points(q, seed=seed),
                        d_obs=None, sigma=0.01, m_prior=sp["m_prior"], precision=prec, rtol=1e-10)
        z = lambda *shape: torch.zeros(shape, dtype=torch.float64, device="cuda")
        eta = z(1, 6 * N * N)
        gp.white_noise(seed, synth.STREAM_TRUTH, 0, eta)
        m_true, u, pp, g, Bu = z(n), z(n), z(n), z(n), z(q)
        gp.prior_sample(eta, m_true)
        gp.forward(m_true, u)
        gp.observe(u, Bu)
        torch.cuda.synchronize()
        sigma = 0.01 * float(u.abs().max())
        gp.set_data(Bu.cpu().numpy() + sigma * synth.obs_noise(q, seed=seed), sigma)
        gp.gradient(m_true, u, pp, g)
        gp.linearize(m_true, u, pp)
        probs.append(gp)
        omegas.append(torch.as_tensor(synth.omega(n, s, seed=seed), device="cuda"))
        Vs.append(z(k, n))
    batch = hv.Batch(ctx, probs)
    torch.cuda.synchronize()
    hvps = 64 * 2 * s

    def batched():
        lam, info = batch.lowrank_eig(omegas, k, Vs, mode=hv.HESS_MISFIT, tprod=tprod)
        assert info["rc"] == 0, info
        return lam

    def sequential():
        lam = np.zeros((64, k))
        for i, gp in enumerate(probs):
            lam[i], info = gp.lowrank_eig(omegas[i], k, Vs[i], mode=hv.HESS_MISFIT, tprod=tprod)
            assert info["rc"] == 0, info
        return lam

    for w in range(a.warmup):
        t0 = time.perf_counter()
        lam_b = batched()
        t1 = time.perf_counter()
        lam_s = sequential()
        t2 = time.perf_counter()
        log(f"warmup {w}: batched {t1 - t0:.3f}s sequential {t2 - t1:.3f}s")
    for name in TIMED_CLASSES:
        ctx.kernel_timer(name, True, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(a.steps):
        lam_b = batched()
        log(f"step {st}: batched done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    roof, kern = roofline(ctx, a.steps, a.tprod, "uneven64")
    for name in TIMED_CLASSES:
        ctx.kernel_timer(name, False, 16)
    t2 = time.perf_counter()
    for st in range(a.steps):
        lam_s = sequential()
    torch.cuda.synchronize()
    dts = time.perf_counter() - t2
    rel = np.max(np.abs(lam_b - lam_s) / np.abs(lam_s[:, :1]))
    sizes = {}
    for sp in specs:
        sizes[sp["N"]] = sizes.get(sp["N"], 0) + 1
    line = {
        "metric": "Hessian-vector products/sec at 1e-10 residual (uneven batch of 64 double passes)",
        "value": hvps * a.steps / dt,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 in f64 refinement" + (", bf16 block product" if a.tprod == "bf16" else ""),
        "data": "synthetic",
        "config": {"workload": "uneven64", "instances": 64, "mesh_sizes": {str(kk): v for kk, v in sorted(sizes.items())},
                   "sum_n": int(sum((sp["N"] + 1) ** 2 for sp in specs)), "k": k, "p": p,
                   "rtol": 1e-10, "linearization": "true parameter", "precision": a.precision,
                   "tprod": a.tprod},
        "sequential_hvp_per_s": hvps * a.steps / dts,
        "batched_over_sequential": dts / dt,
        "max_eig_diff_batched_vs_sequential": float(rel),
        "roofline": roof,
        "kernels": kern,
    }
    print(json.dumps(line), flush=True)


def run_learned(a):
    """Learned correction on the 1024 x 1024 problem (harvest, train, compare)."""
    import torch
    from oracle import cnn as ocnn  # parameter initialisation only (He normal)
    from paper_1909_03948_amd import hinv as hv
    cfg = synth.WORKLOADS["poisson1024"]
    N, q = cfg["N"], cfg["q"]
    n = (N + 1) ** 2
    fields, ppf, crop, steps, B, lr0 = 50, 400, 64, 4000, 32, 2e-3
    ctx = hv.Context(0)

    def field(seed):
        gp = hv.Problem(ctx, N, cfg["gamma"], cfg["delta"], obs_xy=synth.obs_points(q, seed=seed), d_obs=None,
                        sigma=0.01, m_prior=cfg["m_prior"], precision=hv.PREC_AUTO, rtol=1e-10)
        z = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
        eta = z(1, 6 * N * N)
        gp.white_noise(seed, synth.STREAM_TRUTH, 0, eta)
        m, u, pp, g, Bu = z(n), z(n), z(n), z(n), z(q)
        gp.prior_sample(eta, m)
        gp.forward(m, u)
        gp.observe(u, Bu)
        torch.cuda.synchronize()
        sig = 0.01 * float(u.abs().max())
        gp.set_data(Bu.cpu().numpy() + sig * synth.obs_noise(q, seed=seed), sig)
        gp.gradient(m, u, pp, g)
        gp.linearize(m, u, pp)
        return gp

    X = torch.zeros((fields * ppf, 3, crop, crop), dtype=torch.float32, device="cuda")
    T = torch.zeros((fields * ppf, 4, crop, crop), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for f in range(fields):
        gp = field(10000 + f)
        gp.cnn_harvest(ppf, 77 + f, crop, X[f * ppf:(f + 1) * ppf], T[f * ppf:(f + 1) * ppf])
        del gp
        if f % 10 == 9:
            log(f"harvested {(f + 1) * ppf} pairs, {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    harvest_s = time.perf_counter() - t0
    net = hv.Cnn(ctx)
    net.set_params(ocnn.init_params(np.random.default_rng(0)))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    t0 = time.perf_counter()
    losses = []
    for st in range(steps):
        idx = torch.randint(0, X.shape[0], (B,), device="cuda", generator=gen)
        lr = lr0 * 0.5 * (1.0 + np.cos(np.pi * st / steps))
        losses.append(net.train_step(X[idx].contiguous(), T[idx].contiguous(), lr))
        if st % 1000 == 0:
            log(f"train step {st}: energy loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    gp = field(10000 + fields)  # held out
    Xh = torch.zeros((256, 3, crop, crop), dtype=torch.float32, device="cuda")
    Th = torch.zeros((256, 4, crop, crop), dtype=torch.float32, device="cuda")
    gp.cnn_harvest(256, 5, crop, Xh, Th)
    held = float(np.mean([net.gradient(Xh[i:i + 32].contiguous(), Th[i:i + 32].contiguous())[0]
                          for i in range(0, 256, 32)]))
    gp.set_solver(hv.PREC_FP64, 1e-10)
    res = {"fcg_plain": [], "fcg_learned": [], "mg_pcg": []}
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    for trial in range(a.steps + a.warmup):
        b = torch.as_tensor(synth.test_vectors(n, 1, stream=70 + trial)[0], device="cuda")
        for key, fn in (("fcg_plain", lambda: gp.state_solve_fcg(b, x, None, 1e-10, 300)),
                        ("fcg_learned", lambda: gp.state_solve_fcg(b, x, net, 1e-10, 300)),
                        ("mg_pcg", lambda: gp.state_solve(b, x))):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            info = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            if trial >= a.warmup:
                res[key].append((info["iterations"], 1e3 * dt, info.get("fallback", 0),
                                 info.get("relres", info.get("max_relres"))))
    summ = {k: {"iterations": float(np.mean([r[0] for r in v])), "ms": float(np.mean([r[1] for r in v])),
                "fallbacks": int(sum(r[2] for r in v)), "max_relres": float(max(r[3] for r in v))}
            for k, v in res.items()}
    line = {
        "metric": "state solves at 1e-10 relative residual on the 1024x1024 problem: flexible CG with the "
                  "learned correction vs without it vs multigrid PCG (iterations, ms per solve)",
        "value": summ["fcg_learned"]["ms"],
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": summ["fcg_learned"]["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 solve, bf16 network with f32 accumulation",
        "data": "synthetic",
        "config": {"workload": "learned1024", "N": N, "fields": fields, "pairs": fields * ppf, "crop": crop,
                   "train_steps": steps, "batch": B, "lr": lr0, "loss": "relative energy norm"},
        "harvest_s": harvest_s,
        "train_s": train_s,
        "final_train_loss": float(np.mean(losses[-50:])),
        "heldout_energy_loss": held,
        "solvers": summ,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["poisson256", "poisson1024", "uneven64", "learned1024"],
                    default=WORKLOAD)
    ap.add_argument("--samples", type=int, default=1000,
                    help="posterior samples per step (poisson1024 only)")
    ap.add_argument("--precision", choices=["auto", "fp32ir", "fp64"], default="auto")
    ap.add_argument("--tprod", choices=["bf16", "fp64"], default="bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with a 256 MiB device copy (reference for HBM counters)")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the hot path is a "
                                   "single-GPU workload (multi-GPU sharding is design-only)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.workload == "uneven64":
        run_uneven(a)
        return
    if a.workload == "learned1024":
        run_learned(a)
        return
    import torch
    from paper_1909_03948_amd import hinv as hv
    workload = a.workload
    cfg = synth.WORKLOADS[workload]
    prec = {"auto": hv.PREC_AUTO, "fp32ir": hv.PREC_FP32_IR, "fp64": hv.PREC_FP64}[a.precision]
    tprod = hv.TPROD_BF16 if a.tprod == "bf16" else hv.TPROD_FP64
    log("setup", workload, a.precision, a.tprod)
    ctx, prob, omega, meta = setup_gpu(cfg, prec)
    n = meta["n"]
    m_map = torch.zeros(n, dtype=torch.float64, device="cuda")
    V = torch.zeros((cfg["k"], n), dtype=torch.float64, device="cuda")
    samples = None
    if workload != "poisson256" and a.samples > 0:
        chunk = min(a.samples, cfg["k"] + cfg["p"])
        N = cfg["N"]
        samples = (a.samples, chunk,
                   torch.zeros((chunk, 6 * N * N), dtype=torch.float64, device="cuda"),
                   torch.zeros((chunk, n), dtype=torch.float64, device="cuda"))
    for w in range(a.warmup):
        r = run_step(prob, omega, cfg, tprod, m_map, V, samples)
        log(f"warmup {w}: newton {r['newton_s']:.3f}s ({r['newton']['iterations']} it, "
            f"{r['newton']['hessian_applies']} HVP) eig {r['eig_s']:.3f}s "
            f"samples {r['sample_s']:.3f}s")
    for name in TIMED_CLASSES:
        ctx.kernel_timer(name, True, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for k in range(a.steps):
        res.append(run_step(prob, omega, cfg, tprod, m_map, V, samples))
        log(f"step {k}: newton {res[-1]['newton_s']:.3f}s eig {res[-1]['eig_s']:.3f}s "
            f"samples {res[-1]['sample_s']:.3f}s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hvps = sum(r["hvps"] for r in res)
    s = cfg["k"] + cfg["p"]
    eig_s = sum(r["eig_s"] for r in res)
    newton_s = sum(r["newton_s"] for r in res)
    sample_s = sum(r["sample_s"] for r in res)
    line = {
        "metric": "Hessian-vector products/sec at 1e-10 residual; time to MAP + rank-k posterior",
        "value": hvps / dt,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the multigrid V-cycle (the preconditioner) is f32 in every mode
        "dtype": ({"auto": "f64 PCG (single rhs) / f32 PCG in f64 refinement (batched), f32 V-cycle",
                   "fp32ir": "f32 PCG in f64 refinement, f32 V-cycle",
                   "fp64": "f64 PCG, f32 V-cycle"}[a.precision]
                  + (", bf16 block product" if a.tprod == "bf16" else "")),
        "data": "synthetic",
        "config": {"workload": workload, "N": cfg["N"], "n_params": n, "q": cfg["q"],
                   "gamma": cfg["gamma"], "delta": cfg["delta"], "k": cfg["k"], "p": cfg["p"],
                   "rtol": 1e-10, "newton_rel_tol": 1e-6, "precision": a.precision,
                   "tprod": a.tprod},
        "time_to_map_plus_posterior_s": (dt - sample_s) / a.steps,
        "newton_s_per_step": newton_s / a.steps,
        "eigensolver_s_per_step": eig_s / a.steps,
        "batched_hvp_per_s": 2 * s * a.steps / eig_s,
        "newton_iterations": res[-1]["newton"]["iterations"],
        "newton_converged": all(r["newton"]["converged"] for r in res),
        "newton_hvps": res[-1]["newton"]["hessian_applies"],
        "lambda_1": float(res[-1]["lam"][0]),
        "lambda_k": float(res[-1]["lam"][-1]),
    }
    if samples is not None:
        line["config"]["posterior_samples"] = a.samples
        line["posterior_samples_per_s"] = a.samples * a.steps / sample_s
        line["value"] = hvps / (dt - sample_s)
        line["metric"] += " (HVP/s over the MAP + eigensolver part; samples timed separately)"
    roof, kern = roofline(ctx, a.steps, a.tprod, workload)
    for name in TIMED_CLASSES:
        ctx.kernel_timer(name, False, 16)
    line["roofline"] = roof
    line["kernels"] = kern
    if a.calibration_copy:
        # plain device copy of known size for scaling the HBM counters
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: 256 MiB read + 256 MiB written")
    if not a.no_cpu_baseline and workload != "poisson256":
        # the oracle's sparse factorisations alone take minutes at this size
        log("cpu baseline skipped for", workload)
    elif not a.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(cfg, workload, a.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
