"""The launch-shape tuner's persistent cache (HINV_TUNE_CACHE), across processes.

A first process solves with an empty cache file: the tuner times its
candidates and appends its choices.  A second process with the same file
takes every shape from it (no timing) and, running the same launch shapes,
gives bit-identical Hessian actions; both match the oracle to 1e-8.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from cases import col_rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import synth
from paper_1909_03948_amd import hinv as hv
N, q = 64, 50
obs = synth.obs_points(q)
ctx = hv.Context(0)
gp = hv.Problem(ctx, N, 0.1, 0.5, obs_xy=obs, d_obs=np.zeros(q), sigma=0.01, precision=hv.PREC_AUTO)
n = (N + 1) ** 2
dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
m = dev(-2.0 + 0.4 * synth.smooth_field(N))
u, p, g = dev(np.zeros(n)), dev(np.zeros(n)), dev(np.zeros(n))
gp.forward(m, u)
gp.gradient(m, u, p, g)
gp.linearize(m, u, p)
outs = []
for nc in (1, 9):
    mh = dev(synth.test_vectors(n, nc, seed=90 + nc))
    o = dev(np.zeros((nc, n)))
    info = gp.hessian_apply(hv.HESS_GN_MISFIT, mh, o)
    assert info["rc"] == 0, info
    outs.append(o.cpu().numpy().tolist())
print(json.dumps({"counts": hv.tuner_counts(), "outs": outs}))
"""


def run_child(cache):
    env = dict(os.environ, HINV_TUNE_CACHE=cache)
    env.pop("HINV_AUTOTUNE", None)
    env.pop("HINV_SHAPE", None)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_tuner_cache_reused_by_a_later_process(tmp_path):
    cache = str(tmp_path / "tune.jsonl")
    first = run_child(cache)
    lines = [json.loads(l) for l in open(cache)]
    print(f"[gpu-tune] first process: timed {first['counts'][0]}, cached {first['counts'][1]}, "
          f"{len(lines)} lines", flush=True)
    assert first["counts"][0] >= 2 and first["counts"][1] == 0
    assert {l["columns"] for l in lines} >= {1, 9} and all(l["N"] == 64 for l in lines)
    second = run_child(cache)
    print(f"[gpu-tune] second process: timed {second['counts'][0]}, cached {second['counts'][1]}", flush=True)
    assert second["counts"][0] == 0 and second["counts"][1] == first["counts"][0]
    for a, b in zip(first["outs"], second["outs"]):
        assert np.array_equal(np.array(a), np.array(b))
    # and the actions are right
    from oracle import model
    prob = model.Problem(64, 0.1, 0.5, -2.0, obs_xy=synth.obs_points(50), d_obs=np.zeros(50), sigma=0.01)
    m = prob.m_pr + 0.4 * synth.smooth_field(64)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    for nc, got in zip((1, 9), second["outs"]):
        mh = synth.test_vectors(prob.n, nc, seed=90 + nc)
        ref = np.array([prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT) for v in mh])
        assert col_rel(np.array(got), ref) < 1e-8
