"""The no-allocation prior apply (hinv_prior_apply_noalloc) against the
allocating one (hinv_prior_apply) and the oracle's R x (Sec. 5.1, R = K_A
M^-1 K_A), through the C ABI.

Two calls in a row, the second with a smaller input, must each match the
allocating entry point exactly (same kernels, same order of operations) and
the oracle to the bar of applies without solves (1e-10 relative per column).
At the size limit (6 n nrhs <= 8 388 608 doubles) the call is accepted; one
column more is rejected with HINV_EINVAL.
"""
import numpy as np
import pytest

import synth
from cases import col_rel
from oracle import model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")

LIMIT = 8 * 1024 * 1024  # doubles in the fixed scratch


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    return hv.Context(0)


def _both(gp, X):
    ref = dev(np.zeros_like(X))
    out = dev(np.full_like(X, np.nan))
    gp.prior_apply(dev(X), ref)
    gp.prior_apply_noalloc(dev(X), out)
    return host(ref), host(out)


def test_noalloc_prior_apply_two_calls_then_smaller(ctx):
    for N, nc, seed in ((32, 5, 11), (16, 2, 12)):
        print(f"[gpu] prior_apply_noalloc N={N} nrhs={nc}", flush=True)
        prob = model.Problem(N, 0.1, 0.5)
        gp = hv.Problem(ctx, N, 0.1, 0.5, beta=prob.beta)
        X = synth.test_vectors(prob.n, nc, seed=seed)
        ref, out = _both(gp, X)
        assert np.array_equal(ref, out), np.max(np.abs(ref - out))
        orc = np.array([prob.R_apply(x) for x in X])
        assert col_rel(out, orc) <= 1e-10


def test_noalloc_prior_apply_size_limit(ctx):
    N = 512
    n = (N + 1) ** 2
    nmax = LIMIT // (6 * n)
    print(f"[gpu] prior_apply_noalloc N={N} nrhs={nmax} (limit)", flush=True)
    gp = hv.Problem(ctx, N, 0.05, 1.0)
    X = synth.test_vectors(n, nmax, seed=13)
    ref, out = _both(gp, X)
    assert np.array_equal(ref, out)
    big = dev(np.zeros((nmax + 1, n)))
    with pytest.raises(hv.HinvError) as e:
        gp.prior_apply_noalloc(big, dev(np.zeros((nmax + 1, n))))
    assert e.value.code == hv.HINV_EINVAL
    # a rejected call leaves the entry point usable
    X2 = synth.test_vectors(n, 1, seed=14)
    ref, out = _both(gp, X2)
    assert np.array_equal(ref, out)
