"""Exactness of the division-free index arithmetic of the V-cycle and PCG
kernels: node indices are split into (i, j) by a reciprocal multiplication
instead of an integer division, which must agree with the division on every
index the kernels use."""
import numpy as np


def test_small_quotient_by_float_reciprocal_is_exact():
    # the bottom kernel divides node indices q by level widths d as
    # (q + 1/2) * (1/d) in single precision, truncated; exact for q < 2^22
    # (the product errs by at most (q + 1/2) / d * 2^-23, the quotient lies at
    # least 1 / (2 d) from an integer)
    def fdiv(q, d):
        inv = np.float32(1.0) / np.float32(d)
        return ((q.astype(np.float32) + np.float32(0.5)) * inv).astype(np.int64)
    q = np.arange(1 << 16, dtype=np.int64)
    for d in range(1, 130):          # every level width of the bottom kernel and more
        assert np.array_equal(fdiv(q, d), q // d), d
    rng = np.random.default_rng(7)
    for d in rng.integers(1, 1 << 12, 200):  # near multiples of d up to 2^22
        k = rng.integers(0, ((1 << 22) - 1) // d, 500)
        qq = np.concatenate([k * d, k * d + d - 1, np.maximum(k * d - 1, 0)])
        qq = qq[qq < (1 << 22) - 1]
        assert np.array_equal(fdiv(qq, int(d)), qq // d), d


def test_node_row_by_double_reciprocal_is_exact():
    # the PCG apply kernel splits node k = j (N + 1) + i by j = (k + 1/2) * (1/(N + 1))
    # in double precision, truncated
    for n1 in (9, 17, 33, 65, 129, 257, 513, 1025, 2049):
        k = np.arange(n1 * n1, dtype=np.int64)
        inv = 1.0 / n1
        j = ((k.astype(np.float64) + 0.5) * inv).astype(np.int64)
        assert np.array_equal(j, k // n1), n1
