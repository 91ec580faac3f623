"""Pins of the counter-based white-noise generator used for prior and posterior draws.

Philox4x64-10 is written out here from its published definition (Salmon,
Moraes, Dror, Shaw, SC'11: ten rounds of two 64x64-bit multiplications with
Weyl key increments) and checked against NumPy's independent implementation;
the Box-Muller normals of synth.philox_white_noise are checked for their
counter mapping and their statistics.
"""
import numpy as np

import synth

M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
MASK = (1 << 64) - 1


def philox4x64_10(ctr, key):
    R = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0, p1 = M0 * R[0], M1 * R[2]
        R = [(p1 >> 64) ^ R[1] ^ k0, p1 & MASK, (p0 >> 64) ^ R[3] ^ k1, p0 & MASK]
        k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
    return R


def test_published_rounds_match_numpy_philox():
    seed, stream = 1909, 4
    g = np.random.Philox(key=seed | (stream << 64))
    raw = [int(x) for x in g.random_raw(12)]
    mine = sum((philox4x64_10([b, 0, 0, 0], [seed, stream]) for b in (1, 2, 3)), [])
    assert raw == mine


def test_white_noise_counter_mapping_and_box_muller():
    N = 4
    L = 6 * N * N
    z = synth.philox_white_noise(N, 3, seed=7, stream=2)
    # sample 1 drawn alone equals the second row
    np.testing.assert_array_equal(synth.philox_white_noise(N, 1, seed=7, stream=2, first=1)[0], z[1])
    # first normal pair of sample 0 from the first counter block, written out
    w = philox4x64_10([1, 0, 0, 0], [7, 2])
    u1 = ((w[0] >> 11) + 1) * 2.0 ** -53
    u2 = (w[1] >> 11) * 2.0 ** -53
    r = np.sqrt(-2 * np.log(u1))
    np.testing.assert_allclose(z[0, :2], [r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)], rtol=1e-15)
    # block of sample 2 starts at counter 2 L/4 + 1
    w = philox4x64_10([2 * L // 4 + 1, 0, 0, 0], [7, 2])
    u1 = ((w[2] >> 11) + 1) * 2.0 ** -53
    u2 = (w[3] >> 11) * 2.0 ** -53
    assert abs(z[2, 2] - np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)) < 1e-14


def test_white_noise_statistics():
    z = synth.philox_white_noise(64, 4).reshape(-1)  # 98 304 normals
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(z ** 4) - 3) < 0.1           # Gaussian kurtosis
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / np.sqrt(n)
