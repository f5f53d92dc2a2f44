"""Pins of the counter-based batch sampler: published SplitMix64 outputs,
exact multiply-shift, uniformity."""
import json
import os

import numpy as np

from oracle import sampler as S

VEC = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.json")))


def test_splitmix64_known_answers():
    assert S.splitmix64_int(0, 5) == [int(v, 16) for v in VEC["seed_0"]]
    assert S.splitmix64_int(1234567, 5) == VEC["seed_1234567"]


def test_counter_form_is_the_sequence():
    seq = S.splitmix64_int(987654321, 40)
    assert [S.mix_int(987654321 + S.GOLDEN * (c + 1)) for c in range(40)] == seq
    # nested streams: h(seed, stream, step, j) is output j+1 of the generator seeded by
    # output step+1 of the generator seeded by output stream+1 of SplitMix64(seed)
    s1 = S.splitmix64_int(7, 3)[2]
    s2 = S.splitmix64_int(s1, 5)[4]
    assert S.hash_int(7, 2, 4, 9) == S.splitmix64_int(s2, 10)[9]


def test_vectorised_hash_matches_exact():
    j = np.array([0, 1, 2, 1000, 2 ** 22 - 1, 2 ** 31 + 5], dtype=np.uint64)
    got = S.hash_np(12345, 1, 77, j)
    assert [int(v) for v in got] == [S.hash_int(12345, 1, 77, int(x)) for x in j]


def test_mulhi_exact():
    rng = np.random.default_rng(0)
    h = rng.integers(0, 2 ** 63, size=2000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 2000, dtype=np.uint64)
    for n in [1, 2, 3, 43878, 131584, 5_000_000, 2 ** 32 - 1]:
        got = S.mulhi_u64_u32(h, n)
        want = [(int(v) * n) >> 64 for v in h]
        assert got.tolist() == want
        assert got.min() >= 0 and got.max() < n


def test_iid_uniformity_chi2():
    n, B = 1000, 1 << 18
    idx = S.iid_indices(0, 0, 3, B, n)
    counts = np.bincount(idx, minlength=n)
    e = B / n
    chi2 = float(((counts - e) ** 2 / e).sum())
    # dof 999: mean 999, sd ~44.7; 6 sd bounds
    assert 999 - 6 * 44.7 < chi2 < 999 + 6 * 44.7
    # different steps and streams give different batches
    assert not np.array_equal(idx[:64], S.iid_indices(0, 0, 4, 64, n))
    assert not np.array_equal(idx[:64], S.iid_indices(0, 1, 3, 64, n))
