"""Pins of the oracle's hash family (the reading of 'two 2-wise independent
hash functions' in Definitions 1-4): the published SplitMix64 sequence, the
range map, and statistical sanity of h and s."""
import numpy as np
import pytest

import oracle as O
from conftest import read_golden


def test_splitmix64_known_answers():
    # the golden file holds 'seed index output'; the parser keys on the seed
    kat = read_golden("splitmix64_kat.txt")
    seqs = {}
    for key, vals in kat.items():
        for idx, val in vals:
            seqs.setdefault(int(key), {})[int(idx)] = int(val)
    assert seqs[1234567] and seqs[0]
    for seed, want in seqs.items():
        got = O.splitmix64_sequence(seed, max(want) + 1)
        for i, v in want.items():
            assert got[i] == v, (seed, i)


def test_vectorised_mix_matches_scalar():
    x = np.array([0, 1, 2**63 - 1, 2**64 - 1, 0x9E3779B97F4A7C15, 123456789],
                 dtype=np.uint64)
    got = O.fcs_oracle._mix64_array(x)
    for a, b in zip(x.tolist(), got.tolist()):
        assert O.mix64(int(a)) == int(b)


def test_range_map_and_sign_bit():
    seed, d, n, I, J = 99, 3, 2, 257, 1000
    h, s = O.hash_pair(seed, d, n, I, J)
    key = O.hash_key(seed, d, n)
    for i in range(I):
        y = O.mix64((key + i) & O.MASK64)
        assert h[i] == ((y >> 32) * J) >> 32
        assert s[i] == (1 if y % 2 == 0 else -1)
    assert h.min() >= 0 and h.max() < J


@pytest.mark.parametrize("J", [1, 2, 64, 4096, 16384])
def test_h_in_range(J):
    h, s = O.hash_pair(5, 0, 0, 5000, J)
    assert h.dtype == np.int64 and s.dtype == np.int8
    assert h.min() >= 0 and h.max() <= J - 1
    assert set(np.unique(s).tolist()) <= {-1, 1}


def test_h_uniform_chi2_and_s_balanced():
    J, I = 64, 200_000
    h, s = O.hash_pair(2001, 1, 2, I, J)
    counts = np.bincount(h, minlength=J)
    chi2 = ((counts - I / J) ** 2 / (I / J)).sum()
    # 63 degrees of freedom: mean 63, sd ~11.2; 130 is ~6 sd out
    assert chi2 < 130
    assert abs(s.astype(np.int64).sum()) < 5 * np.sqrt(I)


def test_streams_independent_across_sketch_and_mode():
    I, J = 100_000, 128
    hs, ss = O.hash_tables(7, 3, [I, I], [J, J])
    streams = [(d, n) for d in range(3) for n in range(2)]
    for a in range(len(streams)):
        for b in range(a + 1, len(streams)):
            da, na = streams[a]
            db, nb = streams[b]
            sa = ss[da][na].astype(np.float64)
            sb = ss[db][nb].astype(np.float64)
            assert abs(np.mean(sa * sb)) < 5 / np.sqrt(I)
            coll = np.mean(hs[da][na] == hs[db][nb])
            assert abs(coll - 1 / J) < 5 * np.sqrt(1 / J / I)


def test_pairwise_collision_rate():
    I, J = 4000, 256
    h, _ = O.hash_pair(11, 0, 0, I, J)
    same = (h[:, None] == h[None, :])
    rate = (same.sum() - I) / (I * (I - 1))
    assert abs(rate - 1 / J) < 0.1 / J


def test_tables_deterministic_and_seed_sensitive():
    a = O.hash_tables(3, 2, [50, 60], [8, 9])
    b = O.hash_tables(3, 2, [50, 60], [8, 9])
    c = O.hash_tables(4, 2, [50, 60], [8, 9])
    for d in range(2):
        for n in range(2):
            assert np.array_equal(a[0][d][n], b[0][d][n])
            assert np.array_equal(a[1][d][n], b[1][d][n])
    assert not all(np.array_equal(a[0][d][n], c[0][d][n])
                   for d in range(2) for n in range(2))
