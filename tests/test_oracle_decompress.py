"""Pins of the oracle's decompression and contraction compression
(Section 4.3).

* ``decompress_median`` against the paper's 1-based rule
  s1 s2 s3 s4 FCS[mod(h1+h2+h3+h4-4, 4J-3)+1] written as loops over every
  entry and sketch, with the median taken as the order statistic of the
  sorted estimates (mean of the middle pair for even D);
* a tensor with one nonzero entry is recovered exactly at that entry;
* at hash lengths far above the entry count, almost every entry of a
  Kronecker product comes back exactly (collisions are rare and the median
  discards them);
* ``contraction_fcs`` equals the FCS of the materialised contraction.
"""
import itertools

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("D", [1, 2, 3, 4])
def test_decompress_median_matches_paper_rule_by_loops(D):
    I, J = [3, 2, 4, 2], [5, 5, 5, 5]
    hs, ss = O.hash_tables(51, D, I, J)
    Jt = 4 * 5 - 3
    Y = np.random.default_rng(9).standard_normal((D, Jt))
    got = O.decompress_median(Y, hs, ss, I)
    assert got.shape == tuple(I)
    for idx in itertools.product(*[range(i) for i in I]):
        est = []
        for d in range(D):
            h1 = [int(hs[d][n][idx[n]]) + 1 for n in range(4)]    # the paper's 1-based hashes
            pos = (sum(h1) - 4) % Jt + 1
            sign = 1
            for n in range(4):
                sign *= int(ss[d][n][idx[n]])
            est.append(sign * Y[d][pos - 1])
        est.sort()
        m = est[(D - 1) // 2] if D % 2 else 0.5 * (est[D // 2 - 1] + est[D // 2])
        assert got[idx] == m


def test_decompress_recovers_a_lone_entry():
    I, J, D = (6, 5, 7), (16, 16, 16), 5
    hs, ss = O.hash_tables(52, D, I, J)
    T = np.zeros(I)
    T[4, 1, 3] = -2.75
    Y = np.stack([O.fcs_dense(T, hs[d], ss[d], J) for d in range(D)])
    R = O.decompress_median(Y, hs, ss, I)
    assert R[4, 1, 3] == -2.75
    # elsewhere an estimate is nonzero only where its bin collides with the
    # entry's; the median is zero unless most sketches collide there
    assert np.count_nonzero(R) <= 5


def test_decompress_kronecker_is_near_exact_at_long_hashes():
    r = np.random.default_rng(10)
    A = r.uniform(-5, 5, (3, 4))
    B = r.uniform(-5, 5, (2, 5))
    I, J, D = (3, 4, 2, 5), (512, 512, 512, 512), 5
    hs, ss = O.hash_tables(53, D, I, J)
    Y = np.stack([O.kron_fcs(A, B, hs[d], ss[d], J) for d in range(D)])
    R = O.decompress_median(Y, hs, ss, I)
    T = np.einsum("ab,cd->abcd", A, B)
    exact = np.isclose(R, T, rtol=0, atol=1e-9)
    assert exact.mean() >= 0.95
    assert np.linalg.norm(R - T) <= 0.2 * np.linalg.norm(T)


def test_contraction_sketch_is_fcs_of_the_contraction():
    r = np.random.default_rng(11)
    Lc = 4
    A = r.uniform(0, 10, (3, 4, Lc))
    B = r.uniform(0, 10, (Lc, 2, 5))
    I, J = (3, 4, 2, 5), (4, 5, 3, 6)
    hs, ss = O.hash_tables(54, 2, I, J)
    C = np.einsum("abl,lcd->abcd", A, B)
    for d in range(2):
        np.testing.assert_allclose(O.contraction_fcs(A, B, hs[d], ss[d], J),
                                   O.fcs_dense(C, hs[d], ss[d], J), rtol=0, atol=1e-9)
    # one shared index is the Kronecker product
    np.testing.assert_allclose(O.contraction_fcs(A[:, :, :1], B[:1], hs[0], ss[0], J),
                               O.kron_fcs(A[:, :, 0], B[0], hs[0], ss[0], J), rtol=0, atol=1e-12)


def test_decompress_at_equals_the_whole_tensor():
    I, J, D = (5, 3, 4), (7, 6, 5), 4
    hs, ss = O.hash_tables(55, D, I, J)
    Y = np.random.default_rng(12).standard_normal((D, O.sketch_length(J)))
    full = O.decompress_median(Y, hs, ss, I)
    grid = np.indices(I).reshape(3, -1)
    np.testing.assert_array_equal(O.decompress_at(Y, hs, ss, grid), full.reshape(-1))
