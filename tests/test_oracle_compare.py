"""Pins of the oracle's comparison sketches (Definitions 2 and 3) in their
CP forms, of the higher-order count sketch's decompression, and of the two
identities the GPU path uses for them:
* TS (all J_n = J) is FCS folded modulo J (Section 3, item 2);
* HCS, flattened with mode 0 fastest, is FCS under the mode hashes scaled by
  the mixed-radix strides prod_{m<n} J_m (the bins sum_n h_n stride_n are
  exactly the flattened multi-indices (h_0, ..., h_{N-1})).
All CPU, FP64; literal loops over Definitions 2 and 3 are the reference."""
import itertools

import numpy as np
import pytest

import oracle as O


def _ts_loop(T, h, s, J):
    out = np.zeros(J)
    for idx in itertools.product(*[range(n) for n in T.shape]):
        H = sum(int(h[n][idx[n]]) for n in range(T.ndim)) % J
        out[H] += np.prod([int(s[n][idx[n]]) for n in range(T.ndim)]) * T[idx]
    return out


def _hcs_loop(T, h, s, Js):
    out = np.zeros(Js)
    for idx in itertools.product(*[range(n) for n in T.shape]):
        j = tuple(int(h[n][idx[n]]) for n in range(T.ndim))
        out[j] += np.prod([int(s[n][idx[n]]) for n in range(T.ndim)]) * T[idx]
    return out


CP_SHAPES = [([4, 5, 3], 3, 2), ([6, 4], 5, 3), ([3, 2, 4, 2], 4, 2), ([7], 5, 4), ([5, 4, 3], 1, 1)]


@pytest.mark.parametrize("I,J,R", CP_SHAPES)
def test_ts_cp_is_definition_2(I, J, R):
    r = np.random.default_rng(sum(I) + J)
    U = [r.standard_normal((i, R)) for i in I]
    lam = r.standard_normal(R)
    hs, ss = O.hash_tables(31, 1, I, [J] * len(I))
    T = O.cp_full(lam, U)
    want = _ts_loop(T, hs[0], ss[0], J)
    np.testing.assert_allclose(O.ts_dense(T, hs[0], ss[0], J), want, atol=1e-11)
    np.testing.assert_allclose(O.ts_cp(lam, U, hs[0], ss[0], J), want, atol=1e-11)
    # the fold of the FCS (linear convolution) modulo J
    y = O.fcs_cp_conv(lam, U, hs[0], ss[0], [J] * len(I))
    fold = np.zeros(J)
    np.add.at(fold, np.arange(y.size) % J, y)
    np.testing.assert_allclose(fold, want, atol=1e-11)


@pytest.mark.parametrize("I,J,R", [([4, 5, 3], [3, 2, 4], 2), ([6, 4], [5, 3], 3), ([3, 2, 4, 2], [2, 3, 2, 2], 2),
                                   ([7], [4], 3)])
def test_hcs_cp_is_definition_3(I, J, R):
    r = np.random.default_rng(sum(I) + sum(J))
    U = [r.standard_normal((i, R)) for i in I]
    lam = r.standard_normal(R)
    hs, ss = O.hash_tables(32, 1, I, J)
    T = O.cp_full(lam, U)
    want = _hcs_loop(T, hs[0], ss[0], J)
    np.testing.assert_allclose(O.hcs_dense(T, hs[0], ss[0], J), want, atol=1e-11)
    np.testing.assert_allclose(O.hcs_cp(lam, U, hs[0], ss[0], J), want, atol=1e-11)


@pytest.mark.parametrize("I,J", [([4, 5, 3], [3, 2, 4]), ([6, 4], [5, 3]), ([3, 2, 4, 2], [2, 3, 2, 2]), ([9], [4])])
def test_hcs_is_fcs_under_mixed_radix_hashes(I, J):
    r = np.random.default_rng(7 + len(I))
    T = r.standard_normal(I)
    hs, ss = O.hash_tables(33, 1, I, J)
    strides = np.cumprod([1] + list(J[:-1]))
    h2 = [np.asarray(hs[0][n]) * int(strides[n]) for n in range(len(I))]
    J2 = [(int(J[n]) - 1) * int(strides[n]) + 1 for n in range(len(I))]
    assert O.sketch_length(J2) == int(np.prod(J))
    want = _hcs_loop(T, hs[0], ss[0], J)
    np.testing.assert_allclose(O.fcs_dense(T, h2, ss[0], J2), O.vec(want), atol=1e-11)
    # and through the CP route (linear convolution of the scaled count sketches)
    R = 2
    U = [r.standard_normal((i, R)) for i in I]
    np.testing.assert_allclose(O.fcs_cp_conv(None, U, h2, ss[0], J2),
                               O.vec(O.hcs_cp(None, U, hs[0], ss[0], J)), atol=1e-11)


def test_hcs_decompress_is_the_rule():
    r = np.random.default_rng(12)
    I, J, D = [4, 3, 5], [3, 4, 2], 3
    hs, ss = O.hash_tables(34, D, I, J)
    Y = [r.standard_normal(J) for _ in range(D)]
    got = O.hcs_decompress_median(Y, hs, ss, I)
    for idx in itertools.product(*[range(n) for n in I]):
        est = []
        for d in range(D):
            j = tuple(int(hs[d][n][idx[n]]) for n in range(3))
            est.append(np.prod([int(ss[d][n][idx[n]]) for n in range(3)]) * Y[d][j])
        assert got[idx] == pytest.approx(sorted(est)[1], abs=1e-15)
    # a lone entry is recovered exactly from its own sketch
    T = np.zeros(I)
    T[2, 1, 3] = 2.5
    Ys = [O.hcs_dense(T, hs[d], ss[d], J) for d in range(D)]
    assert O.hcs_decompress_median(Ys, hs, ss, I)[2, 1, 3] == pytest.approx(2.5, abs=1e-15)
