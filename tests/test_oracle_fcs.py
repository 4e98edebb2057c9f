"""Pins of the oracle's sketches against what the paper and the mathematics
fix: a hand-worked example, Definition 1 written as a loop, unit impulses,
linearity, the relations to TS (Definition 2) and HCS (Definition 3), the CP
identity of Section 3.1, the Kronecker identity of Section 4.3, and the
independent C brute force."""
import itertools

import numpy as np
import pytest

import oracle as O
import synth
from conftest import read_golden


def _ints(v):
    return [int(x) for x in v]


def _hand():
    g = read_golden("fcs_hand_example.txt")
    I = _ints(g["I"][0])
    J = _ints(g["J"][0])
    h = [np.array(_ints(g["h0"][0])), np.array(_ints(g["h1"][0]))]
    s = [np.array(_ints(g["s0"][0])), np.array(_ints(g["s1"][0]))]
    return g, I, J, h, s


def test_hand_example_dense():
    g, I, J, h, s = _hand()
    T = O.unvec(np.array(_ints(g["A_vec"][0]), dtype=float), I)
    assert O.sketch_length(J) == 3
    np.testing.assert_array_equal(O.fcs_dense(T, h, s, J), _ints(g["A_fcs"][0]))


def test_hand_example_cp():
    g, I, J, h, s = _hand()
    a = np.array(_ints(g["a"][0]), dtype=float)[:, None]
    b = np.array(_ints(g["b"][0]), dtype=float)[:, None]
    want = _ints(g["B_fcs"][0])
    np.testing.assert_array_equal(O.count_sketch(a, h[0], s[0], J[0])[:, 0],
                                  _ints(g["CS0a"][0]))
    np.testing.assert_array_equal(O.count_sketch(b, h[1], s[1], J[1])[:, 0],
                                  _ints(g["CS1b"][0]))
    np.testing.assert_array_equal(O.fcs_dense(O.cp_full(None, [a, b]), h, s, J), want)
    np.testing.assert_allclose(O.fcs_cp_conv(None, [a, b], h, s, J), want, atol=0)
    np.testing.assert_allclose(O.fcs_cp_fft(None, [a, b], h, s, J), want, atol=1e-12)


def _cs_loop(x, h, s, J):
    """Definition 1 as a literal loop."""
    out = [0.0] * J
    for i in range(len(x)):
        out[int(h[i])] += float(s[i]) * float(x[i])
    return np.array(out)


def test_count_sketch_is_definition_1():
    r = np.random.default_rng(0)
    x = r.standard_normal(300)
    h, s = O.hash_pair(1, 0, 0, 300, 37)
    np.testing.assert_allclose(O.count_sketch(x, h, s, 37), _cs_loop(x, h, s, 37),
                               rtol=0, atol=1e-12)
    X = r.standard_normal((300, 4))
    Y = O.count_sketch(X, h, s, 37)
    for c in range(4):
        np.testing.assert_allclose(Y[:, c], _cs_loop(X[:, c], h, s, 37), atol=1e-12)


def test_order_one_fcs_is_count_sketch():
    r = np.random.default_rng(1)
    x = r.standard_normal(500)
    hs, ss = O.hash_tables(3, 1, [500], [61])
    assert O.sketch_length([61]) == 61
    np.testing.assert_allclose(O.fcs_dense(x, hs[0], ss[0], [61]),
                               _cs_loop(x, hs[0][0], ss[0][0], 61), atol=1e-12)


def test_unit_impulses():
    I, J = [4, 3, 5], [3, 4, 2]
    hs, ss = O.hash_tables(17, 1, I, J)
    h, s = hs[0], ss[0]
    for idx in itertools.product(*[range(i) for i in I]):
        T = np.zeros(I)
        T[idx] = 1.0
        y = O.fcs_dense(T, h, s, J)
        H = sum(int(h[n][idx[n]]) for n in range(3))
        S = np.prod([int(s[n][idx[n]]) for n in range(3)])
        want = np.zeros(O.sketch_length(J))
        want[H] = S
        np.testing.assert_array_equal(y, want)


def test_linearity():
    r = np.random.default_rng(2)
    I, J = [6, 5, 4], [5, 5, 3]
    hs, ss = O.hash_tables(5, 1, I, J)
    A, B = r.standard_normal(I), r.standard_normal(I)
    lhs = O.fcs_dense(2.5 * A - 0.75 * B, hs[0], ss[0], J)
    rhs = 2.5 * O.fcs_dense(A, hs[0], ss[0], J) - 0.75 * O.fcs_dense(B, hs[0], ss[0], J)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def _ts_loop(T, h, s, J):
    """Definition 2 as a literal loop: 1-based bin (sum h - N) mod J + 1, here
    with 0-based h (h' = h + 1), i.e. 0-based bin (sum h') mod J."""
    out = np.zeros(J)
    N = T.ndim
    for idx in itertools.product(*[range(n) for n in T.shape]):
        h1 = [int(h[n][idx[n]]) + 1 for n in range(N)]      # 1-based hashes
        bin1 = (sum(h1) - N) % J + 1                        # the paper's formula
        out[bin1 - 1] += np.prod([int(s[n][idx[n]]) for n in range(N)]) * T[idx]
    return out


def _hcs_loop(T, h, s, Js):
    out = np.zeros(Js)
    for idx in itertools.product(*[range(n) for n in T.shape]):
        j = tuple(int(h[n][idx[n]]) for n in range(T.ndim))
        out[j] += np.prod([int(s[n][idx[n]]) for n in range(T.ndim)]) * T[idx]
    return out


def test_ts_is_fold_of_fcs():
    """With equal hash functions and all J_n = J, TS (Definition 2) is FCS
    folded modulo J: the two differ only by the modulo (Section 3, item 2)."""
    r = np.random.default_rng(3)
    I, J = [5, 4, 6], 4
    hs, ss = O.hash_tables(8, 1, I, [J] * 3)
    T = r.standard_normal(I)
    y = O.fcs_dense(T, hs[0], ss[0], [J] * 3)
    fold = np.zeros(J)
    for m, v in enumerate(y):
        fold[m % J] += v
    ts = _ts_loop(T, hs[0], ss[0], J)
    np.testing.assert_allclose(fold, ts, atol=1e-12)
    np.testing.assert_allclose(O.ts_dense(T, hs[0], ss[0], J), ts, atol=1e-12)


def test_hcs_antidiagonal_sum_is_fcs():
    r = np.random.default_rng(4)
    I, J = [4, 5, 3], [3, 4, 2]
    hs, ss = O.hash_tables(9, 1, I, J)
    T = r.standard_normal(I)
    hcs = _hcs_loop(T, hs[0], ss[0], J)
    np.testing.assert_allclose(O.hcs_dense(T, hs[0], ss[0], J), hcs, atol=1e-12)
    want = np.zeros(O.sketch_length(J))
    for j in itertools.product(*[range(n) for n in J]):
        want[sum(j)] += hcs[j]
    np.testing.assert_allclose(O.fcs_dense(T, hs[0], ss[0], J), want, atol=1e-12)


@pytest.mark.parametrize("I,J,R", [([3, 4], [2, 3], 2), ([5, 4, 3], [4, 2, 3], 3),
                                   ([3, 2, 4, 2], [2, 3, 2, 2], 4),
                                   ([4, 3, 2, 3, 2], [2, 2, 3, 2, 2], 2),
                                   ([7], [5], 3)])
def test_cp_routes_equal_brute_force(I, J, R):
    r = np.random.default_rng(sum(I))
    U = [r.standard_normal((i, R)) for i in I]
    lam = r.standard_normal(R)
    hs, ss = O.hash_tables(13, 2, I, J)
    for d in range(2):
        want = O.fcs_dense(O.cp_full(lam, U), hs[d], ss[d], J)
        np.testing.assert_allclose(O.fcs_cp_conv(lam, U, hs[d], ss[d], J), want,
                                   atol=1e-12)
        Jt = O.sketch_length(J)
        for L in (Jt, Jt + 1, 2 * Jt, 1 << int(np.ceil(np.log2(Jt)))):
            np.testing.assert_allclose(O.fcs_cp_fft(lam, U, hs[d], ss[d], J, L), want,
                                       atol=1e-11)


def test_cp_config_cp100_brute_force():
    """The 10^6-entry tensor of the order-3, I_n = 100, R = 10 workload:
    FFT route == direct convolution == brute force (Section 3.1)."""
    cfg = synth.CP100
    U = cfg.factors()
    hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
    T = O.cp_full(None, U)
    assert T.size == 10**6
    for d in range(cfg.D):
        want = O.fcs_dense(T, hs[d], ss[d], cfg.J)
        a = O.fcs_cp_conv(None, U, hs[d], ss[d], cfg.J)
        b = O.fcs_cp_fft(None, U, hs[d], ss[d], cfg.J, 256)
        scale = np.linalg.norm(want)
        assert np.linalg.norm(a - want) <= 1e-13 * scale
        assert np.linalg.norm(b - want) <= 1e-12 * scale


def test_c_brute_force_matches_numpy():
    r = np.random.default_rng(5)
    for I, J in [([7], [5]), ([9, 4], [3, 6]), ([5, 3, 4], [4, 4, 2]),
                 ([3, 2, 4, 3], [2, 3, 2, 4])]:
        T = r.standard_normal(I).astype(np.float32)
        D = 3
        hs, ss = O.hash_tables(21, D, I, J)
        Jt = O.sketch_length(J)
        want = np.stack([O.fcs_dense(T, hs[d], ss[d], J) for d in range(D)])
        got = O.dense_rows(O.vec(T), I, hs, ss, Jt)
        np.testing.assert_allclose(got, want, atol=1e-12)
        # sampled rows add up to the whole sketch (linearity over slabs)
        rows = int(np.prod(I[1:]))
        half = rows // 2
        parts = O.dense_rows(O.vec(T), I, hs, ss, Jt, 0, half) + \
            O.dense_rows(O.vec(T), I, hs, ss, Jt, half, rows)
        np.testing.assert_allclose(parts, want, atol=1e-12)


def test_coo_matches_dense_and_c():
    r = np.random.default_rng(6)
    I, J = [6, 5, 4], [4, 5, 3]
    T = r.standard_normal(I).astype(np.float32)
    T[r.random(I) < 0.6] = 0
    lin = np.flatnonzero(O.vec(T))
    idx = np.stack(np.unravel_index(lin, I, order="F")).astype(np.int32)
    val = O.vec(T)[lin]
    # duplicate a few coordinates with split values: duplicates must add
    dup = lin[:5]
    idx2 = np.concatenate([idx, idx[:, :5]], axis=1)
    val2 = np.concatenate([val, np.zeros(5, np.float32)])
    val2[:5] = val[:5] * 0.25
    val2[-5:] = val[:5] * 0.75
    hs, ss = O.hash_tables(31, 2, I, J)
    Jt = O.sketch_length(J)
    for d in range(2):
        want = O.fcs_dense(T.astype(np.float64), hs[d], ss[d], J)
        np.testing.assert_allclose(O.fcs_coo(idx, val, hs[d], ss[d], J), want, atol=1e-12)
        np.testing.assert_allclose(O.fcs_coo(idx2, val2, hs[d], ss[d], J), want, atol=1e-6)
    got = O.coo(idx2, val2, I, hs, ss, Jt)
    want = np.stack([O.fcs_coo(idx2, val2, hs[d], ss[d], J) for d in range(2)])
    np.testing.assert_allclose(got, want, atol=1e-12)
    del dup


def test_kronecker_identity():
    """Section 4.3: FCS of the order-4 tensor A[i1,i2] B[i3,i4] equals the
    linear convolution of the order-2 sketches of A and B."""
    r = np.random.default_rng(7)
    A = r.uniform(-5, 5, (5, 4))
    B = r.uniform(-5, 5, (3, 6))
    J = [4, 4, 4, 4]
    hs, ss = O.hash_tables(41, 1, [5, 4, 3, 6], J)
    T4 = np.einsum("ab,cd->abcd", A, B)
    want = O.fcs_dense(T4, hs[0], ss[0], J)
    assert O.sketch_length(J) == 4 * 4 - 3
    np.testing.assert_allclose(O.kron_fcs(A, B, hs[0], ss[0], J), want, atol=1e-10)


def test_kronecker_decompress_reading():
    """The paper's 1-based decompression index mod(h1+h2+h3+h4-4, 4J-3)+1
    never wraps, so the 0-based entry is s1 s2 s3 s4 FCS[sum h]."""
    r = np.random.default_rng(8)
    I, J = [3, 4, 2, 5], [6, 6, 6, 6]
    hs, ss = O.hash_tables(42, 1, I, J)
    y = r.standard_normal(O.sketch_length(J))
    got = O.kron_decompress(y, hs[0], ss[0], I)
    for idx in itertools.product(*[range(i) for i in I]):
        h1 = [int(hs[0][n][idx[n]]) + 1 for n in range(4)]
        pos = (sum(h1) - 4) % (4 * 6 - 3) + 1
        S = np.prod([int(ss[0][n][idx[n]]) for n in range(4)])
        assert got[idx] == S * y[pos - 1]
