"""Pins of the oracle's sketched contractions: the inner-product estimator of
Proposition 1 (exact unbiasedness over every hash function on tiny shapes,
statistical unbiasedness over seeds), the median, the T(I, u, v) forms of
Section 4.1 against literal inner products, and the error trend of
Corollary 1."""
import itertools

import numpy as np
import pytest

import oracle as O


def test_median_order_statistics():
    x = np.array([3.0, -1.0, 7.0, 2.0, 5.0])
    assert O.median(x) == 3.0
    y = np.array([4.0, -2.0, 9.0, 1.0])
    assert O.median(y) == (1.0 + 4.0) / 2
    M = np.array([[1.0, 5.0], [3.0, 2.0], [2.0, 9.0], [8.0, 0.0]])
    np.testing.assert_array_equal(O.median(M, axis=0), [2.5, 3.5])


def _all_hash_functions(I, J):
    """Every (h, s) pair for one mode: J^I choices of h times 2^I of s."""
    for hv in itertools.product(range(J), repeat=I):
        for sv in itertools.product((1, -1), repeat=I):
            yield np.array(hv), np.array(sv)


def _enumerate(M, Nt, J):
    """Inner products of the FCS and TS sketches of M and Nt under every
    combination of per-mode hash functions (I_n = 2, three modes)."""
    per_mode = list(_all_hash_functions(2, J))
    f_vals, t_vals = [], []
    for combo in itertools.product(per_mode, repeat=3):
        h = [c[0] for c in combo]
        s = [c[1] for c in combo]
        f_vals.append(np.dot(O.fcs_dense(M, h, s, [J] * 3), O.fcs_dense(Nt, h, s, [J] * 3)))
        t_vals.append(np.dot(O.ts_dense(M, h, s, J), O.ts_dense(Nt, h, s, J)))
    return np.array(f_vals), np.array(t_vals)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("J", [2, 3])
def test_inner_product_exactly_unbiased(seed, J):
    """Proposition 1: <FCS(M), FCS(N)> is an unbiased estimate of <M, N>.
    Enumerating every hash function of every mode gives the exact
    expectation; integer tensors keep every value exact."""
    r = np.random.default_rng(seed)
    I = (2, 2, 2)
    M = r.integers(-3, 4, I).astype(np.float64)
    Nt = M.copy() if seed == 0 else r.integers(-3, 4, I).astype(np.float64)
    f_vals, t_vals = _enumerate(M, Nt, J)
    assert f_vals.size == (J * J * 4) ** 3
    assert abs(np.mean(f_vals) - np.sum(M * Nt)) < 1e-9
    assert abs(np.mean(t_vals) - np.sum(M * Nt)) < 1e-9


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_variance_not_worse_than_ts_at_J3(seed):
    """Proposition 1's variance comparison under equal hash functions, exact
    over all hash functions at J = 3."""
    r = np.random.default_rng(seed)
    I = (2, 2, 2)
    M = r.integers(-3, 4, I).astype(np.float64)
    Nt = M.copy() if seed % 2 == 0 else r.integers(-3, 4, I).astype(np.float64)
    f_vals, t_vals = _enumerate(M, Nt, 3)
    assert np.var(f_vals) <= np.var(t_vals)


def test_variance_comparison_can_fail_at_J2():
    """Reading recorded for Proposition 1: with J = 2 (mod-2 folding) and
    fully random hash functions, the FCS variance exceeds the TS variance for
    some tensors, so the inequality is not universal; unbiasedness still
    holds exactly (previous test)."""
    r = np.random.default_rng(0)
    M = r.integers(-3, 4, (2, 2, 2)).astype(np.float64)
    f_vals, t_vals = _enumerate(M, M, 2)
    assert np.mean(f_vals) == np.sum(M * M)
    assert np.var(f_vals) > np.var(t_vals)


def test_inner_product_unbiased_over_seeds():
    """Statistical check with the SplitMix64 family: the mean over K seeds is
    within 5 standard errors of <M, N>."""
    r = np.random.default_rng(4)
    I, J = [6, 5, 4], [4, 4, 4]
    M = r.standard_normal(I)
    Nt = M + 0.5 * r.standard_normal(I)
    truth = float(np.sum(M * Nt))
    K = 3000
    vals = np.empty(K)
    for k in range(K):
        hs, ss = O.hash_tables(10_000 + k, 1, I, J)
        vals[k] = np.dot(O.fcs_dense(M, hs[0], ss[0], J), O.fcs_dense(Nt, hs[0], ss[0], J))
    se = vals.std(ddof=1) / np.sqrt(K)
    assert abs(vals.mean() - truth) <= 5 * se


def test_inner_median_shapes():
    r = np.random.default_rng(5)
    a, b = r.standard_normal((5, 11)), r.standard_normal((5, 11))
    med, per_d = O.inner_median(a, b)
    np.testing.assert_allclose(per_d, [np.dot(a[d], b[d]) for d in range(5)])
    assert med == np.sort(per_d)[2]


def _fcs_rank1(vecs, h, s, J):
    return O.fcs_dense(O.cp_full(None, [np.asarray(v)[:, None] for v in vecs]), h, s, J)


@pytest.mark.parametrize("free", [0, 1, 2])
def test_contract_free_equals_literal_inner_products(free):
    """Section 4.1: entry i of the T(I, u, v) estimate is <FCS(T), FCS(e_i o u o v)>."""
    r = np.random.default_rng(10 + free)
    I, J = [5, 4, 6], [4, 3, 5]
    T = r.standard_normal(I)
    hs, ss = O.hash_tables(77, 1, I, J)
    h, s = hs[0], ss[0]
    y = O.fcs_dense(T, h, s, J)
    others = [n for n in range(3) if n != free]
    vecs = [r.standard_normal(I[n]) for n in others]
    got = O.contract_free(y, h, s, J, free, vecs)
    for i in range(I[free]):
        parts = [None] * 3
        e = np.zeros(I[free])
        e[i] = 1
        parts[free] = e
        for k, n in enumerate(others):
            parts[n] = vecs[k]
        want = np.dot(y, _fcs_rank1(parts, h, s, J))
        assert abs(got[i] - want) < 1e-10


@pytest.mark.parametrize("L_extra", [0, 1, 17])
def test_contract_free_fft_shortcut(L_extra):
    """The FFT shortcut of Section 4.1 (z = F^-1(F(y) conj F(CS u) conj F(CS v)),
    entry s_0(i) z(h_0(i))) equals the by-definition estimate for any L >= J~."""
    r = np.random.default_rng(20)
    I, J = [7, 5, 6], [5, 4, 6]
    T = r.standard_normal(I)
    hs, ss = O.hash_tables(78, 1, I, J)
    y = O.fcs_dense(T, hs[0], ss[0], J)
    u, v = r.standard_normal(5), r.standard_normal(6)
    L = O.sketch_length(J) + L_extra
    a = O.contract_free_fft(y, hs[0], ss[0], J, L, [u, v])
    b = O.contract_free(y, hs[0], ss[0], J, 0, [u, v])
    np.testing.assert_allclose(a, b, atol=1e-10)


def test_contract_full_equals_literal():
    r = np.random.default_rng(30)
    I, J = [4, 5, 3], [3, 4, 4]
    T = r.standard_normal(I)
    hs, ss = O.hash_tables(79, 1, I, J)
    y = O.fcs_dense(T, hs[0], ss[0], J)
    vecs = [r.standard_normal(i) for i in I]
    want = np.dot(y, _fcs_rank1(vecs, hs[0], ss[0], J))
    assert abs(O.contract_full(y, hs[0], ss[0], J, vecs) - want) < 1e-10


def test_contract_error_shrinks_with_hash_length():
    """Corollary 1: the squared error of the sketched T(I, u, v) scales like
    ||T||_F^2 / J; quadrupling J should cut the mean squared error clearly."""
    r = np.random.default_rng(40)
    I, R = 30, 3
    U = [r.standard_normal((I, R)) for _ in range(3)]
    T = O.cp_full(None, U)
    u, v = r.standard_normal(I), r.standard_normal(I)
    exact = U[0] @ ((U[1].T @ u) * (U[2].T @ v))
    mse = {}
    for J in (32, 512):
        errs = []
        for k in range(40):
            hs, ss = O.hash_tables(500 + k, 1, [I] * 3, [J] * 3)
            y = O.fcs_dense(T, hs[0], ss[0], [J] * 3)
            est = O.contract_free(y, hs[0], ss[0], [J] * 3, 0, [u, v])
            errs.append(np.mean((est - exact) ** 2))
        mse[J] = np.mean(errs)
    assert mse[512] < mse[32] / 4


def test_median_of_sketches_closer_than_single():
    """The median over D independent sketches (Section 4) concentrates."""
    r = np.random.default_rng(50)
    I = [20, 20, 20]
    J = [16, 16, 16]
    M = r.standard_normal(I)
    truth = float(np.sum(M * M))
    single, med = [], []
    for k in range(60):
        hs, ss = O.hash_tables(900 + k, 9, I, J)
        Y = np.stack([O.fcs_dense(M, hs[d], ss[d], J) for d in range(9)])
        m, per_d = O.inner_median(Y, Y)
        single.append(abs(per_d[0] - truth))
        med.append(abs(m - truth))
    assert np.mean(med) < np.mean(single)
