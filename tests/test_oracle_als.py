"""Pin of the oracle's sketched alternating least squares (Section 4.1.2, ALS):

* the update of one mode, given the exact unfolding-times-Khatri-Rao product
  of a rank-R tensor and its true other factors, returns exactly the planted
  factor and weights (the closed form of a least-squares step on an exact
  model);
* from random starting factors, sketched ALS recovers the planted factors
  (up to order and sign) and weights of an asymmetric tensor with
  orthonormal factors; the sketch error bounds the accuracy (J_n = 4096,
  D = 3 here)."""
import numpy as np

import oracle as O
import synth


def test_als_step_is_exact_on_exact_products():
    I, w = 7, np.array([2.5, -1.5, 0.75])
    _, (A, B, C) = synth.asymmetric_cp_tensor(5, I, w)
    # a non-orthonormal third factor makes the Gram product non-diagonal
    C = C + 0.3 * synth.rng(6).standard_normal(C.shape)
    T = np.einsum("r,ir,jr,kr->ijk", w, A, B, C)
    M = np.stack([np.einsum("ijk,j,k->i", T, B[:, r], C[:, r]) for r in range(3)], axis=1)
    lam, U = O.als_step(M, [B, C])
    # A diag(w) = U diag(lam) with unit columns: lam = |w|, U = A sign(w)
    np.testing.assert_allclose(lam, np.abs(w), rtol=1e-12)
    np.testing.assert_allclose(U, A * np.sign(w), atol=1e-12)


def test_oracle_als_recovers_planted_factors():
    I, R, D, J, iters = 16, 3, 3, 4096, 15
    w = np.array([3.0, 2.0, 1.0])
    Tv, F = synth.asymmetric_cp_tensor(12, I, w)
    T = Tv.reshape((I, I, I), order="F")
    hs, ss = O.hash_tables(22, D, (I, I, I), (J, J, J))
    Y = np.stack([O.fcs_dense(T, hs[d], ss[d], (J, J, J)) for d in range(D)])
    lam, G = O.als(Y, hs, ss, (J, J, J), synth.als_init(32, I, R), iters)
    ov = [np.abs(G[n].T @ F[n]) for n in range(3)]          # |<recovered k, planted r>|
    match = ov[0].argmax(axis=1)
    assert sorted(match.tolist()) == [0, 1, 2]
    for n in range(3):
        assert np.all(ov[n][np.arange(R), match] >= 0.99), ov[n]
    assert np.all(np.abs(lam - w[match]) <= 0.08 * w[match]), (lam, match)
    for n in range(3):
        assert np.allclose(np.linalg.norm(G[n], axis=0), 1.0)
