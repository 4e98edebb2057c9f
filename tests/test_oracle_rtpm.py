"""Pin of the oracle's sketched robust tensor power method (Section 4.1.1,
RTPM): on an orthogonally decomposable symmetric tensor
sum_r w_r a_r o a_r o a_r (a_r orthonormal, no noise) it must find the planted
components, in decreasing order of weight, with eigenvalues close to the
weights.  The sketch error bounds the accuracy (J_n = 2048, D = 3 here)."""
import numpy as np

import oracle as O
import synth


def test_oracle_rtpm_recovers_planted_components():
    I, R, D, L, iters, J = 20, 3, 3, 5, 12, 2048
    w = np.array([3.0, 2.0, 1.0])
    Tv, A = synth.symmetric_cp_tensor(11, I, w)
    T = Tv.reshape((I, I, I), order="F")
    hs, ss = O.hash_tables(21, D, (I, I, I), (J, J, J))
    Y = np.stack([O.fcs_dense(T, hs[d], ss[d], (J, J, J)) for d in range(D)])
    lam, U = O.rtpm(Y, hs, ss, (J, J, J), R, synth.rtpm_starts(31, R, L, I), iters)
    overlap = np.abs(U @ A)                       # |<u_k, a_r>|
    assert list(overlap.argmax(axis=1)) == [0, 1, 2]
    assert np.all(overlap.max(axis=1) >= 0.99), overlap
    assert np.all(np.abs(lam - w) <= 0.08 * w), lam
    # unit components
    assert np.allclose(np.linalg.norm(U, axis=1), 1.0)


def test_oracle_rank1_sketch_is_fcs_of_outer_product():
    # fcs_rank1 is the FCS of the materialised rank-1 tensor (Section 3.1)
    I, J = (5, 4, 6), (3, 4, 5)
    hs, ss = O.hash_tables(3, 1, I, J)
    v = [synth.rng(4, n).standard_normal(I[n]) for n in range(3)]
    T = np.einsum("i,j,k->ijk", *v)
    assert np.allclose(O.fcs_rank1(v, hs[0], ss[0], J), O.fcs_dense(T, hs[0], ss[0], J))


def test_oracle_asymmetric_rtpm_recovers_planted_components():
    # alternating rank-1 updates on sum_r w_r a_r o b_r o c_r with
    # orthonormal factors: components in weight order, all three modes
    I, R, D, L, iters, J = 20, 3, 3, 4, 10, 2048
    w = np.array([3.0, 2.0, 1.0])
    Tv, F = synth.asymmetric_cp_tensor(14, I, w)
    T = Tv.reshape((I, I, I), order="F")
    hs, ss = O.hash_tables(24, D, (I, I, I), (J, J, J))
    Y = np.stack([O.fcs_dense(T, hs[d], ss[d], (J, J, J)) for d in range(D)])
    lam, X = O.rtpm_asym(Y, hs, ss, (J, J, J), R, synth.rtpm_asym_starts(34, R, L, I), iters)
    for n in range(3):
        overlap = np.abs(X[n] @ F[n])
        assert list(overlap.argmax(axis=1)) == [0, 1, 2]
        assert np.all(overlap.max(axis=1) >= 0.99), (n, overlap)
        assert np.allclose(np.linalg.norm(X[n], axis=1), 1.0)
    assert np.all(np.abs(lam - w) <= 0.08 * w), lam
