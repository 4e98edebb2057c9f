"""Plain FP64 CPU oracle for fast count sketch (FCS).

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``, by the
``smoke()`` check of ``__graft_entry__`` and by the CPU-baseline leg of
``bench.py``.  The product path (the HIP library and its Python binding) never
imports, links or calls anything under ``oracle/``, and this module imports
nothing from the product path.

Everything here is written from the paper (Cao and Liu, "Efficient Tensor
Contraction via Fast Count Sketch", arXiv 2106.13062) in its own order and
notation, with 0-based indices:

* mode sizes I_n, hash lengths J_n, n = 0..N-1;
* J~ = sum_n J_n - N + 1 (Definition 4);
* the bin of the multi-index (i_0..i_{N-1}) is H = sum_n h_n(i_n) in [0, J~),
  which is the paper's 1-based h_{N+1} = sum h_n - N + 1 shifted down by one;
* its sign is S = prod_n s_n(i_n);
* vec(T) is column-major: mode 0 varies fastest (Section 2.1).

All arithmetic is float64 (inputs given in float32 are upcast first).  Where
the method reaches a result that has a plain definition, the function below is
that definition written out; library primitives used as single steps are
``numpy.bincount`` / ``numpy.add.at`` (scatter-add), ``numpy.convolve``,
``numpy.correlate``, ``numpy.fft`` and ``numpy.median``.

Parity status of each function (what pins it is in ``tests/test_oracle_*.py``):

* ``hash_tables``        pinned by the published SplitMix64 known-answer
                          sequence plus statistical checks; the *choice* of
                          hash family is a reading (the paper only asks for
                          2-wise independence) and is otherwise parity unpinned.
* ``count_sketch``       pinned by an explicit loop over Definition 1.
* ``fcs_dense``/``fcs_coo`` pinned by a hand-worked example, unit impulses,
                          N = 1 == count sketch, the TS fold and HCS
                          anti-diagonal relations, and linearity.
* ``fcs_cp_conv``/``fcs_cp_fft`` pinned against ``fcs_dense`` of the
                          materialised CP tensor (the identity of Section 3.1).
* ``inner`` / ``median`` pinned by exact enumeration of all hash functions on
                          tiny shapes (Proposition 1 unbiasedness) and by the
                          order-statistic definition of the median.
* ``contract_free``      pinned against the literal inner product with the
                          brute-force sketch of e_i o u o v (Section 4.1).
* ``kron_fcs``           pinned against ``fcs_dense`` of the materialised
                          order-4 tensor (Section 4.3).
* ``contraction_fcs``    pinned against ``fcs_dense`` of the materialised
                          contraction (Section 4.3).
* ``ts_cp`` / ``hcs_cp`` pinned against ``ts_dense`` / ``hcs_dense`` of the
                          materialised CP tensor (Definitions 2 and 3; those
                          two are pinned by explicit loops), ``ts_cp`` also
                          against the fold of ``fcs_cp_conv``.
* ``hcs_decompress_median`` pinned by the rule written as explicit loops and
                          by exact recovery of a lone entry.
* ``decompress_median``  pinned by the paper's 1-based decompression rule
                          written as explicit loops, by the order-statistic
                          median, by exact recovery of a lone entry and by
                          near-exact recovery at long hash lengths.
* ``rtpm``               pinned by recovering the planted components and
                          weights of an orthogonally decomposable symmetric
                          tensor (the setting of the RTPM experiments).
* ``rtpm_asym``          pinned by recovering the planted components and
                          weights of an asymmetric tensor with orthonormal
                          factors.
* ``als``                pinned by recovering the planted factors and
                          weights of an asymmetric tensor with orthonormal
                          factors (the setting of the ALS experiment), and by
                          the plain ALS step it reduces to when the
                          contractions are exact.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Hash functions (Definitions 1-4 ask for 2-wise independent pairs h_n, s_n;
# the family is not specified).  Reading used here: one SplitMix64 stream per
# (sketch d, mode n), keyed from a single plan seed.
#   mix(x)    = SplitMix64 finaliser of (x + golden gamma), all mod 2^64
#   key(d, n) = mix(mix(seed) + d * 2^16 + n)
#   y         = mix(key(d, n) + i)
#   h_n(i)    = ((y >> 32) * J_n) >> 32      (Lemire multiply-shift range map)
#   s_n(i)    = +1 if the low bit of y is 0, else -1
# SplitMix64: G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom
# number generators", OOPSLA 2014.
# ---------------------------------------------------------------------------
MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MIX_C1 = 0xBF58476D1CE4E5B9
MIX_C2 = 0x94D049BB133111EB


def mix64(x: int) -> int:
    """SplitMix64 output for a generator whose state is ``x`` before the step."""
    z = (x + GOLDEN_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * MIX_C1) & MASK64
    z = ((z ^ (z >> 27)) * MIX_C2) & MASK64
    return z ^ (z >> 31)


def _mix64_array(x: np.ndarray) -> np.ndarray:
    """Same as ``mix64`` on a uint64 array (numpy wraps mod 2^64)."""
    x = x.astype(np.uint64, copy=False)
    z = x + np.uint64(GOLDEN_GAMMA)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX_C1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX_C2)
    return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of a SplitMix64 generator seeded with ``seed``."""
    out, state = [], seed & MASK64
    for _ in range(count):
        out.append(mix64(state))
        state = (state + GOLDEN_GAMMA) & MASK64
    return out


def hash_key(seed: int, d: int, n: int) -> int:
    return mix64((mix64(seed & MASK64) + (d << 16) + n) & MASK64)


def hash_pair(seed: int, d: int, n: int, I_n: int, J_n: int):
    """(h_n, s_n) of sketch d: h in [0, J_n) as int64, s in {+1, -1} as int8."""
    key = hash_key(seed, d, n)
    i = np.arange(I_n, dtype=np.uint64)
    y = _mix64_array(np.uint64(key) + i)
    h = ((y >> np.uint64(32)) * np.uint64(J_n)) >> np.uint64(32)
    s = np.where((y & np.uint64(1)) == 0, 1, -1).astype(np.int8)
    return h.astype(np.int64), s


def hash_tables(seed: int, D: int, I, J):
    """Per-sketch, per-mode hash pairs: ``h[d][n]``, ``s[d][n]``."""
    hs, ss = [], []
    for d in range(D):
        hd, sd = [], []
        for n, (I_n, J_n) in enumerate(zip(I, J)):
            h, s = hash_pair(seed, d, n, int(I_n), int(J_n))
            hd.append(h)
            sd.append(s)
        hs.append(hd)
        ss.append(sd)
    return hs, ss


def sketch_length(J) -> int:
    """J~ = sum_n J_n - N + 1 (Definition 4)."""
    return int(sum(int(j) for j in J) - len(J) + 1)


# ---------------------------------------------------------------------------
# Definition 1: count sketch, CS(x)_j = sum_{h(i) = j} s(i) x(i); applied
# column by column when x is a matrix.
# ---------------------------------------------------------------------------
def count_sketch(x, h, s, J: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((J,) + x.shape[1:], dtype=np.float64)
    np.add.at(out, np.asarray(h), np.asarray(s, dtype=np.float64).reshape(
        (-1,) + (1,) * (x.ndim - 1)) * x)
    return out


# ---------------------------------------------------------------------------
# Definition 4 / general-tensor formula of Section 3.2: FCS(T)_j is the sum of
# S * T over all multi-indices whose bin H equals j.
# ---------------------------------------------------------------------------
def _bins_and_signs(h, s, shape):
    """H and S over the full index grid, axes in mode order (mode 0 first)."""
    N = len(shape)
    H = np.zeros(shape, dtype=np.int64)
    S = np.ones(shape, dtype=np.float64)
    for n in range(N):
        view = [1] * N
        view[n] = shape[n]
        H = H + np.asarray(h[n], dtype=np.int64).reshape(view)
        S = S * np.asarray(s[n], dtype=np.float64).reshape(view)
    return H, S


def fcs_dense(T, h, s, J) -> np.ndarray:
    """FCS of a dense tensor ``T`` (numpy array, axis n = mode n)."""
    T = np.asarray(T, dtype=np.float64)
    H, S = _bins_and_signs(h, s, T.shape)
    return np.bincount(H.ravel(), weights=(S * T).ravel(),
                       minlength=sketch_length(J)).astype(np.float64)


def fcs_coo(idx, val, h, s, J) -> np.ndarray:
    """FCS of a sparse tensor given as coordinates ``idx[n][k]`` and values
    ``val[k]``; repeated coordinates add (the sketch is linear)."""
    idx = [np.asarray(ix, dtype=np.int64) for ix in idx]
    val = np.asarray(val, dtype=np.float64)
    H = np.zeros(val.shape, dtype=np.int64)
    S = np.ones(val.shape, dtype=np.float64)
    for n, ix in enumerate(idx):
        H += np.asarray(h[n], dtype=np.int64)[ix]
        S *= np.asarray(s[n], dtype=np.float64)[ix]
    return np.bincount(H, weights=S * val,
                       minlength=sketch_length(J)).astype(np.float64)


def vec(T) -> np.ndarray:
    """vec(T) with mode 0 varying fastest (column-major), Section 2.1."""
    return np.asarray(T).ravel(order="F")


def unvec(v, shape) -> np.ndarray:
    return np.asarray(v).reshape(shape, order="F")


# ---------------------------------------------------------------------------
# CP format: T = sum_r lambda_r u_r^(0) o ... o u_r^(N-1) (Section 2.1).
# ---------------------------------------------------------------------------
def cp_full(lam, U) -> np.ndarray:
    """Materialise a CP tensor; ``U[n]`` is I_n x R."""
    U = [np.asarray(u, dtype=np.float64) for u in U]
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    shape = tuple(u.shape[0] for u in U)
    T = np.zeros(shape, dtype=np.float64)
    for r in range(R):
        t = np.array(lam[r])
        for u in U:
            t = np.multiply.outer(t, u[:, r])
        T += t
    return T


def fcs_cp_conv(lam, U, h, s, J) -> np.ndarray:
    """FCS of a CP tensor as sum_r lambda_r CS_0(u_r) * ... * CS_{N-1}(u_r)
    with * the full linear convolution (Section 3.1, second line of the CP
    formula; exact by the polynomial-product identity proved there)."""
    U = [np.asarray(u, dtype=np.float64) for u in U]
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    Y = [count_sketch(U[n], h[n], s[n], int(J[n])) for n in range(len(U))]
    out = np.zeros(sketch_length(J), dtype=np.float64)
    for r in range(R):
        y = Y[0][:, r]
        for n in range(1, len(U)):
            y = np.convolve(y, Y[n][:, r])
        out += lam[r] * y
    return out


def fcs_cp_fft(lam, U, h, s, J, L: int | None = None) -> np.ndarray:
    """Same sketch through zero-padded FFTs (Section 3.1, third line):
    sum_r lambda_r F^-1( prod_n F(CS_n(U_n)(:, r), L) ), truncated to J~.
    The paper pads to L = J~; any L >= J~ gives the same linear convolution."""
    Jt = sketch_length(J)
    L = Jt if L is None else int(L)
    assert L >= Jt
    U = [np.asarray(u, dtype=np.float64) for u in U]
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    P = np.ones((L, R), dtype=np.complex128)
    for n in range(len(U)):
        P *= np.fft.fft(count_sketch(U[n], h[n], s[n], int(J[n])), n=L, axis=0)
    spec = P @ lam
    return np.fft.ifft(spec)[:Jt].real.copy()


def fcs_spectrum(y, L: int) -> np.ndarray:
    """F(y, L): the unnormalised L-point DFT of a zero-padded sketch."""
    return np.fft.fft(np.asarray(y, dtype=np.float64), n=L)


# ---------------------------------------------------------------------------
# Definitions 2 and 3 (the comparison sketches), used only to pin the FCS
# functions above through their stated relations.
# ---------------------------------------------------------------------------
def ts_dense(T, h, s, J: int) -> np.ndarray:
    """Tensor sketch (Definition 2): bin (sum_n h_n(i_n)) mod J, all J_n = J."""
    T = np.asarray(T, dtype=np.float64)
    H, S = _bins_and_signs(h, s, T.shape)
    return np.bincount((H % J).ravel(), weights=(S * T).ravel(),
                       minlength=J).astype(np.float64)


def hcs_dense(T, h, s, J) -> np.ndarray:
    """Higher-order count sketch (Definition 3): a J_0 x ... x J_{N-1} tensor."""
    T = np.asarray(T, dtype=np.float64)
    out = np.zeros(tuple(int(j) for j in J), dtype=np.float64)
    N = T.ndim
    grids = np.meshgrid(*[np.arange(n_) for n_ in T.shape], indexing="ij")
    S = np.ones(T.shape)
    idx = []
    for n in range(N):
        idx.append(np.asarray(h[n])[grids[n]])
        S = S * np.asarray(s[n], dtype=np.float64)[grids[n]]
    np.add.at(out, tuple(idx), S * T)
    return out


def ts_cp(lam, U, h, s, J: int) -> np.ndarray:
    """Tensor sketch of a CP tensor by the FFT form of Definition 2: the sum
    over r of lambda_r F^-1(prod_n F(CS_n(U_n)(:, r))) with J-point
    transforms, i.e. the mode-J circular convolution of the modes' count
    sketches (every mode hashes into the same J bins)."""
    U = [np.asarray(u, dtype=np.float64) for u in U]
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    P = np.ones((int(J), R), dtype=np.complex128)
    for n in range(len(U)):
        P *= np.fft.fft(count_sketch(U[n], h[n], s[n], int(J)), axis=0)
    return np.fft.ifft(P @ lam).real.copy()


def hcs_cp(lam, U, h, s, J) -> np.ndarray:
    """Higher-order count sketch of a CP tensor (Definition 3, rank-1 form):
    sum_r lambda_r CS_0(u_r^(0)) o ... o CS_{N-1}(u_r^(N-1)), materialised as
    a J_0 x ... x J_{N-1} array."""
    U = [np.asarray(u, dtype=np.float64) for u in U]
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    Y = [count_sketch(U[n], h[n], s[n], int(J[n])) for n in range(len(U))]
    out = np.zeros(tuple(int(j) for j in J), dtype=np.float64)
    for r in range(R):
        t = np.array(lam[r])
        for n in range(len(U)):
            t = np.multiply.outer(t, Y[n][:, r])
        out += t
    return out


def hcs_decompress_median(Y, hs, ss, I) -> np.ndarray:
    """The tensor recovered from D higher-order count sketches Y[d] (each a
    J_0 x ... x J_{N-1} array): per sketch, entry i is
    S(i) HCS[h_0(i_0), ..., h_{N-1}(i_{N-1})], the same decompression rule as
    for FCS with the bin taken per mode; the D estimates are reduced by the
    median (Section 4)."""
    I = tuple(int(i) for i in I)
    grids = np.meshgrid(*[np.arange(n) for n in I], indexing="ij")
    est = []
    for d in range(len(Y)):
        idx = tuple(np.asarray(hs[d][n])[grids[n]] for n in range(len(I)))
        S = np.ones(I)
        for n in range(len(I)):
            S = S * np.asarray(ss[d][n], dtype=np.float64)[grids[n]]
        est.append(S * np.asarray(Y[d], dtype=np.float64)[idx])
    return median(np.stack(est), axis=0)


# ---------------------------------------------------------------------------
# Sketched contractions (Section 3.3 and Section 4): inner products of D
# independent sketches reduced by the median.
# ---------------------------------------------------------------------------
def inner(a, b) -> np.ndarray:
    """<a_d, b_d> for each sketch d (rows of a and b)."""
    a = np.atleast_2d(np.asarray(a, dtype=np.float64))
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    return np.sum(a * b, axis=1)


def median(x, axis=0):
    """Median over the D independent sketches (numpy convention: the mean of
    the two middle order statistics when D is even)."""
    return np.median(np.asarray(x, dtype=np.float64), axis=axis)


def inner_median(a, b):
    per_d = inner(a, b)
    return median(per_d), per_d


def contract_free(y, h, s, J, free: int, vecs) -> np.ndarray:
    """Estimate of T(..., I, ...) with the identity at mode ``free`` and the
    given vectors at every other mode, from one sketch y = FCS(T).

    By Section 4.1 the i-th entry is <FCS(T), FCS(e_i o v ...)>.  The sketch of
    that rank-1 tensor is s_f(i) times g shifted by h_f(i), where g is the
    linear convolution of CS_n(v_n) over the modes n != f (Section 3.1), so
    the inner product is s_f(i) * sum_m y[h_f(i) + m] g[m]."""
    y = np.asarray(y, dtype=np.float64)
    N = len(J)
    others = [n for n in range(N) if n != free]
    g = np.ones(1)
    for k, n in enumerate(others):
        g = np.convolve(g, count_sketch(vecs[k], h[n], s[n], int(J[n])))
    corr = np.correlate(y, g, mode="valid")          # length J_free
    assert corr.shape[0] == int(J[free])
    hf = np.asarray(h[free], dtype=np.int64)
    sf = np.asarray(s[free], dtype=np.float64)
    return sf * corr[hf]


def contract_free_fft(y, h, s, J, L: int, vecs) -> np.ndarray:
    """The FFT form of the same estimate for an order-3 tensor with the free
    index at mode 0 (Section 4.1): z = F^-1(F(y) conj(F(CS_1 u)) conj(F(CS_2 v))),
    entry i = s_0(i) z(h_0(i)); F is the L-point DFT, L >= J~."""
    u, v = vecs
    Fy = np.fft.fft(np.asarray(y, dtype=np.float64), n=L)
    F1 = np.fft.fft(count_sketch(u, h[1], s[1], int(J[1])), n=L)
    F2 = np.fft.fft(count_sketch(v, h[2], s[2], int(J[2])), n=L)
    z = np.fft.ifft(Fy * np.conj(F1) * np.conj(F2)).real
    return np.asarray(s[0], dtype=np.float64) * z[np.asarray(h[0])]


def contract_free_median(Y, hs, ss, J, free, vecs) -> np.ndarray:
    """Median over the D sketches (rows of Y, each with its own hash pairs)."""
    est = np.stack([contract_free(Y[d], hs[d], ss[d], J, free, vecs)
                    for d in range(len(Y))])
    return median(est, axis=0)


def contract_full(y, h, s, J, vecs) -> float:
    """T(v_0, ..., v_{N-1}) estimate <FCS(T), FCS(v_0 o ... o v_{N-1})>
    (Section 4.1)."""
    g = np.ones(1)
    for n, v in enumerate(vecs):
        g = np.convolve(g, count_sketch(v, h[n], s[n], int(J[n])))
    return float(np.dot(np.asarray(y, dtype=np.float64), g))


# ---------------------------------------------------------------------------
# Kronecker-product compression (Section 4.3): the order-4 tensor
# T[i1, i2, i3, i4] = A[i1, i2] B[i3, i4] has
# FCS(A (x) B) = F^-1( F(FCS_{1,2}(A), J~) * F(FCS_{3,4}(B), J~) ).
# ---------------------------------------------------------------------------
def kron_fcs(A, B, h, s, J) -> np.ndarray:
    a = fcs_dense(A, h[0:2], s[0:2], J[0:2])
    b = fcs_dense(B, h[2:4], s[2:4], J[2:4])
    Jt = sketch_length(J)
    return np.fft.ifft(np.fft.fft(a, n=Jt) * np.fft.fft(b, n=Jt)).real.copy()


def contraction_fcs(A, B, h, s, J) -> np.ndarray:
    """FCS of the contraction C[i1,i2,i3,i4] = sum_l A[i1,i2,l] B[l,i3,i4]
    (Section 4.3): the sum over l of the Kronecker-product sketches of the
    slices A(:,:,l) and B(l,:,:)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return sum(kron_fcs(A[:, :, l], B[l], h, s, J) for l in range(A.shape[2]))


def decompress_median(Y, hs, ss, I) -> np.ndarray:
    """The tensor recovered from D sketches Y (D x J~): per sketch, entry i
    is S(i) FCS[H(i)] (the decompression rule of Section 4.3, for any
    order), and the D estimates are reduced by the median (Section 4: the
    median over independent sketches)."""
    est = np.stack([kron_decompress(Y[d], hs[d], ss[d], I) for d in range(len(Y))])
    return median(est, axis=0)


def decompress_at(Y, hs, ss, idx) -> np.ndarray:
    """The same recovered entries one by one: idx[n][k] is the mode-n index
    of entry k; returns the median over d of S_d y_d[H_d] for each k."""
    idx = [np.asarray(ix, dtype=np.int64) for ix in idx]
    est = []
    for d in range(len(Y)):
        H = np.zeros(idx[0].shape, dtype=np.int64)
        S = np.ones(idx[0].shape, dtype=np.float64)
        for n, ix in enumerate(idx):
            H += np.asarray(hs[d][n], dtype=np.int64)[ix]
            S *= np.asarray(ss[d][n], dtype=np.float64)[ix]
        est.append(S * np.asarray(Y[d], dtype=np.float64)[H])
    return median(np.stack(est), axis=0)


def kron_decompress(y, h, s, I) -> np.ndarray:
    """Entry (i1,i2,i3,i4) of the recovered order-4 tensor is
    s1 s2 s3 s4 * FCS[h1 + h2 + h3 + h4] (Section 4.3; 0-based, so the
    paper's modulo never wraps)."""
    H, S = _bins_and_signs(h, s, tuple(int(i) for i in I))
    return S * np.asarray(y, dtype=np.float64)[H]


# ---------------------------------------------------------------------------
# Robust tensor power method on sketches (Section 4.1.1: RTPM for a symmetric
# order-3 tensor, with T(I,u,u) and T(u,u,u) estimated from D sketches as in
# Section 4.1).  For each component: power iterations u <- T(I,u,u) /
# ||T(I,u,u)|| from several starting vectors, the eigenvalue T(u,u,u) of
# each, the start with the largest eigenvalue kept, then deflation of the
# sketches by linearity: FCS(T - lam u o u o u) = FCS(T) - lam FCS(u o u o u).
# ---------------------------------------------------------------------------
def fcs_rank1(vecs, h, s, J) -> np.ndarray:
    """FCS of the rank-1 tensor v_0 o ... o v_{N-1}: the linear convolution
    of the mode count sketches (Section 3.1)."""
    g = np.ones(1)
    for n, v in enumerate(vecs):
        g = np.convolve(g, count_sketch(v, h[n], s[n], int(J[n])))
    return g


def rtpm(Y, hs, ss, J, rank: int, inits, iters: int):
    """Y: D x J~ sketches of a symmetric I x I x I tensor (sketch d with hash
    pairs hs[d], ss[d]); inits: rank x L x I starting vectors (the random
    draws are inputs).  Returns (eigenvalues [rank], components rank x I)."""
    Y = np.array(Y, dtype=np.float64)          # deflated in place
    D = Y.shape[0]
    lams, comps = [], []
    for k in range(rank):
        U = np.array(inits[k], dtype=np.float64)
        U = U / np.linalg.norm(U, axis=1, keepdims=True)
        for _ in range(iters):
            W = np.stack([contract_free_median(Y, hs, ss, J, 0, [u, u]) for u in U])
            U = W / np.linalg.norm(W, axis=1, keepdims=True)
        lam = np.array([median([contract_full(Y[d], hs[d], ss[d], J, [u, u, u]) for d in range(D)])
                        for u in U])
        j = int(np.argmax(lam))
        u = U[j]
        lams.append(float(lam[j]))
        comps.append(u)
        for d in range(D):
            Y[d] -= lam[j] * fcs_rank1([u, u, u], hs[d], ss[d], J)
    return np.array(lams), np.stack(comps)



def rtpm_asym(Y, hs, ss, J, rank: int, inits, iters: int):
    """RTPM for an asymmetric order-3 tensor (Section 4.1.1: the power iteration
    becomes an alternating rank-1 update).  Y: D x J~ sketches; inits:
    rank x L x 3 x I_max starting vectors (mode n uses the first I_n
    entries of slot n).  Per component and start: u <- T(I,v,w), then
    v <- T(u,I,w), then w <- T(u,v,I), each normalised, ``iters`` times; the
    eigenvalue T(u,v,w); the start with the largest eigenvalue is kept and
    deflated from the sketches.  Returns (eigenvalues [rank], [U, V, W] with
    the components as rows)."""
    Y = np.array(Y, dtype=np.float64)
    D = Y.shape[0]
    Is = [len(hs[0][n]) for n in range(3)]
    lams, comps = [], [[], [], []]
    for k in range(rank):
        best = None
        for start in inits[k]:
            x = [np.array(start[n][:Is[n]], dtype=np.float64) for n in range(3)]
            x = [v / np.linalg.norm(v) for v in x]
            for _ in range(iters):
                for n in range(3):
                    o = [m for m in range(3) if m != n]
                    g = contract_free_median(Y, hs, ss, J, n, [x[m] for m in o])
                    x[n] = g / np.linalg.norm(g)
            lam = median([contract_full(Y[d], hs[d], ss[d], J, x) for d in range(D)])
            if best is None or lam > best[0]:
                best = (lam, x)
        lam, x = best
        lams.append(float(lam))
        for n in range(3):
            comps[n].append(x[n])
        for d in range(D):
            Y[d] -= lam * fcs_rank1(x, hs[d], ss[d], J)
    return np.array(lams), [np.stack(c) for c in comps]


# ---------------------------------------------------------------------------
# Alternating least squares on sketches (Section 4.1.2, ALS for an order-3
# tensor).  Mode n is updated from the product of the mode-n unfolding with
# the Khatri-Rao product of the other factors; column r of that product is
# the contraction of T with the r-th columns of the other factors at their
# own modes and the identity at mode n (estimated from the D sketches as in
# Section 4.1).  Then, as in plain ALS, the factor is that matrix times the
# inverse of the Hadamard product of the other factors' Gram matrices, and
# its columns are normalised into the weights.
# ---------------------------------------------------------------------------
def als_step(M, others):
    """Plain ALS update of one mode: M (I_n x R) is the mode's
    unfolding-times-Khatri-Rao product, ``others`` the other factor matrices.
    Returns (weights [R], unit-column factor I_n x R)."""
    R = M.shape[1]
    G = np.ones((R, R))
    for F in others:
        G = G * (F.T @ F)
    U = np.linalg.solve(G, np.asarray(M, dtype=np.float64).T).T
    lam = np.linalg.norm(U, axis=0)
    return lam, U / lam


def als(Y, hs, ss, J, init, iters: int):
    """Y: D x J~ sketches of an order-3 tensor; init: three starting factor
    matrices (I_n x R, the random draws are inputs).  Each iteration updates
    modes 0, 1, 2 in turn.  Returns (weights [R], [A_0, A_1, A_2])."""
    F = [np.array(f, dtype=np.float64) for f in init]
    R = F[0].shape[1]
    lam = np.ones(R)
    for _ in range(iters):
        for n in range(3):
            o = [m for m in range(3) if m != n]
            M = np.stack([contract_free_median(Y, hs, ss, J, n, [F[m][:, r] for m in o])
                          for r in range(R)], axis=1)
            lam, F[n] = als_step(M, [F[m] for m in o])
    return lam, F
