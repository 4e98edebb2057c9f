"""Decompression (Section 4.3: entry = S y[H] per sketch, median over the D
sketches) and contraction compression on the GPU against the FP64 oracle.

Decompression parity is bit-exact: every estimate is a sketch value times a
sign, the median of an odd count is one of them, and the mean of the middle
pair is formed in double and rounded once, which the oracle's FP64 mean
rounded to float32 reproduces.  Inputs (sketch values) come from the oracle
or from seeded draws, never from the HIP path.  Cases cover each median
form (D = 1, 2, 3, 4..8, 9..32), vector and scalar stores, staged windows
and in-place reads, rows split into several tiles with a ragged last one,
the Kronecker matrix layout, and sampled entries of a 2^32-entry output."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2106_13062_amd import FcsError, Plan

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _sketches(D, Jt, seed):
    return np.random.default_rng(seed).standard_normal((D, Jt)).astype(np.float32)


def _expected(Y, hs, ss, I, order):
    """Oracle tensor laid out with mode order[0] fastest, flattened."""
    full = O.decompress_median(Y.astype(np.float64), hs, ss, I)
    return np.transpose(full, order).reshape(-1, order="F").astype(np.float32)


@pytest.mark.parametrize("I,J,D,order,seed", [
    ((6, 5, 7), (16, 16, 16), 1, None, 1),
    ((6, 5, 7), (16, 16, 16), 2, None, 2),
    ((8, 5, 7), (16, 16, 16), 3, None, 3),          # vector stores (I_0 % 4 == 0)
    ((8, 5, 7), (16, 16, 16), 5, None, 4),
    ((6, 5, 7), (16, 16, 16), 20, None, 5),
    ((12, 8, 16, 4), (32, 16, 64, 8), 3, (2, 0, 3, 1), 6),   # Kronecker matrix layout
    ((7, 5, 9, 3), (8, 8, 8, 8), 4, (3, 1, 0, 2), 7),       # scalar stores, permuted
    ((256, 300, 3), (64, 64, 64), 1, None, 8),      # 76800-entry rows, 10 tiles, ragged last
    ((40, 30, 20), (4096, 4096, 4096), 20, None, 9),  # windows exceed LDS: reads in place
    ((16, 6, 5), (2048, 64, 64), 3, (1, 0, 2), 10),   # row shorter than its windows
    ((64, 1100, 3, 2), (32, 32, 16, 8), 3, None, 11),     # 6 rows over two outer modes
    ((64, 1100, 3, 2), (4096, 4096, 16, 8), 20, None, 12),  # the same, reads in place
    ((8, 5, 7), (20000, 16, 16), 5, None, 13),            # one window exceeds LDS: reads in place
    ((8, 1100, 3, 2), (2048, 8192, 16, 8), 4, None, 14),  # short rows: reads in place
    ((1000,), (64,), 3, None, 15),                        # order 1: count sketch recovery
    ((1, 7, 1, 5), (1, 4, 1, 8), 2, (3, 0, 2, 1), 16),    # modes of size 1 and hash length 1
    ((4, 1, 3), (1, 1, 1), 1, None, 17),                  # J~ = 1: every entry reads bin 0
])
def test_decompress_matches_oracle(I, J, D, order, seed):
    print(f"decompress I={I} J={J} D={D} order={order}", flush=True)
    N = len(I)
    plan = Plan(I, J, D, 60 + seed, device=DEV)
    hs, ss = O.hash_tables(60 + seed, D, I, J)
    Y = _sketches(D, O.sketch_length(J), seed)
    got = plan.decompress(torch.from_numpy(Y).to(DEV), order=order).cpu().numpy()
    want = _expected(Y, hs, ss, I, list(order) if order else list(range(N)))
    np.testing.assert_array_equal(got, want)


def test_decompress_kronecker_sketch_in_matrix_layout():
    # the paper's Kronecker set-up: A 30 x 40, B 40 x 50 ~ U[-5, 5], D = 20;
    # the sketch comes from the oracle (J_n = 1024 compresses 2.4M entries
    # about 600-fold, so the recovery itself is coarse; parity is the point)
    r = np.random.default_rng(13)
    A = r.uniform(-5, 5, (30, 40))
    B = r.uniform(-5, 5, (40, 50))
    I, J, D = (30, 40, 40, 50), (1024, 1024, 1024, 1024), 20
    hs, ss = O.hash_tables(71, D, I, J)
    Y = np.stack([O.kron_fcs(A, B, hs[d], ss[d], J) for d in range(D)]).astype(np.float32)
    plan = Plan(I, J, D, 71, device=DEV)
    got = plan.decompress(torch.from_numpy(Y).to(DEV), order=(2, 0, 3, 1)).cpu().numpy()
    want = _expected(Y, hs, ss, I, [2, 0, 3, 1])
    np.testing.assert_array_equal(got, want)
    # order (2, 0, 3, 1) is the layout of A (x) B as a column-major matrix
    K = np.kron(A, B)
    T4 = np.einsum("ab,cd->abcd", A, B)
    np.testing.assert_array_equal(np.transpose(T4, (2, 0, 3, 1)).reshape(-1, order="F"), K.reshape(-1, order="F"))


@pytest.mark.parametrize("D", [1, 3])
def test_decompress_full_size_sampled(D):
    # 256 x 256 (x) 256 x 256 in the Kronecker matrix layout: 2^32 entries
    print(f"decompress full size D={D}", flush=True)
    I, J = (256, 256, 256, 256), (4096, 4096, 4096, 4096)
    plan = Plan(I, J, D, 80 + D, device=DEV)
    hs, ss = O.hash_tables(80 + D, D, I, J)
    Y = _sketches(D, O.sketch_length(J), 90 + D)
    out = plan.decompress(torch.from_numpy(Y).to(DEV), order=(2, 0, 3, 1))
    g = np.random.default_rng(14)
    flat = np.concatenate([g.integers(0, 1 << 32, 200000), np.arange(4096), (1 << 32) - 1 - np.arange(4096)])
    got = out[torch.from_numpy(flat).to(DEV)].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    # layout (i2, i0, i3, i1), i2 fastest
    i2, rest = flat % 256, flat // 256
    i0, rest = rest % 256, rest // 256
    i3, i1 = rest % 256, rest // 256
    want = O.decompress_at(Y, hs, ss, [i0, i1, i2, i3]).astype(np.float32)
    np.testing.assert_array_equal(got, want)


def test_decompress_errors():
    plan = Plan((4, 4, 4), (8, 8, 8), 2, 1, device=DEV)
    y = torch.zeros((2, plan.Jt), device=DEV)
    with pytest.raises(FcsError):
        plan.decompress(y, order=(0, 0, 1))
    with pytest.raises(FcsError):
        plan.decompress(y, order=(0, 1, 3))
    big = Plan((4, 4, 4), (8, 8, 8), 33, 1, device=DEV)
    with pytest.raises(FcsError):
        big.decompress(torch.zeros((33, big.Jt), device=DEV))


def _colmajor(X):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(X, dtype=np.float32).reshape(-1, order="F"))).to(DEV)


@pytest.mark.parametrize("I,J,Lc,D,seed", [
    ((6, 5, 4, 7), (8, 9, 7, 10), 5, 3, 1),
    ((30, 40, 40, 30), (64, 64, 64, 64), 50, 20, 2),      # the paper's contraction shapes
    ((33, 17, 9, 21), (512, 256, 1024, 128), 7, 2, 3),   # several transform slices
    ((5, 4, 3, 6), (16, 8, 8, 16), 300, 2, 4),            # long shared index: several chunks of l
])
def test_contraction_matches_oracle(I, J, Lc, D, seed):
    print(f"contraction I={I} J={J} Lc={Lc} D={D}", flush=True)
    r = np.random.default_rng(20 + seed)
    A = r.uniform(0, 10, (I[0], I[1], Lc)).astype(np.float32)
    B = r.uniform(0, 10, (Lc, I[2], I[3])).astype(np.float32)
    plan = Plan(I, J, D, 40 + seed, device=DEV)
    y, spec = plan.sketch_contraction(_colmajor(A), _colmajor(B), want_spec=True)
    y = y.cpu().numpy().astype(np.float64)
    hs, ss = O.hash_tables(40 + seed, D, I, J)
    for d in range(D):
        want = O.contraction_fcs(A, B, hs[d], ss[d], J)
        err = np.linalg.norm(y[d] - want) / np.linalg.norm(want)
        assert err <= 1e-5, (d, err)
    # the spectra are those of the sketch
    spec_y = plan.spectrum(torch.from_numpy(y.astype(np.float32)).to(DEV))
    s1, s2 = spec.cpu().numpy(), spec_y.cpu().numpy()
    assert np.linalg.norm(s1 - s2) <= 1e-5 * np.linalg.norm(s2)


def test_contraction_with_long_hashes():
    """Factor-sketch bins beyond LDS (J = 20000) are summed in global memory."""
    I, J, Lc, D, seed = (30, 40, 40, 30), (20000,) * 4, 5, 2, 44
    r = np.random.default_rng(24)
    A = r.uniform(0, 10, (I[0], I[1], Lc)).astype(np.float32)
    B = r.uniform(0, 10, (Lc, I[2], I[3])).astype(np.float32)
    plan = Plan(I, J, D, seed, device=DEV)
    y, _ = plan.sketch_contraction(_colmajor(A), _colmajor(B))
    y = y.cpu().numpy().astype(np.float64)
    hs, ss = O.hash_tables(seed, D, I, J)
    for d in range(D):
        want = O.contraction_fcs(A, B, hs[d], ss[d], J)
        assert np.linalg.norm(y[d] - want) <= 1e-5 * np.linalg.norm(want), d


def test_contraction_of_one_slice_is_the_kronecker_sketch():
    r = np.random.default_rng(30)
    A = r.uniform(-5, 5, (12, 10, 1)).astype(np.float32)
    B = r.uniform(-5, 5, (1, 9, 14)).astype(np.float32)
    plan = Plan((12, 10, 9, 14), (64, 32, 64, 32), 3, 5, device=DEV)
    yc, _ = plan.sketch_contraction(_colmajor(A), _colmajor(B))
    yk, _ = plan.sketch_kron(_colmajor(A[:, :, 0]), _colmajor(B[0]))
    np.testing.assert_allclose(yc.cpu().numpy(), yk.cpu().numpy(), rtol=0, atol=1e-6 * float(yk.abs().max()))


def test_contraction_errors():
    plan = Plan((4, 4, 4, 4), (8, 8, 8, 8), 1, 1, device=DEV)
    with pytest.raises(ValueError):
        plan.sketch_contraction(torch.zeros(16 * 3, device=DEV), torch.zeros(16 * 2, device=DEV))
    p3 = Plan((4, 4, 4), (8, 8, 8), 1, 1, device=DEV)
    with pytest.raises(ValueError):
        p3.sketch_contraction(torch.zeros(16, device=DEV), torch.zeros(16, device=DEV))
