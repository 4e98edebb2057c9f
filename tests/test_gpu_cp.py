"""GPU parity of the CP sketch (Section 3.1), the sketch spectra and the
T(I, u, v) contraction with the median over D sketches (Section 4.1) against
the FP64 oracle.  Bar: relative L2 error <= 1e-5 per sketch / per estimate
vector."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from paper_2106_13062_amd import FcsError, Plan

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = 1e-5


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    if not (np.iscomplexobj(a) or np.iscomplexobj(b)):
        a = a.astype(np.float64)
        b = b.astype(np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def dev_factors(U):
    """I_n x R factors -> R x I_n device tensors (column-major factors)."""
    return [dev(np.ascontiguousarray(u.T)) for u in U]


CP_CASES = [
    # (I, J, R, D, L)
    ((100, 100, 100), (64, 64, 64), 10, 5, 0),          # the order-3 I_n = 100 workload
    ((100, 100, 100), (64, 64, 64), 10, 5, 256),        # explicit power-of-two L
    ((100, 100, 100), (64, 64, 64), 10, 5, 768),        # L = 3 x 256
    ((57,), (300,), 7, 3, 0),                           # order 1: a plain count sketch
    ((40, 33), (100, 70), 5, 2, 0),
    ((30, 20, 10, 9), (50, 40, 30, 20), 6, 3, 0),
    ((12, 11, 10, 9, 8), (16, 16, 16, 16, 16), 4, 2, 0),
    ((2000, 1500, 700), (1024, 2048, 512), 33, 4, 0),   # folding (J_n > P) and several slices
    ((300, 300, 300), (5000, 5000, 5000), 3, 2, 0),
    # Q = 2: both stored slices are conjugate-symmetric, so both pack modes
    # (0, 1) and (2, 3) into shared transforms
    ((60, 50, 40, 30), (100, 90, 80, 70), 5, 2, 32768),
    # Q = 4: slices 0 and 2 pack modes (0, 1) with mode 2 alone, slice 1 does not pack
    ((60, 50, 40), (100, 90, 80), 4, 3, 65536),
    # order 5 on Q = 2: pairs (0, 1), (2, 3) and mode 4 alone
    ((12, 11, 10, 9, 8), (16, 16, 16, 16, 16), 3, 2, 32768),
    # scatter rounds (8 entries per thread, 64 threads at P = 256, 1024 at
    # P = 16384): exactly one full round, one full round and a one-entry
    # tail, a tail that splits a wave, single entries
    ((512, 513, 511), (64, 64, 64), 3, 2, 0),
    ((1, 1023, 1025), (64, 64, 64), 2, 2, 0),
    ((8192, 8193, 8191), (16384, 16384, 16384), 2, 2, 0),
]


@pytest.mark.parametrize("I,J,R,D,L", CP_CASES)
def test_cp_sketch_parity(I, J, R, D, L):
    print(f"cp I={I} J={J} R={R} D={D} L={L}", flush=True)
    seed = 3
    U = synth.cp_factors(11, I, R)
    lam = np.linspace(0.5, 1.5, R).astype(np.float32)
    plan = Plan(I, J, D, seed, L=L, device=DEV)
    y, _ = plan.sketch_cp(dev_factors(U), lam=dev(lam))
    y = y.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    for d in range(D):
        want = O.fcs_cp_conv(lam, U, hs[d], ss[d], J)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))


def test_cp_sketch_wide_range_columns():
    """Factor columns of very different scales (2^-8 .. 2^8), each with one
    entry up to 2^24 times the rest, and one column whose other entries are
    2^64 below its largest: the count sketches of the factor columns are
    fixed-point sums scaled to each column's maximum, and the sketch still
    matches the FP64 oracle to 1e-5 per sketch (entries more than about
    2^(61 - log2 I_n) below their column's maximum are dropped, far below
    that bar)."""
    I, J, R, D, seed = (300, 200, 250), (256, 128, 512), 8, 3, 21
    rng = np.random.default_rng(5)
    U = synth.cp_factors(13, I, R)
    for n, u in enumerate(U):
        u *= np.float32(2.0) ** rng.integers(-8, 9, size=(1, R)).astype(np.float32)
        rows = rng.integers(0, I[n], size=R)
        u[rows, np.arange(R)] *= np.float32(2.0) ** rng.integers(0, 25, size=R).astype(np.float32)
    U[0][:, 3] *= np.float32(2.0 ** -40)
    U[0][17, 3] = np.float32(2.0 ** 24)
    plan = Plan(I, J, D, seed, device=DEV)
    y, _ = plan.sketch_cp(dev_factors(U))
    y = y.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    for d in range(D):
        want = O.fcs_cp_conv(None, U, hs[d], ss[d], J)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))


@pytest.mark.parametrize("L", [0, 32768])
def test_cp_sketch_zero_columns_and_signed_weights(L):
    """All-zero factor columns (a zero maximum and norm: scale exponent 0,
    in a packed pair and alone) and weights of both signs, at the planner's
    transform length and at Q = 2 (both slices pack)."""
    I, J, R, D, seed = (70, 60, 50), (128, 96, 64), 6, 3, 17
    U = synth.cp_factors(15, I, R)
    U[0][:, 1] = 0.0
    U[1][:, 2] = 0.0
    U[2][:, 4] = 0.0
    lam = np.array([1.5, -2.0, 0.5, -0.25, 3.0, -1.0], dtype=np.float32)
    plan = Plan(I, J, D, seed, L=L, device=DEV)
    y, _ = plan.sketch_cp(dev_factors(U), lam=dev(lam))
    y = y.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    for d in range(D):
        want = O.fcs_cp_conv(lam, U, hs[d], ss[d], J)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))


def test_cp_sketch_non_finite_column():
    """A NaN in one factor column makes every entry of every sketch NaN (the
    FFT spreads it over all bins), as a float sum does; the other sketches of
    a call without it stay finite."""
    I, J, R, D, seed = (50, 40, 30), (64, 32, 16), 4, 2, 8
    U = synth.cp_factors(14, I, R)
    plan = Plan(I, J, D, seed, device=DEV)
    y0, _ = plan.sketch_cp(dev_factors(U))
    assert np.isfinite(y0.cpu().numpy()).all()
    U[1][7, 2] = np.nan
    y, _ = plan.sketch_cp(dev_factors(U))
    assert np.isnan(y.cpu().numpy()).all()


def test_cp_matches_dense_of_materialised_tensor():
    """Section 3.1: the CP route equals the general-tensor formula on the
    materialised tensor (both on the GPU)."""
    I, J, R, D, seed = (40, 30, 20), (32, 16, 24), 6, 4, 9
    U = synth.cp_factors(12, I, R)
    plan = Plan(I, J, D, seed, device=DEV)
    y, _ = plan.sketch_cp(dev_factors(U))
    T = O.vec(O.cp_full(None, U)).astype(np.float32)
    yd = plan.sketch_dense(dev(T))
    for d in range(D):
        assert rel(y[d].cpu().numpy(), yd[d].cpu().numpy()) <= 3 * TOL


def test_cp100_inner_product_of_two_cp_tensors():
    """The order-3 I_n = 100 rank-10 workload (J_n = 64, D = 5): FFT-path
    sketches of two independent rank-10 CP tensors on the GPU, then the
    Proposition 1 inner product of each sketch pair and its median over D
    (fcs_contract_inner), against the oracle's direct-convolution sketches
    (Section 3.1) and their FP64 inner products.  Scalar bar (Cauchy-Schwarz
    scale): |x - x_hat| <= 1e-5 ||a_d|| ||b_d|| per sketch and for the
    median.  The brute-force sketch of the materialised 10^6-entry tensor
    (general formula, GPU) also matches the FFT path."""
    cfg = synth.CP100
    U = cfg.factors()
    V = cfg.factors(stream=1)
    plan = Plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed, device=DEV)
    ya, _ = plan.sketch_cp(dev_factors(U))
    yb, _ = plan.sketch_cp(dev_factors(V))
    med, per_d = plan.contract_inner(ya, yb)
    hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
    wa = np.stack([O.fcs_cp_conv(None, U, hs[d], ss[d], cfg.J) for d in range(cfg.D)])
    wb = np.stack([O.fcs_cp_conv(None, V, hs[d], ss[d], cfg.J) for d in range(cfg.D)])
    w_med, w_per = O.inner_median(wa, wb)
    scale = np.linalg.norm(wa, axis=1) * np.linalg.norm(wb, axis=1)
    got_per = per_d.cpu().numpy()
    assert np.all(np.abs(got_per - w_per) <= TOL * scale), (got_per, w_per)
    assert abs(float(med.cpu()[0]) - w_med) <= TOL * float(np.median(scale))
    # brute force: the general-tensor sketch of the materialised tensor
    T = O.vec(O.cp_full(None, U)).astype(np.float32)
    yd = plan.sketch_dense(dev(T)).cpu().numpy()
    ya = ya.cpu().numpy()
    for d in range(cfg.D):
        assert rel(ya[d], yd[d]) <= 3 * TOL, (d, rel(ya[d], yd[d]))


def test_cp_rank_zero_and_linearity():
    I, J, D = (20, 30, 40), (16, 16, 16), 3
    plan = Plan(I, J, D, 5, device=DEV)
    U = synth.cp_factors(13, I, 4)
    y0, _ = plan.sketch_cp([dev(np.zeros((0, i), np.float32)) for i in I])
    assert torch.count_nonzero(y0).item() == 0
    ya, _ = plan.sketch_cp(dev_factors([u[:, :2] for u in U]))
    yb, _ = plan.sketch_cp(dev_factors([u[:, 2:] for u in U]))
    yab, _ = plan.sketch_cp(dev_factors(U))
    for d in range(D):
        assert rel((ya + yb)[d].cpu().numpy(), yab[d].cpu().numpy()) <= TOL


def _natural_spectrum(spec, Q, P, L):
    """Rebuild X[0..L) of a real sequence from the stored slices."""
    spec = spec[..., 0].astype(np.float64) + 1j * spec[..., 1].astype(np.float64)
    X = np.zeros(L, dtype=np.complex128)
    for q in range(Q // 2 + 1):
        X[q::Q] = spec[q * P:(q + 1) * P]
    for q in range(Q // 2 + 1, Q):
        # X[Qk + q] = conj(X[L - Qk - q])
        k = np.arange(P)
        X[Q * k + q] = np.conj(X[(L - Q * k - q) % L])
    return X


@pytest.mark.parametrize("I,J,L", [((100, 100, 100), (64, 64, 64), 0), ((50, 60), (300, 200), 0),
                                   ((80, 70, 60), (600, 500, 400), 0)])
def test_spectrum_layout_and_values(I, J, L):
    D, seed, R = 3, 21, 5
    U = synth.cp_factors(14, I, R)
    plan = Plan(I, J, D, seed, L=L, device=DEV)
    y, spec = plan.sketch_cp(dev_factors(U), want_spec=True)
    spec2 = plan.spectrum(y)
    hs, ss = O.hash_tables(seed, D, I, J)
    for d in range(D):
        want = O.fcs_cp_conv(None, U, hs[d], ss[d], J)
        F = O.fcs_spectrum(want, plan.L)
        for s_ in (spec, spec2):
            X = _natural_spectrum(s_[d].cpu().numpy(), plan.Q, plan.P, plan.L)
            assert rel(X, F) <= TOL


@pytest.mark.parametrize("I,J,L", [((100, 100, 100), (64, 64, 64), 0), ((50, 60), (300, 200), 0),
                                   ((30, 40, 50), (700, 900, 1100), 3 * 1024),
                                   ((10000, 10000, 10000), (16384, 16384, 16384), 0),
                                   ((10000, 10000, 10000), (16384, 16384, 16384), 65536),
                                   ((100, 100), (40000, 24000), 0)])
def test_twiddle_tables(I, J, L):
    """The plan's twiddle tables exp(-2 pi i k / P) and exp(-2 pi i k / L),
    read back from the bound table memory (layout of fcs_plan_bind): within
    2^-22 of the exact values per component (the argument's rounding and
    sincospif's error, a few ulp), exact at the quarter turns."""
    D = 2
    plan = Plan(I, J, D, 5, L=L, device=DEV)
    tb = plan.tables.cpu().numpy()
    a256 = lambda x: (x + 255) // 256 * 256
    offP = a256(D * sum(I) * 4)
    offL = a256(offP + plan.P * 8)
    print(f"I={I} J={J} L={plan.L} P={plan.P} Q={plan.Q}", flush=True)
    for off, n in ((offP, plan.P), (offL, plan.L)):
        w = tb[off:off + 8 * n].view(np.float32).reshape(n, 2).astype(np.float64)
        k = np.arange(n)
        ex = np.exp(-2j * np.pi * k / n)
        err = np.maximum(np.abs(w[:, 0] - ex.real), np.abs(w[:, 1] - ex.imag))
        assert err.max() <= 2.0 ** -22, (n, err.max(), int(err.argmax()))
        if n % 4 == 0:
            quarter = w[:: n // 4]
            assert np.array_equal(quarter, [[1, 0], [0, -1], [-1, 0], [0, 1]]), quarter


FREE_CASES = [
    # (I, J, D, P, free)
    ((30, 25, 20), (32, 32, 32), 5, 4, 0),
    ((30, 25, 20), (32, 32, 32), 5, 3, 1),
    ((30, 25, 20), (32, 32, 32), 6, 2, 2),
    ((200, 150, 100), (300, 400, 500), 4, 3, 0),
    ((20, 15, 10, 8), (16, 24, 32, 8), 3, 2, 1),
]


@pytest.mark.parametrize("I,J,D,Pn,free", FREE_CASES)
def test_free_mode_contraction_parity(I, J, D, Pn, free):
    print(f"free I={I} J={J} D={D} P={Pn} free={free}", flush=True)
    seed, R = 31, 4
    U = synth.cp_factors(15, I, R)
    plan = Plan(I, J, D, seed, device=DEV)
    y, spec = plan.sketch_cp(dev_factors(U), want_spec=True)
    vecs_np = [None if n == free else synth.unit_vectors(40 + n, Pn, I[n]) for n in range(len(I))]
    vecs = [None if v is None else dev(v) for v in vecs_np]
    out = plan.contract_free_mode(spec, free, vecs).cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    Y = np.stack([O.fcs_cp_conv(None, U, hs[d], ss[d], J) for d in range(D)])
    for p in range(Pn):
        vv = [vecs_np[n][p] for n in range(len(I)) if n != free]
        want = O.median(np.stack([O.contract_free(Y[d], hs[d], ss[d], J, free, vv) for d in range(D)]), axis=0)
        assert rel(out[p], want) <= TOL, (p, rel(out[p], want))


def test_free_mode_from_dense_sketch():
    """T(I, u, v) from a dense sketch through fcs_sketch_spectrum."""
    I, J, D, seed = (64, 48, 40), (128, 128, 128), 5, 8
    T = synth.dense_tensor(3, I)
    plan = Plan(I, J, D, seed, device=DEV)
    y = plan.sketch_dense(dev(T))
    spec = plan.spectrum(y)
    u = synth.unit_vectors(1, 2, I[1])
    v = synth.unit_vectors(2, 2, I[2])
    out = plan.contract_free_mode(spec, 0, [None, dev(u), dev(v)]).cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    Y = O.dense_rows(T, I, hs, ss, plan.Jt)
    for p in range(2):
        want = O.contract_free_median(Y, hs, ss, J, 0, [u[p], v[p]])
        assert rel(out[p], want) <= TOL


@pytest.mark.parametrize("I,J,D,Pn,L", [
    ((30, 20, 10), (64, 32, 16), 3, 5, 0),
    ((50, 40, 30, 20), (128, 64, 64, 32), 4, 3, 0),      # order 4, even D
    ((200, 150, 100), (1024, 512, 256), 5, 7, 8192),     # several transform slices
])
def test_full_contraction_parity(I, J, D, Pn, L):
    """T(v_0, ..., v_{N-1}) for P tuples from the spectra (Parseval) against
    the oracle's literal <y_d, FCS_d(v_0 o ... o v_{N-1})> and its median."""
    print(f"full contraction I={I} J={J} D={D} P={Pn} L={L}", flush=True)
    seed, R = 33, 4
    U = synth.cp_factors(16, I, R)
    plan = Plan(I, J, D, seed, L=L, device=DEV)
    _, spec = plan.sketch_cp(dev_factors(U), want_out=False, want_spec=True)
    vecs_np = [synth.unit_vectors(50 + n, Pn, I[n]) for n in range(len(I))]
    med, per_d = plan.contract_full(spec, [dev(v) for v in vecs_np])
    med, per_d = med.cpu().numpy(), per_d.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    Y = np.stack([O.fcs_cp_conv(None, U, hs[d], ss[d], J) for d in range(D)])
    for p in range(Pn):
        vv = [vecs_np[n][p] for n in range(len(I))]
        want_d = np.array([O.contract_full(Y[d], hs[d], ss[d], J, vv) for d in range(D)])
        scale = max(np.linalg.norm(Y[d]) * np.linalg.norm(O.fcs_rank1(vv, hs[d], ss[d], J)) for d in range(D))
        assert np.all(np.abs(per_d[p] - want_d) <= TOL * scale), (p, per_d[p], want_d)
        assert abs(med[p] - O.median(want_d)) <= TOL * scale


def test_cp_full_size_workload():
    """Order 3, I_n = 10^4, R = 512 unit-norm columns, J_n = 2^14, D = 10,
    and T(I, u, v) for 64 unit vector pairs, in the launch configuration the
    benchmark times.  Oracle: the FFT route in float64 (pinned against the
    direct convolution and the brute force on small shapes)."""
    cfg = synth.CP10K
    U = cfg.factors()
    plan = Plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed, device=DEV)
    y, spec = plan.sketch_cp(dev_factors(U), want_spec=True)
    y = y.cpu().numpy()
    uv = synth.unit_vectors(cfg.data_seed, 2 * cfg.pairs, cfg.I[1], stream=5)
    u, v = uv[:cfg.pairs], uv[cfg.pairs:]
    est = plan.contract_free_mode(spec, 0, [None, dev(u), dev(v)]).cpu().numpy()
    hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
    L = plan.L
    Y = []
    for d in range(cfg.D):
        print(f"cp full size: oracle sketch {d}", flush=True)
        want = O.fcs_cp_fft(None, U, hs[d], ss[d], cfg.J, L)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))
        Y.append(want)
    for p in range(0, cfg.pairs, 8):
        per_d = np.stack([O.contract_free_fft(Y[d], hs[d], ss[d], cfg.J, L, [u[p], v[p]])
                          for d in range(cfg.D)])
        want = O.median(per_d, axis=0)
        assert rel(est[p], want) <= TOL, (p, rel(est[p], want))


def test_cp_argument_errors():
    plan = Plan((8, 8), (4, 4), 2, 1, device=DEV)
    with pytest.raises(ValueError):
        plan.sketch_cp([dev(np.zeros((2, 8), np.float32))])
    z = dev(np.zeros((1, 8), np.float32))
    spec = torch.zeros((2, plan.spec_len, 2), device=DEV)
    with pytest.raises(ValueError):
        plan.contract_free_mode(spec, 5, [z, z])
    # the C entry point itself rejects a bad mode before any device work
    import ctypes
    from paper_2106_13062_amd import _lib as C
    ptrs = (ctypes.c_void_p * 2)(z.data_ptr(), z.data_ptr())
    out = torch.empty(8, dtype=torch.float64, device=DEV)
    ws = plan.workspace(C.OP_FREE_MODE, P=1)
    st = plan.lib.fcs_contract_free_mode(plan.handle, ctypes.c_void_p(spec.data_ptr()), 5, 1, ptrs,
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                         ws.numel(), None)
    assert st == C.FCS_EINVAL
    with pytest.raises(FcsError):
        plan.contract_free_mode(spec, 0, [None, z], ws=torch.empty(16, dtype=torch.uint8, device=DEV))
