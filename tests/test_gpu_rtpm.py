"""Sketched robust tensor power method on the GPU (Section 4.1.1, RTPM) against
the FP64 oracle run on the same inputs: same tensor, same hash tables (the
plan's), same starting vectors.  Every eigenvalue agrees to 1e-5 relative
(the bar of a single FP32 contraction: the power iterations do not amplify
the contractions' rounding, measured maxima are below 1e-6) and every
component to 1 - |<u_gpu, u_oracle>| <= 1e-9 (1 - cos is quadratic in the
angle, about 1e-12 measured)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from paper_2106_13062_amd import Plan
from paper_2106_13062_amd.rtpm import rtpm

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("I,J,D,w,noise,L,iters", [
    (20, 2048, 3, (3.0, 2.0, 1.0), 0.0, 5, 12),
    (32, 1024, 2, (4.0, 3.0, 2.0, 1.0), 0.01, 4, 10),
    (100, 5000, 2, (3.0, 2.0, 1.0), 0.0003, 5, 10),     # the paper's I_n = 100, J_n = 5000, D = 2
])
def test_rtpm_matches_oracle(I, J, D, w, noise, L, iters):
    R = len(w)
    Tv, A = synth.symmetric_cp_tensor(12, I, w, noise)
    starts = synth.rtpm_starts(32, R, L, I)
    plan = Plan((I, I, I), (J, J, J), D, 22, device=DEV)
    y = plan.sketch_dense(torch.from_numpy(Tv.astype(np.float32)).to(DEV))
    lam_g, U_g = rtpm(plan, y, torch.from_numpy(starts).to(DEV), iters)
    torch.cuda.synchronize()
    lam_g = lam_g.numpy()
    U_g = U_g.cpu().numpy().astype(np.float64)
    hs, ss = O.hash_tables(22, D, (I, I, I), (J, J, J))
    T = Tv.astype(np.float32).astype(np.float64).reshape((I, I, I), order="F")
    Y = np.stack([O.fcs_dense(T, hs[d], ss[d], (J, J, J)) for d in range(D)])
    lam_o, U_o = O.rtpm(Y, hs, ss, (J, J, J), R, starts, iters)
    print(f"max relative weight difference {np.max(np.abs(lam_g - lam_o) / np.abs(lam_o)):.3e}", flush=True)
    assert np.all(np.abs(lam_g - lam_o) <= 1e-5 * np.abs(lam_o)), (lam_g, lam_o)
    agree = np.abs(np.sum(U_g * U_o, axis=1)) / np.linalg.norm(U_g, axis=1)
    print(f"max 1 - |cos| {np.max(1.0 - agree):.3e}", flush=True)
    assert np.all(1.0 - agree <= 1e-9), agree
    # and both found the planted basis in weight order
    assert list(np.abs(U_g @ A).argmax(axis=1)) == list(range(R))


@pytest.mark.parametrize("I,J,D,w,noise,L,iters", [
    (20, 2048, 3, (3.0, 2.0, 1.0), 0.0, 4, 10),
    (24, 2048, 2, (4.0, 3.0, 2.0, 1.0), 0.01, 3, 8),
])
def test_asymmetric_rtpm_matches_oracle(I, J, D, w, noise, L, iters):
    from paper_2106_13062_amd.rtpm import rtpm_asym
    print(f"asymmetric rtpm I={I} J={J} D={D} R={len(w)}", flush=True)
    R = len(w)
    Tv, F = synth.asymmetric_cp_tensor(14, I, w, noise)
    starts = synth.rtpm_asym_starts(34, R, L, I)
    plan = Plan((I, I, I), (J, J, J), D, 24, device=DEV)
    y = plan.sketch_dense(torch.from_numpy(Tv.astype(np.float32)).to(DEV))
    lam_g, X_g = rtpm_asym(plan, y, torch.from_numpy(starts).to(DEV), iters)
    torch.cuda.synchronize()
    lam_g = lam_g.numpy()
    X_g = [x.cpu().numpy().astype(np.float64) for x in X_g]
    hs, ss = O.hash_tables(24, D, (I, I, I), (J, J, J))
    T = Tv.astype(np.float32).astype(np.float64).reshape((I, I, I), order="F")
    Y = np.stack([O.fcs_dense(T, hs[d], ss[d], (J, J, J)) for d in range(D)])
    lam_o, X_o = O.rtpm_asym(Y, hs, ss, (J, J, J), R, starts, iters)
    print(f"max relative weight difference {np.max(np.abs(lam_g - lam_o) / np.abs(lam_o)):.3e}", flush=True)
    assert np.all(np.abs(lam_g - lam_o) <= 1e-5 * np.abs(lam_o)), (lam_g, lam_o)
    for n in range(3):
        agree = np.abs(np.sum(X_g[n] * X_o[n], axis=1)) / np.linalg.norm(X_g[n], axis=1)
        print(f"mode {n}: max 1 - |cos| {np.max(1.0 - agree):.3e}", flush=True)
        assert np.all(1.0 - agree <= 1e-9), (n, agree)
        assert list(np.abs(X_g[n] @ F[n]).argmax(axis=1)) == list(range(R))
