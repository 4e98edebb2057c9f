"""Alternating least squares on fast count sketches (Section 4.1.2 of the paper:
ALS for an order-3 tensor, with the contractions of Section 4.1 estimated
from D sketches).

Each iteration updates modes 0, 1, 2 in turn.  The update of mode n needs
the mode-n unfolding of T times the Khatri-Rao product of the other two
factors; its column r is the contraction of T with the r-th columns of the
other factors at their own modes and the identity at mode n, and all R
columns come from one batched free-mode contraction of the sketch spectra
(fcs_contract_free_mode with P = R vector pairs, median over the D
sketches).  The least-squares solve against the Hadamard product of the
other factors' R x R Gram matrices (Cholesky, in double) and the
normalisation of the columns into the weights run in one library call
(fcs_als_update); torch only holds the device memory.
"""
from __future__ import annotations

import torch

from .fcs import Plan, als_update


def als(plan: Plan, y: torch.Tensor, init, iters: int, stream=None):
    """plan: bound Plan of an order-3 shape; y: float32 D x J~ sketch of the
    tensor; init: three float32 I_n x R starting factors (device).
    Returns (weights float64 [R] on the device, three float32 I_n x R
    factors with unit columns on the device)."""
    if plan.N != 3:
        raise ValueError("ALS needs a plan of an order-3 shape")
    if len(init) != 3:
        raise ValueError("ALS needs three starting factors")
    R = int(init[0].shape[1])
    for n, f in enumerate(init):
        if tuple(f.shape) != (plan.I[n], R):
            raise ValueError(f"starting factor {n} must be I_{n} x R")
    s = torch.cuda.current_stream() if stream is None else stream
    with torch.cuda.stream(s):
        spec = plan.spectrum(y, stream=s)
        # factors kept transposed (R x I_n, row-major): the layout of the
        # contraction's vector arguments
        Ft = [f.to(torch.float32).t().contiguous() for f in init]
        lam = torch.ones(R, dtype=torch.float64, device=y.device)
        for _ in range(iters):
            for n in range(3):
                o = [m for m in range(3) if m != n]
                vecs = [None, None, None]
                for m in o:
                    vecs[m] = Ft[m]
                Mt = plan.contract_free_mode(spec, n, vecs, stream=s)       # R x I_n, float64
                Ft[n], lam = als_update(Mt, [Ft[m] for m in o], stream=s)
    return lam, [f.t().contiguous() for f in Ft]
