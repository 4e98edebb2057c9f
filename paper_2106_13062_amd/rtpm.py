"""Robust tensor power method on fast count sketches (Section 4.1.1 of the
paper: RTPM for a symmetric order-3 tensor, with the contractions of
Section 4.1 estimated from D sketches).

For each component k:
  * power iterations u <- T(I,u,u) / ||T(I,u,u)|| from ``L`` starting
    vectors at once: T(I,u,u) is the free-mode contraction of the sketch
    spectra (fcs_contract_free_mode, median over the D sketches);
  * the eigenvalue T(u,u,u) of every start: the median over d of
    <FCS_d(T), FCS_d(u o u o u)>, all L starts in one fcs_contract_full
    launch on the (deflated) spectra;
  * the start with the largest eigenvalue is kept, and the sketch and its
    spectra are deflated by linearity:
    FCS(T - lam u o u o u) = FCS(T) - lam FCS(u o u o u).

The starting vectors are inputs (the random draws of the method).  Every
step runs in the library's kernels: the sketches and contractions, the
normalisation of the estimated vectors (fcs_normalize_rows), the choice of
the best start (fcs_select_max, which leaves the chosen vector and its
eigenvalue on the device) and the deflation (fcs_axpy); torch only holds
the device memory, and the host reads the eigenvalues once at the end.
"""
from __future__ import annotations

import torch

from .fcs import Plan, axpy, normalize_rows, select_max


def rtpm(plan: Plan, y: torch.Tensor, starts: torch.Tensor, iters: int, stream=None):
    """plan: bound Plan of shape (I, I, I); y: float32 D x J~ sketch of the
    tensor (not modified); starts: float32 rank x L x I starting vectors.
    Returns (eigenvalues float64 [rank] on the host, components float32
    rank x I on the device)."""
    if plan.N != 3 or not (plan.I[0] == plan.I[1] == plan.I[2]):
        raise ValueError("RTPM needs a plan of a cubic order-3 shape")
    rank, L, I = (int(x) for x in starts.shape)
    if I != plan.I[0]:
        raise ValueError("starting vectors must have I entries")
    s = torch.cuda.current_stream() if stream is None else stream
    with torch.cuda.stream(s):
        y = y.clone()
        spec = plan.spectrum(y, stream=s)
        lams = torch.empty(rank, dtype=torch.float64, device=y.device)
        lam32 = torch.empty(rank, dtype=torch.float32, device=y.device)
        comps = torch.empty((rank, I), dtype=torch.float32, device=y.device)
        for k in range(rank):
            U = normalize_rows(starts[k].to(torch.float32).contiguous(), stream=s)
            for _ in range(iters):
                W = plan.contract_free_mode(spec, 0, [None, U, U], stream=s)
                U = normalize_rows(W, stream=s)
            lam, _ = plan.contract_full(spec, [U, U, U], stream=s)
            u = comps[k:k + 1]
            select_max(lam, U, row_out=u, val_out=lam32[k:k + 1], val64_out=lams[k:k + 1], stream=s)
            yk, sk = plan.sketch_cp([u, u, u], lam=lam32[k:k + 1], want_spec=True, stream=s)
            axpy(-1.0, yk, y, stream=s)
            axpy(-1.0, sk, spec, stream=s)
    return lams.cpu(), comps


def rtpm_asym(plan: Plan, y: torch.Tensor, starts: torch.Tensor, iters: int, stream=None):
    """RTPM for an asymmetric order-3 tensor: the power iteration becomes an
    alternating rank-1 update, u <- T(I,v,w), v <- T(u,I,w), w <- T(u,v,I),
    each normalised (one batched free-mode contraction per mode and
    iteration, all L starts at once); the eigenvalue T(u,v,w) of every
    start from one full contraction; the best start is deflated from the
    sketch and its spectra by linearity.
    plan: bound Plan of an order-3 shape; y: float32 D x J~ sketch (not
    modified); starts: float32 rank x L x 3 x max(I_n) starting vectors
    (mode n uses the first I_n entries of slot n).  Returns (eigenvalues
    float64 [rank] on the host, three float32 rank x I_n component
    matrices on the device)."""
    if plan.N != 3:
        raise ValueError("RTPM needs a plan of an order-3 shape")
    rank, L, three, Imax = (int(x) for x in starts.shape)
    if three != 3 or Imax < max(plan.I):
        raise ValueError("starting vectors must be rank x L x 3 x max(I_n)")
    s = torch.cuda.current_stream() if stream is None else stream
    with torch.cuda.stream(s):
        y = y.clone()
        spec = plan.spectrum(y, stream=s)
        lams = torch.empty(rank, dtype=torch.float64, device=y.device)
        lam32 = torch.empty(rank, dtype=torch.float32, device=y.device)
        comps = [torch.empty((rank, plan.I[n]), dtype=torch.float32, device=y.device) for n in range(3)]
        for k in range(rank):
            X = [normalize_rows(starts[k, :, n, :plan.I[n]].to(torch.float32).contiguous(), stream=s)
                 for n in range(3)]
            for _ in range(iters):
                for n in range(3):
                    vecs = [None if m == n else X[m] for m in range(3)]
                    G = plan.contract_free_mode(spec, n, vecs, stream=s)
                    X[n] = normalize_rows(G, stream=s)
            lam, _ = plan.contract_full(spec, X, stream=s)
            x = [comps[n][k:k + 1] for n in range(3)]
            for n in range(3):
                select_max(lam, X[n], row_out=x[n], val_out=lam32[k:k + 1], val64_out=lams[k:k + 1], stream=s)
            yk, sk = plan.sketch_cp(x, lam=lam32[k:k + 1], want_spec=True, stream=s)
            axpy(-1.0, yk, y, stream=s)
            axpy(-1.0, sk, spec, stream=s)
    return lams.cpu(), comps
