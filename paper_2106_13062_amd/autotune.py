"""Measured tuning of the batched sketch launch (include/fcs.h, fcs_batch_*).

The batch has four free parameters that the work itself does not fix: the
transform split L = Q * P of every CP item (``tune_lengths``: the weight of
a count-sketch pass against an FFT point in the length model; fewer,
longer transforms repeat fewer count sketches), how many forward FFTs a CP
work tile holds (``tile_ffts``: small tiles balance the queue, large ones
write fewer partial spectra), how many persistent workgroups each FFT size
class keeps per compute unit (``wg_per_cu``: more hide latency, fewer leave
LDS and registers to each) and, per class, the transform structure of the
conjugate-symmetric slices (``no_pack``: two modes packed into one complex
transform and split by one LDS exchange, or one transform per mode).

``tune_batch`` times candidate configurations on the real batch (graph
replays, HIP events on the launch stream) by coordinate descent: first
``tile_ffts``, then the workgroups per CU of each populated class, then the
packing of each populated class, keeping a candidate only when it is faster.
Results can be cached in a JSON file keyed by a signature of the batch
shape.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

import torch

from .fcs import Batch

TILE_FFTS = (8, 16, 32, 64, 128)
WPC = (1, 2, 4, 8)
NCLASS = 7


def choose_length(I, J, gather_weight: float = 16.0, min_fft: int = 256, max_fft: int = 16384) -> int:
    """Transform length L = Q * P for a CP sketch, by the planner's cost
    model with a given weight of a count sketch (per bucket or entry)
    relative to one FFT point-stage: per stored slice, sum_n w (J_n + I_n)
    plus the inverse P log2 P, and P log2 P per forward transform, of which
    the conjugate-symmetric slices (q = 0 and, Q even, Q/2) need one per
    pair of modes when no hash is folded (J_n <= P).  A larger weight
    favours fewer, longer FFTs.  The library planner uses w = 16."""
    Jt = sum(J) - len(J) + 1
    N = len(J)
    best, best_L = None, 0
    P = min_fft
    while P <= max_fft:
        Q = -(-Jt // P)
        if Q <= 64:
            Qh = Q // 2 + 1
            fft = P * math.log2(P)
            folded = any(j > P for j in J)
            nself = 2 if (Q % 2 == 0 and Q > 1) else 1
            packed = N if folded else (N + 1) // 2
            cost = (Qh * (sum(gather_weight * (j + i) for i, j in zip(I, J)) + fft)
                    + fft * (nself * packed + (Qh - nself) * N))
            if best is None or cost < best:
                best, best_L = cost, P * Q
        P *= 2
    return best_L


def plan_for(kind: str, I, J, D: int, seed: int, device=None, gather_weight=None):
    """Bound plan for one batch item.  CP items take the transform length of
    the length model at `gather_weight` (None: the library planner's);
    Kronecker items take a 16384-point (or longer) transform, which gives
    their factor scatters 1024 threads."""
    from .fcs import Plan
    if kind == "kron":
        L = max(4 * int(J[0]), 16384)
    else:
        L = 0 if gather_weight is None else choose_length(I, J, gather_weight)
    return Plan(I, J, D, seed, L=L, device=device)


def batch_signature(items) -> str:
    """Shape signature of a batch: plan shapes, ranks and kinds."""
    h = hashlib.sha1()
    for it in items:
        p = it["plan"]
        R = 1 if it.get("kind") == "kron" else int(it["U"][0].shape[0])
        h.update(repr((it.get("kind", "cp"), p.I, p.J, p.D, p.L, R)).encode())
    return h.hexdigest()


def time_batch(batch: Batch, runs: int = 3, warmup: int = 1, stream=None) -> float:
    """Mean milliseconds of one graph replay of the batch."""
    s = torch.cuda.current_stream() if stream is None else stream
    for _ in range(warmup):
        batch.run(graph=True, stream=s)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(s)
    for _ in range(runs):
        batch.run(graph=True, stream=s)
    end.record(s)
    end.synchronize()
    return start.elapsed_time(end) / runs


def _trial(items, cfg, runs, warmup, device):
    b = Batch(items, config=cfg, device=device)
    try:
        ms = time_batch(b, runs, warmup)
        grids = list(b.grids)
    finally:
        b.close()
        del b
    return ms, grids


def tune_lengths(build_items, weights=(4.0, 16.0, 64.0), runs: int = 2, warmup: int = 1, device=None, log=None):
    """Pick the gather weight of the transform-length model by timing the
    batch built with each candidate (``build_items(weight)`` returns the
    items with plans made for that weight); returns (weight, items, table)."""
    table = []
    best_ms, best_w, best_items = None, None, None
    for w in weights:
        items = build_items(w)
        ms, _ = _trial(items, None, runs, warmup, device)
        table.append({"gather_weight": w, "ms": ms})
        if log:
            log(f"autotune lengths w={w} -> {ms:.3f} ms")
        if best_ms is None or ms < best_ms:
            best_ms, best_w, best_items = ms, w, items
        del items
    return best_w, best_items, table


def tune_batch(items, runs: int = 3, warmup: int = 1, cache: str | None = None, device=None, log=None):
    """Best launch configuration for this batch: (config dict, trial table)."""
    sig = batch_signature(items)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if sig in known:
            return known[sig]["config"], known[sig].get("trials", [])
    trials = []

    def run(cfg):
        ms, grids = _trial(items, cfg, runs, warmup, device)
        trials.append({"config": json.loads(json.dumps(cfg)), "ms": ms})
        if log:
            log(f"autotune {cfg} -> {ms:.3f} ms")
        return ms, grids

    best = {"tile_ffts": 32, "wg_per_cu": [0] * NCLASS, "no_pack": [0] * NCLASS}
    best_ms, grids = run(best)
    for tf in TILE_FFTS:
        if tf == best["tile_ffts"]:
            continue
        cfg = {"tile_ffts": tf, "wg_per_cu": list(best["wg_per_cu"]), "no_pack": list(best["no_pack"])}
        ms, _ = run(cfg)
        if ms < best_ms:
            best, best_ms = cfg, ms
    # classes present in the batch (non-zero persistent grid)
    present = [c for c in range(NCLASS) if grids[c] > 0]
    for c in present:
        for w in WPC:
            cfg = {"tile_ffts": best["tile_ffts"], "wg_per_cu": list(best["wg_per_cu"]),
                   "no_pack": list(best["no_pack"])}
            cfg["wg_per_cu"][c] = w
            if cfg == best:
                continue
            ms, _ = run(cfg)
            if ms < best_ms:
                best, best_ms = cfg, ms
    # transform structure per class: two modes per transform on the
    # conjugate-symmetric slices (fewer transforms, one more LDS exchange and
    # more live registers) or one transform per mode
    for c in present:
        cfg = {"tile_ffts": best["tile_ffts"], "wg_per_cu": list(best["wg_per_cu"]), "no_pack": list(best["no_pack"])}
        cfg["no_pack"][c] = 1 - cfg["no_pack"][c]
        ms, _ = run(cfg)
        if ms < best_ms:
            best, best_ms = cfg, ms
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[sig] = {"config": best, "ms": best_ms, "trials": trials}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(known, f, indent=1)
    return best, trials
