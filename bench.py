"""Benchmark of the fast count sketch hot path on one MI355X.

Default workload (the headline figure): dense general-tensor FCS of a
1024 x 1024 x 1024 float32 N(0,1) tensor, J_n = 4096 (J~ = 12286), D = 8
sketches from one pass over T.  A step is one call of fcs_sketch_dense on the
resident tensor; value = D * steps / elapsed (sketches/s).

Prints ONE JSON line with the metric, a roofline object for the dominant
kernel (algorithmic bytes per launch / HIP-event launch time vs 8 TB/s HBM)
and the CPU oracle timed on a bounded sample of the same workload.
Secondary figures (CP sketch, contractions, batched and served paths) are
added under "secondary" when their paths are built.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
METRIC = "FCS sketches/s + % HBM roofline; batched/served vs plain, p50/p99 ms"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def event_timer(torch, stream, fn, steps):
    """Average HIP-event duration of fn() over `steps` calls on `stream`."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for k in range(steps):
        starts[k].record(stream)
        fn()
        ends[k].record(stream)
    torch.cuda.synchronize()
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return float(np.mean(ms)), ms


def dense_workload(args, torch, dev):
    import synth
    from paper_2106_13062_amd import Plan

    cfg = synth.DENSE1024
    log("generating the 1024^3 tensor")
    T = synth.dense_tensor(cfg.data_seed, cfg.I)
    Td = torch.from_numpy(T).to(dev)
    plan = Plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed, device=dev)
    out = torch.empty((cfg.D, plan.Jt), dtype=torch.float32, device=dev)
    ws = plan.workspace(0)
    stream = torch.cuda.current_stream()

    def step():
        plan.sketch_dense(Td, out=out, ws=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: exactly K steps between two synchronisations
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-launch duration of the dominant kernel with HIP events, same stream
    ev_ms, _ = event_timer(torch, stream, step, args.steps)
    elems = int(np.prod(cfg.I))
    alg_bytes = 4 * elems                   # every entry of T read once
    achieved = alg_bytes / (ev_ms * 1e-3) / 1e9
    res = {
        "value": cfg.D * args.steps / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "event_ms": ev_ms,
        "achieved_gbs": achieved,
        "alg_bytes": alg_bytes,
        "Jt": plan.Jt,
    }
    cpu = None
    if not args.no_cpu_baseline:
        cpu = dense_cpu_baseline(cfg, T, plan.Jt, args.cpu_rows)
    del Td
    torch.cuda.empty_cache()
    return cfg, res, cpu, T


def dense_cpu_baseline(cfg, T, Jt, sample_rows):
    """The oracle (plain C FP64 brute force) on the first `sample_rows` rows
    of the same tensor, scaled to sketches/s of the whole tensor."""
    import oracle as O
    rows = int(np.prod(cfg.I[1:]))
    sample_rows = min(rows, sample_rows)
    hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
    O.dense_rows(T, cfg.I, hs, ss, Jt, 0, 64)    # load and warm the library
    t0 = time.perf_counter()
    O.dense_rows(T, cfg.I, hs, ss, Jt, 0, sample_rows)
    dt = time.perf_counter() - t0
    full = dt * rows / sample_rows
    return {"value": cfg.D / full, "unit": "sketches/s", "cores": 1, "kind": "oracle",
            "sample": f"rows 0..{sample_rows} of {rows} (mode-0 fibres of the 1024^3 tensor), "
                      f"all {cfg.D} sketches, {dt:.2f} s, scaled to the full tensor"}


def cp_workload(args, torch, dev, cfg, pairs=0):
    """CP sketch (and optionally T(I, u, v) for `pairs` vector pairs)."""
    import synth
    from paper_2106_13062_amd import Plan
    U = cfg.factors()
    plan = Plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed, device=dev)
    Ud = [torch.from_numpy(np.ascontiguousarray(u.T)).to(dev) for u in U]
    R = cfg.R
    out = torch.empty((cfg.D, plan.Jt), dtype=torch.float32, device=dev)
    spec = torch.empty((cfg.D, plan.spec_len, 2), dtype=torch.float32, device=dev)
    ws = plan.workspace(2, R=R)
    stream = torch.cuda.current_stream()

    def step():
        plan.sketch_cp(Ud, out=out, spec=spec, want_spec=True, ws=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    ms, _ = event_timer(torch, stream, step, max(3, args.steps // 2))
    lg = np.log2(plan.P)
    # forward transforms: D sketches x stored slices x R ranks x N modes,
    # 5 P log2 P flops each (the usual complex radix-2 count)
    fft_flop = cfg.D * (plan.Q // 2 + 1) * R * len(cfg.I) * 5.0 * plan.P * lg
    res = {"workload": cfg.name, "I": list(cfg.I), "J": list(cfg.J), "R": R, "D": cfg.D, "L": plan.L,
           "P": plan.P, "Q": plan.Q, "ms": ms, "sketches_per_s": cfg.D / (ms * 1e-3),
           "fft_gflop": fft_flop / 1e9, "fft_tflops": fft_flop / (ms * 1e-3) / 1e12,
           "frac_fp32_peak": fft_flop / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
    if pairs:
        uv = synth.unit_vectors(cfg.data_seed, 2 * pairs, cfg.I[1], stream=5)
        u = torch.from_numpy(uv[:pairs]).to(dev)
        v = torch.from_numpy(uv[pairs:]).to(dev)
        outv = torch.empty((pairs, cfg.I[0]), dtype=torch.float64, device=dev)
        wsf = plan.workspace(4, P=pairs)

        def contract():
            plan.contract_free_mode(spec, 0, [None, u, v], out=outv, ws=wsf, stream=stream)

        contract()
        cms, _ = event_timer(torch, stream, contract, max(3, args.steps // 2))
        res.update({"pairs": pairs, "contract_ms": cms, "contractions_per_s": pairs / (cms * 1e-3)})
    return res


def coo_workload(args, torch, dev, T):
    """10 % Bernoulli COO copy of the dense tensor, int32 coordinates."""
    import synth
    from paper_2106_13062_amd import Plan
    cfg = synth.DENSE1024
    idx, val = synth.bernoulli_coo(cfg.data_seed, T, cfg.I, cfg.density)
    nnz = val.size
    idx_d = torch.from_numpy(idx).to(dev)
    val_d = torch.from_numpy(val).to(dev)
    del idx, val
    plan = Plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed, device=dev)
    out = torch.empty((cfg.D, plan.Jt), dtype=torch.float32, device=dev)
    ws = plan.workspace(1)
    stream = torch.cuda.current_stream()

    def step():
        plan.sketch_coo(idx_d, val_d, out=out, ws=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    ms, _ = event_timer(torch, stream, step, max(3, args.steps // 2))
    alg = 16 * nnz
    return {"workload": "dense1024 10% COO", "nnz": nnz, "ms": ms, "sketches_per_s": cfg.D / (ms * 1e-3),
            "alg_bytes": alg, "achieved_gbs": alg / (ms * 1e-3) / 1e9}


def copy_calibration(torch, dev, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the profiled kernels."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1 << 19,
                    help="rows of the tensor the CPU oracle sketches")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "dense1024_traffic.json"))
    ap.add_argument("--mode", default="full", choices=["full", "dense", "copy"],
                    help="full: headline + secondary workloads; dense: headline only; "
                         "copy: plain copy kernel for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.mode == "copy":
        copy_calibration(torch, dev)
        return
    cfg, res, cpu, T = dense_workload(args, torch, dev)
    secondary = {}
    if args.mode == "full":
        import synth
        log("secondary: cp100")
        secondary["cp100"] = cp_workload(args, torch, dev, synth.CP100)
        log("secondary: cp10k + T(I,u,v)")
        secondary["cp10k"] = cp_workload(args, torch, dev, synth.CP10K, pairs=synth.CP10K.pairs)
        log("secondary: coo")
        secondary["coo"] = coo_workload(args, torch, dev, T)
    del T
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            t = json.load(f)
        traffic = t.get("bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "sketches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense1024: order-3 1024^3 float32 N(0,1) tensor, J_n=4096 (J~=12286), "
                               "D=8 sketches in one pass", "I": list(cfg.I), "J": list(cfg.J), "D": cfg.D},
        "roofline": {"bound": "hbm", "achieved": res["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": res["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "dense_scatter_kernel", "launch_ms": res["event_ms"],
                     "alg_bytes_per_launch": res["alg_bytes"]},
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
