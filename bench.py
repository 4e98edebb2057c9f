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


# ---------------------------------------------------------------------------
# CPU baselines: the oracle as it stands, timed on the host cores with a
# process pool over independent pieces of work (sketches d, instances).  The
# pool is forked after the inputs exist, so the workers read them without a
# copy; they run only oracle code (numpy and the plain C brute force).
# ---------------------------------------------------------------------------
_POOL = {}


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pool_map(fn, items, cores):
    """(results, wall seconds, processes used) of fn over items, forked."""
    import multiprocessing as mp
    procs = max(1, min(cores, len(items)))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(fn, items, chunksize=1)
    return res, time.perf_counter() - t0, procs


def _dense_one(d):
    import oracle as O
    st = _POOL
    return O.dense_rows(st["T"], st["I"], [st["hs"][d]], [st["ss"][d]], st["Jt"], 0, st["rows"])


def dense_cpu_baseline(cfg, T, Jt, sample_rows):
    """The oracle (plain C FP64 brute force), one sketch per process, over
    the first `sample_rows` rows of the same tensor, scaled to sketches/s of
    the whole tensor."""
    import oracle as O
    rows = int(np.prod(cfg.I[1:]))
    sample_rows = min(rows, sample_rows)
    hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
    O.dense_rows(T, cfg.I, hs[:1], ss[:1], Jt, 0, 64)    # build and load the library
    _POOL.update(T=T, I=cfg.I, hs=hs, ss=ss, Jt=Jt, rows=sample_rows)
    _, dt, procs = _pool_map(_dense_one, list(range(cfg.D)), host_cores())
    _POOL.clear()
    full = dt * rows / sample_rows
    return {"value": cfg.D / full, "unit": "sketches/s", "cores": procs, "cpu": cpu_model(), "kind": "oracle",
            "sample": f"rows 0..{sample_rows} of {rows} (mode-0 fibres of the 1024^3 tensor), all {cfg.D} "
                      f"sketches, one per process, {dt:.2f} s wall, scaled to the full tensor"}


def _coo_one(d):
    import oracle as O
    st = _POOL
    return O.coo(st["idx"], st["val"], st["I"], [st["hs"][d]], [st["ss"][d]], st["Jt"])


def _cp_one(job):
    import oracle as O
    st = _POOL
    d, r0, r1 = job
    U = [u[:, r0:r1] for u in st["U"]]
    return O.fcs_cp_fft(None, U, st["hs"][d], st["ss"][d], st["J"], st["L"])


def _batch_one(k):
    import oracle as O
    import synth
    st = _POOL
    ins = st["insts"][k]
    F = ins.factors()
    hs, ss = O.hash_tables(ins.hash_seed, 1, ins.I, ins.J)
    if ins.kind == "kron":
        return O.kron_fcs(F[0].astype(np.float64), F[1].astype(np.float64), hs[0], ss[0], ins.J)
    return O.fcs_cp_fft(None, F, hs[0], ss[0], ins.J, int(2 ** np.ceil(np.log2(O.sketch_length(ins.J)))))


def cp_workload(args, torch, dev, cfg, pairs=0, inner=False):
    """CP sketch (and optionally T(I, u, v) for `pairs` vector pairs, and the
    inner product with a second CP tensor's sketch)."""
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
    # algorithmic work: D N R real-to-complex transforms of the power of two
    # L >= J~, 2.5 L log2 L flops each (half a complex transform)
    Lp2 = 1 << int(np.ceil(np.log2(plan.Jt)))
    alg_flop = cfg.D * len(cfg.I) * R * 2.5 * Lp2 * np.log2(Lp2)
    res = {"workload": cfg.name, "I": list(cfg.I), "J": list(cfg.J), "R": R, "D": cfg.D, "L": plan.L,
           "P": plan.P, "Q": plan.Q, "ms": ms, "sketches_per_s": cfg.D / (ms * 1e-3),
           "fft_gflop": fft_flop / 1e9, "fft_tflops": fft_flop / (ms * 1e-3) / 1e12,
           "alg_L": Lp2, "alg_gflop": alg_flop / 1e9, "alg_tflops": alg_flop / (ms * 1e-3) / 1e12,
           "frac_fp32_peak": alg_flop / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
    if Lp2 != plan.L and plan.Jt <= 65536:
        # the same sketch at the power-of-two length L = 2^k >= J~
        p2 = Plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed, L=Lp2, device=dev)
        ws2 = p2.workspace(2, R=R)
        out2 = torch.empty_like(out)
        p2.sketch_cp(Ud, out=out2, ws=ws2, stream=stream)
        ms2, _ = event_timer(torch, stream, lambda: p2.sketch_cp(Ud, out=out2, ws=ws2, stream=stream),
                             max(3, args.steps // 2))
        res["at_alg_L"] = {"L": Lp2, "P": p2.P, "Q": p2.Q, "ms": ms2, "sketches_per_s": cfg.D / (ms2 * 1e-3),
                           "frac_fp32_peak": alg_flop / (ms2 * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                           "rel_diff_vs_default_L": float(torch.linalg.norm((out2 - out).double())
                                                          / torch.linalg.norm(out.double()))}
        p2.close()
    if not args.no_cpu_baseline and cfg.R >= 64:
        import oracle as O
        hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
        rs = 32                                 # ranks per sample job (about 1 s of wall time)
        _POOL.update(U=U, hs=hs, ss=ss, J=cfg.J, L=Lp2)
        _, dt, procs = _pool_map(_cp_one, [(d, 0, rs) for d in range(cfg.D)], host_cores())
        _POOL.clear()
        full = dt * R / rs
        res["cpu_baseline"] = {"value": cfg.D / full, "unit": "sketches/s", "cores": procs, "cpu": cpu_model(),
                               "kind": "oracle", "sample": f"ranks 0..{rs} of {R} (FP64 FFT route, L = {Lp2}), all "
                               f"{cfg.D} sketches, one per process, {dt:.2f} s wall, scaled to all ranks"}
    if inner:
        # the order-3 I_n = 100 outputs: the sketch of a second random rank-R
        # CP tensor, the median over D of the sketch inner products
        # (Proposition 1), and the general-formula sketch of the
        # materialised tensor
        V = cfg.factors(stream=1)
        Vd = [torch.from_numpy(np.ascontiguousarray(v.T)).to(dev) for v in V]
        outb = torch.empty_like(out)
        wsi = plan.workspace(3)

        def inner_step():
            plan.sketch_cp(Ud, out=out, ws=ws, stream=stream)
            plan.sketch_cp(Vd, out=outb, ws=ws, stream=stream)
            return plan.contract_inner(out, outb, ws=wsi, stream=stream)

        med, per_d = inner_step()
        ims, _ = event_timer(torch, stream, inner_step, max(3, args.steps // 2))
        U64 = [u.astype(np.float64) for u in U]
        V64 = [v.astype(np.float64) for v in V]
        G = np.ones((R, R))
        for u, v in zip(U64, V64):
            G *= u.T @ v
        exact = float(G.sum())                 # <M, N> of the two CP tensors
        GM = np.ones((R, R))
        GN = np.ones((R, R))
        for u, v in zip(U64, V64):
            GM *= u.T @ u
            GN *= v.T @ v
        # the size of one sketch's estimation error, ||M|| ||N|| / sqrt(J~)
        noise = float(np.sqrt(GM.sum() * GN.sum() / plan.Jt))
        est = float(med.cpu()[0])
        Tm = np.einsum("ir,jr,kr->kji", *U64).reshape(-1).astype(np.float32)   # vec order, mode 0 fastest
        plan.sketch_cp(Ud, out=out, ws=ws, stream=stream)
        yd = plan.sketch_dense(torch.from_numpy(Tm).to(dev)).cpu().numpy().astype(np.float64)
        yc = out.cpu().numpy().astype(np.float64)
        res.update({"inner_ms": ims, "inner_estimate": est, "inner_exact": exact,
                    "inner_rel_error_vs_exact": abs(est - exact) / max(abs(exact), 1e-300),
                    "inner_noise_scale": noise,
                    "inner_per_sketch": [float(x) for x in per_d.cpu().numpy()],
                    "bruteforce_rel_l2": float(np.linalg.norm(yc - yd) / np.linalg.norm(yd))})
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
    res = {"workload": "dense1024 10% COO", "nnz": nnz, "ms": ms, "sketches_per_s": cfg.D / (ms * 1e-3),
           "alg_bytes": alg, "achieved_gbs": alg / (ms * 1e-3) / 1e9}
    if not args.no_cpu_baseline:
        import oracle as O
        sample = min(nnz, 1 << 24)
        hs, ss = O.hash_tables(cfg.hash_seed, cfg.D, cfg.I, cfg.J)
        _POOL.update(idx=np.ascontiguousarray(idx[:, :sample]), val=np.ascontiguousarray(val[:sample]),
                     I=cfg.I, hs=hs, ss=ss, Jt=plan.Jt)
        _, dt, procs = _pool_map(_coo_one, list(range(cfg.D)), host_cores())
        _POOL.clear()
        full = dt * nnz / sample
        res["cpu_baseline"] = {"value": cfg.D / full, "unit": "sketches/s", "cores": procs, "cpu": cpu_model(),
                               "kind": "oracle", "sample": f"first {sample} of {nnz} entries, all {cfg.D} "
                               f"sketches, one per process, {dt:.2f} s wall, scaled to all entries"}
    del idx, val
    return res


def batch_inputs(torch, dev, count):
    """Instances of the uneven batch (CP, and every 16th a Kronecker pair)
    with their factors resident on the device."""
    import synth
    insts = synth.batch_instances(count)
    facs = []
    for ins, F in synth.instance_inputs(insts):
        # CP: R x I_n rows (column-major factors); KRON: column-major A, B
        facs.append([torch.from_numpy(m).to(dev).t().contiguous() for m in F])
    return insts, facs


def batch_items(torch, dev, insts, facs, gather_weight=None):
    """Plans and outputs of every instance; CP transform lengths from the
    length model with the given gather weight (None: the planner's)."""
    from paper_2106_13062_amd.autotune import plan_for
    items = []
    for ins, U in zip(insts, facs):
        plan = plan_for(ins.kind, ins.I, ins.J, ins.D, ins.hash_seed, device=dev, gather_weight=gather_weight)
        items.append({"plan": plan, "kind": ins.kind, "U": U,
                      "out": torch.empty((ins.D, plan.Jt), dtype=torch.float32, device=dev)})
    return items


def batch_flops(items):
    """Forward and inverse FFT work of the batch (5 P log2 P per P-point
    complex transform), the quantity the batch kernels spend their time on."""
    total = 0.0
    for it in items:
        p = it["plan"]
        Qh = p.Q // 2 + 1
        per = 5.0 * p.P * np.log2(p.P)
        if it["kind"] == "kron":
            total += p.D * Qh * 3 * per
        else:
            R = int(it["U"][0].shape[0])
            total += p.D * Qh * (p.N * R + 1) * per
    return total


def batch_alg_flops(insts):
    """Algorithmic transform work of the batch: per CP instance D N R
    real-to-complex transforms of the power of two L >= J~ (2.5 L log2 L
    flops each); per Kronecker instance D x 2 such transforms (one per factor
    sketch)."""
    import oracle as O
    total = 0.0
    for ins in insts:
        L = 1 << int(np.ceil(np.log2(O.sketch_length(ins.J))))
        per = 2.5 * L * np.log2(L)
        total += ins.D * (2 if ins.kind == "kron" else len(ins.I) * ins.R) * per
    return total


def batch_workload(args, torch, dev):
    """Config of 4096 uneven CP / Kronecker sketches: one instance per
    launch (eager and graph-captured) against the autotuned persistent batch
    launch replayed from one hipGraph."""
    from paper_2106_13062_amd import Batch
    from paper_2106_13062_amd import _lib as C
    from paper_2106_13062_amd.autotune import time_batch, tune_batch, tune_lengths
    t0 = time.perf_counter()
    insts, facs = batch_inputs(torch, dev, args.batch_count)
    items = batch_items(torch, dev, insts, facs)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"batch: {len(items)} instances set up in {setup_s:.1f} s")
    stream = torch.cuda.current_stream()
    plain_out = [torch.empty_like(it["out"]) for it in items]
    wss = []
    for it in items:
        p = it["plan"]
        if it["kind"] == "kron":
            wss.append(p.workspace(C.OP_KRON))
        else:
            wss.append(p.workspace(C.OP_CP, R=int(it["U"][0].shape[0])))

    def plain():
        for it, o, w in zip(items, plain_out, wss):
            p = it["plan"]
            if it["kind"] == "kron":
                p.sketch_kron(it["U"][0], it["U"][1], out=o, ws=w, stream=stream)
            else:
                p.sketch_cp(it["U"], out=o, ws=w, stream=stream)

    plain()
    torch.cuda.synchronize()
    reps = max(1, args.batch_reps)
    t1 = time.perf_counter()
    for _ in range(reps):
        plain()
    torch.cuda.synchronize()
    plain_eager_ms = (time.perf_counter() - t1) * 1e3 / reps
    # the same launches captured into one graph: per-instance kernels
    # without the host's launch loop
    plain_graph_ms = None
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            stream = torch.cuda.current_stream()
            plain()
        stream = torch.cuda.current_stream()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        e1.synchronize()
        plain_graph_ms = e0.elapsed_time(e1) / reps
        del g
    except Exception as exc:  # capture not possible: report the eager path only
        log(f"plain path graph capture failed: {exc}")
        stream = torch.cuda.current_stream()
    # the batch with the planner's lengths and default launch configuration
    bd = Batch(items, device=dev)
    default_ms = time_batch(bd, runs=reps, warmup=1)
    bd.close()
    del bd
    # autotuned batch (tuning is not part of the timed region): transform
    # lengths first, then tile size and persistent grid per FFT size class
    t2 = time.perf_counter()
    cfg, trials, weight, len_table = None, [], None, []
    plain_items = items
    if args.tune:
        weight, items, len_table = tune_lengths(lambda w: batch_items(torch, dev, insts, facs, w),
                                                device=dev, log=log)
        cfg, trials = tune_batch(items, runs=2, warmup=1, device=dev, log=log)
    tune_s = time.perf_counter() - t2
    b = Batch(items, config=cfg, device=dev)
    batch_ms = time_batch(b, runs=reps, warmup=1)
    torch.cuda.synchronize()
    # the one-instance path on the tuned transform lengths as well
    plain_tuned_ms = None
    if items is not plain_items:
        tuned_out = [torch.empty_like(it["out"]) for it in items]
        twss = [it["plan"].workspace(C.OP_KRON) if it["kind"] == "kron"
                else it["plan"].workspace(C.OP_CP, R=int(it["U"][0].shape[0])) for it in items]

        def plain_tuned():
            for it, o, w in zip(items, tuned_out, twss):
                p = it["plan"]
                if it["kind"] == "kron":
                    p.sketch_kron(it["U"][0], it["U"][1], out=o, ws=w, stream=stream)
                else:
                    p.sketch_cp(it["U"], out=o, ws=w, stream=stream)

        plain_tuned()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(reps):
            plain_tuned()
        torch.cuda.synchronize()
        plain_tuned_ms = (time.perf_counter() - t3) * 1e3 / reps
        del tuned_out, twss
    # every batched sketch against its one-instance result
    worst = 0.0
    for it, o in zip(items, plain_out):
        a = it["out"].double()
        r = o.double()
        nr = torch.linalg.vector_norm(r).item()
        err = torch.linalg.vector_norm(a - r).item() / nr if nr > 0 else torch.linalg.vector_norm(a).item()
        worst = max(worst, err)
    n = len(items)
    nsk = sum(it["plan"].D for it in items)
    flops = batch_flops(items)
    plain_flops = batch_flops(plain_items)
    alg = batch_alg_flops(insts)
    base_ms = plain_graph_ms if plain_graph_ms is not None else plain_eager_ms
    if plain_tuned_ms is not None:
        base_ms = min(base_ms, plain_tuned_ms)
    res = {"workload": f"batch{n}: uneven CP (N 3-5, I_n log-uniform [32,4096], R 1-256, J_n 2^8-2^13), "
                       "every 16th a 256x256 Kronecker pair, D=1",
           "instances": n, "kron": sum(1 for i in insts if i.kind == "kron"), "tiles": b.tiles,
           "plain_eager_ms": plain_eager_ms, "plain_graph_ms": plain_graph_ms,
           "plain_tuned_lengths_ms": plain_tuned_ms,
           "batched_ms": batch_ms, "batched_default_cfg_ms": default_ms,
           "sketches_per_s_batched": nsk / (batch_ms * 1e-3),
           "sketches_per_s_plain": nsk / (base_ms * 1e-3),
           "speedup_vs_plain": base_ms / batch_ms,
           "speedup_vs_plain_eager": plain_eager_ms / batch_ms,
           "fft_tflops_batched": flops / (batch_ms * 1e-3) / 1e12,
           "fft_tflop_batched": flops / 1e12, "fft_tflop_plain": plain_flops / 1e12,
           "alg_tflop": alg / 1e12, "alg_tflops_batched": alg / (batch_ms * 1e-3) / 1e12,
           "frac_fp32_peak": alg / (batch_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
           "max_rel_err_vs_plain": worst, "tuned_config": cfg, "tuned_gather_weight": weight,
           "length_trials": len_table, "tune_s": tune_s, "tune_trials": len(trials), "setup_s": setup_s}
    b.close()
    if not args.no_cpu_baseline:
        step = max(1, n // 128)
        sample = list(range(0, n, step))
        _POOL.update(insts=insts)
        _, dt, procs = _pool_map(_batch_one, sample, host_cores())
        _POOL.clear()
        full = dt * n / len(sample)
        res["cpu_baseline"] = {"value": nsk / full, "unit": "sketches/s", "cores": procs, "cpu": cpu_model(),
                               "kind": "oracle", "sample": f"every {step}th instance ({len(sample)} of {n}, FP64 "
                               f"FFT route at L = 2^k >= J~), one per process, {dt:.2f} s wall, scaled to all"}
    return res


def serve_setup(torch, dev, args):
    """Server with the resident order-3 10^4 sketch (D = 10) and its bank of
    (u, v) pairs, CP build inputs from the uneven-batch shape distribution
    (D = 10) and COO tensors of order 3 (1024^3, J_n = 4096, D = 8) with nnz
    log-uniform in [1e4, 1e8], all pre-staged on the device."""
    import synth
    from paper_2106_13062_amd.serve import Server
    srv = Server(dev, streams=4, cap_bytes=200e9, max_group=256, max_inflight=8)
    cfg = synth.CP10K
    plan = srv.plan(cfg.I, cfg.J, cfg.D, cfg.hash_seed)
    U = [torch.from_numpy(u).to(dev).t().contiguous() for u in cfg.factors()]
    _, spec = plan.sketch_cp(U, want_out=False, want_spec=True)
    del U
    npairs = args.serve_pairs
    uv = synth.unit_vectors(cfg.data_seed, 2 * npairs, cfg.I[1], stream=6)
    srv.add_resident_sketch("cp10k", plan, spec, torch.from_numpy(uv[:npairs]).to(dev),
                            torch.from_numpy(uv[npairs:]).to(dev))
    insts = synth.batch_instances(args.serve_cp, seed=synth.DATA_SEED["batch4096"] + 17,
                                  hash_seed=synth.HASH_SEED["batch4096"] + 17, kron_every=0)
    for k, (ins, F) in enumerate(synth.instance_inputs(insts)):
        p = srv.plan(ins.I, ins.J, 10, ins.hash_seed)
        srv.add_input(f"cp{k}", "cp", p, [torch.from_numpy(u).to(dev).t().contiguous() for u in F])
    d = synth.DENSE1024
    pc = srv.plan(d.I, d.J, d.D, d.hash_seed)
    g = torch.Generator(device=dev)
    g.manual_seed(synth.DATA_SEED["dense1024"] + 5)
    nnzs = synth.coo_nnz_sizes(synth.DATA_SEED["dense1024"] + 5, args.serve_coo)
    for k, nnz in enumerate(nnzs):
        idx = torch.stack([torch.randint(0, i, (nnz,), generator=g, device=dev, dtype=torch.int32) for i in d.I])
        val = torch.randn(nnz, generator=g, device=dev)
        srv.add_input(f"coo{k}", "coo", pc, idx.contiguous(), val)
    torch.cuda.synchronize()
    return srv, nnzs


def serve_requests(srv, args, rate, count, seed):
    import synth
    reqs = []
    for rid, (t, kind, i) in enumerate(synth.serving_requests(seed, rate, count, args.serve_pairs,
                                                              args.serve_cp, args.serve_coo)):
        key = {"contract": "cp10k", "cp": f"cp{i}", "coo": f"coo{i}"}[kind]
        reqs.append(srv.make_request(rid, kind, t, key, index=i if kind == "contract" else 0))
    return reqs


def noise_std(sigma, R, I):
    """Per-entry standard deviation of the Gaussian noise at level sigma for
    the decomposition experiments: sigma is read as the noise-to-signal
    energy ratio, ||N||^2 = sigma ||T_clean||^2, with ||T_clean|| = sqrt(R)
    for unit weights and orthonormal factors (plain ALS then leaves exactly
    the residual sqrt(sigma), the value the paper prints for it)."""
    return np.sqrt(sigma) * np.sqrt(R) / I ** 1.5


def rtpm_workload(args, torch, dev):
    """Sketched robust tensor power method (Section 4.1.1, RTPM) in the setting of
    the paper's synthetic experiment: a symmetric 100^3 tensor of CP rank 10
    (orthonormal basis, unit weights) plus Gaussian noise at level 0.01 (an
    energy ratio, ||N|| = 0.1 ||T||), D = 2 sketches, 15 starts, 20 power
    iterations, J_n = 5000.  Timed: the dense sketch of the tensor plus the
    whole decomposition.  Quality: residual ||T - sum lam u o u o u|| / ||T||
    against the noisy and against the clean tensor, and the overlap of each
    component with the planted basis."""
    import synth
    from paper_2106_13062_amd import Plan
    from paper_2106_13062_amd.rtpm import rtpm
    I, R, D, L, iters, J, sigma = 100, 10, 2, 15, 20, 5000, 0.01
    Tv, A = synth.symmetric_cp_tensor(synth.DATA_SEED["rtpm100"], I, np.ones(R), noise_std(sigma, R, I))
    starts = torch.from_numpy(synth.rtpm_starts(synth.DATA_SEED["rtpm100"], R, L, I, stream=7)).to(dev)
    plan = Plan((I, I, I), (J, J, J), D, synth.HASH_SEED["rtpm100"], device=dev)
    T = torch.from_numpy(Tv.astype(np.float32)).to(dev)

    def run():
        y = plan.sketch_dense(T)
        return rtpm(plan, y, starts, iters)

    run()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        lam, U = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    Ud = U.double()
    approx = torch.einsum("r,ir,jr,kr->kji", lam.to(dev), Ud.T, Ud.T, Ud.T).reshape(-1)
    Td = T.double()
    resid = (torch.linalg.vector_norm(Td - approx) / torch.linalg.vector_norm(Td)).item()
    clean = torch.from_numpy(synth.symmetric_cp_tensor(synth.DATA_SEED["rtpm100"], I, np.ones(R))[0]).to(dev)
    resid_clean = (torch.linalg.vector_norm(clean - approx) / torch.linalg.vector_norm(clean)).item()
    overlap = np.abs(U.double().cpu().numpy() @ A).max(axis=1)
    return {"workload": "rtpm100: symmetric 100^3 CP rank 10 (orthonormal basis, unit weights) + Gaussian noise "
                        "at energy ratio 0.01 (||N|| = 0.1 ||T||), D=2, 15 starts, 20 iterations, J_n=5000", "ms": ms,
            "residual": resid, "noise_floor": float(np.sqrt(sigma)),
            "residual_vs_clean": resid_clean, "min_overlap": float(overlap.min()),
            "eigenvalues": [round(float(x), 5) for x in lam]}


def rtpm_asym_workload(args, torch, dev):
    """RTPM by alternating rank-1 updates (the asymmetric form of Section 4.1.1)
    on an asymmetric 100^3 tensor of CP rank 10 (three independent
    orthonormal factors, unit weights) plus Gaussian noise at energy ratio
    0.01, D = 10 (the paper's asymmetric experiments use 10 and 15),
    15 starts, 20 iterations, J_n = 5000.  Timed: the dense sketch plus the
    whole decomposition.  Quality: residual and the smallest overlap of a
    recovered vector with its planted factor."""
    import synth
    from paper_2106_13062_amd import Plan
    from paper_2106_13062_amd.rtpm import rtpm_asym
    I, R, D, L, iters, J, sigma = 100, 10, 10, 15, 20, 5000, 0.01
    Tv, F = synth.asymmetric_cp_tensor(synth.DATA_SEED["rtpm_asym100"], I, np.ones(R), noise_std(sigma, R, I))
    starts = torch.from_numpy(synth.rtpm_asym_starts(synth.DATA_SEED["rtpm_asym100"], R, L, I, stream=7)).to(dev)
    plan = Plan((I, I, I), (J, J, J), D, synth.HASH_SEED["rtpm_asym100"], device=dev)
    T = torch.from_numpy(Tv.astype(np.float32)).to(dev)

    def run():
        y = plan.sketch_dense(T)
        return rtpm_asym(plan, y, starts, iters)

    run()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        lam, X = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    Xd = [x.double() for x in X]
    approx = torch.einsum("r,ri,rj,rk->kji", lam.to(dev), *Xd).reshape(-1)
    Td = T.double()
    resid = (torch.linalg.vector_norm(Td - approx) / torch.linalg.vector_norm(Td)).item()
    overlap = min(float(np.abs(Xd[n].cpu().numpy() @ F[n]).max(axis=1).min()) for n in range(3))
    plan.close()
    return {"workload": "rtpm_asym100: asymmetric 100^3 CP rank 10 (orthonormal factors, unit weights) + noise at "
                        "energy ratio 0.01, D=10, 15 starts, 20 iterations, J_n=5000", "ms": ms, "residual": resid,
            "min_overlap": overlap, "eigenvalues": [round(float(x), 5) for x in lam]}


def rtpm50_workload(args, torch, dev):
    """Sketched RTPM in the setting of the paper's HCS-versus-FCS table: a
    symmetric 50^3 tensor of CP rank 10 (orthonormal basis, unit weights)
    plus Gaussian noise at energy ratio sigma in {0.01, 0.1}, J_n in
    {200, 300, 400} and D in {10, 20}, 15 starts and 20 iterations per
    component.  Each cell is timed (sketch plus decomposition) and reports
    the relative residual against the noisy tensor and against the clean
    one (the paper's values fall below the noise level at sigma = 0.1, so
    they measure the recovery of the clean tensor)."""
    import synth
    from paper_2106_13062_amd import Plan
    from paper_2106_13062_amd.rtpm import rtpm
    I, R, L, iters = 50, 10, 15, 20
    starts = torch.from_numpy(synth.rtpm_starts(synth.DATA_SEED["rtpm50"], R, L, I, stream=7)).to(dev)
    clean = torch.from_numpy(synth.symmetric_cp_tensor(synth.DATA_SEED["rtpm50"], I, np.ones(R))[0]).to(dev)
    cells = []
    for sigma in (0.01, 0.1):
        Tv, A = synth.symmetric_cp_tensor(synth.DATA_SEED["rtpm50"], I, np.ones(R), noise_std(sigma, R, I))
        T = torch.from_numpy(Tv.astype(np.float32)).to(dev)
        Td = T.double()
        for D in (10, 20):
            for J in (200, 300, 400):
                plan = Plan((I, I, I), (J, J, J), D, synth.HASH_SEED["rtpm50"], device=dev)

                def run():
                    y = plan.sketch_dense(T)
                    return rtpm(plan, y, starts, iters)

                run()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lam, U = run()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                Ud = U.double()
                approx = torch.einsum("r,ir,jr,kr->kji", lam.to(dev), Ud.T, Ud.T, Ud.T).reshape(-1)
                resid = (torch.linalg.vector_norm(Td - approx) / torch.linalg.vector_norm(Td)).item()
                resid_clean = (torch.linalg.vector_norm(clean - approx) / torch.linalg.vector_norm(clean)).item()
                cells.append({"sigma": sigma, "D": D, "J": J, "ms": ms, "residual": resid,
                              "residual_vs_clean": resid_clean})
                plan.close()
    return {"workload": "rtpm50: symmetric 50^3 CP rank 10 + noise at energy ratio 0.01 and 0.1, 15 starts, "
                        "20 iterations", "cells": cells}


def als_workload(args, torch, dev):
    """Sketched alternating least squares (Section 4.1.2, ALS) in the setting of
    the paper's synthetic experiment: an asymmetric 400^3 tensor of CP rank
    10 (three independent orthonormal factors, unit weights) plus Gaussian
    noise at energy ratio sigma in {0.01, 0.1} (plain ALS would leave
    residual sqrt(sigma): 0.1 and 0.316), D = 10 sketches, J_n = 5000, 20
    iterations.  Two starts: N(0, 1) factors, and the factors found by the
    sketched asymmetric power method (15 starts, 20 iterations) on the same
    sketch.  Timed: the dense sketch plus the whole decomposition (and the
    power method for the second start).  Quality: residual
    ||T - sum lam a o b o c|| / ||T|| against the noisy and the clean tensor,
    and the overlap of each recovered column with the planted factors."""
    import synth
    from paper_2106_13062_amd import Plan
    from paper_2106_13062_amd.als import als
    from paper_2106_13062_amd.rtpm import rtpm_asym
    I, R, D, iters, J = 400, 10, 10, 20, 5000
    plan = Plan((I, I, I), (J, J, J), D, synth.HASH_SEED["als400"], device=dev)
    rand_init = [torch.from_numpy(f).to(dev) for f in synth.als_init(synth.DATA_SEED["als400"], I, R, stream=9)]
    starts = torch.from_numpy(synth.rtpm_asym_starts(synth.DATA_SEED["als400"], R, 15, I, stream=11)).to(dev)
    cleanv, F = synth.asymmetric_cp_tensor(synth.DATA_SEED["als400"], I, np.ones(R))
    clean = torch.from_numpy(cleanv).to(dev)
    del cleanv
    runs = []
    for sigma in (0.01, 0.1):
        Tv, _ = synth.asymmetric_cp_tensor(synth.DATA_SEED["als400"], I, np.ones(R), noise_std(sigma, R, I))
        T = torch.from_numpy(Tv.astype(np.float32)).to(dev)
        del Tv
        Td = T.double()
        for start in ("random", "rtpm"):

            def run():
                y = plan.sketch_dense(T)
                if start == "random":
                    init = rand_init
                else:
                    _, X = rtpm_asym(plan, y, starts, 20)
                    init = [x.t().contiguous() for x in X]
                return als(plan, y, init, iters)

            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, G = run()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            Gd = [g.double() for g in G]
            approx = torch.einsum("r,ir,jr,kr->kji", lam, *Gd).reshape(-1)
            resid = (torch.linalg.vector_norm(Td - approx) / torch.linalg.vector_norm(Td)).item()
            resid_clean = (torch.linalg.vector_norm(clean - approx) / torch.linalg.vector_norm(clean)).item()
            del approx
            overlap = min(float(np.abs(Gd[n].cpu().numpy().T @ F[n]).max(axis=1).min()) for n in range(3))
            runs.append({"sigma": sigma, "start": start, "ms": ms, "residual": resid,
                         "residual_vs_clean": resid_clean, "plain_als_residual": float(np.sqrt(sigma)),
                         "min_overlap": overlap, "weights": [round(float(x), 5) for x in lam.cpu()]})
        del T, Td
        torch.cuda.empty_cache()
    plan.close()
    return {"workload": "als400: asymmetric 400^3 CP rank 10 (orthonormal factors, unit weights) + Gaussian noise "
                        "at energy ratio 0.01 and 0.1, D=10, J_n=5000, 20 iterations from random or power-method "
                        "starts", "runs": runs}


def decompress_workload(args, torch, dev):
    """Decompression (Section 4.3) of the Kronecker product of two 256 x 256
    U[-5, 5] matrices: 2^32 recovered entries (16 GiB) written as the
    column-major (I_0 I_2) x (I_1 I_3) matrix, J_n = 4096, D = 1, 3 and 20
    sketches (median over D).  Timed with HIP events on the launch stream;
    algorithmic HBM bytes per launch are the output (4 B per entry) plus one
    read of the sketches and hash words.  Also, end to end on the paper's
    set-ups with D = 20 and J_n = 4096: the Kronecker product of A 30 x 40
    and B 40 x 50, and the contraction of A 30 x 40 x 50 with B 50 x 40 x 30
    over the shared index (compression, then decompression)."""
    import synth
    from paper_2106_13062_amd import Plan
    stream = torch.cuda.current_stream()
    I, J = (256, 256, 256, 256), (4096, 4096, 4096, 4096)
    g = synth.rng(synth.DATA_SEED["batch4096"], 31)
    A = torch.from_numpy(g.uniform(-5, 5, 256 * 256).astype(np.float32)).to(dev)
    B = torch.from_numpy(g.uniform(-5, 5, 256 * 256).astype(np.float32)).to(dev)
    M = 1 << 32
    out = torch.empty(M, dtype=torch.float32, device=dev)
    runs = []
    for D in (1, 3, 20):
        plan = Plan(I, J, D, synth.HASH_SEED["batch4096"] + D, device=dev)
        y, _ = plan.sketch_kron(A, B)

        def step():
            plan.decompress(y, order=(2, 0, 3, 1), out=out, stream=stream)

        step()
        ms, _ = event_timer(torch, stream, step, max(3, args.steps // 4))
        nbytes = 4.0 * M + 4.0 * D * plan.Jt + 4.0 * D * sum(I)
        gbs = nbytes / (ms * 1e-3) / 1e9
        runs.append({"D": D, "ms": ms, "entries_per_s": M / (ms * 1e-3), "GB_per_s": gbs,
                     "frac_hbm": gbs / HBM_PEAK_GBS, "bytes_per_launch": nbytes})
        plan.close()
    del out
    torch.cuda.empty_cache()
    # the paper's set-ups, compression and decompression, D = 20
    D, Jp = 20, (4096, 4096, 4096, 4096)
    Ak = torch.from_numpy(g.uniform(-5, 5, 30 * 40).astype(np.float32)).to(dev)
    Bk = torch.from_numpy(g.uniform(-5, 5, 40 * 50).astype(np.float32)).to(dev)
    pk = Plan((30, 40, 40, 50), Jp, D, 77, device=dev)
    outk = torch.empty(30 * 40 * 40 * 50, dtype=torch.float32, device=dev)
    wsk = pk.workspace(6)
    yk = torch.empty((D, pk.Jt), dtype=torch.float32, device=dev)
    kc, _ = event_timer(torch, stream, lambda: pk.sketch_kron(Ak, Bk, out=yk, ws=wsk, stream=stream), 5)
    kd, _ = event_timer(torch, stream, lambda: pk.decompress(yk, order=(2, 0, 3, 1), out=outk, stream=stream), 5)
    Ac = torch.from_numpy(g.uniform(0, 10, 30 * 40 * 50).astype(np.float32)).to(dev)
    Bc = torch.from_numpy(g.uniform(0, 10, 50 * 40 * 30).astype(np.float32)).to(dev)
    pc = Plan((30, 40, 40, 30), Jp, D, 78, device=dev)
    outc = torch.empty(30 * 40 * 40 * 30, dtype=torch.float32, device=dev)
    wsc = pc.workspace(7, R=50)
    yc = torch.empty((D, pc.Jt), dtype=torch.float32, device=dev)
    cc, _ = event_timer(torch, stream, lambda: pc.sketch_contraction(Ac, Bc, out=yc, ws=wsc, stream=stream), 5)
    cd, _ = event_timer(torch, stream, lambda: pc.decompress(yc, out=outc, stream=stream), 5)
    return {"workload": "decompress256: A (x) B of two 256 x 256 matrices, 2^32 entries (16 GiB) in matrix "
                        "layout, J_n=4096", "runs": runs,
            "paper_kron_30x40_40x50_D20": {"compress_ms": kc, "decompress_ms": kd},
            "paper_contraction_30x40x50_50x40x30_D20": {"compress_ms": cc, "decompress_ms": cd}}


def serve_workload(args, torch, dev):
    """Poisson request streams at several rates through the continuous
    batching server, against the same requests served one at a time."""
    from paper_2106_13062_amd.serve import Request, latency_stats, run_alone
    t0 = time.perf_counter()
    srv, nnzs = serve_setup(torch, dev, args)
    log(f"serve: set up in {time.perf_counter() - t0:.1f} s (COO nnz {nnzs})")
    # warm every kind of launch (allocator, first-use attributes)
    for r in serve_requests(srv, args, 1e3, 64, 999):
        run_alone(srv, r)
    srv.run(serve_requests(srv, args, 5e4, 256, 998), timeout=120)
    torch.cuda.synchronize()
    rates = [float(x) for x in args.serve_rates.split(",")]
    out = {"workload": "serve: Poisson mix of 90% T(I,u,v) on the resident order-3 10^4 D=10 sketch, "
                       "8% CP builds (uneven-batch shapes, D=10), 2% COO sketches (1024^3, D=8, nnz "
                       "log-uniform 1e4-1e8); admission cap 200 GB, 4 streams",
           "rates": []}
    for k, rate in enumerate(rates):
        n = int(min(args.serve_max, max(200, rate * args.serve_seconds)))
        reqs = serve_requests(srv, args, rate, n, 100 + k)
        wall = srv.run(reqs, timeout=300)
        st = latency_stats(reqs)
        sk = sum(r.sketches for r in reqs)
        row = {"offered_req_s": rate, "requests": n, "wall_s": wall, "served_req_s": n / wall,
               "sketches_per_s": sk / wall, **st}
        out["rates"].append(row)
        log(f"serve rate {rate:g}: {row}")
        for r in reqs:
            r.result = None
    # one request at a time on the same stream, each waited for
    reqs = serve_requests(srv, args, rates[-1], int(min(args.serve_max, 4000)), 100 + len(rates) - 1)
    torch.cuda.synchronize()
    service = {}
    t1 = time.perf_counter()
    for r in reqs:
        ta = time.perf_counter()
        run_alone(srv, r)
        service.setdefault(r.kind, []).append(time.perf_counter() - ta)
        r.result = None
    plain_s = time.perf_counter() - t1
    sk = sum(r.sketches for r in reqs)
    out["plain"] = {"requests": len(reqs), "wall_s": plain_s, "req_s": len(reqs) / plain_s,
                    "sketches_per_s": sk / plain_s,
                    "mean_service_ms": {k: 1e3 * float(np.mean(v)) for k, v in service.items()}}
    best = max(out["rates"], key=lambda x: x["served_req_s"])
    out["served_vs_plain_req_s"] = best["served_req_s"] / out["plain"]["req_s"]
    # the plain path at each offered rate: the same arrivals through one
    # first-come first-served server whose service times are the measured
    # one-at-a-time times of requests of the same kind
    for k, row in enumerate(out["rates"]):
        reqs = serve_requests(srv, args, row["offered_req_s"], row["requests"], 100 + k)
        pos = {kind: 0 for kind in service}
        free = 0.0
        lat = []
        for r in sorted(reqs, key=lambda q: q.arrival):
            v = service[r.kind]
            sv = v[pos[r.kind] % len(v)]
            pos[r.kind] += 1
            start = max(r.arrival, free)
            free = start + sv
            lat.append(free - r.arrival)
        makespan = free - min(r.arrival for r in reqs)
        plain_rate = len(reqs) / makespan
        row["plain_req_s"] = plain_rate
        row["plain_p50_ms"] = float(np.percentile(lat, 50) * 1e3)
        row["plain_p99_ms"] = float(np.percentile(lat, 99) * 1e3)
        row["served_vs_plain_req_s"] = row["served_req_s"] / plain_rate
        arr = sorted(r.arrival for r in reqs)
        row["arrival_req_s"] = (len(arr) - 1) / max(arr[-1] - arr[0], 1e-9)
        # saturated: completions fall clearly behind the arrivals
        row["saturated"] = bool(row["served_req_s"] < 0.9 * row["arrival_req_s"])
        row["plain_saturated"] = bool(plain_rate < 0.9 * row["arrival_req_s"])
    # the highest offered rate the loop keeps up with, and its latencies
    ok = [row for row in out["rates"] if not row["saturated"]]
    if ok:
        top = max(ok, key=lambda x: x["offered_req_s"])
        out["highest_unsaturated"] = {"offered_req_s": top["offered_req_s"], "served_req_s": top["served_req_s"],
                                      "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
                                      "vs_plain_capacity": top["served_req_s"] / out["plain"]["req_s"]}
    # alone-versus-mix parity on a sample of a mixed run
    reqs = serve_requests(srv, args, rates[len(rates) // 2], 600, 4242)
    srv.run(reqs, timeout=120)
    worst = 0.0
    for r in reqs[::6]:
        alone = Request(r.rid, r.kind, 0.0, r.key, r.index)
        run_alone(srv, alone)
        a = (r.result[0][r.result[1]] if r.kind == "contract" else r.result).double()
        b = (alone.result[0][alone.result[1]] if r.kind == "contract" else alone.result).double()
        nb = torch.linalg.vector_norm(b).item()
        worst = max(worst, torch.linalg.vector_norm(a - b).item() / (nb if nb > 0 else 1.0))
    out["max_rel_err_mix_vs_alone"] = worst
    return out


def copy_ceiling_gbs(torch, dev, nbytes=1 << 30, reps=10):
    """Measured HBM ceiling: a plain device-to-device copy of nbytes (read
    once, written once), timed with HIP events, in GB/s of bytes moved."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def lds_atomic_ceiling(torch, dev, cfg, kernel_ms, reps=5):
    """LDS-atomic ceiling of the dense scatter: fcs_probe_lds_atomics on the
    dense kernel's grid (one 1024-thread workgroup per last-mode slab and
    group of four sketches, every row of the slab adding its I_0 = 1024
    columns to four windows of J_0 + J_1 - 1 bins), the same atomics with no
    loads or conversions, timed with HIP events on the launch stream; with
    random column bins and with conflict-free bins."""
    from paper_2106_13062_amd.fcs import probe_lds_atomics
    I, J = list(cfg.I), list(cfg.J)
    rows = int(np.prod(I[1:-1]))
    blocks = I[-1] * (cfg.D // 4)
    window, span = J[0] + J[1] - 1, J[0]
    stream = torch.cuda.current_stream()
    sink = torch.empty(blocks, dtype=torch.int32, device=dev)
    res = {"atomics_per_launch": blocks * rows * 1024 * 4, "kernel_ms": kernel_ms}
    for name, pattern in (("random_bins", 0), ("conflict_free", 1)):
        def fn():
            probe_lds_atomics(blocks, rows, window, span, pattern, 1, sink=sink, stream=stream)
        fn()
        torch.cuda.synchronize()
        ms, _ = event_timer(torch, stream, fn, reps)
        if not bool((sink == rows * 4096).all().item()):
            raise RuntimeError("LDS-atomic probe lost additions")
        res[name + "_ms"] = ms
        res["kernel_vs_" + name] = ms / kernel_ms
    return res


def lds_atomic_sweep(torch, dev, reps=5):
    """fcs_probe_lds_atomics over window sizes at the dense1024 launch's
    atomic count (2048 workgroups x 1024 rows x 4096 atomics): four
    8191-bin windows fill LDS (one workgroup per CU, as in the dense
    scatter); 4096 bins and below let two or more workgroups share a CU.
    Rate = lanes added per clock and CU at 2.4 GHz."""
    from paper_2106_13062_amd.fcs import probe_lds_atomics
    stream = torch.cuda.current_stream()
    blocks, rows = 2048, 1024
    sink = torch.empty(blocks, dtype=torch.int32, device=dev)
    out = []
    for window, span in ((8191, 4096), (4096, 2048), (2048, 1024), (1024, 1024)):
        for pattern in (0, 1):
            def fn():
                probe_lds_atomics(blocks, rows, window, span, pattern, 1, sink=sink, stream=stream)
            fn()
            torch.cuda.synchronize()
            ms, _ = event_timer(torch, stream, fn, reps)
            if not bool((sink == rows * 4096).all().item()):
                raise RuntimeError("LDS-atomic probe lost additions")
            lanes = blocks * rows * 4096 / (256 * ms * 1e-3 * 2.4e9)
            out.append({"window": window, "span": span,
                        "bins": "random" if pattern == 0 else "conflict-free",
                        "ms": ms, "lanes_per_clock_per_cu": lanes})
    return out


def copy_calibration(torch, dev, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the profiled kernels."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def _recovery_error(torch, got, want):
    return float(torch.linalg.norm(got.double() - want.double()) / torch.linalg.norm(want.double()))


def compare_workload(args, torch, dev):
    """The paper's Kronecker and contraction compression experiments (Section
    4.3) with FCS against the long-hash count sketch (CS: Definition 1 on
    vec(T), an order-1 plan over all prod I_n entries) and the higher-order
    count sketch (HCS: Definition 3, an HCS plan with the same per-mode hash
    pairs), D = 20, at compression ratios CR = prod I_n / J~ (HCS: per-mode
    hash length round(J~^(1/4))).  Kronecker: A 30 x 40 and B 40 x 50, U[-5, 5];
    contraction: A 30 x 40 x 50 and B 50 x 40 x 30, U[0, 10], over the shared
    index.  Per method: compression and decompression time (HIP events),
    relative error of the recovered tensor, hash-function memory (the packed
    (h, s) words, 4 B per index and sketch) and the bound plan's table
    bytes.  FCS compresses from the factors; CS and HCS compress the
    materialised tensor, whose construction (torch, on the device) is timed
    apart.  Also Proposition 1's variance comparison under equal hash
    functions: inner-product estimates of FCS, TS (the mod-J fold of the
    same sketches) and HCS over many independent hash draws."""
    import synth
    from paper_2106_13062_amd import Plan, inner_median
    stream = torch.cuda.current_stream()
    g = synth.rng(synth.DATA_SEED["batch4096"], 41)
    D = 20
    reps = max(3, args.steps // 4)
    out = {}

    def methods(name, I, make_full, fcs_compress, crs):
        n = int(np.prod(I))
        full = make_full()
        t_mat, _ = event_timer(torch, stream, make_full, reps)
        rows = []
        for cr in crs:
            Jt = n // cr
            row = {"CR": cr, "Jt_target": Jt}
            J = (Jt + 3) // 4
            try:
                pf = Plan(I, (J,) * 4, D, 91, device=dev)
            except Exception as e:          # no transform length fits
                pf = None
                row["fcs"] = {"error": str(e)}
            if pf is not None:
                y = fcs_compress(pf)
                c_ms, _ = event_timer(torch, stream, lambda: fcs_compress(pf), reps)
                rec = pf.decompress(y)
                d_ms, _ = event_timer(torch, stream, lambda: pf.decompress(y, out=rec, stream=stream), reps)
                row["fcs"] = {"J": J, "Jt": pf.Jt, "compress_ms": c_ms, "decompress_ms": d_ms,
                              "rel_error": _recovery_error(torch, rec, full),
                              "hash_bytes": 4 * D * sum(I), "plan_table_bytes": int(pf.tables.numel())}
                pf.close()
            pc = Plan((n,), (Jt,), D, 92, device=dev)
            wsc = pc.workspace(0)
            y = pc.sketch_dense(full, ws=wsc)
            c_ms, _ = event_timer(torch, stream, lambda: pc.sketch_dense(full, out=y, ws=wsc, stream=stream), reps)
            rec = pc.decompress(y)
            d_ms, _ = event_timer(torch, stream, lambda: pc.decompress(y, out=rec, stream=stream), reps)
            row["cs"] = {"Jt": pc.Jt, "compress_ms": c_ms, "compress_with_materialise_ms": c_ms + t_mat,
                         "decompress_ms": d_ms, "rel_error": _recovery_error(torch, rec, full),
                         "hash_bytes": 4 * D * n, "plan_table_bytes": int(pc.tables.numel())}
            pc.close()
            Jh = max(1, int(round(Jt ** 0.25)))
            ph = Plan(I, (Jh,) * 4, D, 93, device=dev, hcs=True)
            wsh = ph.workspace(0)
            y = ph.sketch_dense(full, ws=wsh)
            c_ms, _ = event_timer(torch, stream, lambda: ph.sketch_dense(full, out=y, ws=wsh, stream=stream), reps)
            rec = ph.decompress(y)
            d_ms, _ = event_timer(torch, stream, lambda: ph.decompress(y, out=rec, stream=stream), reps)
            row["hcs"] = {"J": Jh, "Jt": ph.Jt, "compress_ms": c_ms, "compress_with_materialise_ms": c_ms + t_mat,
                          "decompress_ms": d_ms, "rel_error": _recovery_error(torch, rec, full),
                          "hash_bytes": 4 * D * sum(I), "plan_table_bytes": int(ph.tables.numel())}
            ph.close()
            if "hash_bytes" in row.get("fcs", {}):
                row["fcs_hash_memory_vs_cs"] = row["fcs"]["hash_bytes"] / row["cs"]["hash_bytes"]
            rows.append(row)
            torch.cuda.empty_cache()
        out[name] = {"I": list(I), "entries": n, "materialise_ms": t_mat, "rows": rows}

    # Kronecker product A (x) B as the order-4 tensor T[a, b, c, d] = A[a, b] B[c, d]
    A = torch.from_numpy(g.uniform(-5, 5, (30, 40)).astype(np.float32)).to(dev)
    B = torch.from_numpy(g.uniform(-5, 5, (40, 50)).astype(np.float32)).to(dev)
    Ak, Bk = A.t().contiguous(), B.t().contiguous()          # column-major matrices
    wsk = {}

    def kron_fcs(p):
        if p.Jt not in wsk:
            wsk[p.Jt] = p.workspace(6)
        return p.sketch_kron(Ak, Bk, ws=wsk[p.Jt], stream=stream)[0]

    methods("kron_30x40_40x50", (30, 40, 40, 50),
            lambda: torch.einsum("ab,cd->dcba", A, B).contiguous().reshape(-1), kron_fcs, (4, 8, 16, 32, 64))
    wsk.clear()
    # contraction C[a, b, c, d] = sum_l A[a, b, l] B[l, c, d]
    Ac = torch.from_numpy(g.uniform(0, 10, (30, 40, 50)).astype(np.float32)).to(dev)
    Bc = torch.from_numpy(g.uniform(0, 10, (50, 40, 30)).astype(np.float32)).to(dev)
    Acm = Ac.permute(2, 1, 0).contiguous().reshape(-1)       # column-major (a fastest)
    Bcm = Bc.permute(2, 1, 0).contiguous().reshape(-1)       # column-major (l fastest)
    wsc = {}

    def contraction_fcs(p):
        if p.Jt not in wsc:
            wsc[p.Jt] = p.workspace(7, R=50)
        return p.sketch_contraction(Acm, Bcm, ws=wsc[p.Jt], stream=stream)[0]

    methods("contraction_30x40x50_50x40x30", (30, 40, 40, 30),
            lambda: torch.einsum("abl,lcd->dcba", Ac, Bc).contiguous().reshape(-1), contraction_fcs,
            (4, 8, 16, 32, 64))
    wsc.clear()
    torch.cuda.empty_cache()

    # Proposition 1: variance of the inner-product estimate under equal hash
    # functions, FCS (J~ = 3J - 2 bins) against TS (its fold modulo J) and
    # HCS (per-mode length round((3J - 2)^(1/3))), one sketch per hash draw
    I, J, K = (30, 30, 30), 64, 2000
    M = synth.dense_tensor(50, I)
    Nn = (M + synth.dense_tensor(51, I)).astype(np.float32)
    exact = float(np.dot(M.astype(np.float64), Nn.astype(np.float64)))
    Md, Nd = torch.from_numpy(M).to(dev), torch.from_numpy(Nn).to(dev)
    Jh = int(round((3 * J - 2) ** (1.0 / 3.0)))
    est = {"fcs": [], "ts": [], "hcs": []}
    for k in range(K):
        p = Plan(I, (J,) * 3, 1, 10_000 + k, device=dev)
        ya, yb = p.sketch_dense(Md), p.sketch_dense(Nd)
        est["fcs"].append(p.contract_inner(ya, yb)[0])
        est["ts"].append(inner_median(p.ts_fold(ya), p.ts_fold(yb))[0])
        h = Plan(I, (Jh,) * 3, 1, 10_000 + k, device=dev, hcs=True)
        est["hcs"].append(h.contract_inner(h.sketch_dense(Md), h.sketch_dense(Nd))[0])
    prop1 = {"I": list(I), "J": J, "hcs_J": Jh, "draws": K, "exact": exact,
             "norm_M_norm_N": float(np.linalg.norm(M) * np.linalg.norm(Nn))}
    for k_, v in est.items():
        v = torch.cat(v).cpu().numpy()
        prop1[k_] = {"mean": float(v.mean()), "var": float(v.var(ddof=1)),
                     "mean_within_5_std_err": bool(abs(v.mean() - exact) <= 5 * v.std(ddof=1) / np.sqrt(K))}
    prop1["var_fcs_over_var_ts"] = prop1["fcs"]["var"] / prop1["ts"]["var"]
    out["prop1_variance"] = prop1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1 << 20,
                    help="rows of the tensor the CPU oracle sketches")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "dense1024_traffic.json"))
    ap.add_argument("--mode", default="full", choices=["full", "dense", "coo", "cp", "batch", "serve", "rtpm", "als", "decompress", "compare",
                                                       "copy", "lds"],
                    help="full: headline + secondary workloads; dense: headline only; cp: the CP "
                         "sketches and T(I,u,v) only; batch: the uneven batch only; serve: the "
                         "serving loop only; copy: plain copy kernel for counter calibration; lds: "
                         "LDS-atomic probe over window sizes")
    ap.add_argument("--batch-count", type=int, default=4096, help="instances of the uneven batch")
    ap.add_argument("--batch-reps", type=int, default=3, help="timed passes of each batch path")
    ap.add_argument("--no-tune", dest="tune", action="store_false", help="skip the batch autotuner")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000,30000,40000,50000",
                    help="offered request rates (1/s)")
    ap.add_argument("--serve-seconds", type=float, default=0.5, help="arrival span per rate")
    ap.add_argument("--serve-max", type=int, default=25000, help="most requests per rate")
    ap.add_argument("--serve-pairs", type=int, default=1024, help="(u, v) pairs in the bank")
    ap.add_argument("--serve-cp", type=int, default=32, help="pre-staged CP build inputs")
    ap.add_argument("--serve-coo", type=int, default=6, help="pre-staged COO tensors")
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
    if args.mode == "lds":
        print(json.dumps({"lds_atomic_sweep": lds_atomic_sweep(torch, dev)}), flush=True)
        return
    if args.mode == "batch":
        print(json.dumps({"batch": batch_workload(args, torch, dev)}), flush=True)
        return
    if args.mode == "serve":
        print(json.dumps({"serve": serve_workload(args, torch, dev)}), flush=True)
        return
    if args.mode == "rtpm":
        print(json.dumps({"rtpm": rtpm_workload(args, torch, dev),
                          "rtpm50": rtpm50_workload(args, torch, dev),
                          "rtpm_asym": rtpm_asym_workload(args, torch, dev)}), flush=True)
        return
    if args.mode == "als":
        print(json.dumps({"als": als_workload(args, torch, dev)}), flush=True)
        return
    if args.mode == "coo":
        import synth
        cfg = synth.DENSE1024
        T = synth.dense_tensor(cfg.data_seed, cfg.I)
        print(json.dumps({"coo": coo_workload(args, torch, dev, T)}), flush=True)
        return
    if args.mode == "decompress":
        print(json.dumps({"decompress": decompress_workload(args, torch, dev)}), flush=True)
        return
    if args.mode == "compare":
        print(json.dumps({"compare": compare_workload(args, torch, dev)}), flush=True)
        return
    if args.mode == "cp":
        import synth
        print(json.dumps({"cp100": cp_workload(args, torch, dev, synth.CP100, inner=True),
                          "cp10k": cp_workload(args, torch, dev, synth.CP10K, pairs=synth.CP10K.pairs)}),
              flush=True)
        return
    cfg, res, cpu, T = dense_workload(args, torch, dev)
    copy_gbs = copy_ceiling_gbs(torch, dev)
    lds_ceiling = lds_atomic_ceiling(torch, dev, cfg, res["event_ms"])
    secondary = {}
    if args.mode == "full":
        import synth
        log("secondary: cp100")
        secondary["cp100"] = cp_workload(args, torch, dev, synth.CP100, inner=True)
        log("secondary: cp10k + T(I,u,v)")
        secondary["cp10k"] = cp_workload(args, torch, dev, synth.CP10K, pairs=synth.CP10K.pairs)
        log("secondary: coo")
        secondary["coo"] = coo_workload(args, torch, dev, T)
        del T
        T = None
        log("secondary: uneven batch")
        secondary["batch"] = batch_workload(args, torch, dev)
        torch.cuda.empty_cache()
        log("secondary: serving loop")
        secondary["serve"] = serve_workload(args, torch, dev)
        log("secondary: sketched RTPM")
        secondary["rtpm"] = rtpm_workload(args, torch, dev)
        secondary["rtpm50"] = rtpm50_workload(args, torch, dev)
        secondary["rtpm_asym"] = rtpm_asym_workload(args, torch, dev)
        log("secondary: sketched ALS")
        secondary["als"] = als_workload(args, torch, dev)
        torch.cuda.empty_cache()
        log("secondary: decompression and contraction compression")
        secondary["decompress"] = decompress_workload(args, torch, dev)
        torch.cuda.empty_cache()
        log("secondary: CS / HCS / FCS comparison and Proposition 1 variances")
        secondary["compare"] = compare_workload(args, torch, dev)
    del T
    # HBM traffic per launch from the committed FETCH_SIZE / WRITE_SIZE
    # summary, only while the kernel source is the one that was measured
    traffic = None
    if os.path.exists(args.traffic_json):
        import hashlib
        with open(args.traffic_json) as f:
            t = json.load(f)
        src = os.path.join(ROOT, t.get("source", ""))
        if os.path.isfile(src):
            with open(src, "rb") as f:
                if hashlib.sha1(f.read()).hexdigest()[:12] == t.get("source_sha1"):
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
                     "alg_bytes_per_launch": res["alg_bytes"],
                     "copy_ceiling": copy_gbs, "frac_of_copy_ceiling": res["achieved_gbs"] / copy_gbs,
                     "lds_atomic": lds_ceiling},
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
