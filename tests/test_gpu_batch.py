"""GPU parity of the Kronecker sketch (Section 4.3) and of the batched uneven
CP / Kronecker path: every item of a batch equals the same computation done
alone (fcs_sketch_cp / fcs_sketch_kron), graph replays equal direct
launches, and sampled items match the FP64 oracle.  Bar: relative L2 error
<= 1e-5 per sketch."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from paper_2106_13062_amd import Batch, FcsError, Plan

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = 1e-5


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def colmajor(M):
    """Matrix -> device tensor holding it in column-major order."""
    return dev(np.ascontiguousarray(np.asarray(M, dtype=np.float32).T))


@pytest.mark.parametrize("I,J,D,L", [
    ((20, 30, 25, 15), (16, 32, 8, 16), 3, 0),
    ((256, 256, 256, 256), (256, 256, 256, 256), 2, 1024),
    ((256, 256, 256, 256), (8192, 8192, 8192, 8192), 1, 32768),
    ((7, 1, 1, 9), (1, 5, 3, 2), 2, 0),
])
def test_kron_parity(I, J, D, L):
    print(f"kron I={I} J={J} D={D}", flush=True)
    seed = 17
    A = synth.uniform_matrix(5, (I[0], I[1]), stream=1)
    B = synth.uniform_matrix(5, (I[2], I[3]), stream=2)
    plan = Plan(I, J, D, seed, L=L, device=DEV)
    y, spec = plan.sketch_kron(colmajor(A), colmajor(B), want_spec=True)
    y = y.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    for d in range(D):
        want = O.kron_fcs(A32, B32, hs[d], ss[d], J)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))
    # the spectrum is that of the sketch
    spec2 = plan.spectrum(torch.from_numpy(y).to(DEV))
    assert rel(spec.cpu().numpy(), spec2.cpu().numpy()) <= 10 * TOL


def test_kron_nonfinite_and_errors():
    I, J = (4, 5, 6, 3), (8, 8, 8, 8)
    plan = Plan(I, J, 1, 3, device=DEV)
    A = np.ones((4, 5), np.float32)
    A[1, 2] = np.inf
    y, _ = plan.sketch_kron(colmajor(A), colmajor(np.ones((6, 3), np.float32)))
    assert torch.isnan(y).all()
    p3 = Plan((4, 5, 6), (8, 8, 8), 1, 3, device=DEV)
    with pytest.raises(ValueError):
        p3.sketch_kron(colmajor(A), colmajor(A))
    with pytest.raises(FcsError):   # J~ = 1.2e6 exceeds every transform length (64 x 16384)
        Plan((2, 2, 2, 2), (300000,) * 4, 1, 3, device=DEV).sketch_kron(dev(np.ones(4, np.float32)),
                                                                        dev(np.ones(4, np.float32)))


@pytest.mark.parametrize("J", [20000, 150000])
def test_kron_long_hashes_sum_factor_bins_in_global_memory(J):
    """The paper's Kronecker set-up (A 30 x 40, B 40 x 50, U[-5, 5]) at hash
    lengths whose 64-bit factor-sketch bins exceed LDS (J~ = 4J - 3 up to
    about 6e5, a compression ratio of 4): the bins are summed in global
    memory, and the sketch still matches the oracle."""
    I, D, seed = (30, 40, 40, 50), 2, 23
    A = synth.uniform_matrix(21, (30, 40), stream=1)
    B = synth.uniform_matrix(21, (40, 50), stream=2)
    plan = Plan(I, (J,) * 4, D, seed, device=DEV)
    y, _ = plan.sketch_kron(colmajor(A), colmajor(B))
    y = y.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, (J,) * 4)
    for d in range(D):
        want = O.kron_fcs(A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64),
                          hs[d], ss[d], (J,) * 4)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))


def test_kron_dense_factors_with_global_64bit_bins():
    """Factor matrices with more than four entries per factor-sketch bin
    (400 x 400 and 300 x 300 into J_0 + J_1 - 1 = 29999 bins, too many for
    LDS): the bins stay 64-bit fixed point, in global memory, and the sketch
    (three stored slices, so computed as a one-slice contraction) matches
    the oracle."""
    I, J, D, seed = (400, 400, 300, 300), (15000,) * 4, 2, 29
    A = synth.uniform_matrix(22, (400, 400), stream=1)
    B = synth.uniform_matrix(22, (300, 300), stream=2)
    plan = Plan(I, J, D, seed, device=DEV)
    y, _ = plan.sketch_kron(colmajor(A), colmajor(B))
    y = y.cpu().numpy()
    hs, ss = O.hash_tables(seed, D, I, J)
    for d in range(D):
        want = O.kron_fcs(A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64),
                          hs[d], ss[d], J)
        assert rel(y[d], want) <= TOL, (d, rel(y[d], want))


def _instances(count, seed, kron_every=5, I_range=(8, 400), R_range=(1, 40), logJ_range=(5, 11)):
    return synth.batch_instances(count, seed=seed, hash_seed=seed + 7, kron_every=kron_every,
                                 I_range=I_range, R_range=R_range, logJ_range=logJ_range)


def _make_items(insts, D=1, kron_I=None):
    items, plans, host = [], [], []
    for k, ins in enumerate(insts):
        if ins.kind == "kron":
            I = kron_I or ins.I
            A = synth.uniform_matrix(ins.seed, (I[0], I[1]), stream=1)
            B = synth.uniform_matrix(ins.seed, (I[2], I[3]), stream=2)
            plan = Plan(I, ins.J, D, ins.hash_seed, L=max(4 * ins.J[0], 256), device=DEV)
            items.append({"plan": plan, "kind": "kron", "U": [colmajor(A), colmajor(B)]})
            host.append(("kron", I, [A, B], None))
        else:
            U = synth.cp_factors(ins.seed, ins.I, ins.R)
            lam = np.linspace(0.5, 1.5, ins.R).astype(np.float32) if k % 3 == 0 else None
            plan = Plan(ins.I, ins.J, D, ins.hash_seed, device=DEV)
            items.append({"plan": plan, "kind": "cp", "U": [dev(np.ascontiguousarray(u.T)) for u in U],
                          "lam": None if lam is None else dev(lam)})
            host.append(("cp", ins.I, U, lam))
        plans.append(plan)
    return items, plans, host


def _alone(item):
    plan = item["plan"]
    if item["kind"] == "kron":
        y, _ = plan.sketch_kron(*item["U"])
    else:
        y, _ = plan.sketch_cp(item["U"], lam=item.get("lam"))
    return y


def _oracle(plan, host, d):
    kind, I, F, lam = host
    hs, ss = O.hash_tables(plan.seed, plan.D, I, plan.J)
    if kind == "kron":
        A32, B32 = (x.astype(np.float32).astype(np.float64) for x in F)
        return O.kron_fcs(A32, B32, hs[d], ss[d], plan.J)
    return O.fcs_cp_fft(lam, F, hs[d], ss[d], plan.J, plan.L)


@pytest.mark.parametrize("D,cfg", [(1, None), (3, {"tile_ffts": 4}), (2, {"tile_ffts": 200, "wg_per_cu": [1] * 7}),
                                   (2, {"no_pack": [1, 0, 1, 0, 1, 0, 1]})])
def test_batch_equals_alone_and_oracle(D, cfg):
    insts = _instances(40, seed=900 + D)
    items, plans, host = _make_items(insts, D=D, kron_I=(40, 30, 20, 50))
    print(f"batch D={D} cfg={cfg}: {len(items)} items", flush=True)
    b = Batch(items, config=cfg, device=DEV)
    outs = b.run(graph=False)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    for k, it in enumerate(items):
        want = _alone(it).cpu().numpy()
        for d in range(D):
            assert rel(got[k][d], want[d]) <= TOL, (k, d, rel(got[k][d], want[d]))
    for k in range(0, len(items), 7):
        for d in range(D):
            w = _oracle(plans[k], host[k], d)
            assert rel(got[k][d], w) <= TOL, (k, d, rel(got[k][d], w))


def test_batch_graph_replays():
    """One captured graph replayed several times, with other device work and
    synchronisations in between: every replay equals the direct launch."""
    insts = _instances(24, seed=77)
    items, _, _ = _make_items(insts, D=2, kron_I=(16, 24, 32, 8))
    b = Batch(items, device=DEV)
    ref = [o.clone() for o in b.run(graph=False)]
    torch.cuda.synchronize()
    for rep in range(4):
        for it in items:
            it["out"].fill_(float("nan"))
        x = torch.randn(1 << 20, device=DEV)
        (x * 2).sum().item()
        b.run(graph=True)
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            assert rel(it["out"].cpu().numpy(), ref[k].cpu().numpy()) <= TOL, (rep, k)


def test_batch_rank_zero_and_spec_only():
    I, J = (30, 20, 10), (16, 16, 16)
    p1 = Plan(I, J, 2, 1, device=DEV)
    p2 = Plan(I, J, 2, 2, device=DEV)
    U = synth.cp_factors(3, I, 4)
    spec = torch.empty((2, p2.spec_len, 2), device=DEV)
    items = [{"plan": p1, "kind": "cp", "U": [torch.empty((0, i), device=DEV) for i in I]},
             {"plan": p2, "kind": "cp", "U": [dev(np.ascontiguousarray(u.T)) for u in U], "spec": spec}]
    items[0]["out"] = torch.full((2, p1.Jt), 7.0, device=DEV)
    b = Batch(items, device=DEV)
    b.run(graph=True)
    torch.cuda.synchronize()
    assert torch.count_nonzero(items[0]["out"]).item() == 0
    _, want = p2.sketch_cp([dev(np.ascontiguousarray(u.T)) for u in U], want_out=False, want_spec=True)
    assert rel(spec.cpu().numpy(), want.cpu().numpy()) <= TOL


def test_batch_errors():
    p = Plan((8, 8, 8), (4, 4, 4), 1, 1, device=DEV)
    with pytest.raises(ValueError):
        Batch([{"plan": p, "kind": "kron", "U": []}], device=DEV)
    with pytest.raises(ValueError):
        Batch([{"plan": p, "kind": "bogus", "U": []}], device=DEV)
    b = Batch([], device=DEV)
    b.run(graph=True)
    b.run(graph=False)


def test_batch_full_size_sampled_parity():
    """The 4096-instance uneven batch (order 3-5, I_n up to 4096, R up to
    256, J_n up to 2^13, every 16th a 256 x 256 Kronecker pair) built and
    replayed from one graph as the benchmark does; sampled instances of every
    FFT size class and both kinds against the FP64 oracle."""
    from paper_2106_13062_amd.autotune import plan_for
    insts = synth.batch_instances(4096)
    items, hostF = [], {}
    for k, (ins, F) in enumerate(synth.instance_inputs(insts)):
        plan = plan_for(ins.kind, ins.I, ins.J, ins.D, ins.hash_seed, device=DEV, gather_weight=16.0)
        U = [torch.from_numpy(m).to(DEV).t().contiguous() for m in F]
        items.append({"plan": plan, "kind": ins.kind, "U": U})
        hostF[k] = F
    b = Batch(items, config={"tile_ffts": 32, "wg_per_cu": [0, 2, 0, 0, 0, 0, 2]}, device=DEV)
    print(f"full batch: {len(items)} items, {b.tiles} tiles", flush=True)
    b.run(graph=True)
    b.run(graph=True)      # second replay: counters and queues reset themselves
    torch.cuda.synchronize()
    # one CP instance per FFT size class (the smallest rank, to keep the
    # oracle quick) plus the largest-rank one, and two Kronecker instances
    by_class = {}
    for k, (ins, it) in enumerate(zip(insts, items)):
        if ins.kind == "cp":
            P = it["plan"].P
            if P not in by_class or ins.R < insts[by_class[P]].R:
                by_class[P] = k
    sample = sorted(by_class.values())
    sample.append(max((k for k, i in enumerate(insts) if i.kind == "cp"), key=lambda k: insts[k].R * len(insts[k].I)))
    sample += [k for k, i in enumerate(insts) if i.kind == "kron"][:2]
    for k in sample:
        ins, plan = insts[k], items[k]["plan"]
        got = items[k]["out"][0].cpu().numpy()
        hs, ss = O.hash_tables(ins.hash_seed, 1, ins.I, ins.J)
        if ins.kind == "kron":
            A, B = (x.astype(np.float32).astype(np.float64) for x in hostF[k])
            want = O.kron_fcs(A, B, hs[0], ss[0], ins.J)
        else:
            want = O.fcs_cp_fft(None, hostF[k], hs[0], ss[0], ins.J, plan.L)
        print(f"instance {k} {ins.kind} I={ins.I} J={ins.J} R={ins.R} P={plan.P} Q={plan.Q}: "
              f"{rel(got, want):.2e}", flush=True)
        assert rel(got, want) <= TOL, (k, rel(got, want))
