"""Serving loop on the GPU: a Poisson stream of mixed requests (T(I, u, v)
against a resident sketch, CP builds, COO sketches) served with continuous
batching on several streams gives, for every request, the same result as
the request run alone (relative L2 error <= 1e-5), also under a tight
memory cap; every request completes and gets a latency."""
import numpy as np
import pytest
import torch

import synth
from paper_2106_13062_amd.serve import Request, Server, latency_stats, run_alone

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


def build_server(cap):
    srv = Server(DEV, streams=3, cap_bytes=cap, max_group=16, max_inflight=6)
    I, J, D = (300, 200, 150), (512, 512, 512), 5
    plan = srv.plan(I, J, D, 41)
    U = synth.cp_factors(42, I, 8, normalize=True)
    _, spec = plan.sketch_cp([dev(u.T) for u in U], want_out=False, want_spec=True)
    uv = synth.unit_vectors(43, 128, I[1])
    vv = synth.unit_vectors(44, 64, I[2])
    srv.add_resident_sketch("S", plan, spec, dev(uv[:64]), dev(vv))
    for k, ins in enumerate(synth.batch_instances(3, seed=45, hash_seed=46, kron_every=0, I_range=(16, 300),
                                                   R_range=(1, 20), logJ_range=(6, 10))):
        p = srv.plan(ins.I, ins.J, 3, ins.hash_seed)
        srv.add_input(f"cp{k}", "cp", p, [dev(u.T) for u in ins.factors()])
    Ic = (64, 50, 40)
    pc = srv.plan(Ic, (128, 128, 128), 4, 47)
    T = synth.dense_tensor(48, Ic)
    for k, dens in enumerate((0.01, 0.3)):
        idx, val = synth.bernoulli_coo(49 + k, T, Ic, dens)
        srv.add_input(f"coo{k}", "coo", pc, dev(idx), dev(val))
    torch.cuda.synchronize()
    return srv


def make_requests(srv, n, rate, seed):
    reqs = []
    for rid, (t, kind, i) in enumerate(synth.serving_requests(seed, rate, n, 64, 3, 2, mix=(0.7, 0.2, 0.1))):
        key = {"contract": "S", "cp": f"cp{i}", "coo": f"coo{i}"}[kind]
        reqs.append(srv.make_request(rid, kind, t, key, index=i if kind == "contract" else 0))
    return reqs


def result_of(r):
    if r.kind == "contract":
        out, k = r.result
        return out[k].cpu().numpy()
    return r.result.cpu().numpy()


@pytest.mark.parametrize("cap", [200e9, 0])
def test_served_equals_alone(cap):
    srv = build_server(200e9)
    if cap == 0:
        # tight cap: resident data plus room for about two requests in flight
        srv.sched.cap = srv.sched.resident_bytes + 2.5 * max(r.footprint for r in make_requests(srv, 50, 1e4, 5))
    reqs = make_requests(srv, 240, 2e4, 7)
    print(f"serving {len(reqs)} requests, cap {srv.sched.cap:.3g}", flush=True)
    srv.run(reqs, timeout=60.0)
    torch.cuda.synchronize()
    assert all(r.done is not None for r in reqs)
    st = latency_stats(reqs)
    assert st["served"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    assert srv.sched.inflight_bytes == 0 and srv.sched.inflight_groups == 0
    # merged launches happened: some contraction result rows share a tensor
    groups = {id(r.result[0]) for r in reqs if r.kind == "contract"}
    ncontract = sum(1 for r in reqs if r.kind == "contract")
    if cap != 0:
        assert len(groups) < ncontract
    for r in reqs:
        alone = Request(r.rid, r.kind, 0.0, r.key, r.index)
        got = result_of(r)
        run_alone(srv, alone)
        want = result_of(alone)
        assert rel(got, want) <= TOL, (r.rid, r.kind, rel(got, want))
