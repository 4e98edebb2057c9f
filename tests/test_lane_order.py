"""Lane order of the dense scatter (host logic, no GPU).

The dense kernel adds a row of mode 0 to the LDS bins of a group of sketches
with one wave of 64 lanes per 256-column segment, 4 columns per lane, and
each LDS atomic is served as two half-waves of 32 lanes whose time grows with
the largest number of lanes that fall on one of the 32 banks.  The bank of
column c in sketch d is h_0(c) plus a row-uniform offset (mod 32).  Checked
here: for every group and every 1024-column set the block order is a
permutation over the set's waves (each column is added exactly once), and
it lowers the mean largest bank load per half-wave against the plain order,
with h_0 taken from the oracle's hash tables (the same hash definition)."""
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_2106_13062_amd as F
from paper_2106_13062_amd import _lib as L


def _plan(I, J, D, seed):
    lib = F.load()
    N = len(I)
    desc = L.PlanDesc(N, (ctypes.c_int64 * N)(*I), (ctypes.c_int64 * N)(*J), D, seed, 0)
    h = ctypes.c_void_p()
    assert lib.fcs_plan_create(ctypes.byref(desc), ctypes.byref(h)) == L.FCS_OK
    return lib, h


def _order(I, J, D, seed):
    lib, h = _plan(I, J, D, seed)
    try:
        n = lib.fcs_plan_dense_order_bytes(h)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        g = ctypes.c_int32()
        assert lib.fcs_plan_dense_order(h, out.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(g)) == L.FCS_OK
        if n:
            # a short buffer is rejected
            assert lib.fcs_plan_dense_order(h, out.ctypes.data_as(ctypes.c_void_p), n - 1, None) == L.FCS_EINVAL
        return out[:n], g.value
    finally:
        lib.fcs_plan_destroy(h)


def _half_load(h0_mod, cols_of_half):
    # largest bank load of one half-wave, for one sketch and one column slot
    return np.bincount(h0_mod[cols_of_half], minlength=32).max()


@pytest.mark.parametrize("I,J,D,seed", [
    ((1024, 64, 8), (4096, 512, 64), 8, 2002),     # 4 segments: one full set
    ((1536, 16, 8), (1024, 16, 16), 3, 7),         # 6 segments: a full and a partial set
    ((1000, 32, 4), (2048, 64, 8), 5, 11),         # partial last segment
])
def test_dense_lane_order_is_a_permutation_and_spreads_banks(I, J, D, seed):
    order, dg = _order(I, J, D, seed)
    assert dg >= 1
    I0 = I[0]
    segs = -(-I0 // 256)
    ngroups = -(-D // dg)
    assert order.size == D * segs * 64
    order = order.reshape(D, segs, 64).astype(np.int64)
    hs, _ = O.hash_tables(seed, D, I, J)
    before = after = 0
    for g in range(ngroups):
        d_group = range(g * dg, min(D, g * dg + dg))
        for st in range(0, segs, 4):
            ns = min(4, segs - st)
            blocks = order[g, st:st + ns].reshape(-1)
            assert sorted(blocks.tolist()) == list(range(ns * 64)), (g, st)
            plain = np.arange(ns * 64)
            for d in d_group:
                hm = np.asarray(hs[d][0]) % 32
                for half in range(2 * ns):
                    for e in range(4):
                        for lay, acc in ((plain, "b"), (blocks, "a")):
                            cols = st * 256 + 4 * lay[half * 32:half * 32 + 32] + e
                            cols = cols[cols < I0]
                            if cols.size == 0:
                                continue
                            v = _half_load(hm, cols)
                            if acc == "b":
                                before += v
                            else:
                                after += v
    assert after < 0.85 * before, (after, before)


def test_dense_lane_order_deterministic():
    a, _ = _order((1024, 64, 8), (4096, 512, 64), 8, 2002)
    b, _ = _order((1024, 64, 8), (4096, 512, 64), 8, 2002)
    assert np.array_equal(a, b)
