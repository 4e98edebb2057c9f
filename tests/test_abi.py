"""Host-side checks of the C ABI that need no GPU: the library loads, every
entry point declared in include/fcs.h is exported, and plan validation
rejects bad descriptions before any device work."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

import paper_2106_13062_amd as F
from paper_2106_13062_amd import _lib as L


def _declared():
    with open(os.path.join(ROOT, "include", "fcs.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^FCS_API\s+[\w\s\*]+?\b(fcs_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ["fcs_plan_create", "fcs_plan_bind", "fcs_plan_export", "fcs_sketch_dense",
                 "fcs_sketch_coo", "fcs_sketch_cp", "fcs_contract_inner",
                 "fcs_contract_free_mode", "fcs_status_str"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert set(_declared()) <= set(L.SIGNATURES)
    F.load()


def _create(N, I, J, D, seed=1, Lreq=0):
    lib = F.load()
    Ia = (ctypes.c_int64 * max(N, 1))(*I)
    Ja = (ctypes.c_int64 * max(N, 1))(*J)
    desc = L.PlanDesc(N, Ia, Ja, D, seed, Lreq)
    h = ctypes.c_void_p()
    st = lib.fcs_plan_create(ctypes.byref(desc), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("N,I,J,D", [
    (0, [1], [1], 1),            # order 0
    (9, [2] * 9, [2] * 9, 1),    # order above the maximum
    (3, [4, 0, 4], [2, 2, 2], 1),  # empty mode
    (3, [4, 4, 4], [2, 0, 2], 1),  # zero hash length
    (3, [4, 4, 4], [2, 2, 2], 0),  # no sketches
    (3, [4, 4, 4], [2, 2, 2], 65),  # too many sketches
])
def test_plan_create_rejects(N, I, J, D):
    st, h = _create(N, I, J, D)
    assert st == L.FCS_EINVAL
    assert h.value is None
    assert F.load().fcs_last_error()


def test_plan_create_and_sizes():
    lib = F.load()
    st, h = _create(3, [100, 100, 100], [64, 64, 64], 5)
    assert st == L.FCS_OK
    Jt, Lt, Pt, Qt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    assert lib.fcs_plan_info(h, ctypes.byref(Jt), ctypes.byref(Lt), ctypes.byref(Pt), ctypes.byref(Qt)) == 0
    assert Jt.value == 190
    assert Lt.value >= 190 and Lt.value == Pt.value * Qt.value
    assert Pt.value & (Pt.value - 1) == 0
    assert lib.fcs_plan_table_bytes(h) >= 5 * 300 * 4
    assert lib.fcs_plan_spec_len(h) == (Qt.value // 2 + 1) * Pt.value
    assert lib.fcs_workspace_bytes(h, 99, 0, 0) == 0
    assert lib.fcs_plan_destroy(h) == 0


def test_transform_length_choices():
    lib = F.load()
    # the large CP workload: J~ = 49150 fits a 3 x 16384 transform
    st, h = _create(3, [10000] * 3, [16384] * 3, 10)
    assert st == 0
    Lt, Pt, Qt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    lib.fcs_plan_info(h, None, ctypes.byref(Lt), ctypes.byref(Pt), ctypes.byref(Qt))
    assert Lt.value >= 49150
    lib.fcs_plan_destroy(h)
    # explicit L: power of two accepted, too short or badly factored rejected
    st, h = _create(3, [10000] * 3, [16384] * 3, 10, Lreq=65536)
    assert st == 0
    lib.fcs_plan_info(h, None, ctypes.byref(Lt), ctypes.byref(Pt), ctypes.byref(Qt))
    assert Lt.value == 65536 and Pt.value * Qt.value == 65536
    lib.fcs_plan_destroy(h)
    st, _ = _create(3, [100] * 3, [64] * 3, 1, Lreq=100)
    assert st == L.FCS_EINVAL
    st, _ = _create(3, [100] * 3, [64] * 3, 1, Lreq=255)
    assert st == L.FCS_EUNSUPPORTED


def test_unbound_plan_rejected_without_device_work():
    lib = F.load()
    st, h = _create(2, [8, 8], [4, 4], 2)
    assert st == 0
    x = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    assert lib.fcs_sketch_dense(h, x, x, None, 0, None) == L.FCS_EINVAL
    assert lib.fcs_sketch_coo(h, 4, x, x, x, None, 0, None) == L.FCS_EINVAL
    assert lib.fcs_plan_export(h, 0, 0, x, x, None) == L.FCS_EINVAL
    assert lib.fcs_plan_bind(h, None, None) == L.FCS_EINVAL
    assert lib.fcs_plan_bind(h, ctypes.c_void_p(8), None) == L.FCS_EINVAL   # misaligned
    assert lib.fcs_plan_destroy(h) == 0


def test_status_strings():
    lib = F.load()
    for code in range(6):
        assert lib.fcs_status_str(code)


def test_hcs_plan_sizes():
    """A higher-order count sketch plan flattens J_0 x ... x J_{N-1}: J~ is
    the product of the hash lengths; products beyond the 31-bit range are
    refused before any device work."""
    lib = F.load()
    I, J = [50, 40, 30], [14, 9, 5]
    Ia = (ctypes.c_int64 * 3)(*I)
    Ja = (ctypes.c_int64 * 3)(*J)
    h = ctypes.c_void_p()
    assert lib.fcs_plan_create_hcs(ctypes.byref(L.PlanDesc(3, Ia, Ja, 2, 7, 0)), ctypes.byref(h)) == 0
    Jt = ctypes.c_int64()
    lib.fcs_plan_info(h, ctypes.byref(Jt), None, None, None)
    assert Jt.value == 14 * 9 * 5
    lib.fcs_plan_destroy(h)
    Jb = (ctypes.c_int64 * 3)(*[2048, 2048, 1024])
    assert lib.fcs_plan_create_hcs(ctypes.byref(L.PlanDesc(3, Ia, Jb, 2, 7, 0)), ctypes.byref(h)) == \
        L.FCS_EUNSUPPORTED


def test_ts_fold_and_inner_median_validate_before_device_work():
    lib = F.load()
    st, h = _create(2, [8, 8], [4, 5], 2)
    x = ctypes.c_void_p(16)
    assert lib.fcs_ts_fold(h, x, x, None) == L.FCS_EINVAL        # unequal hash lengths
    assert lib.fcs_inner_median(0, 10, x, x, x, None, None, 0, None) == L.FCS_EINVAL
    assert lib.fcs_inner_median(2, 0, x, x, x, None, None, 0, None) == L.FCS_EINVAL
    assert lib.fcs_inner_median(2, 10, x, x, x, None, None, 0, None) == L.FCS_EINVAL   # no workspace
    lib.fcs_plan_destroy(h)


@pytest.mark.parametrize("args", [
    (0, 4, 8191, 4096, 0), (4, 0, 8191, 4096, 0), (4, 1 << 20, 8191, 4096, 0),
    (4, 4, 8191, 4096, 2), (4, 4, 8191, 1000, 0), (4, 4, 4000, 4096, 0), (4, 4, 10001, 4096, 0),
])
def test_probe_rejects_before_launch(args):
    lib = F.load()
    sink = ctypes.c_void_p(256)      # never dereferenced: the arguments are rejected first
    assert lib.fcs_probe_lds_atomics(*args, 1, sink, None) == L.FCS_EINVAL
    assert lib.fcs_last_error()


def test_probe_rejects_null_sink():
    assert F.load().fcs_probe_lds_atomics(4, 4, 8191, 4096, 0, 1, None, None) == L.FCS_EINVAL
