"""Python binding of libfcs: argument marshalling only.

PyTorch provides device memory and streams; every step of every sketch runs
in the HIP kernels behind the C ABI.  Tensors passed in must already be on the
current HIP device, contiguous and of the stated dtype; outputs and
workspaces are allocated here with torch and handed to the library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as C

_I64 = ctypes.c_int64


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """A bound FCS plan: D sketches of an order-N tensor with mode sizes I and
    hash lengths J, hash pairs drawn from ``seed`` (see include/fcs.h)."""

    def __init__(self, I, J, D: int, seed: int, L: int = 0, device=None, stream=None, hcs: bool = False):
        """hcs: a plan of the higher-order count sketch (Definition 3) with
        the same hash pairs, its sketches flattened to prod(J) entries."""
        self.lib = C.load()
        self.hcs = bool(hcs)
        self.I = tuple(int(i) for i in I)
        self.J = tuple(int(j) for j in J)
        self.N = len(self.I)
        self.D = int(D)
        self.seed = int(seed) & ((1 << 64) - 1)
        Ia = (_I64 * self.N)(*self.I)
        Ja = (_I64 * self.N)(*self.J)
        desc = C.PlanDesc(self.N, Ia, Ja, self.D, self.seed, int(L))
        h = ctypes.c_void_p()
        create = self.lib.fcs_plan_create_hcs if self.hcs else self.lib.fcs_plan_create
        C.check(create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        Jt, Lt, Pt, Qt = _I64(), _I64(), _I64(), ctypes.c_int32()
        C.check(self.lib.fcs_plan_info(h, ctypes.byref(Jt), ctypes.byref(Lt), ctypes.byref(Pt),
                                       ctypes.byref(Qt)))
        self.Jt, self.L, self.P, self.Q = Jt.value, Lt.value, Pt.value, Qt.value
        self.spec_len = int(self.lib.fcs_plan_spec_len(h))
        self.device = torch.device("cuda") if device is None else torch.device(device)
        nbytes = int(self.lib.fcs_plan_table_bytes(h))
        self.tables = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        C.check(self.lib.fcs_plan_bind(h, _ptr(self.tables), _stream(stream)))

    # ------------------------------------------------------------------ utils
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.fcs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def workspace(self, op: int, R: int = 0, P: int = 0) -> torch.Tensor:
        n = int(self.lib.fcs_workspace_bytes(self._h, op, R, P))
        return torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)

    def export(self, d: int, n: int, stream=None):
        h = np.empty(self.I[n], dtype=np.int32)
        s = np.empty(self.I[n], dtype=np.int8)
        C.check(self.lib.fcs_plan_export(self._h, d, n, h.ctypes.data_as(ctypes.c_void_p),
                                         s.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return h, s

    def _ws(self, ws, op, R=0, P=0):
        if ws is None:
            ws = self.workspace(op, R, P)
        return ws, ctypes.c_size_t(ws.numel() * ws.element_size())

    # --------------------------------------------------------------- sketches
    def sketch_dense(self, T: torch.Tensor, out=None, ws=None, stream=None) -> torch.Tensor:
        """T: float32 with prod(I) entries in vec order (mode 0 fastest)."""
        _need(T, torch.float32, "T")
        if T.numel() != int(np.prod(self.I)):
            raise ValueError("T has the wrong number of entries")
        out = torch.empty((self.D, self.Jt), dtype=torch.float32, device=self.device) if out is None else out
        _need(out, torch.float32, "out")
        ws, nb = self._ws(ws, C.OP_DENSE)
        C.check(self.lib.fcs_sketch_dense(self._h, _ptr(T), _ptr(out), _ptr(ws), nb, _stream(stream)))
        return out

    def sketch_coo(self, idx: torch.Tensor, val: torch.Tensor, out=None, ws=None, stream=None):
        """idx: int32 N x nnz (mode-major), val: float32 nnz."""
        _need(idx, torch.int32, "idx")
        _need(val, torch.float32, "val")
        nnz = val.numel()
        if idx.shape != (self.N, nnz):
            raise ValueError("idx must be N x nnz")
        out = torch.empty((self.D, self.Jt), dtype=torch.float32, device=self.device) if out is None else out
        _need(out, torch.float32, "out")
        ws, nb = self._ws(ws, C.OP_COO)
        C.check(self.lib.fcs_sketch_coo(self._h, nnz, _ptr(idx), _ptr(val), _ptr(out), _ptr(ws), nb,
                                        _stream(stream)))
        return out

    def sketch_cp(self, U, lam=None, out=None, spec=None, want_out=True, want_spec=False,
                  ws=None, stream=None):
        """U: list of N float32 tensors of shape (R, I_n) (each row is one
        factor column, i.e. the I_n x R factor in column-major order)."""
        if len(U) != self.N:
            raise ValueError("need N factors")
        R = int(U[0].shape[0])
        for n, u in enumerate(U):
            _need(u, torch.float32, f"U[{n}]")
            if tuple(u.shape) != (R, self.I[n]):
                raise ValueError(f"U[{n}] must be R x I_n = {(R, self.I[n])}")
        if lam is not None:
            _need(lam, torch.float32, "lambda")
        if want_out and out is None:
            out = torch.empty((self.D, self.Jt), dtype=torch.float32, device=self.device)
        if want_spec and spec is None:
            spec = torch.empty((self.D, self.spec_len, 2), dtype=torch.float32, device=self.device)
        ptrs = (ctypes.c_void_p * self.N)(*[u.data_ptr() for u in U])
        ws, nb = self._ws(ws, C.OP_CP, R=R)
        C.check(self.lib.fcs_sketch_cp(self._h, R, ptrs, _ptr(lam), _ptr(out), _ptr(spec), _ptr(ws), nb,
                                       _stream(stream)))
        return out, spec

    def sketch_cp_noalloc(self, U, lam=None, out=None, spec=None, want_out=True, want_spec=False, stream=None):
        """fcs_sketch_cp_noalloc: the CP sketch with the library's own
        device scratch array instead of a workspace (the library allocates
        nothing; outputs not given are allocated here)."""
        if len(U) != self.N:
            raise ValueError("need N factors")
        R = int(U[0].shape[0])
        for n, u in enumerate(U):
            _need(u, torch.float32, f"U[{n}]")
            if tuple(u.shape) != (R, self.I[n]):
                raise ValueError(f"U[{n}] must be R x I_n = {(R, self.I[n])}")
        if lam is not None:
            _need(lam, torch.float32, "lambda")
        if want_out and out is None:
            out = torch.empty((self.D, self.Jt), dtype=torch.float32, device=self.device)
        if want_spec and spec is None:
            spec = torch.empty((self.D, self.spec_len, 2), dtype=torch.float32, device=self.device)
        ptrs = (ctypes.c_void_p * self.N)(*[u.data_ptr() for u in U])
        C.check(self.lib.fcs_sketch_cp_noalloc(self._h, R, ptrs, _ptr(lam), _ptr(out), _ptr(spec),
                                               _stream(stream)))
        return out, spec

    def sketch_kron(self, A: torch.Tensor, B: torch.Tensor, out=None, spec=None, want_out=True,
                    want_spec=False, ws=None, stream=None):
        """Kronecker product A (x) B of an order-4 plan: A is I_0 x I_1 and B
        is I_2 x I_3, each given as a float32 tensor of shape (I_1, I_0)
        (resp. (I_3, I_2)), i.e. the matrix in column-major order."""
        if self.N != 4:
            raise ValueError("a Kronecker sketch needs an order-4 plan")
        _need(A, torch.float32, "A")
        _need(B, torch.float32, "B")
        if A.numel() != self.I[0] * self.I[1] or B.numel() != self.I[2] * self.I[3]:
            raise ValueError("A must have I_0 * I_1 and B I_2 * I_3 entries")
        if want_out and out is None:
            out = torch.empty((self.D, self.Jt), dtype=torch.float32, device=self.device)
        if want_spec and spec is None:
            spec = torch.empty((self.D, self.spec_len, 2), dtype=torch.float32, device=self.device)
        ws, nb = self._ws(ws, C.OP_KRON)
        C.check(self.lib.fcs_sketch_kron(self._h, _ptr(A), _ptr(B), _ptr(out), _ptr(spec), _ptr(ws), nb,
                                         _stream(stream)))
        return out, spec

    def sketch_contraction(self, A: torch.Tensor, B: torch.Tensor, out=None, spec=None, want_out=True,
                           want_spec=False, ws=None, stream=None):
        """Contraction sum_l A[i0, i1, l] B[l, i2, i3] of an order-4 plan: A
        is I_0 x I_1 x Lc and B is Lc x I_2 x I_3, each a float32 tensor in
        column-major order (shape (Lc, I_1, I_0), resp. (I_3, I_2, Lc))."""
        if self.N != 4:
            raise ValueError("a contraction sketch needs an order-4 plan")
        _need(A, torch.float32, "A")
        _need(B, torch.float32, "B")
        sa, sb = self.I[0] * self.I[1], self.I[2] * self.I[3]
        if A.numel() == 0 or A.numel() % sa != 0:
            raise ValueError("A must have I_0 * I_1 * Lc entries")
        Lc = A.numel() // sa
        if B.numel() != Lc * sb:
            raise ValueError("B must have Lc * I_2 * I_3 entries")
        if want_out and out is None:
            out = torch.empty((self.D, self.Jt), dtype=torch.float32, device=self.device)
        if want_spec and spec is None:
            spec = torch.empty((self.D, self.spec_len, 2), dtype=torch.float32, device=self.device)
        ws, nb = self._ws(ws, C.OP_CONTRACTION, R=Lc)
        C.check(self.lib.fcs_sketch_contraction(self._h, Lc, _ptr(A), _ptr(B), _ptr(out), _ptr(spec), _ptr(ws),
                                                nb, _stream(stream)))
        return out, spec

    def decompress(self, y: torch.Tensor, order=None, out=None, stream=None) -> torch.Tensor:
        """Recovered tensor (median over the D sketches) as a flat float32
        tensor of prod I_n entries, laid out with mode order[0] fastest
        (vec order when order is None)."""
        _need(y, torch.float32, "y")
        if tuple(y.shape) != (self.D, self.Jt):
            raise ValueError("y must be D x J~")
        n = 1
        for i in self.I:
            n *= i
        out = torch.empty(n, dtype=torch.float32, device=self.device) if out is None else out
        _need(out, torch.float32, "out")
        if out.numel() != n:
            raise ValueError("out must have prod I_n entries")
        ords = None
        if order is not None:
            if len(order) != self.N:
                raise ValueError("order must list every mode once")
            ords = (ctypes.c_int32 * self.N)(*[int(k) for k in order])
        C.check(self.lib.fcs_decompress(self._h, _ptr(y), ords, _ptr(out), _stream(stream)))
        return out

    def spectrum(self, y: torch.Tensor, spec=None, ws=None, stream=None):
        _need(y, torch.float32, "y")
        spec = torch.empty((self.D, self.spec_len, 2), dtype=torch.float32, device=self.device) \
            if spec is None else spec
        ws, nb = self._ws(ws, C.OP_SPECTRUM)
        C.check(self.lib.fcs_sketch_spectrum(self._h, _ptr(y), _ptr(spec), _ptr(ws), nb, _stream(stream)))
        return spec

    # ----------------------------------------------------------- contractions
    def contract_inner(self, a: torch.Tensor, b: torch.Tensor, ws=None, stream=None):
        _need(a, torch.float32, "a")
        _need(b, torch.float32, "b")
        med = torch.empty(1, dtype=torch.float64, device=self.device)
        per_d = torch.empty(self.D, dtype=torch.float64, device=self.device)
        ws, nb = self._ws(ws, C.OP_INNER)
        C.check(self.lib.fcs_contract_inner(self._h, _ptr(a), _ptr(b), _ptr(med), _ptr(per_d), _ptr(ws), nb,
                                            _stream(stream)))
        return med, per_d

    def ts_fold(self, y: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """Tensor sketch (Definition 2, all J_n equal) of the tensor whose
        fast count sketches under this plan are y (D x J~): D x J."""
        _need(y, torch.float32, "y")
        if tuple(y.shape) != (self.D, self.Jt):
            raise ValueError("y must be D x J~")
        out = torch.empty((self.D, self.J[0]), dtype=torch.float32, device=self.device) if out is None else out
        _need(out, torch.float32, "out")
        C.check(self.lib.fcs_ts_fold(self._h, _ptr(y), _ptr(out), _stream(stream)))
        return out

    def contract_free_mode(self, spec: torch.Tensor, free_mode: int, vecs, out=None, ws=None, stream=None):
        """vecs: list of N entries; vecs[free_mode] is ignored (may be None);
        the others are float32 P x I_n."""
        _need(spec, torch.float32, "spec")
        if not 0 <= int(free_mode) < self.N:
            raise ValueError(f"free_mode must be in [0, {self.N})")
        Pn = None
        ptrs = (ctypes.c_void_p * self.N)()
        for n in range(self.N):
            if n == free_mode:
                ptrs[n] = None
                continue
            v = _need(vecs[n], torch.float32, f"vecs[{n}]")
            if Pn is None:
                Pn = int(v.shape[0])
            if tuple(v.shape) != (Pn, self.I[n]):
                raise ValueError(f"vecs[{n}] must be P x I_n")
            ptrs[n] = v.data_ptr()
        Pn = 0 if Pn is None else Pn
        out = torch.empty((Pn, self.I[free_mode]), dtype=torch.float64, device=self.device) \
            if out is None else out
        ws, nb = self._ws(ws, C.OP_FREE_MODE, P=Pn)
        C.check(self.lib.fcs_contract_free_mode(self._h, _ptr(spec), int(free_mode), Pn, ptrs, _ptr(out),
                                                _ptr(ws), nb, _stream(stream)))
        return out


    def contract_full(self, spec: torch.Tensor, vecs, out=None, per_d=None, ws=None, stream=None):
        """T(v_0, ..., v_{N-1}) for P tuples: vecs is a list of N float32
        P x I_n tensors.  Returns (medians float64 [P], per-sketch float64
        P x D)."""
        _need(spec, torch.float32, "spec")
        if len(vecs) != self.N:
            raise ValueError("one vector block per mode")
        ptrs = (ctypes.c_void_p * self.N)()
        Pn = None
        for n in range(self.N):
            v = _need(vecs[n], torch.float32, f"vecs[{n}]")
            if Pn is None:
                Pn = int(v.shape[0])
            if tuple(v.shape) != (Pn, self.I[n]):
                raise ValueError(f"vecs[{n}] must be P x I_n")
            ptrs[n] = v.data_ptr()
        out = torch.empty(Pn, dtype=torch.float64, device=self.device) if out is None else out
        per_d = torch.empty((Pn, self.D), dtype=torch.float64, device=self.device) if per_d is None else per_d
        C.check(self.lib.fcs_contract_full(self._h, _ptr(spec), Pn, ptrs, _ptr(out), _ptr(per_d), None, 0,
                                           _stream(stream)))
        return out, per_d


class Batch:
    """Many uneven CP / Kronecker sketch computations run together by the
    persistent batch kernels (include/fcs.h, fcs_batch_*).

    items: list of dicts with keys
      plan   a bound Plan (kept alive by the batch)
      kind   "cp" or "kron"
      U      CP: list of N float32 (R, I_n) tensors; KRON: [A, B] as for
             Plan.sketch_kron
      lam    optional float32 R weights (CP)
      out    float32 (D, J~) output tensor (allocated when missing)
      spec   optional float32 (D, spec_len, 2) spectrum output
    config: optional dict with "tile_ffts", "wg_per_cu" (7 ints) and
    "no_pack" (7 flags: one transform per mode in that FFT size class)."""

    def __init__(self, items, config=None, device=None):
        self.lib = C.load()
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.items = list(items)
        n = len(self.items)
        arr = (C.BatchItem * max(n, 1))()
        self._keep = []
        for k, it in enumerate(self.items):
            plan = it["plan"]
            kind = it.get("kind", "cp")
            U = it["U"]
            if kind == "cp":
                if len(U) != plan.N:
                    raise ValueError(f"item {k}: need N factors")
                R = int(U[0].shape[0])
                for n_, u in enumerate(U):
                    _need(u, torch.float32, f"item {k} U[{n_}]")
                    if tuple(u.shape) != (R, plan.I[n_]):
                        raise ValueError(f"item {k}: U[{n_}] must be R x I_n")
                kd = C.ITEM_CP
            elif kind == "kron":
                if plan.N != 4 or len(U) != 2:
                    raise ValueError(f"item {k}: a Kronecker item needs an order-4 plan and [A, B]")
                _need(U[0], torch.float32, f"item {k} A")
                _need(U[1], torch.float32, f"item {k} B")
                if U[0].numel() != plan.I[0] * plan.I[1] or U[1].numel() != plan.I[2] * plan.I[3]:
                    raise ValueError(f"item {k}: factor matrices have the wrong sizes")
                R = 1
                kd = C.ITEM_KRON
            else:
                raise ValueError(f"item {k}: unknown kind {kind!r}")
            if it.get("out") is None and it.get("spec") is None:
                it["out"] = torch.empty((plan.D, plan.Jt), dtype=torch.float32, device=self.device)
            if it.get("out") is not None:
                _need(it["out"], torch.float32, f"item {k} out")
            if it.get("spec") is not None:
                _need(it["spec"], torch.float32, f"item {k} spec")
            ptrs = (ctypes.c_void_p * len(U))(*[u.data_ptr() for u in U])
            self._keep.append((plan, U, ptrs, it.get("lam"), it.get("out"), it.get("spec")))
            arr[k] = C.BatchItem(plan.handle, kd, R, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)),
                                 _ptr(it.get("lam")), _ptr(it.get("out")), _ptr(it.get("spec")))
        cfg = None
        if config:
            cfg = C.BatchConfig(int(config.get("tile_ffts", 0)),
                                (ctypes.c_int32 * 7)(*[int(x) for x in config.get("wg_per_cu", [0] * 7)]),
                                (ctypes.c_int32 * 7)(*[int(x) for x in config.get("no_pack", [0] * 7)]))
        h = ctypes.c_void_p()
        C.check(self.lib.fcs_batch_create(arr, n, None if cfg is None else ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        nbytes = int(self.lib.fcs_batch_workspace_bytes(h))
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        tiles = ctypes.c_int64()
        grids = (ctypes.c_int32 * 7)()
        C.check(self.lib.fcs_batch_info(h, ctypes.byref(tiles), grids))
        self.tiles = tiles.value
        self.grids = list(grids)
        self.prepared = False

    def prepare(self, stream=None):
        C.check(self.lib.fcs_batch_prepare(self._h, _ptr(self.ws), self.ws.numel(), _stream(stream)))
        self.prepared = True

    def run(self, graph: bool = True, stream=None):
        if not self.prepared:
            self.prepare(stream)
        C.check(self.lib.fcs_batch_run(self._h, _ptr(self.ws), self.ws.numel(), 1 if graph else 0,
                                       _stream(stream)))
        return [it.get("out") for it in self.items]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.fcs_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def inner_median(a: torch.Tensor, b: torch.Tensor, stream=None):
    """fcs_inner_median: per-row inner products of two D x len float32
    tensors (double) and their median, e.g. for tensor sketches."""
    lib = C.load()
    _need(a, torch.float32, "a")
    _need(b, torch.float32, "b")
    if a.dim() != 2 or a.shape != b.shape:
        raise ValueError("a and b must be D x len of equal shape")
    D, n = int(a.shape[0]), int(a.shape[1])
    med = torch.empty(1, dtype=torch.float64, device=a.device)
    per_d = torch.empty(D, dtype=torch.float64, device=a.device)
    C.check(lib.fcs_inner_median(D, n, _ptr(a), _ptr(b), _ptr(med), _ptr(per_d), None, 0, _stream(stream)))
    return med, per_d


# ---------------------------------------------------------------------------
# small dense steps of the decomposition drivers (argument marshalling only)
# ---------------------------------------------------------------------------
def normalize_rows(x: torch.Tensor, out=None, norms=None, stream=None) -> torch.Tensor:
    """fcs_normalize_rows: unit rows of a P x n float64 or float32 tensor,
    returned as float32."""
    lib = C.load()
    if x.dtype not in (torch.float64, torch.float32):
        raise TypeError("x must be float64 or float32")
    _need(x, x.dtype, "x")
    if x.dim() != 2:
        raise ValueError("x must be P x n")
    out = torch.empty(x.shape, dtype=torch.float32, device=x.device) if out is None else out
    _need(out, torch.float32, "out")
    in64 = x if x.dtype == torch.float64 else None
    in32 = x if x.dtype == torch.float32 else None
    C.check(lib.fcs_normalize_rows(int(x.shape[0]), int(x.shape[1]), _ptr(in64), _ptr(in32), _ptr(out),
                                   _ptr(norms), _stream(stream)))
    return out


def select_max(vals: torch.Tensor, rows: torch.Tensor, row_out=None, val_out=None, val64_out=None,
               stream=None):
    """fcs_select_max: the row of the largest value (first on ties) into
    row_out (1 x n float32), its value as float32 and float64 device
    scalars."""
    lib = C.load()
    _need(vals, torch.float64, "vals")
    _need(rows, torch.float32, "rows")
    P, n = int(rows.shape[0]), int(rows.shape[1])
    if vals.numel() != P:
        raise ValueError("one value per row")
    dev = rows.device
    row_out = torch.empty((1, n), dtype=torch.float32, device=dev) if row_out is None else row_out
    val_out = torch.empty(1, dtype=torch.float32, device=dev) if val_out is None else val_out
    val64_out = torch.empty(1, dtype=torch.float64, device=dev) if val64_out is None else val64_out
    C.check(lib.fcs_select_max(P, _ptr(vals), n, _ptr(rows), _ptr(row_out), _ptr(val_out), _ptr(val64_out),
                               None, _stream(stream)))
    return row_out, val_out, val64_out


def axpy(a: float, x: torch.Tensor, y: torch.Tensor, stream=None) -> torch.Tensor:
    """fcs_axpy: y += a x (float32, same number of entries), in place."""
    lib = C.load()
    _need(x, torch.float32, "x")
    _need(y, torch.float32, "y")
    if x.numel() != y.numel():
        raise ValueError("x and y must have the same number of entries")
    C.check(lib.fcs_axpy(y.numel(), float(a), _ptr(x), _ptr(y), _stream(stream)))
    return y


def als_update(Mt: torch.Tensor, others, out=None, lam=None, ws=None, stream=None):
    """fcs_als_update: solve (Hadamard product of F_m F_m^T) X = Mt by
    Cholesky and normalise the rows of X.  Mt: R x In float64; others: list
    of R x I_m float32 (factors with their columns as rows).  Returns
    (float32 R x In unit rows, float64 R weights)."""
    lib = C.load()
    _need(Mt, torch.float64, "Mt")
    R, In = int(Mt.shape[0]), int(Mt.shape[1])
    for m, f in enumerate(others):
        _need(f, torch.float32, f"others[{m}]")
        if f.dim() != 2 or int(f.shape[0]) != R:
            raise ValueError("every other factor must be R x I_m")
    dev = Mt.device
    out = torch.empty((R, In), dtype=torch.float32, device=dev) if out is None else out
    lam = torch.empty(R, dtype=torch.float64, device=dev) if lam is None else lam
    nb = int(lib.fcs_als_workspace_bytes(R, In))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev) if ws is None else ws
    ptrs = (ctypes.c_void_p * max(1, len(others)))(*[f.data_ptr() for f in others])
    Is = (_I64 * max(1, len(others)))(*[int(f.shape[1]) for f in others])
    C.check(lib.fcs_als_update(R, In, _ptr(Mt), len(others), ptrs, Is, _ptr(out), _ptr(lam), _ptr(ws),
                               ctypes.c_size_t(ws.numel() * ws.element_size()), _stream(stream)))
    return out, lam


def probe_lds_atomics(blocks: int, rows: int, window: int, span: int, pattern: int, seed: int = 1,
                      sink=None, device=None, stream=None) -> torch.Tensor:
    """fcs_probe_lds_atomics: the LDS atomics of the dense scatter's access
    pattern alone (a measurement probe); returns the per-workgroup bin sums
    (uint32 as int32, each rows * 4096)."""
    lib = C.load()
    if sink is None:
        sink = torch.empty(blocks, dtype=torch.int32, device=device)
    _need(sink, torch.int32, "sink")
    if sink.numel() < blocks:
        raise ValueError("sink holds fewer than `blocks` entries")
    C.check(lib.fcs_probe_lds_atomics(int(blocks), int(rows), int(window), int(span), int(pattern),
                                      int(seed) & 0xFFFFFFFF, _ptr(sink), _stream(stream)))
    return sink
