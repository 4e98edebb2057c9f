"""Precision of the built kernels, read from the library's own gfx950 code.

Sketches and spectra are formed in single precision; double precision on
the device belongs only to the final reductions (medians over the D
sketches, the bin sums of sketched inner products and full contractions)
and to norms (column and block norms, the decomposition drivers' row norms,
Gram matrices and solves).  The test disassembles the code objects of
libfcs.so (built here from this repository's sources) and checks that no
sketch-forming kernel holds a double-precision instruction and that every
kernel that does hold one is a reduction of that kind.
"""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2106_13062_amd", "libfcs.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"

# kernels that form sketches, spectra or plan tables: single precision only
FP32_ONLY = [
    "dense_scatter_kernel", "dense_scatter_global_kernel",
    "coo_scatter_kernel", "coo_scatter_global_kernel",
    "cp_forward_kernel", "reduce_chunks_kernel", "cp_finalize_kernel", "sum_slices_kernel",
    "spectrum_kernel", "free_mode_kernel",
    "kron_kernel", "contraction_factor_kernel", "contraction_forward_kernel",
    "batch_kernel", "ts_fold_kernel",
    "twiddle_kernel", "hash_tables_kernel", "axpy_kernel",
    "lds_atomic_probe_kernel",
]
# final reductions and norms: double precision allowed
FP64_ALLOWED = [
    "median_kernel", "median_rows_kernel", "median_tuples_kernel",
    "decompress_kernel", "decompress_phase_kernel",          # median over d
    "inner_kernel", "full_contract_kernel",                  # bin sums of contractions
    "column_absmax_kernel", "batch_absmax_kernel",           # column 2-norm exponents
    "dense_exact_kernel", "dense_exact_exponent",            # block root mean square
    "normalize_rows_kernel", "select_max_kernel",            # driver norms, max of medians
    "als_gram_kernel", "als_solve_kernel",                   # R x R Gram and Cholesky
]


def _named(sym, name):
    # Itanium mangling writes an identifier as <length><name>
    return f"{len(name)}{name}" in sym


def _disassemble(tmp_path):
    lib = os.path.join(str(tmp_path), "libfcs.so")
    shutil.copy(LIB, lib)
    subprocess.run([OBJDUMP, "--offloading", lib], cwd=str(tmp_path), check=True,
                   capture_output=True)
    objs = sorted(glob.glob(os.path.join(str(tmp_path), "libfcs.so.*gfx950")))
    assert objs, "no gfx950 code object in libfcs.so"
    f64 = {}
    for obj in objs:
        out = subprocess.run([OBJDUMP, "-d", "--no-show-raw-insn", obj], check=True,
                             capture_output=True, text=True).stdout
        cur = None
        for line in out.splitlines():
            m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
            if m:
                cur = m.group(1)
                f64.setdefault(cur, 0)
            elif cur is not None and re.match(r"^\s+v_\w*f64", line):
                f64[cur] += 1
    return f64


@pytest.mark.skipif(not (os.path.exists(LIB) and os.path.exists(OBJDUMP)),
                    reason="libfcs.so not built or llvm-objdump missing")
def test_fp64_only_in_final_reductions(tmp_path):
    f64 = _disassemble(tmp_path)
    for name in FP32_ONLY:
        syms = [s for s in f64 if _named(s, name)]
        assert syms, f"{name} not found in the code objects"
        bad = {s: f64[s] for s in syms if f64[s]}
        assert not bad, f"double-precision instructions in {name}: {bad}"
    for sym, n in f64.items():
        if n:
            assert any(_named(sym, a) for a in FP64_ALLOWED), \
                f"{sym} holds {n} double-precision instructions"
