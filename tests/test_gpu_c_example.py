"""The C ABI without Python: paper_2106_13062_amd/examples/fcs_dense_example
(plain C against include/fcs.h, libfcs.so and the HIP runtime) sketches an
integer-valued order-3 tensor; its printed sketches equal the FP64 oracle's
exactly (integer data: every partial sum is exact)."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2106_13062_amd", "examples", "fcs_dense_example")


def test_c_program_dense_sketch_matches_oracle():
    assert os.path.exists(EXE), "build() compiles the C example"
    run = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    lines = run.stdout.strip().split("\n")
    D, Jt = (int(x) for x in lines[0].split())
    got = np.array([[float(v) for v in ln.split()] for ln in lines[1:1 + D]])
    assert got.shape == (D, Jt)
    I, J, seed = (20, 15, 10), (16, 8, 4), 5
    n = int(np.prod(I))
    T = (((np.arange(n, dtype=np.uint64) * np.uint64(7919)) % np.uint64(7)).astype(np.int64) - 3).astype(np.float32)
    hs, ss = O.hash_tables(seed, D, I, J)
    want = O.dense_rows(T, I, hs, ss, Jt)
    np.testing.assert_array_equal(got, want)
