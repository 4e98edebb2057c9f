"""The LDS-atomic probe of the dense scatter's access pattern
(fcs_probe_lds_atomics): every atomic lands, so each workgroup's bins sum to
rows x 1024 columns x 4 windows, for random and for conflict-free bins, at
the dense1024 grid's window and at the extremes of the accepted sizes."""
import numpy as np
import pytest
import torch

from paper_2106_13062_amd import FcsError
from paper_2106_13062_amd.fcs import probe_lds_atomics

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("pattern", [0, 1])
@pytest.mark.parametrize("blocks,rows,window,span", [
    (8, 64, 8191, 4096),        # the dense1024 window and column span
    (3, 5, 1024, 1024),         # smallest window, row count not a multiple of 4
    (300, 16, 10000, 2048),     # largest window, more workgroups than CUs
])
def test_probe_every_atomic_lands(pattern, blocks, rows, window, span):
    print(f"probe pattern={pattern} blocks={blocks} rows={rows} window={window} span={span}", flush=True)
    sink = probe_lds_atomics(blocks, rows, window, span, pattern, seed=7, device=DEV)
    torch.cuda.synchronize()
    got = sink.cpu().numpy().astype(np.int64)
    assert (got == rows * 4096).all(), got[:8]


@pytest.mark.parametrize("args", [
    (0, 4, 8191, 4096, 0), (4, 0, 8191, 4096, 0), (4, 1 << 20, 8191, 4096, 0),
    (4, 4, 8191, 4096, 2), (4, 4, 8191, 1000, 0), (4, 4, 4000, 4096, 0), (4, 4, 10001, 4096, 0),
])
def test_probe_rejects(args):
    with pytest.raises(FcsError):
        probe_lds_atomics(*args, seed=1, device=DEV)
