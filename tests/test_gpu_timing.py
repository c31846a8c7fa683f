"""Kernel timing through the dispatch timestamps: every launch of a timed
block is counted under its kind (the history copy inside the reduction's
launch), the durations are positive and add up to
no more than the wall time of the same work, and timing changes no result."""
import numpy as np
import pytest

from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


# the tap-history copy rides in the dump reduction's launch (kind dump_reduce)
# whenever a block completes spectra, as these do
@pytest.mark.parametrize("N,kinds", [(1024, ("single_pass", "dump_reduce")),
                                     (32768, ("column_pass", "row_pass", "dump_reduce"))])
def test_timing_counts_every_launch(N, kinds):
    torch = require_gpu()
    x = synth.generate(synth.spec_c2(n_ref=N), 0, 40 * N)
    blk = torch.from_numpy(x).cuda()
    d0 = torch.empty((8, 4, N), dtype=torch.float32, device="cuda")
    d1 = torch.empty_like(d0)
    a = pf.Plan(N, 8, n_pol=2, n_int=5)
    b = pf.Plan(N, 8, n_pol=2, n_int=5)
    b.timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n0 = a.execute(blk, d0)
    e0.record()
    n1 = b.execute(blk, d1)
    e1.record()
    torch.cuda.synchronize()
    t = b.timing_read()
    assert n0 == n1 and torch.equal(d0[:n0], d1[:n1])
    wall = e0.elapsed_time(e1)
    for k in kinds:
        ms, cnt = t[k]
        assert cnt >= 1 and ms > 0, (k, t)
    assert t["tap_history"][1] == 0, t
    assert sum(ms for ms, cnt in t.values()) <= wall * 1.05 + 0.01
    assert b.timing_read()["dump_reduce"] == (0.0, 0)  # read once, then forgotten
