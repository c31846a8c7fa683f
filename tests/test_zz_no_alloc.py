"""The allocation-free entry point (pfbs_execute_noalloc) against
pfbs_execute: the same dumps bit for bit on two calls in a row, the second
with a smaller block, through the C ABI; the plan's device memory does not
grow; a block whose scratch exceeds the fixed array is rejected before
anything is queued."""
import numpy as np
import pytest

from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,P,n_int,frames", [
    (32768, 8, 64, [300, 97]),     # two-pass FFT, several intermediate groups
    (4096, 8, 40, [200, 57]),      # single pass
])
def test_noalloc_equals_execute_on_two_calls(N, P, n_int, frames):
    torch = require_gpu()
    x = synth.generate(synth.spec_c2(n_ref=N), 0, sum(frames) * N, workers=synth.default_workers())
    a = pf.Plan(N, P, n_pol=2, n_int=n_int)
    b = pf.Plan(N, P, n_pol=2, n_int=n_int)
    bytes0 = b.info()["device_bytes"]
    pos = 0
    for f in frames:
        blk = torch.from_numpy(np.ascontiguousarray(x[pos:pos + f * N])).cuda()
        nd = a.dumps_in(f * N)
        assert nd == b.dumps_in(f * N) and nd >= 1
        da = torch.full((nd, 4, N), -1.0, dtype=torch.float32, device="cuda")
        db = torch.full((nd, 4, N), -2.0, dtype=torch.float32, device="cuda")
        assert a.execute(blk, da) == nd
        assert b.execute_noalloc(blk, db) == nd
        torch.cuda.synchronize()
        assert torch.equal(da, db)
        pos += f * N
    pa = torch.empty((4, N), dtype=torch.float32, device="cuda")
    pb = torch.empty((4, N), dtype=torch.float32, device="cuda")
    assert a.flush(pa) == b.flush(pb)
    torch.cuda.synchronize()
    assert torch.equal(pa, pb)
    # the plan's own scratch buffers were never allocated
    assert b.info()["device_bytes"] == bytes0
    assert a.info()["device_bytes"] > bytes0
    a.close()
    b.close()


def test_noalloc_rejects_blocks_beyond_the_scratch():
    torch = require_gpu()
    N = 1 << 19
    plan = pf.Plan(N, 8, n_pol=2, n_int=64)       # one chunk of 16 spectra: 128 MiB of intermediate
    blk = torch.zeros((24 * N, 2, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(pf.PfbsError) as ei:
        plan.execute_noalloc(blk, torch.empty((1, 4, N), device="cuda"))
    assert ei.value.status == pf.ERR_INVALID
    assert plan.info()["frames_seen"] == 0
    # a smaller chunk fits
    small = pf.Plan(N, 8, n_pol=2, n_int=64, chunk=4)
    assert small.execute_noalloc(blk, torch.empty((1, 4, N), device="cuda")) == 0
    torch.cuda.synchronize()
    assert small.info()["frames_seen"] == 24
    plan.close()
    small.close()
