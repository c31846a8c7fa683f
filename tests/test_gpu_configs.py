"""The benchmark configurations end to end against the FP64 oracle, and the
production kernels' tap/frame indexing bit for bit.

* One-hot taps: with h[p*N + n] = 1 for p = p0 and 0 otherwise, every
  pre-filter output is exactly frame j + p0 (fmaf(0, x, y) = y and 1*x = x
  in FP32), so a PFB plan's dumps must equal, bit for bit, those of a
  direct-mode plan fed the stream shifted by p0 frames, cut so that each of
  its blocks completes the same spectra.  This runs through the production
  column, pair and single-pass kernels (not a debug kernel), across block
  cuts shorter than P-1 frames.
* The largest mode (N = 2^19, 8 taps, two polarisations, 256 MB blocks, 64
  spectra per dump) over three blocks: every dump and the flushed tail
  within 1e-5 of the oracle, in FP32 and in the MIXED matrix-core precision.
* The eight uneven sub-bands of the batched form at their real shapes
  (N = 2^10 .. 2^19, direct and 4/8-tap PFB, 2^23 samples per sub-band per
  block): batched dumps equal per-sub-band plans bit for bit, and each
  sub-band's first dump is within 1e-5 of the oracle.
* N = 2^20, the paper's largest direct transform length, with the PFB.
"""
import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import rel_err, require_gpu, run_stream

pytestmark = pytest.mark.gpu

TOL = 1e-5
W = synth.default_workers()


def _cores():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


# ------------------------------------------------- one-hot tap indexing ----

@pytest.mark.parametrize("N,P,p0,split,frames", [
    (4096, 8, 5, 0, [3, 9, 2, 12, 6]),            # single pass
    (32768, 8, 2, 0, [9, 3, 1, 11]),              # 128-point columns
    (1 << 19, 8, 6, 0, [3, 9, 2, 10]),            # 512-point columns (FP32 default)
    (1 << 19, 8, 3, 256, [10, 5, 1, 9]),          # two-spectra column kernel
])
def test_one_hot_taps_equal_shifted_direct_bitwise(N, P, p0, split, frames):
    torch = require_gpu()
    n_int = 3
    h = np.zeros(P * N, dtype=np.float64)
    h[p0 * N:(p0 + 1) * N] = 1.0
    rng = np.random.default_rng(N + p0)
    T = sum(frames) * N
    x = rng.integers(-128, 128, size=(T, 2, 2)).astype(np.int8)   # -128 included
    kw = {"split_n2": split} if split else {}
    a = pf.Plan(N, P, window=pf.WINDOW_CUSTOM, custom_taps=h, n_pol=2, n_int=n_int, **kw)
    b = pf.Plan(N, 1, mode=pf.MODE_DIRECT, n_pol=2, n_int=n_int, **kw)
    if split:
        assert a.info()["split_n2"] == split == b.info()["split_n2"]
    da, db = [], []
    pos = 0
    for f in frames:
        j_lo = a.info()["spectra_done"]
        blk = torch.from_numpy(np.ascontiguousarray(x[pos:pos + f * N])).cuda()
        nd = a.dumps_in(f * N)
        d = torch.empty((max(nd, 1), 4, N), dtype=torch.float32, device="cuda")
        assert a.execute(blk, d) == nd
        if nd:
            da.append(d[:nd].cpu().numpy())
        pos += f * N
        j_hi = a.info()["spectra_done"]
        if j_hi > j_lo:
            # the direct plan gets frames j_lo + p0 .. j_hi + p0 - 1: the same spectra
            seg = x[(j_lo + p0) * N:(j_hi + p0) * N]
            nd = b.dumps_in(seg.shape[0])
            d = torch.empty((max(nd, 1), 4, N), dtype=torch.float32, device="cuda")
            assert b.execute(torch.from_numpy(np.ascontiguousarray(seg)).cuda(), d) == nd
            if nd:
                db.append(d[:nd].cpu().numpy())
    pa = torch.empty((4, N), dtype=torch.float32, device="cuda")
    pb = torch.empty((4, N), dtype=torch.float32, device="cuda")
    ca, cb = a.flush(pa), b.flush(pb)
    torch.cuda.synchronize()
    assert a.info()["spectra_done"] == b.info()["spectra_done"] == T // N - P + 1
    da = np.concatenate(da) if da else np.zeros((0, 4, N), np.float32)
    db = np.concatenate(db) if db else np.zeros((0, 4, N), np.float32)
    assert da.shape == db.shape and da.shape[0] == (T // N - P + 1) // n_int
    assert np.array_equal(da, db)
    assert ca == cb and np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())
    a.close()
    b.close()


# ----------------------------------------------- largest mode, 3 blocks ----

C3_N, C3_BLOCK, C3_BLOCKS, C3_NINT = 1 << 19, 1 << 26, 3, 64


@pytest.fixture(scope="module")
def c3_stream():
    x = synth.generate(synth.spec_c3(), 0, C3_BLOCKS * C3_BLOCK, workers=W)
    h = oracle.taps(C3_N, 8)
    ref = oracle.dumps(x, C3_N, 8, h, False, C3_NINT, n_threads=_cores())
    tail, cnt = oracle.tail(x, C3_N, 8, h, False, C3_NINT, n_threads=_cores())
    return x, ref, tail, cnt


@pytest.mark.parametrize("prec", [pf.PREC_FP32, pf.PREC_MIXED])
def test_config3_three_blocks_every_dump_and_tail(c3_stream, prec):
    x, ref, tail, cnt = c3_stream
    plan = pf.Plan(C3_N, 8, n_pol=2, n_int=C3_NINT, precision=prec)
    dumps, part, c = run_stream(plan, x, [C3_BLOCK // C3_N])
    plan.close()
    S = C3_BLOCKS * (C3_BLOCK // C3_N) - 7
    assert dumps.shape[0] == S // C3_NINT == ref.shape[0] == 5
    assert c == cnt == S - 5 * C3_NINT == 57
    errs = [rel_err(dumps[d], ref[d]).max() for d in range(dumps.shape[0])]
    et = rel_err(part, tail).max()
    print("config3 precision %d: dump errors %s, tail %.3g" % (prec, ["%.3g" % e for e in errs], et))
    assert max(errs) <= TOL and et <= TOL, (errs, et)


# ------------------------------------------------ eight uneven sub-bands ----

C5 = [  # N, P, mode, n_int
    (1024, 1, pf.MODE_DIRECT, 8192), (4096, 1, pf.MODE_DIRECT, 2048),
    (16384, 1, pf.MODE_DIRECT, 512), (32768, 1, pf.MODE_DIRECT, 256),
    (65536, 4, pf.MODE_PFB, 128), (131072, 8, pf.MODE_PFB, 64),
    (262144, 8, pf.MODE_PFB, 32), (524288, 4, pf.MODE_PFB, 16),
]
C5_BLOCK, C5_BLOCKS = 1 << 23, 2


def test_eight_subband_shapes_batched_bitwise_and_first_dumps():
    torch = require_gpu()
    xs = [synth.generate(synth.spec_subband(s, N), 0, C5_BLOCK * C5_BLOCKS, workers=W)
          for s, (N, _, _, _) in enumerate(C5)]
    descs = [pf.make_desc(N=N, P=P, mode=m, n_pol=2, n_int=ni) for (N, P, m, ni) in C5]
    batch = pf.Batch(descs)
    got = [[] for _ in C5]
    for k in range(C5_BLOCKS):
        blocks = [torch.from_numpy(np.ascontiguousarray(x[k * C5_BLOCK:(k + 1) * C5_BLOCK])).cuda() for x in xs]
        dumps = [torch.empty((max(p.dumps_in(C5_BLOCK), 1), 4, p.N), dtype=torch.float32, device="cuda")
                 for p in batch.plans]
        nd = batch.execute(blocks, dumps)
        torch.cuda.synchronize()
        for i in range(len(C5)):
            if nd[i]:
                got[i].append(dumps[i][:nd[i]].cpu().numpy())
        del blocks, dumps
    tails = []
    for p in batch.plans:
        t = torch.empty((4, p.N), dtype=torch.float32, device="cuda")
        tails.append((p.flush(t), t))
    torch.cuda.synchronize()
    tails = [(c, t.cpu().numpy()) for c, t in tails]
    batch.close()
    for i, ((N, P, m, ni), x) in enumerate(zip(C5, xs)):
        g = np.concatenate(got[i])
        plan = pf.Plan(N, P, mode=m, n_pol=2, n_int=ni)
        want, part, cnt = run_stream(plan, x, [C5_BLOCK // N])
        plan.close()
        assert g.shape == want.shape and g.shape[0] >= 1, i
        assert np.array_equal(g, want), i
        assert tails[i][0] == cnt and np.array_equal(tails[i][1], part), i
        direct = m == pf.MODE_DIRECT
        ref = oracle.integrate(x, N, P, None if direct else oracle.taps(N, P), direct, 0, ni, _cores())
        e = rel_err(g[0], ref).max()
        print("sub-band %d (N=%d, P=%d, n_int=%d): first dump error %.3g" % (i, N, P, ni, e))
        assert e <= TOL, (i, e)


# ------------------------------------------------------------- N = 2^20 ----

def test_two_to_the_twenty_channels_first_dump():
    """N = 2^20 (the paper's largest direct FFT), 8-tap PFB, dual
    polarisation, 64 spectra per dump across two blocks."""
    N, P, n_int = 1 << 20, 8, 64
    frames = [40, 31]
    x = synth.generate(synth.spec_c2(n_ref=N), 0, sum(frames) * N, workers=W)
    plan = pf.Plan(N, P, n_pol=2, n_int=n_int)
    dumps, part, cnt = run_stream(plan, x, frames)
    plan.close()
    assert dumps.shape[0] == 1 and cnt == sum(frames) - P + 1 - n_int
    ref = oracle.integrate(x, N, P, oracle.taps(N, P), False, 0, n_int, _cores())
    e = rel_err(dumps[0], ref).max()
    print("N=2^20 first dump error %.3g" % e)
    assert e <= TOL, e
