"""Batched multi-sub-band launches: three launches per block for all
sub-bands (front phase, row phase, tail; optionally replayed from a HIP
graph) must give bit-identical dumps to each sub-band's own plan, in FP32 and
MIXED, and match the oracle."""
import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import require_gpu, run_stream, within_fp32_bound

pytestmark = pytest.mark.gpu

# (N, P, mode, n_int): single pass and two-pass, PFB and direct, uneven dumps
SUBBANDS = [
    (1024, 1, pf.MODE_DIRECT, 48),
    (4096, 4, pf.MODE_PFB, 10),
    (16384, 8, pf.MODE_PFB, 6),
    (32768, 1, pf.MODE_DIRECT, 4),
    (65536, 4, pf.MODE_PFB, 3),
]
BLOCK = 1 << 19          # time samples per sub-band per block
BLOCKS = 4


def _streams():
    return [synth.generate(synth.spec_subband(s, N), 0, BLOCK * BLOCKS) for s, (N, *_rest) in enumerate(SUBBANDS)]


def _descs():
    return [pf.make_desc(N=N, P=P, mode=m, n_pol=2, n_int=ni) for (N, P, m, ni) in SUBBANDS]


def _run_batch(xs, use_graph, descs=None, subs=SUBBANDS, launches=None):
    torch = require_gpu()
    b = pf.Batch(descs or _descs())
    outs = [[] for _ in SUBBANDS]
    for k in range(BLOCKS):
        blocks = [torch.from_numpy(np.ascontiguousarray(x[k * BLOCK:(k + 1) * BLOCK])).cuda() for x in xs]
        dumps = [torch.empty((max(p.dumps_in(BLOCK), 1), 4, p.N), dtype=torch.float32, device="cuda")
                 for p in b.plans]
        nd = b.execute(blocks, dumps, use_graph=use_graph)
        if launches is not None:
            launches.append(b.launches)
        torch.cuda.synchronize()
        for i in range(len(subs)):
            if nd[i]:
                outs[i].append(dumps[i][:nd[i]].cpu().numpy())
    parts = []
    for p in b.plans:
        part = torch.empty((4, p.N), dtype=torch.float32, device="cuda")
        parts.append((p.flush(part), part))
    torch.cuda.synchronize()
    res = [np.concatenate(o) if o else np.zeros((0, 4, subs[i][0]), np.float32) for i, o in enumerate(outs)]
    flushed = [(c, t.cpu().numpy()) for c, t in parts]
    b.close()
    return res, flushed


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_equals_individual_plans_bitwise(use_graph):
    require_gpu()
    xs = _streams()
    launches = []
    got, flushed = _run_batch(xs, use_graph, launches=launches)
    assert launches == [3] * BLOCKS
    for i, ((N, P, m, ni), x) in enumerate(zip(SUBBANDS, xs)):
        plan = pf.Plan(N, P, mode=m, n_pol=2, n_int=ni)
        want, part, cnt = run_stream(plan, x, [BLOCK // N])
        assert got[i].shape == want.shape, i
        assert np.array_equal(got[i], want), i
        assert flushed[i][0] == cnt and np.array_equal(flushed[i][1], part), i


def test_batched_graph_replays_match_oracle():
    require_gpu()
    xs = _streams()
    got, _ = _run_batch(xs, True)
    for i in (0, 1, 2, 3):
        N, P, m, ni = SUBBANDS[i]
        direct = m == pf.MODE_DIRECT
        ref = oracle.dumps(xs[i], N, P, None if direct else oracle.taps(N, P), direct, ni,
                           which=list(range(min(3, got[i].shape[0]))))
        for d in range(ref.shape[0]):
            assert within_fp32_bound(got[i][d], ref[d], N) <= 1.0, (i, d)


@pytest.mark.parametrize("n_pol", [2, 1])
def test_two_spectra_column_kernel_bitwise(n_pol):
    """Where the tap table is large (P*N >= 2^21 floats) an FP32 column pass
    filters two spectra per workgroup step, in a plan's own launch and in the
    batched front phase alike: one sub-band batched and alone agree bit for
    bit, with odd and even spectrum counts per block (5, 11 and 10 here)."""
    torch = require_gpu()
    N, P, ni = 262144, 8, 3
    frames = [12, 11, 10]
    x = synth.generate(synth.spec_subband(5, N), 7, N * sum(frames))
    if n_pol == 1:
        x = np.ascontiguousarray(x[:, :1, :])
    kw = dict(N=N, P=P, mode=pf.MODE_PFB, n_pol=n_pol, n_int=ni, split_n2=256)
    want, part, cnt = run_stream(pf.Plan(**kw), x, frames)
    b = pf.Batch([pf.make_desc(**kw)])
    got, pos = [], 0
    for f in frames:
        blk = torch.from_numpy(np.ascontiguousarray(x[pos:pos + f * N])).cuda()
        pos += f * N
        d = torch.empty((max(b.plans[0].dumps_in(f * N), 1), 4 if n_pol == 2 else 1, N), dtype=torch.float32,
                        device="cuda")
        nd = b.execute([blk], [d])
        torch.cuda.synchronize()
        if nd[0]:
            got.append(d[:nd[0]].cpu().numpy())
    bpart = torch.empty((4 if n_pol == 2 else 1, N), dtype=torch.float32, device="cuda")
    bcnt = b.plans[0].flush(bpart)
    torch.cuda.synchronize()
    b.close()
    got = np.concatenate(got)
    assert got.shape == want.shape and want.shape[0] == (5 + 11 + 10) // ni
    assert np.array_equal(got, want)
    assert bcnt == cnt and np.array_equal(bpart.cpu().numpy(), part)


def test_graph_grid_covers_padded_column_items():
    """The captured graph launches the column pass with an upper-bound grid;
    it must cover the item count padded to a multiple of 8 per column tile
    (blocks of 9 and 13 frames: 2, 9 and 13 spectra, 4 and 16 tiles)."""
    torch = require_gpu()
    subs = [(16384, 8, pf.MODE_PFB, 3), (65536, 4, pf.MODE_PFB, 2)]
    frames = [9, 13, 9]
    xs = [synth.generate(synth.spec_subband(s, N), 3, N * sum(frames)) for s, (N, *_r) in enumerate(subs)]
    b = pf.Batch([pf.make_desc(N=N, P=P, mode=m, n_pol=2, n_int=ni) for (N, P, m, ni) in subs])
    got = [[] for _ in subs]
    pos = [0] * len(subs)
    for f in frames:
        blocks, dumps = [], []
        for i, (N, *_r) in enumerate(subs):
            blocks.append(torch.from_numpy(np.ascontiguousarray(xs[i][pos[i]:pos[i] + f * N])).cuda())
            pos[i] += f * N
            dumps.append(torch.empty((max(b.plans[i].dumps_in(f * N), 1), 4, N), dtype=torch.float32, device="cuda"))
        nd = b.execute(blocks, dumps, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(subs)):
            if nd[i]:
                got[i].append(dumps[i][:nd[i]].cpu().numpy())
    b.close()
    for i, (N, P, m, ni) in enumerate(subs):
        want, _part, _cnt = run_stream(pf.Plan(N, P, mode=m, n_pol=2, n_int=ni), xs[i], frames)
        g = np.concatenate(got[i])
        assert g.shape == want.shape and np.array_equal(g, want), i


# FP32 and MIXED sub-bands in one batch: single pass, one-spectrum and
# two-spectra column passes, FP32, FP64 and split-FP16 row passes
MIXED_SUBBANDS = [
    (1024, 8, pf.MODE_PFB, 40, pf.PREC_MIXED),
    (16384, 4, pf.MODE_PFB, 6, pf.PREC_MIXED),
    (65536, 1, pf.MODE_DIRECT, 3, pf.PREC_FP32),
    (131072, 8, pf.MODE_PFB, 2, pf.PREC_MIXED),
    (262144, 8, pf.MODE_PFB, 2, pf.PREC_FP32),
    (524288, 4, pf.MODE_PFB, 2, pf.PREC_MIXED),
]
MIXED_BLOCK = 1 << 21


@pytest.mark.parametrize("use_graph", [False, True])
def test_mixed_precision_batch_bitwise(use_graph):
    require_gpu()
    subs = [s[:4] for s in MIXED_SUBBANDS]
    descs = [pf.make_desc(N=N, P=P, mode=m, n_pol=2, n_int=ni, precision=pr) for (N, P, m, ni, pr) in MIXED_SUBBANDS]
    xs = [synth.generate(synth.spec_subband(s, N), 11, MIXED_BLOCK * 3) for s, (N, *_r) in enumerate(subs)]
    torch = require_gpu()
    b = pf.Batch(descs)
    assert [p.info()["row_arith"] for p in b.plans[1:]] == [2, 0, 2, 3, 2]
    outs = [[] for _ in subs]
    for k in range(3):
        blocks = [torch.from_numpy(np.ascontiguousarray(x[k * MIXED_BLOCK:(k + 1) * MIXED_BLOCK])).cuda() for x in xs]
        dumps = [torch.empty((max(p.dumps_in(MIXED_BLOCK), 1), 4, p.N), dtype=torch.float32, device="cuda")
                 for p in b.plans]
        nd = b.execute(blocks, dumps, use_graph=use_graph)
        assert b.launches == 3
        torch.cuda.synchronize()
        for i in range(len(subs)):
            if nd[i]:
                outs[i].append(dumps[i][:nd[i]].cpu().numpy())
    b.close()
    for i, (N, P, m, ni, pr) in enumerate(MIXED_SUBBANDS):
        want, _part, _cnt = run_stream(pf.Plan(N, P, mode=m, n_pol=2, n_int=ni, precision=pr), xs[i],
                                       [MIXED_BLOCK // N] * 3)
        g = np.concatenate(outs[i])
        assert g.shape == want.shape and np.array_equal(g, want), i


def test_batch_of_single_pass_sub_bands_only_has_two_launches():
    """Only single-pass sub-bands: the single passes (in the row-phase
    kernel, which has a single-pass workgroup's threads) and the tail."""
    torch = require_gpu()
    subs = [(256, 4, pf.MODE_PFB, 16), (4096, 1, pf.MODE_DIRECT, 8)]
    xs = [synth.generate(synth.spec_subband(s, N), 2, 1 << 17) for s, (N, *_r) in enumerate(subs)]
    b = pf.Batch([pf.make_desc(N=N, P=P, mode=m, n_pol=2, n_int=ni) for (N, P, m, ni) in subs])
    dumps = [torch.empty((max(p.dumps_in(1 << 17), 1), 4, p.N), dtype=torch.float32, device="cuda") for p in b.plans]
    nd = b.execute([torch.from_numpy(x).cuda() for x in xs], dumps)
    assert b.launches == 2
    torch.cuda.synchronize()
    got = [dumps[i][:nd[i]].cpu().numpy() for i in range(2)]
    b.close()
    for i, (N, P, m, ni) in enumerate(subs):
        want, _p, _c = run_stream(pf.Plan(N, P, mode=m, n_pol=2, n_int=ni), xs[i], [(1 << 17) // N])
        assert np.array_equal(got[i], want), i


def test_single_passes_beside_4096_point_rows_bitwise():
    """A batch whose rows are 4096 points long (N = 2^20) keeps its single
    passes in the front phase (the row phase's 4096-point tiles have twice a
    single-pass workgroup's threads); dumps equal per-sub-band plans."""
    torch = require_gpu()
    subs = [(1024, 8, pf.MODE_PFB, 64), (1 << 20, 4, pf.MODE_PFB, 2)]
    blk = 1 << 22
    xs = [synth.generate(synth.spec_subband(s, N), 9, blk * 2) for s, (N, *_r) in enumerate(subs)]
    b = pf.Batch([pf.make_desc(N=N, P=P, mode=m, n_pol=2, n_int=ni) for (N, P, m, ni) in subs])
    got = [[] for _ in subs]
    for k in range(2):
        blocks = [torch.from_numpy(np.ascontiguousarray(x[k * blk:(k + 1) * blk])).cuda() for x in xs]
        dumps = [torch.empty((max(p.dumps_in(blk), 1), 4, p.N), dtype=torch.float32, device="cuda") for p in b.plans]
        nd = b.execute(blocks, dumps)
        assert b.launches == 3
        torch.cuda.synchronize()
        for i in range(len(subs)):
            if nd[i]:
                got[i].append(dumps[i][:nd[i]].cpu().numpy())
    b.close()
    for i, (N, P, m, ni) in enumerate(subs):
        want, _p, _c = run_stream(pf.Plan(N, P, mode=m, n_pol=2, n_int=ni), xs[i], [blk // N])
        g = np.concatenate(got[i])
        assert g.shape == want.shape and np.array_equal(g, want), i
