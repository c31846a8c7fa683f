"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Integer work (unpack, tap/frame indexing, history carry) must be bit-exact.
Integrated products over the long integrations of the benchmark
configurations must agree within 1e-5 relative per channel (cross terms
scaled by sqrt(XX*YY)).  Short integrations (a few spectra, used here to
exercise dump and block boundaries, on tone-bearing streams) are held to the
bound that FP32 arithmetic itself implies (tests/gpu_util.fp32_bound): with
only a few spectra some channels carry almost no power and any FP32 FFT's
absolute error is then a large fraction of it.  Identities that hold exactly in FP32
(one rectangular tap equals direct mode, chunk-aligned block splits, reruns)
are bitwise."""
import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import plan_n2, rel_err, require_gpu, run_stream, tone_stream, within_fp32_bound

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _plan(N, P, mode, n_pol, n_int, **kw):
    return pf.Plan(N, P, mode=mode, n_pol=n_pol, n_int=n_int, **kw)


# ------------------------------------------------------------ bit-exact ----

@pytest.mark.parametrize("n_pol", [1, 2])
def test_unpack_all_256_values_bit_exact(n_pol):
    torch = require_gpu()
    N = 256
    t = np.arange(4 * N)
    x = np.empty((4 * N, n_pol, 2), dtype=np.int8)
    for p in range(n_pol):
        x[:, p, 0] = ((t + 37 * p) % 256).astype(np.uint8).view(np.int8)
        x[:, p, 1] = ((t * 7 + 11 + p) % 256).astype(np.uint8).view(np.int8)
    plan = _plan(N, 1, pf.MODE_DIRECT, n_pol, 1)
    y = torch.empty((4, n_pol, N, 2), dtype=torch.float32, device="cuda")
    n = plan.debug_pfb(torch.from_numpy(x).cuda(), y)
    assert n == 4
    got = y.cpu().numpy()
    want = x.astype(np.float32).reshape(4, N, n_pol, 2).transpose(0, 2, 1, 3)
    assert np.array_equal(got, want)
    assert got.min() == -128.0 and got.max() == 127.0


@pytest.mark.parametrize("N,P,n_pol,frames", [
    (64, 5, 2, [3, 1, 7, 2, 9]),      # blocks shorter than P-1 frames too
    (32, 8, 1, [4, 4, 12]),
    (8192, 3, 2, [2, 5]),
])
def test_prefilter_indexing_and_history_bit_exact(N, P, n_pol, frames):
    """Asymmetric integer taps: every partial sum is an exact integer, so the
    GPU pre-filter must equal the oracle's bit for bit across block cuts."""
    torch = require_gpu()
    h = np.array([((7 * m) % 23) - 11 for m in range(P * N)], dtype=np.float64)
    rng = np.random.default_rng(N + P)
    T = sum(frames) * N
    x = rng.integers(-128, 128, size=(T, n_pol, 2)).astype(np.int8)
    plan = _plan(N, P, pf.MODE_PFB, n_pol, 3, window=pf.WINDOW_CUSTOM, custom_taps=h)
    pos = 0
    j = 0
    for f in frames:
        blk = torch.from_numpy(np.ascontiguousarray(x[pos:pos + f * N])).cuda()
        y = torch.empty((max(f, 1), n_pol, N, 2), dtype=torch.float32, device="cuda")
        n = plan.debug_pfb(blk, y)
        got = y[:n].cpu().numpy()
        for i in range(n):
            want = oracle.pfb(x, N, P, h, False, j + i)
            assert np.array_equal(got[i][..., 0], want.real.astype(np.float32)), (j + i)
            assert np.array_equal(got[i][..., 1], want.imag.astype(np.float32)), (j + i)
        j += n
        plan.execute(blk, torch.empty((8, plan.n_prod, N), device="cuda"))
        pos += f * N
    assert j == oracle.num_spectra(T, N, P, False)


@pytest.mark.parametrize("N", [256, 8192])
def test_one_rect_tap_equals_direct_bitwise(N):
    x = synth.generate(synth.spec_c2(n_ref=N), 0, 20 * N)
    a = _plan(N, 1, pf.MODE_PFB, 2, 6, window=pf.WINDOW_RECT)
    b = _plan(N, 1, pf.MODE_DIRECT, 2, 6)
    da, pa, _ = run_stream(a, x, [7])
    db, pb, _ = run_stream(b, x, [7])
    assert da.shape[0] == 3
    assert np.array_equal(da, db) and np.array_equal(pa, pb)


def test_taps_table_within_one_ulp_of_fp64():
    torch = require_gpu()
    for N, P in [(1024, 8), (32768, 8), (65536, 4)]:
        plan = _plan(N, P, pf.MODE_PFB, 2, 1)
        out = torch.empty(P * N, dtype=torch.float32, device="cuda")
        plan.debug_taps(out)
        got = out.cpu().numpy()
        ref = oracle.taps(N, P)
        r32 = ref.astype(np.float32)
        ulp = np.spacing(np.abs(r32)).astype(np.float64)
        # the FP64 reference itself carries ~1e-16 absolute rounding (e.g. its
        # sin(pi*q) at the sinc zeros is ~1e-17, not 0)
        assert np.all(np.abs(got.astype(np.float64) - ref) <= ulp + 1e-15)


# -------------------------------------------------------------- parity -----

CASES = [
    # N, P, mode, n_pol, n_int, block frames, extra plan args
    (16, 4, pf.MODE_PFB, 2, 5, [9, 4], {}),
    (64, 4, pf.MODE_PFB, 2, 7, [5, 9, 3, 20], {}),
    (256, 8, pf.MODE_PFB, 1, 10, [16, 16, 17], {}),
    (1024, 8, pf.MODE_PFB, 2, 16, [40, 8], {}),
    (2048, 1, pf.MODE_DIRECT, 2, 9, [11, 5], {}),
    (4096, 8, pf.MODE_PFB, 2, 5, [12, 12], {}),
    (4096, 1, pf.MODE_DIRECT, 1, 8, [9, 9], {}),
    (8192, 8, pf.MODE_PFB, 2, 6, [14, 14], {}),
    (16384, 4, pf.MODE_PFB, 2, 5, [10, 10], {}),
    (32768, 8, pf.MODE_PFB, 2, 4, [12, 10], {}),
    (32768, 1, pf.MODE_DIRECT, 2, 4, [8, 8], {}),
    (32768, 8, pf.MODE_PFB, 2, 4, [12, 10], {"split_n2": 128}),
    (65536, 8, pf.MODE_PFB, 1, 3, [12], {"split_n2": 512}),
    (65536, 2, pf.MODE_PFB, 2, 3, [6, 2], {"chunk": 2}),
]


@pytest.mark.parametrize("N,P,mode,n_pol,n_int,frames,kw", CASES)
def test_dumps_match_oracle(N, P, mode, n_pol, n_int, frames, kw):
    # noise plus the correlated tone of the dual-polarisation workload: the
    # short integrations here are held to the FP32 bound, whose row term
    # covers the rounding that a strong tone concentrates on its row
    spec = tone_stream(n_pol, N, 100 + N % 97)
    T = sum(frames) * N
    x = synth.generate(spec, 0, T)
    plan = _plan(N, P, mode, n_pol, n_int, **kw)
    dumps, part, cnt = run_stream(plan, x, frames)
    direct = mode == pf.MODE_DIRECT
    h = None if direct else oracle.taps(N, P)
    S = oracle.num_spectra(T, N, P, direct)
    assert dumps.shape[0] == S // n_int
    assert cnt == S - (S // n_int) * n_int
    ref = oracle.dumps(x, N, P, h, direct, n_int)
    n2 = plan_n2(plan)
    for d in range(dumps.shape[0]):
        r = within_fp32_bound(dumps[d], ref[d], N, n2=n2)
        assert r <= 1.0, (d, r, rel_err(dumps[d], ref[d]).max())
    if cnt:
        tail, c2 = oracle.tail(x, N, P, h, direct, n_int)
        assert c2 == cnt
        assert within_fp32_bound(part, tail, N, n2=n2) <= 1.0


def test_config1_single_pol_full():
    """2^20 single-polarisation samples, N=1024, 8-tap PFB and direct mode,
    everything integrated into one output."""
    x = synth.generate(synth.spec_c1(), 0, 1 << 20)
    for mode, P, S in [(pf.MODE_PFB, 8, 1017), (pf.MODE_DIRECT, 1, 1024)]:
        plan = _plan(1024, P, mode, 1, S)
        dumps, _, cnt = run_stream(plan, x, [1024])
        assert dumps.shape == (1, 1, 1024) and cnt == 0
        direct = mode == pf.MODE_DIRECT
        ref = oracle.dumps(x, 1024, P, None if direct else oracle.taps(1024, P), direct, S)
        assert rel_err(dumps[0], ref[0]).max() <= TOL
        # the tone at bin 100.25 dominates its bin
        assert np.argmax(dumps[0][0]) == 100


def test_config2_shape_first_dump():
    """N=32768 dual-pol, 8-tap PFB, 64 MB blocks (2^24 samples), 1024 spectra
    per dump: the first dump completes in the third block."""
    N, blk = 32768, 1 << 24
    x = synth.generate(synth.spec_c2(), 0, 3 * blk, workers=synth.default_workers())
    plan = _plan(N, 8, pf.MODE_PFB, 2, 1024)
    dumps, _, cnt = run_stream(plan, x, [blk // N])
    assert dumps.shape[0] == 1
    ref = oracle.dumps(x, N, 8, oracle.taps(N, 8), False, 1024, which=[0])
    e = rel_err(dumps[0], ref[0])
    assert e.max() <= TOL, e.max()
    ph = np.angle(dumps[0][2][5000] + 1j * dumps[0][3][5000])
    assert abs(ph + 0.7) < 0.05


def test_config3_shape_first_dump():
    """N=524288 dual-pol, 8-tap PFB, one 256 MB block (2^26 samples), 64
    spectra per dump: the first dump against the oracle."""
    N, blk = 1 << 19, 1 << 26
    x = synth.generate(synth.spec_c3(), 0, blk, workers=synth.default_workers())
    plan = _plan(N, 8, pf.MODE_PFB, 2, 64)
    dumps, _, cnt = run_stream(plan, x, [blk // N])
    assert dumps.shape[0] == 1 and cnt == 121 - 64
    ref = oracle.dumps(x, N, 8, oracle.taps(N, 8), False, 64, which=[0])
    e = rel_err(dumps[0], ref[0])
    assert e.max() <= TOL, e.max()


# ------------------------------------------------ invariances (bitwise) ----

@pytest.mark.parametrize("N,chunk", [(1024, 16), (32768, 4)])
def test_chunk_aligned_block_split_invariance_and_rerun(N, chunk):
    P, n_int = 8, 32
    x = synth.generate(synth.spec_c2(n_ref=N), 0, 120 * N)
    one = _plan(N, P, pf.MODE_PFB, 2, n_int, chunk=chunk)
    d1, p1, c1 = run_stream(one, x, [120])
    # every block ends on a chunk boundary of the spectrum index
    two = _plan(N, P, pf.MODE_PFB, 2, n_int, chunk=chunk)
    d2, p2, c2 = run_stream(two, x, [chunk * 2 + P - 1] + [chunk * 3, chunk, chunk * 5] * 40)
    assert np.array_equal(d1, d2) and np.array_equal(p1, p2) and c1 == c2
    three = _plan(N, P, pf.MODE_PFB, 2, n_int, chunk=chunk)
    d3, p3, _ = run_stream(three, x, [120])
    assert np.array_equal(d1, d3) and np.array_equal(p1, p3)
    # an unaligned split differs only by rounding
    four = _plan(N, P, pf.MODE_PFB, 2, n_int, chunk=chunk)
    d4, _, _ = run_stream(four, x, [13, 7, 29])
    assert d4.shape == d1.shape
    assert max(rel_err(a, b).max() for a, b in zip(d4, d1)) <= 1e-5


def test_reset_restarts_the_stream():
    torch = require_gpu()
    N = 512
    x = synth.generate(synth.spec_c2(n_ref=N), 0, 40 * N)
    plan = _plan(N, 8, pf.MODE_PFB, 2, 8)
    d1, _, _ = run_stream(plan, x, [40])
    plan.reset()
    info = plan.info()
    assert info["frames_seen"] == 0 and info["dumps_done"] == 0
    d2, _, _ = run_stream(plan, x, [40])
    assert np.array_equal(d1, d2)


def test_execute_rejects_bad_blocks():
    torch = require_gpu()
    plan = _plan(1024, 8, pf.MODE_PFB, 2, 4)
    blk = torch.zeros((1024 * 3 + 5, 2, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(pf.PfbsError) as ei:
        plan.execute(blk)
    assert ei.value.status == pf.ERR_INVALID
    blk = torch.zeros((1024 * 64, 2, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(pf.PfbsError):
        plan.execute(blk, None)       # dumps complete but no buffer
    assert plan.info()["frames_seen"] == 0   # rejected calls change nothing
    raw = torch.zeros(1024 * 8 * 4 + 16, dtype=torch.int8, device="cuda")
    with pytest.raises(pf.PfbsError):
        plan.execute(raw[1:1 + 1024 * 8 * 4])   # misaligned


def test_plan_execute_is_three_launches_with_the_history_in_the_reduction():
    """A two-pass PFB plan's block is three launches: the column pass, the row
    pass, and one launch holding the dump reduction and the tap-history copy
    (the history copy has no launch of its own once spectra complete)."""
    N, P, frames = 32768, 8, [12, 9]
    x = synth.generate(tone_stream(2, N, 5), 0, N * sum(frames))
    plan = _plan(N, P, pf.MODE_PFB, 2, 4)
    plan.timing(True)
    d_split, _, _ = run_stream(plan, x, frames)
    kt = plan.timing_read()
    plan.close()
    assert kt["column_pass"][1] == kt["row_pass"][1] == kt["dump_reduce"][1] == len(frames)
    assert kt["tap_history"][1] == 0
    # the history copied in the first block's reduction launch feeds the second
    ref = oracle.dumps(x, N, P, oracle.taps(N, P), False, 4)
    assert d_split.shape == ref.shape
    for d in range(ref.shape[0]):
        assert within_fp32_bound(d_split[d], ref[d], N, n2=128) <= 1.0
