"""Parity of the matrix-core precisions with the FP64 oracle.

MFMA_FP16X2 (DFT matrix and data split into FP16 hi + lo pairs, three
products per radix-16 stage, FP32 accumulation) keeps about 22 significant
bits per operand, so it is held to the same bars as the FP32 path: 1e-5
relative per channel on the long integrations of the precision study, and
the FP32 arithmetic bound on short noise-only integrations.  MFMA_FP16
(single FP16 operands) is held to the same form of bound with the FP16 unit
roundoff 2^-11 in place of 2^-24 and c = 64 instead of 8: its matrix
rounding is the same for every spectrum, so its error does not average down
over an integration (measured normwise constant 28-35 at N = 2^16..2^19,
against about 2.4 for FP32), and its error is reported beside the others."""
import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import U16, U32, plan_n2, rel_err, run_stream, tone_stream, within_fp32_bound

pytestmark = pytest.mark.gpu

TOL = 1e-5
C16 = 64.0
X2, F16, MIX = pf.PREC_MFMA_FP16X2, pf.PREC_MFMA_FP16, pf.PREC_MIXED


@pytest.mark.parametrize("N,n_int", [(4096, 1024), (65536, 1024), (524288, 128)])
def test_precision_study_first_dump(N, n_int):
    """The c2 stream (sigma=20 noise + correlated tone) at the three lengths
    of the precision study, 8-tap PFB, first dump: FP32, FP16X2 and MIXED
    within 1e-5 of the oracle, FP16 within its roundoff bound."""
    P = 8
    n = (n_int + P - 1) * N
    x = synth.generate(synth.spec_c2(n_ref=N), 0, n)
    ref = oracle.dumps(x, N, P, oracle.taps(N, P), False, n_int, which=[0])[0]
    errs = {}
    for prec in (pf.PREC_FP32, X2, F16, MIX):
        plan = pf.Plan(N, P, n_pol=2, n_int=n_int, precision=prec)
        d, _, _ = run_stream(plan, x, [max(P, (1 << 24) // N)])
        plan.close()
        assert d.shape[0] == 1
        errs[prec] = rel_err(d[0], ref).max()
        if prec == F16:
            assert within_fp32_bound(d[0], ref, N, u=U16, c=C16) <= 1.0, errs
        else:
            assert errs[prec] <= TOL, errs
    print("max relative error N=%d: fp32 %.3g fp16x2 %.3g fp16 %.3g mixed %.3g"
          % (N, errs[0], errs[X2], errs[F16], errs[MIX]))


def test_mixed_config3_first_dump_within_1e5():
    """N=524288 dual-pol, 8-tap PFB, the three-tone + pulse stream, first dump
    of 64 spectra: the MIXED precision (FP32 column pass, FP16X2 row pass) at
    its default 256-point column split stays within 1e-5, where an all-FP32
    FFT with that split does not (1.2e-5 at the strongest tone's row)."""
    N, blk = 1 << 19, 1 << 26
    x = synth.generate(synth.spec_c3(), 0, blk, workers=synth.default_workers())
    plan = pf.Plan(N, 8, n_pol=2, n_int=64, precision=MIX)
    assert plan.info()["split_n2"] == 256
    dumps, _, cnt = run_stream(plan, x, [blk // N])
    assert dumps.shape[0] == 1
    ref = oracle.dumps(x, N, 8, oracle.taps(N, 8), False, 64, which=[0])
    e = rel_err(dumps[0], ref[0])
    assert e.max() <= TOL, e.max()


CASES = [
    # N, P, mode, n_pol, n_int, block frames, extra plan args
    (16, 4, pf.MODE_PFB, 2, 5, [9, 4], {}),
    (128, 8, pf.MODE_PFB, 1, 6, [7, 9], {}),
    (1024, 8, pf.MODE_PFB, 2, 8, [20, 8], {}),
    (2048, 1, pf.MODE_DIRECT, 1, 9, [11, 5], {}),
    (4096, 8, pf.MODE_PFB, 2, 5, [12, 12], {}),
    (8192, 8, pf.MODE_PFB, 2, 6, [14, 14], {}),
    (32768, 1, pf.MODE_DIRECT, 2, 4, [8, 8], {}),
    (32768, 8, pf.MODE_PFB, 2, 4, [12, 10], {"split_n2": 128}),
    (65536, 8, pf.MODE_PFB, 1, 3, [12], {"split_n2": 512}),
    (131072, 4, pf.MODE_PFB, 2, 3, [5, 4], {"split_n2": 64}),
]


@pytest.mark.parametrize("prec", [X2, F16, MIX])
@pytest.mark.parametrize("N,P,mode,n_pol,n_int,frames,kw", CASES)
def test_dumps_match_oracle(prec, N, P, mode, n_pol, n_int, frames, kw):
    """Every sub-FFT length and pass layout of both kernels (single pass,
    column and row passes of the two-pass FFT, one and two polarisations,
    PFB and direct), across block cuts, dumps and the flushed tail."""
    spec = tone_stream(n_pol, N, 200 + N % 89)
    T = sum(frames) * N
    x = synth.generate(spec, 0, T)
    plan = pf.Plan(N, P, mode=mode, n_pol=n_pol, n_int=n_int, precision=prec, **kw)
    dumps, part, cnt = run_stream(plan, x, frames)
    direct = mode == pf.MODE_DIRECT
    h = None if direct else oracle.taps(N, P)
    S = oracle.num_spectra(T, N, P, direct)
    assert dumps.shape[0] == S // n_int and cnt == S - (S // n_int) * n_int
    ref = oracle.dumps(x, N, P, h, direct, n_int)
    u, c = (U16, C16) if prec == F16 else (U32, 8.0)
    n2 = plan_n2(plan)
    for d in range(dumps.shape[0]):
        r = within_fp32_bound(dumps[d], ref[d], N, u=u, c=c, n2=n2)
        assert r <= 1.0, (d, r, rel_err(dumps[d], ref[d]).max())
    if cnt:
        tail, c2 = oracle.tail(x, N, P, h, direct, n_int)
        assert c2 == cnt
        assert within_fp32_bound(part, tail, N, u=u, c=c, n2=n2) <= 1.0


def test_fp16x2_full_scale_input_keeps_range():
    """Full-scale int8 tones (|x| = 127) in both polarisations: the growth of
    a coherent tone through the stages (x 2^19 at N=524288) must not overflow
    the FP16 operands; the per-butterfly scaling keeps them in range."""
    N, P, n_int = 524288, 1, 4
    x = synth.exact_tone((n_int + P - 1) * N, 2, N, N // 4, 127)
    ref = oracle.dumps(x, N, P, None, True, n_int)[0]
    plan = pf.Plan(N, P, mode=pf.MODE_DIRECT, n_pol=2, n_int=n_int, precision=X2)
    d, _, _ = run_stream(plan, x, [n_int])
    assert np.all(np.isfinite(d))
    k0 = N // 4
    # the tone bin carries (127 N)^2 per spectrum
    assert abs(d[0][0][k0] / ref[0][k0] - 1.0) <= TOL
    assert abs(d[0][1][k0] / ref[1][k0] - 1.0) <= TOL


def test_fp16x2_silence_and_tiny_signal():
    """All-zero input gives exact zeros; a +-1 LSB signal (values far below
    the FP16 normal range after the stage growth is divided out) still meets
    the FP32 bound, since each butterfly is scaled to its own maximum."""
    N, P, n_int = 4096, 8, 6
    z = np.zeros(((n_int + P - 1) * N, 2, 2), dtype=np.int8)
    plan = pf.Plan(N, P, n_pol=2, n_int=n_int, precision=X2)
    d, _, _ = run_stream(plan, z, [n_int + P - 1])
    assert d.shape[0] == 1 and not np.any(d)
    rng = np.random.default_rng(5)
    x = rng.integers(-1, 2, size=z.shape).astype(np.int8)
    plan = pf.Plan(N, P, n_pol=2, n_int=n_int, precision=X2)
    d, _, _ = run_stream(plan, x, [n_int + P - 1])
    ref = oracle.dumps(x, N, P, oracle.taps(N, P), False, n_int)[0]
    assert within_fp32_bound(d[0], ref, N) <= 1.0


def test_batch_rejects_matrix_core_front_precisions_and_output_forms():
    for kw in (dict(precision=X2), dict(precision=F16), dict(output=pf.OUT_STOKES), dict(fftshift=1)):
        desc = pf.make_desc(N=4096, P=8, n_pol=2, n_int=4, **kw)
        with pytest.raises(pf.PfbsError):
            pf.Batch([desc])


@pytest.mark.parametrize("prec,n_pol", [(X2, 2), (F16, 2), (X2, 1), (pf.PREC_FP32, 2)])
@pytest.mark.parametrize("unroll", [1, 2])
def test_two_spectra_column_kernel_equals_one_spectrum_kernel(prec, n_pol, unroll):
    """The two-spectra column kernel (col_pair=1) runs the same pre-filter and
    column FFT, in the same order, as the one-spectrum kernel (col_pair=2), in
    every precision and with either tap loop: the dumps agree bit for bit,
    with odd and even spectrum counts per block."""
    N, P, ni = 262144, 8, 3
    frames = [12, 11, 10]
    x = synth.generate(synth.spec_subband(5, N), 7, N * sum(frames))
    if n_pol == 1:
        x = np.ascontiguousarray(x[:, :1, :])
    out = []
    for pair in (1, 2):
        plan = pf.Plan(N, P, n_pol=n_pol, n_int=ni, precision=prec, split_n2=256, col_pair=pair,
                       tap_unroll=unroll)
        out.append(run_stream(plan, x, frames))
        plan.close()
    (d1, p1, c1), (d2, p2, c2) = out
    assert d1.shape == d2.shape and d1.shape[0] == (5 + 11 + 10) // ni
    assert np.array_equal(d1, d2) and np.array_equal(p1, p2) and c1 == c2
