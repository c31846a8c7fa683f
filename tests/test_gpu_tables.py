"""The plan's device tables, generated on the device in FP64 and rounded once
(Section 4, initialisation): every FP32 twiddle within one unit in the last
place of the FP64 value, the FP64 row-pass twiddles within a few units of
double rounding, the matrix-core DFT operands' hi + lo pairs within 2^-22 of
the exact DFT-16 entries.  References are computed here with numpy in FP64
from the definitions (exp(-2 pi i m / M)), not taken from the library."""
import numpy as np
import pytest

from paper_1411_0436_amd import pfbspec as pf
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _radix16_table(L):
    """W_(16 Ns)^(k r), k < Ns, r = 1..15, passes Ns = r0, 16 r0, ..."""
    logL = int(np.log2(L))
    r0 = 1 << (logL % 4)
    out = []
    Ns = r0
    for _ in range(logL // 4):
        k = np.arange(Ns)[:, None]
        r = np.arange(1, 16)[None, :]
        M = 16 * Ns
        out.append(np.exp(-2j * np.pi * ((k * r) % M) / M).ravel())
        Ns *= 16
    return np.concatenate(out)


def _as_complex(t, dtype):
    a = t.cpu().numpy().view(dtype)
    return a[0::2] + 1j * a[1::2]


def _within_one_ulp32(got, ref):
    # numpy's FP64 exp carries ~1e-16 of its own (e.g. 6e-17 where the exact
    # value, and the device's sincospi, is 0)
    for part in (np.real, np.imag):
        g, r = part(got).astype(np.float64), part(ref)
        ulp = np.spacing(np.abs(r).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(g - r) <= ulp + 2e-16), np.max(np.abs(g - r) - ulp)


@pytest.mark.parametrize("N,prec", [(4096, pf.PREC_FP32), (1 << 15, pf.PREC_FP32),
                                    (1 << 19, pf.PREC_FP32), (1 << 19, pf.PREC_MIXED),
                                    (1 << 20, pf.PREC_FP32)])
def test_twiddle_tables_within_one_ulp_of_fp64(N, prec):
    require_gpu()
    plan = pf.Plan(N, 8, n_pol=2, n_int=4, precision=prec)
    info = plan.info()
    n1, n2 = info["split_n1"], info["split_n2"]
    first = _as_complex(plan.debug_table(pf.TABLE_TW_FIRST), np.float32)
    _within_one_ulp32(first, _radix16_table(n2 if n1 > 1 else N))
    if n1 > 1:
        rows = _as_complex(plan.debug_table(pf.TABLE_TW_ROWS), np.float32)
        ref_rows = _radix16_table(n1)
        _within_one_ulp32(rows, ref_rows)
        step = _as_complex(plan.debug_table(pf.TABLE_TW_STEP), np.float32)
        m = (np.arange(n1)[:, None] * np.arange(n2)[None, :]) % N
        _within_one_ulp32(step, np.exp(-2j * np.pi * m / N).ravel())
        t64 = plan.debug_table(pf.TABLE_TW_ROWS_F64)
        if info["row_arith"] == 3:
            rows64 = _as_complex(t64, np.float64)
            assert np.max(np.abs(rows64 - ref_rows)) <= 1e-15
        else:
            assert t64 is None
    plan.close()


def test_matrix_core_operands_split_the_dft16_matrix():
    """Lane l holds, for output row m = l mod 16 and contraction columns
    k = 8 (l / 16) + j, the real form of W16: Re-row operand [Re W, -Im W]
    pairs and Im-row operand [Im W, Re W] pairs, each as FP16 hi + lo."""
    require_gpu()
    plan = pf.Plan(65536, 8, n_pol=2, n_int=4, precision=pf.PREC_MFMA_FP16X2)
    t = plan.debug_table(pf.TABLE_MFMA).cpu().numpy().view(np.float16).astype(np.float64).reshape(64, 4, 8)
    hr, hi, lr, li = t[:, 0], t[:, 1], t[:, 2], t[:, 3]
    W = np.exp(-2j * np.pi * np.outer(np.arange(16), np.arange(16)) / 16)
    for lane in range(64):
        m, kb = lane % 16, lane // 16
        for j in range(8):
            r = 4 * kb + j // 2
            w = W[m, r]
            want_r = w.real if j % 2 == 0 else -w.imag
            want_i = w.imag if j % 2 == 0 else w.real
            assert abs(hr[lane, j] + lr[lane, j] - want_r) <= 2.0 ** -22
            assert abs(hi[lane, j] + li[lane, j] - want_i) <= 2.0 ** -22
            assert abs(hr[lane, j] - want_r) <= 2.0 ** -11
    plan.close()
