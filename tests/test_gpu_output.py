"""Output forms of the dumps: Stokes parameters and the shifted channel
order, applied in place to the integrated FP32 products.  Same kernels up to
the dump, so the Stokes dumps equal the FP32 combination of a products run
bit for bit and the shifted dumps are a permutation of it; against the FP64
oracle the Stokes parameters stay within 1e-5 of I (each is a sum of
products whose own errors are within 1e-5 of XX, YY or sqrt(XX YY) <= I/2)."""
import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import require_gpu, run_stream

pytestmark = pytest.mark.gpu


def _stokes32(p):
    p = np.asarray(p, dtype=np.float32)
    xx, yy, re, im = p[..., 0, :], p[..., 1, :], p[..., 2, :], p[..., 3, :]
    return np.stack([xx + yy, xx - yy, np.float32(2) * re, np.float32(-2) * im], axis=-2)


@pytest.mark.parametrize("N,P,n_int,frames", [(1024, 8, 12, [30, 17]), (32768, 8, 5, [9, 8, 6])])
def test_stokes_and_shift_follow_the_products_bitwise(N, P, n_int, frames):
    x = synth.generate(synth.spec_c2(n_ref=N), 0, sum(frames) * N)
    runs = {}
    for out, shift in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        plan = pf.Plan(N, P, n_pol=2, n_int=n_int, output=out, fftshift=shift)
        runs[(out, shift)] = run_stream(plan, x, frames)
        plan.close()
    d0, p0, c0 = runs[(0, 0)]
    assert d0.shape[0] >= 2 and c0 > 0
    for (out, shift), (d, p, c) in runs.items():
        want_d, want_p = d0, p0
        if out:
            want_d, want_p = _stokes32(want_d), _stokes32(want_p)
        if shift:
            want_d, want_p = np.fft.fftshift(want_d, axes=-1), np.fft.fftshift(want_p, axes=-1)
        assert c == c0
        assert np.array_equal(d, want_d), (out, shift)
        assert np.array_equal(p, want_p), (out, shift)


def test_stokes_against_oracle():
    require_gpu()
    N, P, n_int = 4096, 8, 256
    x = synth.generate(synth.spec_c2(n_ref=N), 0, (n_int + P - 1) * N)
    plan = pf.Plan(N, P, n_pol=2, n_int=n_int, output=pf.OUT_STOKES, fftshift=1)
    d, _, _ = run_stream(plan, x, [n_int + P - 1])
    ref = oracle.fftshift(oracle.stokes(oracle.dumps(x, N, P, oracle.taps(N, P), False, n_int, which=[0])))[0]
    I = ref[0]
    err = np.abs(d[0].astype(np.float64) - ref) / I
    assert err.max() <= 1e-5, err.max()
    # the correlated tone (Y leading X by 0.7 rad) shows up in U and V
    k = int(np.argmax(I))
    assert abs(np.arctan2(d[0][3][k], d[0][2][k]) - 0.7) < 0.05
