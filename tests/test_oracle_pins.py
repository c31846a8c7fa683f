"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each check reaches the same
quantity by another route (a library FFT, a brute-force DFT written as a
matrix, the windowed-DTFT form of the pre-filter, closed forms of tones,
Parseval, noise statistics, an impulse response, exact integer arithmetic).
A dropped term, a wrong sign or index, or a transposed operand in the oracle
fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import synth


def _dtft_spectrum(xs_pol: np.ndarray, h: np.ndarray, N: int, j: int) -> np.ndarray:
    """Windowed DTFT at the N bins: X_j[k] = sum_{m<PN} h[m] x[jN+m] e^{-2pi i k m/N}.

    This is the pre-filter + DFT written as one sum over the P*N window
    (weighted overlap-add form, paper Section 4), not folded into frames."""
    L = h.size
    m = np.arange(L)
    k = np.arange(N)
    E = np.exp(-2j * np.pi * np.outer(k, m % N) / N)
    return E @ (h * xs_pol[j * N:j * N + L])


# ---------------------------------------------------------------- unpack ----

def test_unpack_all_256_bytes():
    raw = np.arange(256, dtype=np.uint8).view(np.int8)
    got = oracle.unpack(raw)
    want = np.array([b - 256 if b >= 128 else b for b in range(256)], dtype=np.float64)
    assert np.array_equal(got, want)
    assert got[128] == -128.0


# ------------------------------------------------------------ transforms ----

@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 64, 256])
def test_fft_equals_bruteforce_matrix_dft(N):
    rng = np.random.default_rng(N)
    z = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    n = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(n, n) / N)
    want = F @ z
    got = oracle.fft(z)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("N", [512, 4096, 32768])
def test_fft_matches_library_fft(N):
    rng = np.random.default_rng(7)
    z = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    got = oracle.fft(z)
    want = np.fft.fft(z)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-13


def test_bruteforce_dft_matches_library_fft():
    rng = np.random.default_rng(3)
    z = rng.standard_normal(96) + 1j * rng.standard_normal(96)  # not a power of two
    assert np.max(np.abs(oracle.dft(z) - np.fft.fft(z))) < 1e-11


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12))


def test_fft_sign_and_order_single_exponential():
    # e^{+2pi i 3n/N} lands in bin +3 (forward kernel e^{-2pi i kn/N}), gain N.
    N = 32
    n = np.arange(N)
    X = oracle.fft(np.exp(2j * np.pi * 3 * n / N))
    assert abs(X[3] - N) < 1e-12
    X[3] = 0
    assert np.max(np.abs(X)) < 1e-12


# ------------------------------------------------------------------ taps ----

@pytest.mark.parametrize("N,P", [(1024, 8), (64, 4), (16, 8), (32768, 8)])
def test_taps_closed_form_points(N, P):
    h = oracle.taps(N, P)
    L = P * N
    c = L // 2
    assert h.size == L
    assert h[c] == 1.0                       # sinc(0) * hann(centre) = 1
    assert abs(h[0]) == 0.0                  # hann(0) = 0
    for q in range(1, P // 2):               # zeros of sinc at every N from the centre
        assert abs(h[c + q * N]) < 1e-15
        assert abs(h[c - q * N]) < 1e-15
    d = np.arange(1, c)
    assert np.max(np.abs(h[c + d] - h[c - d])) < 1e-15  # symmetric about P*N/2
    # half a frame from the centre: sinc(1/2) = 2/pi, periodic Hann
    want = (2.0 / np.pi) * (0.5 - 0.5 * np.cos(2 * np.pi * (c + N // 2) / L))
    assert abs(h[c + N // 2] - want) < 1e-15


def test_taps_rect_is_ones():
    assert np.array_equal(oracle.taps(16, 3, oracle.WINDOW_RECT), np.ones(48))


def test_taps_rejects_unknown_window():
    with pytest.raises(ValueError):
        oracle.taps(16, 2, 7)


# ------------------------------------------------------------ pre-filter ----

def test_pfb_integer_asymmetric_taps_impulse_response():
    """An impulse at t0 (n0 = t0 mod N) shows up in spectrum j only at n0,
    weighted by h[t0 - jN]; asymmetric integer taps make a reversed or
    shifted tap order visible exactly."""
    N, P = 8, 4
    h = np.array([((7 * m) % 23) - 11 for m in range(P * N)], dtype=np.float64)
    T = 12 * N
    t0 = 5 * N + 3
    x = np.zeros((T, 2, 2), dtype=np.int8)
    x[t0, 0, 0] = 1     # X real impulse
    x[t0, 1, 1] = -2    # Y imaginary impulse
    S = oracle.num_spectra(T, N, P, False)
    for j in range(S):
        y = oracle.pfb(x, N, P, h, False, j)
        wx = np.zeros(N, dtype=complex)
        wy = np.zeros(N, dtype=complex)
        if 0 <= t0 - j * N < P * N:
            wx[t0 % N] = h[t0 - j * N]
            wy[t0 % N] = -2j * h[t0 - j * N]
        assert np.array_equal(y[0], wx), j
        assert np.array_equal(y[1], wy), j


def test_pfb_integer_taps_exact_against_integer_arithmetic():
    """With integer taps every partial sum is an exact integer, so the
    pre-filter must agree exactly with integer arithmetic done frame by frame."""
    N, P = 16, 5
    h = np.array([((7 * m) % 23) - 11 for m in range(P * N)], dtype=np.int64)
    rng = np.random.default_rng(11)
    T = 9 * N
    x = rng.integers(-128, 128, size=(T, 2, 2)).astype(np.int8)
    xi = x.astype(np.int64)
    for j in range(oracle.num_spectra(T, N, P, False)):
        y = oracle.pfb(x, N, P, h.astype(np.float64), False, j)
        frames = xi[j * N:(j + P) * N].reshape(P, N, 2, 2)   # [p, n, pol, re/im]
        taps = h.reshape(P, N)                                 # [p, n]
        acc = np.einsum("pn,pnqc->qnc", taps, frames)
        assert np.array_equal(y.real, acc[..., 0].astype(np.float64))
        assert np.array_equal(y.imag, acc[..., 1].astype(np.float64))


@pytest.mark.parametrize("N,P", [(16, 8), (32, 4), (64, 2)])
def test_pfb_plus_fft_equals_windowed_dtft(N, P):
    h = oracle.taps(N, P)
    rng = np.random.default_rng(N + P)
    T = (P + 3) * N
    x = rng.integers(-127, 128, size=(T, 2, 2)).astype(np.int8)
    xs = x[..., 0].astype(float) + 1j * x[..., 1].astype(float)
    for j in range(oracle.num_spectra(T, N, P, False)):
        y = oracle.pfb(x, N, P, h, False, j)
        for pol in range(2):
            got = oracle.fft(y[pol])
            want = _dtft_spectrum(xs[:, pol], h, N, j)
            assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def test_one_tap_rect_filter_equals_direct_mode():
    N = 64
    rng = np.random.default_rng(5)
    x = rng.integers(-128, 128, size=(10 * N, 2, 2)).astype(np.int8)
    h1 = oracle.taps(N, 1, oracle.WINDOW_RECT)
    a = oracle.integrate(x, N, 1, h1, False, 0, 10)
    b = oracle.integrate(x, N, 1, None, True, 0, 10)
    assert np.array_equal(a, b)


def test_num_spectra_startup_rule():
    # the first spectrum needs P frames; direct mode needs one
    assert oracle.num_spectra(1 << 20, 1024, 8, False) == 1017
    assert oracle.num_spectra(1 << 20, 1024, 8, True) == 1024
    assert oracle.num_spectra(7 * 1024 + 5, 1024, 8, False) == 0


# --------------------------------------------------------------- Parseval ----

def test_parseval_per_spectrum_and_integrated():
    N, P = 256, 8
    h = oracle.taps(N, P)
    x = synth.generate(synth.noise_only(2, 20.0, 9), 0, 20 * N)
    S = oracle.num_spectra(x.shape[0], N, P, False)
    tot_y = np.zeros(2)
    for j in range(S):
        y = oracle.pfb(x, N, P, h, False, j)
        for pol in range(2):
            X = oracle.fft(y[pol])
            e_y = np.sum(np.abs(y[pol]) ** 2)
            assert abs(np.sum(np.abs(X) ** 2) - N * e_y) <= 1e-12 * N * e_y
            tot_y[pol] += e_y
    D = oracle.integrate(x, N, P, h, False, 0, S)
    assert abs(D[0].sum() - N * tot_y[0]) <= 1e-12 * N * tot_y[0]
    assert abs(D[1].sum() - N * tot_y[1]) <= 1e-12 * N * tot_y[1]


# ----------------------------------------------------------- tone closed forms

@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_exact_bin_centred_tone_direct_mode(q):
    N, A = 128, 100
    k0 = q * N // 4
    x = synth.exact_tone(4 * N, 2, N, k0, A)
    D = oracle.integrate(x, N, 1, None, True, 0, 4)
    want = np.zeros(N)
    want[k0] = 4 * (A * N) ** 2
    assert np.max(np.abs(D[0] - want)) <= 1e-9 * want[k0]
    assert np.max(np.abs(D[1] - want)) <= 1e-9 * want[k0]
    assert np.max(np.abs(D[2] - want)) <= 1e-9 * want[k0]   # X = Y: Re XY* = |X|^2
    assert np.max(np.abs(D[3])) <= 1e-9 * want[k0]          # Im XY* = 0


def test_exact_bin_centred_tone_pfb_equals_filter_response():
    """Tone at integer bin k0: |X_j[k]|^2 = A^2 |H((k-k0)/N)|^2 with
    H(f) = sum_m h[m] e^{-2 pi i f m}; at k0 this is A^2 (sum h)^2."""
    N, P, A = 64, 8, 50
    k0 = N // 4
    h = oracle.taps(N, P)
    x = synth.exact_tone((P + 2) * N, 1, N, k0, A)
    D = oracle.integrate(x, N, P, h, False, 0, 3)
    m = np.arange(P * N)
    H = np.array([np.sum(h * np.exp(-2j * np.pi * ((k - k0) / N) * m)) for k in range(N)])
    want = 3 * A * A * np.abs(H) ** 2
    assert np.max(np.abs(D[0] - want)) <= 1e-10 * want.max()
    assert abs(D[0][k0] - 3 * (A * h.sum()) ** 2) <= 1e-10 * D[0][k0]


@pytest.mark.parametrize("k0", [5.5, 10.25, 31.75])
def test_off_bin_tone_direct_mode_dirichlet(k0):
    N, A = 64, 3.0
    t = np.arange(N)
    xs = (A * np.exp(2j * np.pi * k0 * t / N))[:, None]
    y = oracle.pfb_f64(xs, N, 1, None, True, 0)
    X = oracle.fft(y[0])
    k = np.arange(N)
    want = A * A * np.sin(np.pi * (k0 - k)) ** 2 / np.sin(np.pi * (k0 - k) / N) ** 2
    assert np.max(np.abs(np.abs(X) ** 2 - want)) <= 1e-9 * want.max()
    # half-bin scalloping of the rectangular window: about -3.92 dB
    if k0 == 5.5:
        loss = 10 * np.log10(np.abs(X[5]) ** 2 / (A * N) ** 2)
        assert abs(loss - (-3.9224)) < 1e-3


@pytest.mark.parametrize("k0", [5.5, 12.3])
def test_off_bin_tone_pfb_equals_filter_response(k0):
    N, P, A = 64, 8, 2.0
    h = oracle.taps(N, P)
    t = np.arange((P + 1) * N)
    xs = (A * np.exp(2j * np.pi * k0 * t / N))[:, None]
    m = np.arange(P * N)
    k = np.arange(N)
    H = np.array([np.sum(h * np.exp(-2j * np.pi * ((kk - k0) / N) * m)) for kk in k])
    for j in range(2):
        X = oracle.fft(oracle.pfb_f64(xs, N, P, h, False, j)[0])
        assert np.max(np.abs(np.abs(X) ** 2 - A * A * np.abs(H) ** 2)) <= 1e-9 * (A * A * np.abs(H) ** 2).max()


# ------------------------------------------------------- noise statistics ----

def test_white_noise_mean_power_pfb_and_direct():
    """E|X_j[k]|^2 = E|x|^2 * sum_m h[m]^2 for white input (every k); with
    rounding to integers E|x|^2 = sigma^2 + 1/6 (1/12 per component)."""
    N, P, sigma = 256, 8, 20.0
    h = oracle.taps(N, P)
    x = synth.generate(synth.noise_only(1, sigma, 21), 0, 400 * N)
    S = oracle.num_spectra(x.shape[0], N, P, False)
    D = oracle.integrate(x, N, P, h, False, 0, S)[0]
    ex2 = sigma ** 2 + 1.0 / 6.0
    ratio = D.mean() / (S * ex2 * np.sum(h ** 2))
    assert abs(ratio - 1.0) < 5.0 / np.sqrt(N * S / P)
    Dd = oracle.integrate(x, N, 1, None, True, 0, 400)[0]
    ratio_d = Dd.mean() / (400 * ex2 * N)
    assert abs(ratio_d - 1.0) < 5.0 / np.sqrt(N * 400)


# -------------------------------------------------------- cross spectrum ----

def test_cross_spectrum_phase_and_cauchy_schwarz():
    """Shared tone, Y leading by 0.7 rad: X Y* has phase -0.7 at the tone."""
    N = 1024
    spec = synth.spec_c2(n_ref=N)
    x = synth.generate(spec, 0, 64 * N)
    h = oracle.taps(N, 8)
    S = oracle.num_spectra(x.shape[0], N, 8, False)
    D = oracle.integrate(x, N, 8, h, False, 0, S)
    k_t = int(np.floor(5000.5 * N / 32768.0))
    ph = np.angle(D[2][k_t] + 1j * D[3][k_t])
    assert abs(ph - (-0.7)) < 0.02
    assert np.all(D[2] ** 2 + D[3] ** 2 <= D[0] * D[1] * (1 + 1e-12))


def test_products_sign_convention():
    X = np.array([[1 + 2j, 3 - 1j]])
    Y = np.array([[-2 + 0.5j, 1j]])
    p = oracle.products(np.concatenate([X, Y]))
    xy = X[0] * np.conj(Y[0])
    assert np.allclose(p[0], np.abs(X[0]) ** 2)
    assert np.allclose(p[1], np.abs(Y[0]) ** 2)
    assert np.allclose(p[2], xy.real)
    assert np.allclose(p[3], xy.imag)


# --------------------------------------------------------------- Stokes -----

@pytest.mark.parametrize("jones,iquv", [
    ((1.0, 0.0), (1, 1, 0, 0)),                              # linear along X
    ((0.0, 1.0), (1, -1, 0, 0)),                             # linear along Y
    ((2 ** -0.5, 2 ** -0.5), (1, 0, 1, 0)),                  # linear at +45 degrees
    ((2 ** -0.5, -2 ** -0.5), (1, 0, -1, 0)),                # linear at -45 degrees
    ((2 ** -0.5, 1j * 2 ** -0.5), (1, 0, 0, 1)),             # circular, Y leading X by 90 degrees
    ((2 ** -0.5, -1j * 2 ** -0.5), (1, 0, 0, -1)),           # circular, Y lagging
])
def test_stokes_of_pure_polarisation_states(jones, iquv):
    """Fully polarised unit-power waves of known polarisation state, through
    the oracle's products and Stokes: the textbook parameters of linear feeds
    (with V signed by the phase of Y relative to X)."""
    X = np.array([[jones[0], 0.3 * jones[0]]])
    Y = np.array([[jones[1], 0.3 * jones[1]]])
    S = oracle.stokes(oracle.products(np.concatenate([X, Y])))
    assert S.shape == (4, 2)
    assert np.allclose(S[:, 0], iquv, atol=1e-12)
    assert np.allclose(S[:, 1], 0.09 * np.array(iquv), atol=1e-12)


def test_stokes_fully_polarised_identity_and_unpolarised_noise():
    """I^2 = Q^2 + U^2 + V^2 for any single Jones vector; independent equal-power
    noise in X and Y integrates to Q, U, V small against I."""
    rng = np.random.default_rng(3)
    XY = rng.normal(size=(2, 64)) + 1j * rng.normal(size=(2, 64))
    S = oracle.stokes(oracle.products(XY))
    assert np.allclose(S[0] ** 2, S[1] ** 2 + S[2] ** 2 + S[3] ** 2, rtol=1e-12)
    Xn = rng.normal(size=(2, 4000, 8)) + 1j * rng.normal(size=(2, 4000, 8))
    acc = sum(oracle.products(Xn[:, t, :]) for t in range(4000))
    Sn = oracle.stokes(acc)
    assert np.all(np.abs(Sn[1:]) < 0.1 * Sn[0])


@pytest.mark.parametrize("N", [16, 1024])
def test_shifted_order_equals_library_fftshift(N):
    rows = np.random.default_rng(N).normal(size=(3, 4, N))
    assert np.array_equal(oracle.fftshift(rows), np.fft.fftshift(rows, axes=-1))


# ---------------------------------------------------------------- dumps -----

@pytest.mark.parametrize("n_pol", [1, 2])
def test_dumps_equal_windowed_dtft_route(n_pol):
    N, P, n_int = 16, 4, 5
    h = oracle.taps(N, P)
    rng = np.random.default_rng(2 + n_pol)
    T = 30 * N + 7   # ragged tail: the last partial frame is ignored
    x = rng.integers(-128, 128, size=(T, n_pol, 2)).astype(np.int8)
    xs = x[..., 0].astype(float) + 1j * x[..., 1].astype(float)
    S = (T // N) - P + 1
    assert oracle.num_spectra(T, N, P, False) == S
    spectra = np.array([[_dtft_spectrum(xs[:, p], h, N, j) for p in range(n_pol)]
                        for j in range(S)])             # [S, n_pol, N]
    if n_pol == 2:
        Xs, Ys = spectra[:, 0], spectra[:, 1]
        prods = np.stack([np.abs(Xs) ** 2, np.abs(Ys) ** 2,
                          (Xs * np.conj(Ys)).real, (Xs * np.conj(Ys)).imag], axis=1)
    else:
        prods = (np.abs(spectra[:, 0]) ** 2)[:, None, :]
    n_d = S // n_int
    got = oracle.dumps(x, N, P, h, False, n_int)
    assert got.shape == (n_d, 2 * n_pol if n_pol == 2 else 1, N) or got.shape[0] == n_d
    for d in range(n_d):
        want = prods[d * n_int:(d + 1) * n_int].sum(axis=0)
        assert np.max(np.abs(got[d] - want)) <= 1e-9 * np.max(np.abs(want))
    part, cnt = oracle.tail(x, N, P, h, False, n_int)
    assert cnt == S - n_d * n_int
    assert np.max(np.abs(part - prods[n_d * n_int:].sum(axis=0))) <= 1e-9 * np.max(np.abs(part))


def test_integrate_rejects_short_stream():
    x = np.zeros((10 * 16, 1, 2), dtype=np.int8)
    with pytest.raises(ValueError):
        oracle.integrate(x, 16, 8, oracle.taps(16, 8), False, 0, 4)
