"""Seeded synthetic voltage streams shaped like the spectrometer's inputs.

The paper benchmarks on recorded disk files that are not available (Section 5),
so every input here is synthetic: complex Gaussian noise plus tones and, for the
largest mode, a broadband pulse, rounded and clipped to two's-complement int8,
in the sample layout of Section 4 (dual-polarisation, 8-bit, complex).

This module holds no arithmetic of the spectrometer itself (no window, no
filter, no transform, no products).  It is shared by the tests, the benchmark
and the CPU oracle's callers; both sides consume the same bytes.

Layout of a stream: int8 array ``[T, n_pol, 2]`` (time-major, per time sample
X_re, X_im[, Y_re, Y_im]).

Determinism: the stream is cut into fixed generation chunks of ``GEN_CHUNK``
time samples; chunk ``c`` draws its noise from
``numpy.random.default_rng(SeedSequence([seed, c]))``.  Any window
``[t0, t0 + n)`` is therefore identical whether it is generated at once or in
pieces, whatever the processing block size.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

GEN_CHUNK = 1 << 20


@dataclasses.dataclass(frozen=True)
class Tone:
    """A complex exponential at ``bin_`` cycles per ``n_ref`` samples.

    ``phases`` holds the start phase (radians) per polarisation.
    """

    bin_: float
    n_ref: int
    amp: float
    phases: Tuple[float, ...] = (0.0, 0.0)


@dataclasses.dataclass(frozen=True)
class Pulse:
    """Additive complex Gaussian burst of std ``sigma`` during the first
    ``duty`` fraction of every ``period`` time samples (all polarisations)."""

    period: int
    duty: float
    sigma: float


@dataclasses.dataclass(frozen=True)
class StreamSpec:
    n_pol: int
    sigma: float
    seed: int
    tones: Tuple[Tone, ...] = ()
    pulse: Optional[Pulse] = None


def _tone_phase(t: np.ndarray, tone: Tone) -> np.ndarray:
    # 2*pi*bin*t/n_ref with the cycle count reduced modulo n_ref first, so the
    # phase keeps full float64 precision for t up to 2^30 and beyond.
    num = np.mod(t.astype(np.float64) * tone.bin_, float(tone.n_ref))
    return 2.0 * np.pi * num / float(tone.n_ref)


def _chunk(spec: StreamSpec, c: int) -> np.ndarray:
    """Float64 complex samples of generation chunk ``c`` as ``[L, n_pol]``."""
    rng = np.random.default_rng(np.random.SeedSequence([spec.seed, c]))
    L = GEN_CHUNK
    g = rng.standard_normal((L, spec.n_pol, 2))
    v = (g[..., 0] + 1j * g[..., 1]) * (spec.sigma / np.sqrt(2.0))
    t = np.arange(c * L, (c + 1) * L, dtype=np.int64)
    for tone in spec.tones:
        ph = _tone_phase(t, tone)
        for p in range(spec.n_pol):
            v[:, p] += tone.amp * np.exp(1j * (ph + tone.phases[p]))
    if spec.pulse is not None:
        pu = spec.pulse
        gp = rng.standard_normal((L, spec.n_pol, 2))
        on = (t % pu.period) < int(round(pu.duty * pu.period))
        burst = (gp[..., 0] + 1j * gp[..., 1]) * (pu.sigma / np.sqrt(2.0))
        v += burst * on[:, None]
    return v


def quantise(v: np.ndarray) -> np.ndarray:
    """Complex float ``[..., n_pol]`` -> int8 ``[..., n_pol, 2]``: clip each
    component to [-127, 127] and round half to even."""
    out = np.empty(v.shape + (2,), dtype=np.int8)
    out[..., 0] = np.rint(np.clip(v.real, -127.0, 127.0)).astype(np.int8)
    out[..., 1] = np.rint(np.clip(v.imag, -127.0, 127.0)).astype(np.int8)
    return out


def generate(spec: StreamSpec, t0: int, n: int, workers: int = 1) -> np.ndarray:
    """Time samples ``[t0, t0 + n)`` of the stream as int8 ``[n, n_pol, 2]``.
    ``workers`` > 1 generates the chunks on that many threads (numpy releases
    the interpreter lock inside its array routines); the bytes are the same."""
    if n < 0 or t0 < 0:
        raise ValueError("negative window")
    out = np.empty((n, spec.n_pol, 2), dtype=np.int8)
    pieces = []
    pos = 0
    while pos < n:
        t = t0 + pos
        c = t // GEN_CHUNK
        off = t - c * GEN_CHUNK
        take = min(GEN_CHUNK - off, n - pos)
        pieces.append((pos, c, off, take))
        pos += take

    def fill(piece):
        p, c, off, take = piece
        out[p:p + take] = quantise(_chunk(spec, c)[off:off + take])

    if workers > 1 and len(pieces) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(workers, len(pieces))) as ex:
            list(ex.map(fill, pieces))
    else:
        for piece in pieces:
            fill(piece)
    return out


def default_workers() -> int:
    """Generator threads: the cores this process may use, at most 16."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


# ---------------------------------------------------------------------------
# Stream recipes for the workloads (shapes from the paper's VEGAS modes,
# Table 1, and the benchmark configurations).
# ---------------------------------------------------------------------------

def spec_c1() -> StreamSpec:
    """Single polarisation, N=1024 reference: 20*g + 40*exp(2*pi*i*100.25*n/1024)."""
    return StreamSpec(n_pol=1, sigma=20.0, seed=0,
                      tones=(Tone(100.25, 1024, 40.0, (0.0,)),))


def spec_c2(n_ref: int = 32768) -> StreamSpec:
    """Dual polarisation, sigma=20 each, shared tone at bin 5000.5 (of 32768),
    amplitude 30, Y leading X by 0.7 rad.  ``n_ref`` rescales the tone bin for
    the same physical frequency at another channel count."""
    b = 5000.5 * n_ref / 32768.0
    return StreamSpec(n_pol=2, sigma=20.0, seed=1,
                      tones=(Tone(b, n_ref, 30.0, (0.0, 0.7)),))


def spec_c3() -> StreamSpec:
    """Dual polarisation at N=524288: sigma=16, three off-bin tones with
    independent phases per polarisation, and a 5%-duty 4-sigma broadband pulse
    of period 2^21 samples."""
    N = 524288
    tones = (
        Tone(12345.25, N, 24.0, (0.3, 1.9)),
        Tone(131072.5, N, 12.0, (2.2, -0.4)),
        Tone(400000.75, N, 6.0, (-1.1, 0.8)),
    )
    return StreamSpec(n_pol=2, sigma=16.0, seed=2, tones=tones,
                      pulse=Pulse(period=1 << 21, duty=0.05, sigma=64.0))


def spec_subband(s: int, N: int) -> StreamSpec:
    """Sub-band ``s`` of the eight-sub-band mode: sigma=20 noise plus one tone
    at bin N/4 + 0.3, amplitude 30."""
    return StreamSpec(n_pol=2, sigma=20.0, seed=4 + s,
                      tones=(Tone(N / 4 + 0.3, N, 30.0, (0.0, 0.5)),))


def noise_only(n_pol: int, sigma: float, seed: int) -> StreamSpec:
    return StreamSpec(n_pol=n_pol, sigma=sigma, seed=seed)


def exact_tone(n: int, n_pol: int, N: int, k0: int, amp: int,
               t0: int = 0) -> np.ndarray:
    """Noise-free tone at bin k0 in {0, N/4, N/2, 3N/4} of integer amplitude:
    exactly representable in int8, so its spectrum has a closed form."""
    if (4 * k0) % N != 0:
        raise ValueError("k0 must be a multiple of N/4")
    q = (4 * k0) // N
    t = np.arange(t0, t0 + n, dtype=np.int64)
    step = (q * t) % 4  # power of i
    re = np.array([1, 0, -1, 0], dtype=np.int64)[step] * amp
    im = np.array([0, 1, 0, -1], dtype=np.int64)[step] * amp
    out = np.zeros((n, n_pol, 2), dtype=np.int8)
    for p in range(n_pol):
        out[:, p, 0] = re
        out[:, p, 1] = im
    return out
