"""Observing-mode presets of the spectrometer, from the instrument's mode
table (the paper's Table 1, Section 3): single-sub-band modes with 100-187.5
MHz or 11.72-23.44 MHz bandwidth, and eight-sub-band modes with 15.625-23.44
MHz per sub-band.  Each preset takes one end of a row of that table.

A sub-band's bandwidth is its complex sample rate per polarisation (complex
sampling), so a mode needs 2 x sub-bands x bandwidth complex samples per
second to keep up in real time; `real_time_factor` compares a measured rate
with that.  The spectra per dump follow from the minimum integration time:
n_int = ceil(t_min * bandwidth / N)."""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class Mode:
    name: str
    subbands: int       # sub-bands per polarisation
    bw_hz: float        # sub-band bandwidth = complex samples/s per polarisation
    N: int              # channels per sub-band
    min_int_s: float    # minimum integration time
    P: int = 8          # pre-filter taps

    @property
    def resolution_hz(self) -> float:
        return self.bw_hz / self.N

    @property
    def n_int(self) -> int:
        """Spectra per dump at the minimum integration time."""
        return max(1, math.ceil(self.min_int_s * self.bw_hz / self.N - 1e-9))

    @property
    def dump_interval_s(self) -> float:
        return self.n_int * self.N / self.bw_hz

    @property
    def required_samples_per_s(self) -> float:
        """Complex samples per second of both polarisations of all sub-bands."""
        return 2.0 * self.subbands * self.bw_hz


MODES = {m.name: m for m in (
    # single sub-band, wide: 100-187.5 MHz, 32768-131072 channels, 10-30 ms
    Mode("wide-32k", 1, 187.5e6, 32768, 0.010),
    Mode("wide-128k", 1, 100.0e6, 131072, 0.030),
    # single sub-band, narrow: 11.72-23.44 MHz, 32768-524288 channels, 5-75 ms
    Mode("narrow-32k", 1, 23.4375e6, 32768, 0.005),
    Mode("narrow-512k", 1, 11.71875e6, 524288, 0.075),
    # eight sub-bands: 15.625-23.44 MHz each, 4096-65536 channels, 5-100 ms
    Mode("eight-4k", 8, 23.4375e6, 4096, 0.005),
    Mode("eight-64k", 8, 15.625e6, 65536, 0.100),
)}


def real_time_factor(mode: Mode, achieved_samples_per_s: float) -> float:
    """Measured throughput over the mode's real-time requirement (> 1 keeps up)."""
    return achieved_samples_per_s / mode.required_samples_per_s
