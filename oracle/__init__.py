"""FP64 CPU oracle of the spectrometer hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and this package never
imports the product library: the two share no code.  See ``pfb_oracle.c`` for
what is computed and which passage of the paper each step follows.

Python side: thin ctypes marshalling around the C functions, plus the dump
bookkeeping (which spectra form which integration), written out plainly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pfb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WINDOW_HANN_SINC = 0
WINDOW_RECT = 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP).  Returns the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        i32 = ctypes.c_int32
        L.orc_unpack.argtypes = [ctypes.c_void_p, i64, ctypes.c_void_p]
        L.orc_taps.argtypes = [i64, i32, i32, ctypes.c_void_p]
        L.orc_taps.restype = ctypes.c_int
        L.orc_dft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, i64, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_fft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, i64]
        L.orc_fft.restype = ctypes.c_int
        L.orc_pfb_f64.argtypes = [ctypes.c_void_p, i32, i64, i32, ctypes.c_void_p, i32, i64, ctypes.c_void_p]
        L.orc_pfb.argtypes = [ctypes.c_void_p, i32, i64, i32, ctypes.c_void_p, i32, i64, ctypes.c_void_p]
        L.orc_products.argtypes = [ctypes.c_void_p, i32, i64, ctypes.c_void_p]
        L.orc_integrate.argtypes = [ctypes.c_void_p, i64, i32, i64, i32, ctypes.c_void_p, i32,
                                    i64, i64, ctypes.c_void_p, i32]
        L.orc_integrate.restype = ctypes.c_int
        L.orc_num_spectra.argtypes = [i64, i64, i32, i32]
        L.orc_num_spectra.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def unpack(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int8)
    out = np.empty(x.shape, dtype=np.float64)
    lib().orc_unpack(_p(x), x.size, _p(out))
    return out


def taps(N: int, P: int, window: int = WINDOW_HANN_SINC) -> np.ndarray:
    h = np.empty(P * N, dtype=np.float64)
    if lib().orc_taps(N, P, window, _p(h)) != 0:
        raise ValueError("bad taps arguments")
    return h


def fft(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.complex128)
    re = np.ascontiguousarray(z.real)
    im = np.ascontiguousarray(z.imag)
    if lib().orc_fft(_p(re), _p(im), z.size) != 0:
        raise ValueError("N must be a power of two")
    return re + 1j * im


def dft(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.complex128)
    re = np.ascontiguousarray(z.real)
    im = np.ascontiguousarray(z.imag)
    ore = np.empty_like(re)
    oim = np.empty_like(im)
    lib().orc_dft(_p(re), _p(im), z.size, _p(ore), _p(oim))
    return ore + 1j * oim


def pfb_f64(xs: np.ndarray, N: int, P: int, h: Optional[np.ndarray], direct: bool, j: int) -> np.ndarray:
    """Pre-filter output of spectrum j from complex samples xs[T, n_pol]
    (float64 complex).  Returns complex [n_pol, N]."""
    xs = np.asarray(xs, dtype=np.complex128)
    n_pol = xs.shape[1]
    frames = 1 if direct else P
    if (j + frames) * N > xs.shape[0]:
        raise ValueError("stream too short for spectrum %d" % j)
    flat = np.ascontiguousarray(np.stack([xs.real, xs.imag], axis=-1))
    y = np.empty((n_pol, N, 2), dtype=np.float64)
    hh = np.ascontiguousarray(h if h is not None else np.zeros(1), dtype=np.float64)
    lib().orc_pfb_f64(_p(flat), n_pol, N, P, _p(hh), int(direct), j, _p(y))
    return y[..., 0] + 1j * y[..., 1]


def pfb(x: np.ndarray, N: int, P: int, h: Optional[np.ndarray], direct: bool, j: int) -> np.ndarray:
    """Pre-filter output of spectrum j from the int8 stream x[T, n_pol, 2].
    Returns complex [n_pol, N]."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    n_pol = x.shape[1]
    frames = 1 if direct else P
    if (j + frames) * N > x.shape[0]:
        raise ValueError("stream too short for spectrum %d" % j)
    y = np.empty((n_pol, N, 2), dtype=np.float64)
    hh = np.ascontiguousarray(h if h is not None else np.zeros(1), dtype=np.float64)
    lib().orc_pfb(_p(x), n_pol, N, P, _p(hh), int(direct), j, _p(y))
    return y[..., 0] + 1j * y[..., 1]


def products(X: np.ndarray) -> np.ndarray:
    """X complex [n_pol, N] -> products [n_prod, N] (float64)."""
    X = np.asarray(X, dtype=np.complex128)
    n_pol, N = X.shape
    flat = np.ascontiguousarray(np.stack([X.real, X.imag], axis=-1))
    out = np.empty((4 if n_pol == 2 else 1, N), dtype=np.float64)
    lib().orc_products(_p(flat), n_pol, N, _p(out))
    return out


def num_spectra(T: int, N: int, P: int, direct: bool) -> int:
    return int(lib().orc_num_spectra(T, N, P, int(direct)))


def integrate(x: np.ndarray, N: int, P: int, h: Optional[np.ndarray], direct: bool,
              j0: int, j1: int, n_threads: int = 0) -> np.ndarray:
    """Sum of the products of spectra [j0, j1) of the int8 stream
    x[T, n_pol, 2], in spectrum order.  Returns float64 [n_prod, N]."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    T, n_pol = x.shape[0], x.shape[1]
    out = np.empty((4 if n_pol == 2 else 1, N), dtype=np.float64)
    hh = np.ascontiguousarray(h if h is not None else np.zeros(1), dtype=np.float64)
    rc = lib().orc_integrate(_p(x), T, n_pol, N, P, _p(hh), int(direct), j0, j1, _p(out), n_threads)
    if rc != 0:
        raise ValueError("bad integrate arguments")
    return out


def dumps(x: np.ndarray, N: int, P: int, h: Optional[np.ndarray], direct: bool, n_int: int,
          which: Optional[List[int]] = None, n_threads: int = 0) -> np.ndarray:
    """Integrations of n_int consecutive valid spectra: dump d covers spectra
    [d*n_int, (d+1)*n_int).  Only complete dumps exist.  ``which`` selects dump
    indices (default: all).  Returns float64 [len(which), n_prod, N]."""
    S = num_spectra(x.shape[0], N, P, direct)
    n_d = S // n_int
    idx = list(range(n_d)) if which is None else list(which)
    for d in idx:
        if not (0 <= d < n_d):
            raise ValueError("dump %d does not exist (have %d)" % (d, n_d))
    n_prod = 4 if x.shape[1] == 2 else 1
    out = np.empty((len(idx), n_prod, N), dtype=np.float64)
    for i, d in enumerate(idx):
        out[i] = integrate(x, N, P, h, direct, d * n_int, (d + 1) * n_int, n_threads)
    return out


def tail(x: np.ndarray, N: int, P: int, h: Optional[np.ndarray], direct: bool, n_int: int,
         n_threads: int = 0) -> Tuple[np.ndarray, int]:
    """Partial integration after the last complete dump, and its spectrum count."""
    S = num_spectra(x.shape[0], N, P, direct)
    j0 = (S // n_int) * n_int
    return integrate(x, N, P, h, direct, j0, S, n_threads), S - j0


def stokes(prod: np.ndarray) -> np.ndarray:
    """Integrated products [..., 4, N] (|X|^2, |Y|^2, Re XY*, Im XY*) -> Stokes
    parameters of linear feeds [..., 4, N] = I, Q, U, V with I = |X|^2 + |Y|^2,
    Q = |X|^2 - |Y|^2, U = 2 Re XY*, V = -2 Im XY* (the paper notes that the
    Stokes parameters follow from the four products, Section 4; the sign of V
    is the reading recorded with the library's output option)."""
    p = np.asarray(prod, dtype=np.float64)
    xx, yy, re, im = p[..., 0, :], p[..., 1, :], p[..., 2, :], p[..., 3, :]
    return np.stack([xx + yy, xx - yy, 2.0 * re, -2.0 * im], axis=-2)


def fftshift(rows: np.ndarray) -> np.ndarray:
    """Channel order of the shifted output: position m holds channel
    (m + N/2) mod N along the last axis (negative frequencies first)."""
    r = np.asarray(rows)
    N = r.shape[-1]
    return r[..., (np.arange(N) + N // 2) % N]
