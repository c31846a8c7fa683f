"""Helpers for the GPU parity tests: run a stream through a plan block by
block and compare dumps with the oracle."""
from __future__ import annotations

import numpy as np


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def rel_err(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-channel relative error of integrated products [n_prod, N]:
    |dXX|/XX, |dYY|/YY, and for the cross terms |d|/sqrt(XX*YY) (the
    Cauchy-Schwarz scale, since Re/Im XY* may be near zero)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.shape[0] == 1:
        return np.abs(got[0] - ref[0]) / ref[0]
    xx, yy = ref[0], ref[1]
    sc = np.sqrt(xx * yy)
    return np.stack([np.abs(got[0] - xx) / xx, np.abs(got[1] - yy) / yy,
                     np.abs(got[2] - ref[2]) / sc, np.abs(got[3] - ref[3]) / sc])


U32 = 2.0 ** -24


U16 = 2.0 ** -11


def fp32_bound(ref: np.ndarray, N: int, c: float = 8.0, u: float = U32) -> np.ndarray:
    """Per-channel error bound of integrated products from FP32 arithmetic.

    A floating-point FFT has a normwise error |dX_jk| <= c*u*sqrt(log2 N)*rms_j
    (u = 2^-24, rms_j^2 = mean_k |X_jk|^2).  Summed over the spectra of a dump
    and bounded with Cauchy-Schwarz this gives
        |dD_k| <= 2 c u sqrt(log2 N) sqrt(D_k <D>)        (<D> = mean_k D_k),
    plus the 1e-5 relative allowance of the integrated power itself.  For the
    cross terms D_k is replaced by sqrt(XX_k YY_k).  The measured constant of
    the FP32 path is about 2.4; c = 8 leaves margin."""
    ref = np.asarray(ref, dtype=np.float64)
    if ref.shape[0] == 1:
        scale = ref[0][None]
    else:
        sc = np.sqrt(ref[0] * ref[1])
        scale = np.stack([ref[0], ref[1], sc, sc])
    mean = scale.mean(axis=1, keepdims=True)
    return 1e-5 * scale + 2 * c * u * np.sqrt(np.log2(N)) * np.sqrt(scale * mean)


def within_fp32_bound(got, ref, N, u: float = U32, c: float = 8.0) -> float:
    """max over channels of |got - ref| / bound (<= 1 passes).  ``u`` is the
    unit roundoff of the arithmetic (2^-24 for FP32, 2^-11 for FP16)."""
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref) / fp32_bound(ref, N, c=c, u=u)))


def run_stream(plan, x: np.ndarray, block_frames, keep_device=False):
    """Feed x[T, n_pol, 2] in blocks of the given frame counts (cycled until
    the stream is used up; a short last block takes what is left).  Returns
    (dumps [nd, n_prod, N] float32 numpy, partial [n_prod, N], partial count)."""
    torch = require_gpu()
    N = plan.N
    T = (x.shape[0] // N) * N
    out = []
    pos = 0
    i = 0
    while pos < T:
        f = block_frames[i % len(block_frames)]
        i += 1
        n = min(f * N, T - pos)
        blk = torch.from_numpy(np.ascontiguousarray(x[pos:pos + n])).cuda()
        nd = plan.dumps_in(n)
        d = torch.empty((max(nd, 1), plan.n_prod, N), dtype=torch.float32, device="cuda")
        got = plan.execute(blk, d if nd > 0 else None)
        assert got == nd
        if nd:
            out.append(d[:nd].cpu().numpy())
        pos += n
    part = torch.empty((plan.n_prod, N), dtype=torch.float32, device="cuda")
    cnt = plan.flush(part)
    torch.cuda.synchronize()
    dumps = np.concatenate(out) if out else np.zeros((0, plan.n_prod, N), np.float32)
    return dumps, part.cpu().numpy(), cnt
