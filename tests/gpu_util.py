"""Helpers for the GPU parity tests: run a stream through a plan block by
block and compare dumps with the oracle."""
from __future__ import annotations

import numpy as np


def tone_stream(n_pol: int, N: int, seed: int):
    """Noise (sigma 20) plus the dual-polarisation workload's correlated tone
    (bin 5000.5 of 32768 rescaled to N, amplitude 30, Y leading by 0.7 rad);
    one polarisation: the same tone alone."""
    from paper_1411_0436_amd import synth
    if n_pol == 2:
        s = synth.spec_c2(n_ref=N)
        return synth.StreamSpec(n_pol=2, sigma=s.sigma, seed=seed, tones=s.tones)
    b = 5000.5 * N / 32768.0
    return synth.StreamSpec(n_pol=1, sigma=20.0, seed=seed, tones=(synth.Tone(b, N, 30.0, (0.0,)),))


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


def fp32_bound(ref: np.ndarray, N: int, c: float = 8.0, u: float = U32, n2: int = 0) -> np.ndarray:
    """Per-channel error bound of integrated products from FP32 arithmetic.

    A floating-point FFT pass has a normwise error: the outputs of a pass over
    a vector v carry errors of rms c*u*sqrt(log2 L)*rms(v) (u = 2^-24, L the
    pass length).  In a two-pass FFT, N = N1*N2, the column pass transforms
    columns whose energy, summed, is the whole spectrum's, and its errors
    reach every channel: rms c*u*sqrt(log2 N2)*rms_j over all channels.  The
    row pass transforms row k2, whose outputs are exactly the channels
    k = k2 (mod N2), so its errors scale with that row's own power: a strong
    tone's row carries a large error on every channel of the row.  Per
    spectrum, |dX_jk|^2 <= c^2 u^2 log2 N (<|X_j|^2> + <|X_j|^2>_row(k)).
    Summed over the spectra of a dump and bounded with Cauchy-Schwarz:
        |dD_k| <= 2 c u sqrt(log2 N) sqrt(D_k (<D> + <D>_row(k))),
    plus the 1e-5 relative allowance of the integrated power itself.  With
    n2 = 0 (single-pass FFT) the row mean is the global mean.  For the cross
    terms D_k is replaced by sqrt(XX_k YY_k).  The measured constant of the
    FP32 path is about 2.4; c = 8 leaves margin."""
    ref = np.asarray(ref, dtype=np.float64)
    if ref.shape[0] == 1:
        scale = ref[0][None]
    else:
        sc = np.sqrt(ref[0] * ref[1])
        scale = np.stack([ref[0], ref[1], sc, sc])
    mean = scale.mean(axis=1, keepdims=True)
    if n2 and n2 < N:
        # channel k belongs to row k mod n2
        rows = scale.reshape(scale.shape[0], N // n2, n2).mean(axis=1)  # [q, n2]
        row_mean = np.tile(rows, (1, N // n2))
    else:
        row_mean = np.broadcast_to(mean, scale.shape)
    return 1e-5 * scale + 2 * c * u * np.sqrt(np.log2(N)) * np.sqrt(scale * (mean + row_mean))


def within_fp32_bound(got, ref, N, u: float = U32, c: float = 8.0, n2: int = 0) -> float:
    """max over channels of |got - ref| / bound (<= 1 passes).  ``u`` is the
    unit roundoff of the arithmetic (2^-24 for FP32, 2^-11 for FP16); ``n2``
    the column length of a two-pass FFT (0: single pass)."""
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref) / fp32_bound(ref, N, c=c, u=u, n2=n2)))


def plan_n2(plan) -> int:
    """Column length of the plan's two-pass FFT, 0 for a single pass."""
    i = plan.info()
    return int(i["split_n2"]) if i["split_n1"] > 1 else 0


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
