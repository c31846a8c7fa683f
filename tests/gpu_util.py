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
