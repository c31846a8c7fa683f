"""The autotuner: it times candidate settings on the device, returns a valid
one, records it in the cache file, and plans built from the cache compute the
same dumps as the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_1411_0436_amd import pfbspec as pf
from paper_1411_0436_amd import synth
from tests.gpu_util import rel_err, require_gpu, run_stream, within_fp32_bound

pytestmark = pytest.mark.gpu


def test_autotune_returns_valid_setting_and_caches_it(tmp_path, monkeypatch):
    require_gpu()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PFBS_TUNE_CACHE", str(cache))
    N = 8192
    fields, sps = pf.autotune(block_samples=64 * N, max_candidates=8, N=N, P=8, n_pol=2, n_int=16)
    assert sps > 0
    assert fields["split_n2"] in (128, 256, 512)  # rows no longer than the default split's
    assert fields["chunk"] in (0, 4, 8, 16, 32, 64)
    assert fields["row_tile"] in (0, 2048, 4096)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert f[0] == "pfbs-tune-v4" and f[1] == "gfx950" and "pfbspec " + f[2] == pf.version()
    assert len(f) == 18
    assert f[3:9] == ["8192", "8", "0", "2", "16", "0"]
    plan = pf.Plan(N, 8, n_pol=2, n_int=16, tune=1)
    info = plan.info()
    assert info["split_n2"] == fields["split_n2"]
    assert fields["chunk"] == 0 or info["chunk"] == fields["chunk"]
    assert info["row_tile"] == (fields["row_tile"] or 1024)
    x = synth.generate(synth.noise_only(2, 20.0, 77), 0, 60 * N)
    dumps, _, _ = run_stream(plan, x, [23, 37])
    ref = oracle.dumps(x, N, 8, oracle.taps(N, 8), False, 16)
    assert dumps.shape[0] == ref.shape[0] == 3
    for d in range(3):
        assert within_fp32_bound(dumps[d], ref[d], N) <= 1.0


def test_tune_without_cache_entry_keeps_defaults(tmp_path, monkeypatch):
    require_gpu()
    monkeypatch.setenv("PFBS_TUNE_CACHE", str(tmp_path / "empty.txt"))
    plan = pf.Plan(32768, 8, n_pol=2, n_int=4, tune=1)
    assert plan.info()["split_n2"] == 128  # the built-in choice for 2^15 channels


def test_single_pass_shape_tunes_chunk_only(tmp_path, monkeypatch):
    require_gpu()
    monkeypatch.delenv("PFBS_TUNE_CACHE", raising=False)
    fields, sps = pf.autotune(block_samples=256 * 1024, N=1024, P=8, n_pol=1, n_int=64)
    assert sps > 0 and fields["split_n2"] == 0 and fields["col_run"] == 0


def test_tuned_fp32_largest_mode_stays_within_1e5(tmp_path, monkeypatch):
    """Whatever split the tuner picks for an FP32 plan at N = 2^19, the plan
    keeps the largest mode's first dump within 1e-5 of the oracle: from 2^18
    channels the FP32 row pass runs in FP64, where a strong tone's row would
    otherwise carry more than 1e-5 of rounding."""
    require_gpu()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PFBS_TUNE_CACHE", str(cache))
    N = 1 << 19
    fields, sps = pf.autotune(N=N, P=8, n_pol=2, n_int=64, precision=pf.PREC_FP32, max_candidates=12)
    assert sps > 0 and fields["split_n2"] in (0, 128, 256, 512), fields
    plan = pf.Plan(N, 8, n_pol=2, n_int=64, tune=1)
    info = plan.info()
    assert info["row_arith"] == 3
    assert fields["split_n2"] in (0, info["split_n2"])
    blk = 1 << 26
    x = synth.generate(synth.spec_c3(), 0, blk, workers=synth.default_workers())
    dumps, _, _ = run_stream(plan, x, [blk // N])
    plan.close()
    ref = oracle.integrate(x, N, 8, oracle.taps(N, 8), False, 0, 64, synth.default_workers())
    assert rel_err(dumps[0], ref).max() <= 1e-5


def test_tuner_full_search_and_row_tiles_give_same_bits(tmp_path, monkeypatch):
    """A full coordinate search on a 2^17-channel MIXED shape (every field),
    and plans that differ only in the row-pass tile width (1024, 2048 and
    4096 points: 2, 4 and 8 rows of 512 per workgroup step) and in the column
    kernel's form (one or two spectra per workgroup) give the same dumps bit
    for bit."""
    require_gpu()
    monkeypatch.delenv("PFBS_TUNE_CACHE", raising=False)
    N = 1 << 17
    fields, sps = pf.autotune(block_samples=16 * N, N=N, P=8, n_pol=2, n_int=3, precision=pf.PREC_MIXED)
    assert sps > 0 and fields["split_n2"] in (256, 512) and fields["col_pair"] in (0, 1, 2)
    x = synth.generate(synth.spec_subband(6, N), 5, 25 * N)
    ref = None
    for rt in (0, 2048, 4096):
        for cp in (1, 2):
            plan = pf.Plan(N, 8, n_pol=2, n_int=3, precision=pf.PREC_MIXED, split_n2=256, row_tile=rt, col_pair=cp)
            assert plan.info()["row_tile"] == (rt or 1024)
            d, _, _ = run_stream(plan, x, [9, 16])
            plan.close()
            if ref is None:
                ref = d
            assert d.shape == ref.shape and np.array_equal(d, ref), (rt, cp)


def test_row_tile_rejected_when_shorter_than_rows():
    require_gpu()
    with pytest.raises(pf.PfbsError):
        pf.Plan(1 << 19, 8, n_pol=2, n_int=4, split_n2=128, row_tile=2048)   # rows of 4096
