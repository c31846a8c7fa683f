"""Python binding of the pfbspec C ABI (include/pfbspec.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the spectrometer runs in the library's HIP kernels.
There is no fallback: if libpfbspec.so is missing or fails to load, every
call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfbspec.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_NOMEM, ERR_DEVICE, ERR_STATE = range(6)
WINDOW_HANN_SINC, WINDOW_RECT, WINDOW_CUSTOM = 0, 1, 2
MODE_PFB, MODE_DIRECT = 0, 1
PREC_FP32, PREC_MFMA_FP16, PREC_MFMA_FP16X2, PREC_MIXED = 0, 1, 2, 3
OUT_PRODUCTS, OUT_STOKES = 0, 1
TABLE_TAPS, TABLE_TW_FIRST, TABLE_TW_ROWS, TABLE_TW_ROWS_F64, TABLE_TW_STEP, TABLE_MFMA = range(6)

# Every entry point declared in include/pfbspec.h.
EXPORTS = (
    "pfbs_plan_create", "pfbs_plan_create_ex", "pfbs_plan_destroy", "pfbs_dumps_in",
    "pfbs_execute", "pfbs_flush", "pfbs_plan_reset", "pfbs_debug_pfb", "pfbs_debug_taps",
    "pfbs_plan_get_info", "pfbs_last_error", "pfbs_batch_create", "pfbs_batch_execute",
    "pfbs_batch_destroy", "pfbs_batch_plan", "pfbs_plan_timing", "pfbs_plan_timing_read",
    "pfbs_autotune", "pfbs_host_alloc", "pfbs_host_free", "pfbs_hstream_create", "pfbs_hstream_push",
    "pfbs_hstream_sync", "pfbs_hstream_destroy", "pfbs_hstream_plan", "pfbs_version", "pfbs_plan_timing_kinds",
    "pfbs_execute_noalloc", "pfbs_debug_table", "pfbs_batch_launches",
)

KERNEL_KINDS = ("single_pass", "column_pass", "row_pass", "dump_reduce", "tap_history")


class PfbsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("pfbspec status %d: %s" % (status, msg))
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("P", ctypes.c_int32), ("window", ctypes.c_int32),
        ("mode", ctypes.c_int32), ("n_pol", ctypes.c_int32), ("n_int", ctypes.c_int64),
        ("precision", ctypes.c_int32), ("device", ctypes.c_int32),
        ("custom_taps", ctypes.c_void_p), ("tune", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("split_n2", ctypes.c_int64), ("group_bytes", ctypes.c_int64),
        ("col_run", ctypes.c_int32), ("stream_z", ctypes.c_int32),
        ("output", ctypes.c_int32), ("fftshift", ctypes.c_int32),
        ("tap_unroll", ctypes.c_int32), ("col_pair", ctypes.c_int32), ("row_tile", ctypes.c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("P", ctypes.c_int32), ("n_pol", ctypes.c_int32),
        ("n_prod", ctypes.c_int32), ("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("chunk", ctypes.c_int32), ("n_int", ctypes.c_int64), ("split_n1", ctypes.c_int64),
        ("split_n2", ctypes.c_int64), ("frames_seen", ctypes.c_int64),
        ("spectra_done", ctypes.c_int64), ("dumps_done", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("row_arith", ctypes.c_int32), ("row_tile", ctypes.c_int32),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpfbspec.so and declare the signatures.  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpfbspec.so not built (%s); run __graft_entry__.build()" % path)
    # PyTorch ships its own HIP runtime under the same soname; loading it
    # first makes the library bind to that one runtime instead of bringing a
    # second one into the process (two runtimes do not share the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pi64 = ctypes.POINTER(ctypes.c_int64)
    L.pfbs_plan_create.argtypes = [ctypes.POINTER(vp), i64, i32, i32, i32, i32, i64]
    L.pfbs_plan_create_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc)]
    L.pfbs_plan_destroy.argtypes = [vp]
    L.pfbs_dumps_in.argtypes = [vp, i64]
    L.pfbs_dumps_in.restype = i64
    L.pfbs_execute.argtypes = [vp, vp, i64, vp, i64, pi64, vp]
    L.pfbs_execute_noalloc.argtypes = [vp, vp, i64, vp, i64, pi64, vp]
    L.pfbs_flush.argtypes = [vp, vp, pi64, vp]
    L.pfbs_plan_reset.argtypes = [vp]
    L.pfbs_debug_pfb.argtypes = [vp, vp, i64, vp, i64, pi64, vp]
    L.pfbs_debug_taps.argtypes = [vp, vp, vp]
    L.pfbs_debug_table.argtypes = [vp, i32, vp, i64, pi64, vp]
    L.pfbs_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.pfbs_last_error.restype = ctypes.c_char_p
    L.pfbs_version.restype = ctypes.c_char_p
    L.pfbs_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc), i32]
    L.pfbs_batch_execute.argtypes = [vp, ctypes.POINTER(vp), pi64, ctypes.POINTER(vp), pi64, pi64, i32, vp]
    L.pfbs_batch_destroy.argtypes = [vp]
    L.pfbs_batch_launches.argtypes = [vp]
    L.pfbs_batch_launches.restype = i32
    L.pfbs_plan_timing.argtypes = [vp, i32]
    L.pfbs_plan_timing_kinds.argtypes = [vp, ctypes.c_uint32]
    L.pfbs_plan_timing_kinds.restype = ctypes.c_int
    L.pfbs_plan_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), pi64, i32]
    L.pfbs_autotune.argtypes = [ctypes.POINTER(PlanDesc), i64, i32, ctypes.POINTER(PlanDesc),
                                ctypes.POINTER(ctypes.c_double)]
    L.pfbs_batch_plan.argtypes = [vp, i32]
    L.pfbs_batch_plan.restype = vp
    L.pfbs_host_alloc.argtypes = [ctypes.POINTER(vp), i64]
    L.pfbs_host_free.argtypes = [vp]
    L.pfbs_hstream_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc), i64, i32]
    L.pfbs_hstream_push.argtypes = [vp, vp, i64, vp, i64, pi64]
    L.pfbs_hstream_sync.argtypes = [vp]
    L.pfbs_hstream_destroy.argtypes = [vp]
    L.pfbs_hstream_plan.argtypes = [vp]
    L.pfbs_hstream_plan.restype = vp
    for name in ("pfbs_plan_create", "pfbs_plan_create_ex", "pfbs_plan_destroy", "pfbs_execute",
                 "pfbs_execute_noalloc", "pfbs_debug_table",
                 "pfbs_flush", "pfbs_plan_reset", "pfbs_debug_pfb", "pfbs_debug_taps",
                 "pfbs_plan_get_info", "pfbs_batch_create", "pfbs_batch_execute", "pfbs_batch_destroy",
                 "pfbs_plan_timing", "pfbs_plan_timing_read", "pfbs_autotune", "pfbs_host_alloc",
                 "pfbs_host_free", "pfbs_hstream_create", "pfbs_hstream_push", "pfbs_hstream_sync",
                 "pfbs_hstream_destroy"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def version() -> str:
    return load().pfbs_version().decode()


def last_error() -> str:
    return load().pfbs_last_error().decode(errors="replace")


def _check(st: int):
    if st != OK:
        raise PfbsError(st, last_error())


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_desc(N: int, P: int, window: int = WINDOW_HANN_SINC, mode: int = MODE_PFB, n_pol: int = 2,
              n_int: int = 1, precision: int = PREC_FP32, device: int = -1, custom_taps=None,
              tune: int = 0, chunk: int = 0, split_n2: int = 0, group_bytes: int = 0,
              col_run: int = 0, stream_z: int = 0, output: int = 0, fftshift: int = 0,
              tap_unroll: int = 0, col_pair: int = 0, row_tile: int = 0):
    """A PlanDesc; ``custom_taps`` (float64 numpy array) is kept alive on the
    returned object until the plan is created."""
    import numpy as np
    d = PlanDesc(N=N, P=P, window=window, mode=mode, n_pol=n_pol, n_int=n_int,
                 precision=precision, device=device, custom_taps=None, tune=tune,
                 chunk=chunk, split_n2=split_n2, group_bytes=group_bytes,
                 col_run=col_run, stream_z=stream_z, output=output, fftshift=fftshift,
                 tap_unroll=tap_unroll, col_pair=col_pair, row_tile=row_tile)
    keep = None
    if custom_taps is not None:
        keep = np.ascontiguousarray(custom_taps, dtype=np.float64)
        if keep.size != N * P:
            raise ValueError("custom_taps needs P*N values")
        d.custom_taps = keep.ctypes.data
    d._keep = keep
    return d


def autotune(block_samples: int = 0, max_candidates: int = 0, **desc_kw):
    """Time candidate settings for a plan shape (see pfbs_autotune).
    Returns (dict of the tuned fields, complex samples per second)."""
    L = load()
    d = make_desc(**desc_kw)
    best = PlanDesc()
    sps = ctypes.c_double(0.0)
    _check(L.pfbs_autotune(ctypes.byref(d), block_samples, max_candidates, ctypes.byref(best),
                           ctypes.byref(sps)))
    fields = ("split_n2", "chunk", "col_run", "stream_z", "tap_unroll", "col_pair", "row_tile")
    return {f: getattr(best, f) for f in fields}, sps.value


class Plan:
    """One spectrometer stream (pfbs_plan)."""

    def __init__(self, N: int, P: int, window: int = WINDOW_HANN_SINC, mode: int = MODE_PFB,
                 n_pol: int = 2, n_int: int = 1, **kw):
        self._lib = load()
        self._h = ctypes.c_void_p()
        d = make_desc(N, P, window, mode, n_pol, n_int, **kw)
        _check(self._lib.pfbs_plan_create_ex(ctypes.byref(self._h), ctypes.byref(d)))
        self.N, self.P, self.n_pol, self.n_int = N, P, n_pol, n_int
        self.n_prod = 4 if n_pol == 2 else 1

    @classmethod
    def _wrap(cls, handle: int, owner) -> "Plan":
        self = cls.__new__(cls)
        self._lib = load()
        self._h = ctypes.c_void_p(handle)
        self._owner = owner
        i = self.info()
        self.N, self.P, self.n_pol, self.n_int, self.n_prod = i["N"], i["P"], i["n_pol"], i["n_int"], i["n_prod"]
        return self

    def close(self):
        if getattr(self, "_owner", None) is None and self._h:
            _check(self._lib.pfbs_plan_destroy(self._h))
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dumps_in(self, n_time_samples: int) -> int:
        return int(self._lib.pfbs_dumps_in(self._h, n_time_samples))

    def execute(self, block, dumps=None, stream=None) -> int:
        """block: int8 cuda tensor [n, n_pol, 2] (or flat); dumps: float32 cuda
        tensor [cap, n_prod, N] or None.  Returns dumps written."""
        n = block.numel() // (2 * self.n_pol)
        cap = 0 if dumps is None else dumps.numel() // (self.n_prod * self.N)
        out = ctypes.c_int64(0)
        _check(self._lib.pfbs_execute(self._h, block.data_ptr(), n,
                                      None if dumps is None else dumps.data_ptr(), cap,
                                      ctypes.byref(out), _stream_ptr(stream)))
        return out.value

    def execute_noalloc(self, block, dumps=None, stream=None) -> int:
        """execute() through pfbs_execute_noalloc: the library's fixed scratch
        array instead of the plan's buffers; no device allocation."""
        n = block.numel() // (2 * self.n_pol)
        cap = 0 if dumps is None else dumps.numel() // (self.n_prod * self.N)
        out = ctypes.c_int64(0)
        _check(self._lib.pfbs_execute_noalloc(self._h, block.data_ptr(), n,
                                              None if dumps is None else dumps.data_ptr(), cap,
                                              ctypes.byref(out), _stream_ptr(stream)))
        return out.value

    def flush(self, partial, stream=None) -> int:
        cnt = ctypes.c_int64(0)
        _check(self._lib.pfbs_flush(self._h, partial.data_ptr(), ctypes.byref(cnt), _stream_ptr(stream)))
        return cnt.value

    def reset(self):
        _check(self._lib.pfbs_plan_reset(self._h))

    def debug_pfb(self, block, y, stream=None) -> int:
        n = block.numel() // (2 * self.n_pol)
        cap = y.numel() // (self.n_pol * self.N * 2)
        cnt = ctypes.c_int64(0)
        _check(self._lib.pfbs_debug_pfb(self._h, block.data_ptr(), n, y.data_ptr(), cap,
                                        ctypes.byref(cnt), _stream_ptr(stream)))
        return cnt.value

    def debug_taps(self, out, stream=None):
        _check(self._lib.pfbs_debug_taps(self._h, out.data_ptr(), _stream_ptr(stream)))

    def debug_table(self, which: int):
        """One of the plan's device tables (TABLE_*) as a uint8 cuda tensor,
        or None when the plan has none."""
        import torch
        n = ctypes.c_int64(0)
        _check(self._lib.pfbs_debug_table(self._h, which, None, 0, ctypes.byref(n), _stream_ptr(None)))
        if n.value == 0:
            return None
        out = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        _check(self._lib.pfbs_debug_table(self._h, which, out.data_ptr(), n.value, ctypes.byref(n),
                                          _stream_ptr(None)))
        return out

    def timing(self, enable: bool = True, kinds=None):
        """Time every launch (enable), or only the named kernel kinds."""
        if kinds is None:
            _check(self._lib.pfbs_plan_timing(self._h, int(enable)))
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << KERNEL_KINDS.index(k)
            _check(self._lib.pfbs_plan_timing_kinds(self._h, mask if enable else 0))

    def timing_read(self) -> dict:
        """{kind: (total ms, launches)} since the last read (waits for the events)."""
        n = len(KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(self._lib.pfbs_plan_timing_read(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}

    def info(self) -> dict:
        i = PlanInfo()
        _check(self._lib.pfbs_plan_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_}


class Batch:
    """Several sub-band streams run by three launches per block (pfbs_batch)."""

    def __init__(self, descs: Sequence[PlanDesc]):
        self._lib = load()
        self._h = ctypes.c_void_p()
        arr = (PlanDesc * len(descs))(*descs)
        _check(self._lib.pfbs_batch_create(ctypes.byref(self._h), arr, len(descs)))
        self.n = len(descs)
        self.plans = [Plan._wrap(self._lib.pfbs_batch_plan(self._h, i), self) for i in range(self.n)]

    def execute(self, blocks, dumps, use_graph: bool = False, stream=None):
        n = self.n
        vp = ctypes.c_void_p
        blk = (vp * n)(*[b.data_ptr() for b in blocks])
        ns = (ctypes.c_int64 * n)(*[b.numel() // (2 * p.n_pol) for b, p in zip(blocks, self.plans)])
        dp = (vp * n)(*[None if d is None else d.data_ptr() for d in dumps])
        caps = (ctypes.c_int64 * n)(*[0 if d is None else d.numel() // (p.n_prod * p.N)
                                      for d, p in zip(dumps, self.plans)])
        nd = (ctypes.c_int64 * n)()
        _check(self._lib.pfbs_batch_execute(self._h, blk, ns, dp, caps, nd, int(use_graph),
                                            _stream_ptr(stream)))
        return list(nd)

    @property
    def launches(self) -> int:
        """Kernel launches (or graph kernel nodes) of the last execute."""
        return int(self._lib.pfbs_batch_launches(self._h))

    def close(self):
        if self._h:
            for p in self.plans:
                p._h = ctypes.c_void_p()
            _check(self._lib.pfbs_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostBuffer:
    """Page-locked host memory (pfbs_host_alloc) seen as a numpy array."""

    def __init__(self, shape, dtype):
        import numpy as np
        self._lib = load()
        dt = np.dtype(dtype)
        n = int(np.prod(shape)) * dt.itemsize
        self._p = ctypes.c_void_p()
        _check(self._lib.pfbs_host_alloc(ctypes.byref(self._p), n))
        raw = (ctypes.c_uint8 * n).from_address(self._p.value)
        self.array = np.frombuffer(raw, dtype=dt).reshape(shape)

    @property
    def ptr(self) -> int:
        return self._p.value

    def close(self):
        if self._p:
            self.array = None
            _check(self._lib.pfbs_host_free(self._p))
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostStream:
    """A plan fed from host memory (pfbs_hstream): push() queues a block's
    host-to-device copy, its execution and the copy of its dumps back, on
    three streams; sync() waits for all of them."""

    def __init__(self, N: int, P: int, max_block_samples: int, depth: int = 3, **kw):
        self._lib = load()
        self._h = ctypes.c_void_p()
        d = make_desc(N, P, **kw)
        _check(self._lib.pfbs_hstream_create(ctypes.byref(self._h), ctypes.byref(d), max_block_samples, depth))
        self.plan = Plan._wrap(self._lib.pfbs_hstream_plan(self._h), self)
        self.N, self.n_pol, self.n_prod = self.plan.N, self.plan.n_pol, self.plan.n_prod

    def push(self, block, dumps=None) -> int:
        """block: C-contiguous int8 numpy array [n, n_pol, 2] (page-locked for an
        asynchronous copy); dumps: float32 numpy array [cap, n_prod, N] or None.
        Both must be left alone until the push has completed (sync, or `depth`
        later pushes)."""
        import numpy as np
        assert block.dtype == np.int8 and block.flags.c_contiguous
        n = block.size // (2 * self.n_pol)
        cap = 0 if dumps is None else dumps.size // (self.n_prod * self.N)
        if dumps is not None:
            assert dumps.dtype == np.float32 and dumps.flags.c_contiguous
        out = ctypes.c_int64(0)
        _check(self._lib.pfbs_hstream_push(self._h, block.ctypes.data, n,
                                           None if dumps is None else dumps.ctypes.data, cap,
                                           ctypes.byref(out)))
        return out.value

    def sync(self):
        _check(self._lib.pfbs_hstream_sync(self._h))

    def close(self):
        if self._h:
            self.plan._h = ctypes.c_void_p()
            _check(self._lib.pfbs_hstream_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
