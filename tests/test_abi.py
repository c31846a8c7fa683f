"""The C-ABI library: it loads, exports every entry point the header declares,
and rejects bad arguments on the host before any device call (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1411_0436_amd import pfbspec as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfbspec.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfbs_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(pf.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = pf.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pfbs_[a-z_]+)\b", out))
    assert set(_declared()) <= exported


def _create(**kw):
    lib = pf.load()
    h = ctypes.c_void_p()
    d = pf.make_desc(**kw)
    st = lib.pfbs_plan_create_ex(ctypes.byref(h), ctypes.byref(d))
    return st, h


@pytest.mark.parametrize("kw", [
    dict(N=1000, P=8),                    # not a power of two
    dict(N=8, P=8),                       # too small
    dict(N=1 << 21, P=8),                 # too large
    dict(N=1024, P=0),
    dict(N=1024, P=17),
    dict(N=1024, P=8, mode=1),            # direct needs P=1
    dict(N=1024, P=8, mode=5),
    dict(N=1024, P=8, window=9),
    dict(N=1024, P=8, window=2),          # custom without taps
    dict(N=1024, P=8, n_pol=3),
    dict(N=1024, P=8, n_int=0),
    dict(N=1024, P=8, precision=7),
    dict(N=1024, P=8, n_pol=1, output=1),  # Stokes needs two polarisations
    dict(N=1024, P=8, output=5),
    dict(N=1024, P=8, fftshift=2),
    dict(N=1024, P=8, tap_unroll=3),
    dict(N=1024, P=8, split_n2=256),      # single-pass size with a split
    dict(N=1 << 15, P=8, split_n2=100),
    dict(N=1 << 15, P=8, split_n2=2048),  # N1 = 16 too small
    dict(N=1024, P=8, chunk=-1),
])
def test_invalid_arguments_rejected_before_device(kw):
    kw.setdefault("n_int", 4)
    st, h = _create(**kw)
    assert st == pf.ERR_INVALID, pf.last_error()
    assert not h.value
    assert pf.last_error()


def test_null_out_and_null_handles():
    lib = pf.load()
    assert lib.pfbs_plan_create(None, 1024, 8, 0, 0, 2, 4) == pf.ERR_INVALID
    assert lib.pfbs_plan_destroy(None) == pf.OK
    assert lib.pfbs_batch_destroy(None) == pf.OK
    assert lib.pfbs_dumps_in(None, 1024) == -1
    n = ctypes.c_int64(0)
    assert lib.pfbs_execute(None, None, 0, None, 0, ctypes.byref(n), None) == pf.ERR_STATE
    assert lib.pfbs_flush(None, None, ctypes.byref(n), None) == pf.ERR_STATE
    assert lib.pfbs_plan_reset(None) == pf.ERR_STATE
    assert lib.pfbs_batch_plan(None, 0) is None


def test_batch_validation_before_device():
    lib = pf.load()
    h = ctypes.c_void_p()
    good = pf.make_desc(N=1024, P=8, n_int=4)
    bad = pf.make_desc(N=1000, P=8, n_int=4)
    arr = (pf.PlanDesc * 2)(good, bad)
    assert lib.pfbs_batch_create(ctypes.byref(h), arr, 2) == pf.ERR_INVALID
    assert "sub-band 1" in pf.last_error()
    one = pf.make_desc(N=1024, P=8, n_int=4, n_pol=1)
    arr = (pf.PlanDesc * 2)(good, one)
    assert lib.pfbs_batch_create(ctypes.byref(h), arr, 2) == pf.ERR_INVALID
    assert lib.pfbs_batch_create(ctypes.byref(h), arr, 0) == pf.ERR_INVALID


def test_no_device_gives_device_error_not_crash():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _create(N=1024, P=8, n_int=4)
    assert st in (pf.ERR_DEVICE, pf.ERR_NOMEM, pf.ERR_UNSUPPORTED)
    assert not h.value


def test_library_shares_torchs_hip_runtime():
    """Loading the library must not bring a second HIP runtime into a process
    that uses PyTorch: the library binds libamdhip64 by soname to the copy
    PyTorch loaded (two runtimes in one process do not share the device)."""
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1411_0436_amd import pfbspec as pf\n"
            "pf.load()\n"
            "import re\n"
            "print(sorted(set(re.findall(r'/\\S*libamdhip64\\S*', open('/proc/self/maps').read()))))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr
    paths = eval(out.stdout.strip().splitlines()[-1])
    assert len(paths) == 1, paths
