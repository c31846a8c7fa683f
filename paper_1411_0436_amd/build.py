"""Build the HIP library libpfbspec.so for gfx950, in-tree.

Every HIP source is compiled with hipcc for --offload-arch=gfx950 only, with
packed FP32 instructions disabled (-packed-fp32-ops), and linked into one
shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpfbspec.so")
RUNNER = os.path.join(HERE, "pfbs_run")
SOURCES = ["k_single.hip", "k_fourstep.hip", "k_rows_f32.hip", "k_rows_mfma.hip", "k_batch.hip", "k_aux.hip", "plan.cpp", "autotune.cpp", "host_stream.cpp"]
HEADERS = ["pfbs_internal.h", "fft_common.h", "fft_bodies.h", "k_rows.h", os.path.join("..", "..", "include", "pfbspec.h")]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    # matrix-core results in ordinary VGPRs (no accumulator-register copies)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I" + os.path.join(ROOT, "include"),
]


def _objdir() -> str:
    d = os.path.join(HERE, "_build")
    os.makedirs(d, exist_ok=True)
    return d


def source_digest() -> str:
    """Digest of every library source and the public header: the library
    version that autotune cache entries are keyed on."""
    import hashlib
    h = hashlib.sha1()
    for name in sorted(os.listdir(CSRC)) + ["../../include/pfbspec.h"]:
        path = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(path):
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link libpfbspec.so.  Returns its path."""
    od = _objdir()
    objs = []
    procs = []
    version = ['-DPFBS_SOURCE_DIGEST="%s"' % source_digest()]
    for src in SOURCES:
        obj = os.path.join(od, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [HIPCC] + FLAGS + version + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errs = []
    for cmd, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            errs.append(" ".join(cmd) + "\n" + out.decode(errors="replace"))
        elif verbose and out:
            print(out.decode(errors="replace"))
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the plain C-ABI driver (for hardware-counter runs and as a C example)
    tmp = RUNNER + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp, os.path.join(CSRC, "pfbs_run.cpp"), "-L" + HERE, "-lpfbspec",
                             "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, RUNNER)
    return LIB


def build_host_sanitized(outdir: str, verbose: bool = False) -> str:
    """The same library with the address and undefined-behaviour sanitizers
    in its host code (device code is built as usual), linked into outdir.
    For host-side tests without a GPU.  Returns the library path."""
    os.makedirs(outdir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    version = ['-DPFBS_SOURCE_DIGEST="%s"' % source_digest()]
    for src in SOURCES:
        obj = os.path.join(outdir, src + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + san + version + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errs = []
    for cmd, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            errs.append(" ".join(cmd) + "\n" + out.decode(errors="replace"))
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    lib = os.path.join(outdir, "libpfbspec.so")
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    cmd = [clang, "-shared", "-fPIC", "-fsanitize=address,undefined", "-o", lib] + objs + \
          ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
