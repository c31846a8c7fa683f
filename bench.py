#!/usr/bin/env python3
"""Throughput of the spectrometer hot path on one MI355X.

One step = the whole workload stream pushed through pfbs_execute block by
block (unpack -> 8-tap polyphase pre-filter -> N-point FFT -> polarisation
products -> integration and dumps), with every block already resident in
device memory.  The default workload is the largest mode: dual polarisation,
N = 524288 channels, 8-tap PFB, four 256 MB blocks (2^26 time samples each)
of the three-tone + pulse stream, 64 spectra per dump, timed for the
matrix-core MIXED path, FP32 and FP16X2 on the same blocks.

Prints ONE JSON line:
  value       : Gsamples/s (complex int8 samples of all polarisations / s)
                of the fastest path whose first dump is within 1e-5 of the
                FP64 oracle (named by dtype); every path is listed in paths;
  roofline    : that path's dominant kernel: method flops per launch over its
                average launch time from the library's dispatch timestamps,
                against the published FP32 vector peak, and the same launch's
                algorithmic HBM bytes (input + dumps) against 8 TB/s;
  step_roofline: the whole step against both roofs;
  cpu_baseline: the FP64 CPU oracle on a bounded sample of the same stream,
                all host cores and one thread.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_VECTOR_UNPACKED_TFLOPS = 78.6
FP32_VECTOR_UNPACKED_TFLOPS = 78.6

# Eight sub-bands of the batched mode: (N, P, direct, n_int); each sub-band
# gets 2^23 time samples (32 MB) per block, so every sub-band dumps once per block.
SUBBANDS = [(1024, 1, True, 8192), (4096, 1, True, 2048), (16384, 1, True, 512), (32768, 1, True, 256),
            (65536, 4, False, 128), (131072, 8, False, 64), (262144, 8, False, 32), (524288, 4, False, 16)]
SUB_BLOCK = 1 << 23

WORKLOADS = {
    # name: N, P, mode, n_pol, n_int, time samples per block, blocks, stream recipe
    "c2": dict(N=32768, P=8, direct=False, n_pol=2, n_int=1024, block=1 << 24, blocks=8, spec="c2",
               cpu_spectra=256),
    "c2-direct": dict(N=32768, P=1, direct=True, n_pol=2, n_int=1024, block=1 << 24, blocks=8, spec="c2"),
    # the largest mode: N=2^19, 256 MB blocks; the matrix-core paths beside FP32
    "c3": dict(N=1 << 19, P=8, direct=False, n_pol=2, n_int=64, block=1 << 26, blocks=4, spec="c3",
               precisions="mixed,fp32,fp16x2", cpu_spectra=4),
    "c1": dict(N=1024, P=8, direct=False, n_pol=1, n_int=1017, block=1 << 20, blocks=1, spec="c1"),
    # precision study: the c2 stream at three lengths (run with --precisions)
    "c4-4096": dict(N=4096, P=8, direct=False, n_pol=2, n_int=1024, block=1 << 24, blocks=8, spec="c2",
                    precisions="fp32,fp16x2,fp16,mixed", cpu_spectra=2048),
    "c4-65536": dict(N=65536, P=8, direct=False, n_pol=2, n_int=1024, block=1 << 24, blocks=8, spec="c2",
                     precisions="fp32,fp16x2,fp16,mixed", cpu_spectra=128),
    "c4-524288": dict(N=1 << 19, P=8, direct=False, n_pol=2, n_int=128, block=1 << 24, blocks=8, spec="c2",
                      precisions="fp32,fp16x2,fp16,mixed", cpu_spectra=4),
}
PRECISIONS = {"fp32": 0, "fp16": 1, "fp16x2": 2, "mixed": 3}

# Sources that define the spectrometer kernels: a traffic summary under
# profiles/ applies only while their digest is unchanged.
KERNEL_SOURCES = ["fft_common.h", "fft_bodies.h", "k_single.hip", "k_fourstep.hip", "k_rows.h",
                  "k_rows_f32.hip", "k_rows_mfma.hip", "pfbs_internal.h"]


def kernel_digest():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_0436_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the counter summary in profiles/
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when there is
    none for the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.txt" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha1") != kernel_digest():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_stream(w, procs):
    """The workload's blocks (the generator is per-window reproducible; its
    chunks are made on `procs` threads)."""
    from paper_1411_0436_amd import synth
    spec = {"c1": synth.spec_c1, "c2": synth.spec_c2, "c3": synth.spec_c3}[w["spec"]]()
    if w["spec"] == "c2" and w["N"] != 32768:
        spec = synth.spec_c2(n_ref=w["N"])
    x = synth.generate(spec, 0, w["blocks"] * w["block"], workers=procs)
    return [x[b * w["block"]:(b + 1) * w["block"]] for b in range(w["blocks"])]


def flops_per_pol_sample(kind, w, N1, N2):
    """Algorithmic (method) flops per complex pol-sample attributed to one
    kernel: pre-filter 4P (P real-by-complex multiply-adds), FFT 5 log2(L) per
    point of each L-point pass (5 log2 N in all), products 6 and accumulation
    2 (one polarisation: 4).  The four-step twiddle between the passes is an
    artefact of the two-pass algorithm, not method work, and is not counted."""
    P = 0 if w["direct"] else w["P"]
    prods = 8 if w["n_pol"] == 2 else 4
    if kind == "single_pass":
        return 4 * P + 5 * np.log2(w["N"]) + prods
    if kind == "column_pass":
        return 4 * P + 5 * np.log2(N2)
    if kind == "row_pass":
        return 5 * np.log2(N1) + prods
    return 0.0


def step_flops_per_pol_sample(w):
    """Method flops of the whole path per complex pol-sample: 4P + 5 log2 N + 8."""
    P = 0 if w["direct"] else w["P"]
    return 4 * P + 5 * np.log2(w["N"]) + (8 if w["n_pol"] == 2 else 4)


MFMA_FP16_PEAK_TFLOPS = 2500.0   # dense FP16 matrix-core peak (no sparsity)


def mfma_flops_per_pol_sample(kind, prec_name, w, N1, N2):
    """Dense matrix-core flops per complex pol-sample of one kernel: every
    radix-16 pass on the matrix cores runs 16x16x32 FP16 products (16384
    flops each) on 16 butterflies (256 points): 2 per group with single FP16
    (128 flops per point and pass), 6 with the hi/lo split (384).  MIXED:
    FP32 column/single pass, split-FP16 rows."""
    front = {"fp16": 128, "fp16x2": 384}.get(prec_name, 0)
    back = {"fp16": 128, "fp16x2": 384, "mixed": 384}.get(prec_name, 0)
    if kind == "single_pass":
        return front * (int(np.log2(w["N"])) // 4)
    if kind == "column_pass":
        return front * (int(np.log2(N2)) // 4)
    if kind == "row_pass":
        return back * (int(np.log2(N1)) // 4)
    return 0.0


def hbm_probe_gbps(mib=1024, reps=5):
    """Bandwidth of a plain device-to-device copy on this GPU (bytes read +
    written per second), the practical HBM ceiling beside the 8 TB/s peak."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def alg_bytes_per_pol_sample(kind, w):
    """Algorithmic HBM bytes per complex pol-sample: the int8 input (2 B, read
    by the kernel that pre-filters) and the dumps (4 B per product and channel
    per dump of n_int spectra, written by the reduction).  The two-pass
    intermediate, partial sums, tap table and tap history are not algorithmic."""
    n_prod = 4 if w["n_pol"] == 2 else 1
    dump = 4.0 * n_prod / (w["n_int"] * w["n_pol"])
    if kind in ("single_pass", "column_pass"):
        return 2.0
    if kind == "dump_reduce":
        return dump
    return 0.0


def _gen_sub(args):
    s, N, t0, n = args
    from paper_1411_0436_amd import synth
    return synth.generate(synth.spec_subband(s, N), t0, n)


def bench_subbands(args):
    """Eight uneven sub-bands per block: the batched form (three launches per
    block) replayed from a HIP graph, the same without the graph, and one
    execute per sub-band, all on the same device-resident blocks."""
    import torch
    from paper_1411_0436_amd import pfbspec as pf
    nblk = args.blocks or 2
    sub = args.sub_block
    prec = PRECISIONS[args.c5_precision]
    procs = min(16, len(os.sched_getaffinity(0)))
    jobs = [(s, N, b * sub, sub) for b in range(nblk) for s, (N, _, _, _) in enumerate(SUBBANDS)]
    import multiprocessing as mp
    t_gen = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_gen_sub, jobs)
    t_gen = time.perf_counter() - t_gen
    blocks = [[torch.from_numpy(parts[b * len(SUBBANDS) + s]).cuda() for s in range(len(SUBBANDS))]
              for b in range(nblk)]
    # every sub-band's speed-only fields from the autotuner at the sub-block
    # size (or the chunk given on the command line)
    t_tune = time.perf_counter()
    knobs = []
    for (N, P, d, ni) in SUBBANDS:
        if args.no_tune or args.chunk:
            knobs.append({"chunk": args.chunk})
        else:
            f, _ = pf.autotune(block_samples=sub, N=N, P=P, mode=pf.MODE_DIRECT if d else pf.MODE_PFB, n_pol=2,
                               n_int=ni, precision=prec)
            knobs.append({k: f[k] for k in KNOBS})
    t_tune = time.perf_counter() - t_tune
    descs = [pf.make_desc(N=N, P=P, mode=pf.MODE_DIRECT if d else pf.MODE_PFB, n_pol=2, n_int=ni,
                          precision=prec, **kn)
             for (N, P, d, ni), kn in zip(SUBBANDS, knobs)]
    samples_per_block = len(SUBBANDS) * sub * 2
    # the first few dozen executes of a process stall now and then (runtime
    # start-up); run them before any timed mode
    batch = pf.Batch(descs)
    dumps = [torch.empty((2, 4, p.N), dtype=torch.float32, device="cuda") for p in batch.plans]
    for i in range(40):
        batch.execute(blocks[i % nblk], dumps)
    torch.cuda.synchronize()
    batch.close()
    results = {}
    for mode in ("batched", "graph", "individual"):
        if mode == "individual":
            plans = [pf.Plan(N, P, mode=pf.MODE_DIRECT if d else pf.MODE_PFB, n_pol=2, n_int=ni, precision=prec,
                             **kn)
                     for (N, P, d, ni), kn in zip(SUBBANDS, knobs)]
        else:
            batch = pf.Batch(descs)
            plans = batch.plans
        dumps = [torch.empty((2, 4, p.N), dtype=torch.float32, device="cuda") for p in plans]

        def step(b):
            if mode == "individual":
                for p, blk, d in zip(plans, blocks[b], dumps):
                    p.execute(blk, d)
            else:
                batch.execute(blocks[b], dumps, use_graph=(mode == "graph"))
        # graph replays: the first few after instantiation are slow on this
        # runtime, so the graph mode gets a longer warm-up
        for i in range(max(args.warmup, 10) if mode == "graph" else args.warmup):
            step(i % nblk)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(args.steps):
            step(i % nblk)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        results[mode] = {"ms_per_block": round(ms, 4), "Gsamples_s": round(samples_per_block / (ms * 1e-3) / 1e9, 2)}
        if mode != "individual":
            results[mode]["launches_per_block"] = batch.launches
            batch.close()
        else:
            for p in plans:
                p.close()
    results["knobs"] = knobs
    results["tune_s"] = round(t_tune, 1)
    return results, t_gen


def bench_host_fed(args):
    """The C2 stream fed from page-locked host memory through pfbs_hstream
    (copy in, compute, copy out on three streams), against the same blocks
    already in device memory.  Returns both rates and the copy bandwidth."""
    import numpy as np
    import torch
    from paper_1411_0436_amd import pfbspec as pf
    w = dict(WORKLOADS["c2"])
    if args.blocks:
        w["blocks"] = args.blocks
    procs = min(16, len(os.sched_getaffinity(0)))
    host = make_stream(w, procs)
    N, P, B = w["N"], w["P"], w["block"]
    bufs = []
    for b in host:
        hb = pf.HostBuffer(b.shape, np.int8)
        hb.array[...] = b
        bufs.append(hb)
    hs = pf.HostStream(N, P, B, depth=args.depth, n_pol=2, n_int=w["n_int"])
    cap = hs.plan.dumps_in(B) + 1
    outs = [pf.HostBuffer((cap, 4, N), np.float32) for _ in bufs]

    def push_all():
        for hb, o in zip(bufs, outs):
            hs.push(hb.array, o.array)
    push_all()
    hs.sync()
    t = time.perf_counter()
    for _ in range(args.steps):
        push_all()
    hs.sync()
    dt = (time.perf_counter() - t) / args.steps
    samples = len(bufs) * B * 2
    host_rate = samples / dt / 1e9
    # the same plan shape on device-resident copies of the blocks
    dev = [torch.from_numpy(b).cuda() for b in host]
    plan = pf.Plan(N, P, n_pol=2, n_int=w["n_int"])
    d = torch.empty((cap, 4, N), dtype=torch.float32, device="cuda")
    for b in dev:
        plan.execute(b, d)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        for b in dev:
            plan.execute(b, d)
    torch.cuda.synchronize()
    dev_rate = samples / ((time.perf_counter() - t) / args.steps) / 1e9
    plan.close()
    hs.close()
    for b in bufs + outs:
        b.close()
    return {"host_fed_Gsamples_s": round(host_rate, 2), "device_resident_Gsamples_s": round(dev_rate, 2),
            "h2d_GBps": round(host_rate * 2, 2), "depth": args.depth, "blocks": len(host), "block_MB": B * 4 >> 20}


def bench_mode(args):
    """One observing-mode preset (the instrument's mode table) on device-resident
    blocks: a single plan, or a batch of eight plans for the eight-sub-band
    modes.  Returns Gsamples/s and the real-time factor."""
    import torch
    from paper_1411_0436_amd import pfbspec as pf
    from paper_1411_0436_amd import synth
    from paper_1411_0436_amd.modes import MODES, real_time_factor
    m = MODES[args.mode]
    nblk = args.blocks or 2
    sub = (1 << 24) if m.subbands == 1 else (1 << 23)
    streams = [[torch.from_numpy(synth.generate(synth.spec_c2(n_ref=m.N), b * sub + s * (1 << 30), sub)).cuda()
                for s in range(m.subbands)] for b in range(nblk)]
    descs = [pf.make_desc(N=m.N, P=m.P, n_pol=2, n_int=m.n_int) for _ in range(m.subbands)]
    cap = sub // m.N // m.n_int + 2
    if m.subbands == 1:
        plan = pf.Plan(m.N, m.P, n_pol=2, n_int=m.n_int)
        d = torch.empty((cap, 4, m.N), dtype=torch.float32, device="cuda")
        run = lambda b: plan.execute(streams[b][0], d)
    else:
        batch = pf.Batch(descs)
        ds = [torch.empty((cap, 4, m.N), dtype=torch.float32, device="cuda") for _ in range(m.subbands)]
        run = lambda b: batch.execute(streams[b], ds)
    for i in range(args.warmup):
        run(i % nblk)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        run(i % nblk)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    rate = m.subbands * sub * 2 / (ms * 1e-3)
    return {"Gsamples_s": round(rate / 1e9, 2), "ms_per_block": round(ms, 4),
            "real_time_factor": round(real_time_factor(m, rate), 1),
            "mode": {"name": m.name, "subbands": m.subbands, "bandwidth_MHz": m.bw_hz / 1e6, "N": m.N,
                     "n_int": m.n_int, "dump_interval_ms": round(m.dump_interval_s * 1e3, 3),
                     "required_Gsamples_s": m.required_samples_per_s / 1e9}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, blocks, spectra, min_seconds=10.0):
    """The FP64 oracle, as written, on the host cores: the first `spectra`
    valid spectra of the stream (0 = every spectrum of it), run again until at
    least `min_seconds` have passed, once with one thread and once with every
    core this process may use."""
    import oracle
    n_all = len(os.sched_getaffinity(0))
    N, P, direct = w["N"], w["P"], w["direct"]
    x = np.concatenate(blocks)
    total = oracle.num_spectra(x.shape[0], N, P, direct)
    S1 = total if spectra <= 0 else min(spectra, total)
    # the oracle spreads spectra over its threads: give every core two
    S_all = total if spectra <= 0 else min(max(spectra, 2 * n_all), total)
    x = x[:(S_all + (1 if direct else P) - 1) * N]
    h = None if direct else oracle.taps(N, P)
    oracle.integrate(x, N, P, h, direct, 0, 1, n_all)  # warm (page in, build)
    legs = {}
    for thr, S in ((1, S1), (n_all, S_all)):
        reps = 0
        t = time.perf_counter()
        while True:
            oracle.integrate(x, N, P, h, direct, 0, S, thr)
            reps += 1
            dt = time.perf_counter() - t
            if dt >= min_seconds:
                break
        legs[thr] = (reps * S * N * w["n_pol"] / dt / 1e9, reps, dt, S)
    v_all, reps, dt, S = legs[n_all]
    return {"value": v_all, "unit": "Gsamples/s", "cores": n_all, "kind": "oracle",
            "value_1_thread": legs[1][0], "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": "valid spectra from the start of the stream (N=%d, %s, %d pol), FP64 oracle; "
                      "%d threads: the first %d spectra, %d pass(es) in %.1f s; 1 thread: the first %d, "
                      "%d pass(es) in %.1f s"
                      % (N, "direct" if direct else "P=%d PFB" % P, w["n_pol"], n_all, S, reps, dt,
                         legs[1][3], legs[1][1], legs[1][2])}


def first_dump_error(w, prec, dev_blocks, ref, **plan_kw):
    """Max and median per-channel relative error (cross terms on the
    sqrt(XX*YY) scale) of the stream's first dump from a fresh plan of
    precision `prec`, against the oracle's `ref` [n_prod, N]."""
    import torch
    from paper_1411_0436_amd import pfbspec as pf
    N = w["N"]
    plan = pf.Plan(N, w["P"], mode=pf.MODE_DIRECT if w["direct"] else pf.MODE_PFB, n_pol=w["n_pol"],
                   n_int=w["n_int"], precision=prec, **plan_kw)
    cap = max(plan.dumps_in(w["block"]) + 1, 2)
    d = torch.empty((cap, plan.n_prod, N), dtype=torch.float32, device="cuda")
    for b in dev_blocks:
        if plan.execute(b, d) > 0:
            break
    torch.cuda.synchronize()
    got = d[0].cpu().numpy().astype(np.float64)
    plan.close()
    if ref.shape[0] == 1:
        e = np.abs(got[0] - ref[0]) / ref[0]
    else:
        sc = np.sqrt(ref[0] * ref[1])
        e = np.concatenate([np.abs(got[0] - ref[0]) / ref[0], np.abs(got[1] - ref[1]) / ref[1],
                            np.abs(got[2] - ref[2]) / sc, np.abs(got[3] - ref[3]) / sc])
    return float(np.max(e)), float(np.median(e))


KNOBS = ("split_n2", "chunk", "col_run", "stream_z", "tap_unroll", "col_pair", "row_tile")


def plan_knobs(w, prec_name, args):
    """The speed-only plan fields of one path: the autotuner's choice for this
    shape and block size (pfbs_autotune's coordinate search), or the ones given
    on the command line (then nothing is tuned)."""
    from paper_1411_0436_amd import pfbspec as pf
    given = {"split_n2": args.split_n2, "chunk": args.chunk, "tap_unroll": args.tap_unroll,
             "col_pair": args.col_pair, "row_tile": args.row_tile}
    if args.no_tune or any(given.values()):
        return dict(given), False
    fields, _ = pf.autotune(block_samples=w["block"], N=w["N"], P=w["P"],
                            mode=pf.MODE_DIRECT if w["direct"] else pf.MODE_PFB, n_pol=w["n_pol"],
                            n_int=w["n_int"], precision=PRECISIONS[prec_name])
    return {k: fields[k] for k in KNOBS}, True


def time_path(w, prec_name, dev_blocks, args, knobs):
    """Time `steps` passes of the whole stream through one plan of the given
    precision (after `warmup` untimed ones).  Kernel times come from the
    library's dispatch timestamps: every kind during the warm-up, only the
    dominant kind during the timed steps."""
    import torch
    from paper_1411_0436_amd import pfbspec as pf
    N = w["N"]
    plan = pf.Plan(N, w["P"], mode=pf.MODE_DIRECT if w["direct"] else pf.MODE_PFB, n_pol=w["n_pol"],
                   n_int=w["n_int"], group_bytes=args.group_mb << 20, precision=PRECISIONS[prec_name], **knobs)
    info = plan.info()
    cap = max(plan.dumps_in(w["block"]) + 1, 2)
    dumps = torch.empty((cap, plan.n_prod, N), dtype=torch.float32, device="cuda")

    def step():
        for b in dev_blocks:
            plan.execute(b, dumps)

    plan.timing(True)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    kt_all = plan.timing_read()
    dom = max(kt_all, key=lambda k: kt_all[k][0])
    plan.timing(True, kinds=[dom])
    # one event at every step boundary: the total and the median step
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(args.steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1])
    step_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    kt = plan.timing_read()
    plan.timing(False)
    plan.close()
    samples_per_step = w["blocks"] * w["block"] * w["n_pol"]
    value = args.steps * samples_per_step / (ms * 1e-3) / 1e9
    dom_ms, dom_n = kt[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    per_launch = samples_per_step * args.steps / max(dom_n, 1)
    return {"value": value, "ms_per_step": ms / args.steps, "ms_per_step_median": step_ms[len(step_ms) // 2],
            "info": info, "dominant": dom,
            "dom_avg_ms": avg_ms, "dom_pol_samples_per_launch": per_launch,
            "kernel_ms": {k: round(v[0] / max(v[1], 1), 5) for k, v in kt_all.items() if v[1]},
            "kernel_launches_per_step": {k: v[1] // max(1, args.warmup) for k, v in kt_all.items() if v[1]}}


DTYPES = {"fp32": "f32", "fp16": "f16 mfma (f32 accumulate)", "fp16x2": "f16x2 mfma (f32 accumulate)",
          "mixed": "f32 + f16x2 mfma (f32 accumulate)"}


def bench_stream(args):
    """The standard workloads: every requested precision timed on the same
    device-resident blocks, each with the max relative error of its first
    dump against the FP64 oracle; `value` is the fastest path within 1e-5."""
    import torch
    import oracle
    w = dict(WORKLOADS[args.workload])
    if args.blocks:
        w["blocks"] = args.blocks
    N, n_pol = w["N"], w["n_pol"]
    procs = min(16, len(os.sched_getaffinity(0)))
    t_gen = time.perf_counter()
    host_blocks = make_stream(w, procs)
    t_gen = time.perf_counter() - t_gen
    dev_blocks = [torch.from_numpy(b).cuda() for b in host_blocks]
    precs = [p.strip() for p in (args.precisions or w.get("precisions", "fp32")).split(",") if p.strip()]
    for p in precs:
        if p not in PRECISIONS:
            raise SystemExit("unknown precision %r" % p)

    # the first dump of the stream from the oracle: the sampled output every
    # path is checked against
    ref = None
    if not args.no_check:
        x = np.concatenate(host_blocks)
        S = oracle.num_spectra(x.shape[0], N, w["P"], w["direct"])
        if S >= w["n_int"]:
            h = None if w["direct"] else oracle.taps(N, w["P"])
            ref = oracle.integrate(x, N, w["P"], h, w["direct"], 0, w["n_int"], procs)
        del x

    paths = {}
    t_tune = 0.0
    for p in precs:
        t0 = time.perf_counter()
        knobs, tuned = plan_knobs(w, p, args)
        t_tune += time.perf_counter() - t0
        r = time_path(w, p, dev_blocks, args, knobs)
        r["knobs"], r["tuned"] = knobs, tuned
        if ref is not None:
            r["max_rel_err"], r["median_rel_err"] = first_dump_error(w, PRECISIONS[p], dev_blocks, ref,
                                                                     group_bytes=args.group_mb << 20, **knobs)
        paths[p] = r
        print("bench: %s %.2f Gsamples/s%s, %s %s" % (p, r["value"], "" if ref is None else
                                                      ", first-dump error %.3g" % r["max_rel_err"],
                                                      "tuned" if tuned else "given", knobs),
              file=sys.stderr, flush=True)
    ok = [p for p in precs if ref is None or paths[p]["max_rel_err"] <= 1e-5]
    best = max(ok or precs, key=lambda p: paths[p]["value"])
    r = paths[best]
    info = r["info"]
    dom = r["dominant"]
    avg_ms = r["dom_avg_ms"]
    per_launch = r["dom_pol_samples_per_launch"]
    fl = flops_per_pol_sample(dom, w, info["split_n1"], info["split_n2"]) * per_launch
    by = alg_bytes_per_pol_sample(dom, w) * per_launch
    tflops = fl / (avg_ms * 1e-3) / 1e12
    gbps = by / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, args.workload, best)
    value = r["value"]
    step_s = r["ms_per_step"] * 1e-3
    samples_per_step = w["blocks"] * w["block"] * n_pol
    dumps_per_step = samples_per_step / n_pol / N / w["n_int"]
    step_bytes = 2.0 * samples_per_step + dumps_per_step * 4.0 * (4 if n_pol == 2 else 1) * N
    step_flops = step_flops_per_pol_sample(w) * samples_per_step
    probe = hbm_probe_gbps()
    # the matrix cores: dense flops of each kernel that uses them, against its
    # own average launch time, and over the whole step
    mfma = {}
    step_mfma = 0.0
    for kind, kms in r["kernel_ms"].items():
        f = mfma_flops_per_pol_sample(kind, best, w, info["split_n1"], info["split_n2"])
        if f <= 0:
            continue
        launches = r["kernel_launches_per_step"][kind]
        per_launch_samples = samples_per_step / max(launches, 1)
        tf = f * per_launch_samples / (kms * 1e-3) / 1e12
        mfma[kind] = {"dense_flops_per_pol_sample": f, "TFLOPs": round(tf, 1), "peak": MFMA_FP16_PEAK_TFLOPS,
                      "frac": round(tf / MFMA_FP16_PEAK_TFLOPS, 4)}
        step_mfma += f * samples_per_step
    out = {
        "metric": "Gsamples/s PFB+FFT+integrate (dual-pol) at N=32K..512K; MFMA vs FP32 at 1e-5",
        "value": round(value, 2),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "ms_per_step_median": round(r["ms_per_step_median"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[best],
        "data": "synthetic (seeded int8 noise + tones%s, device-resident blocks)"
                % (" + broadband pulse" if w["spec"] == "c3" else ""),
        "config": {"workload": args.workload, "N": N, "P": w["P"], "mode": "direct" if w["direct"] else "pfb",
                   "n_pol": n_pol, "n_int": w["n_int"], "block_samples": w["block"],
                   "block_MB": w["block"] * 2 * n_pol >> 20, "blocks": w["blocks"], "precision": best,
                   "split_n1": info["split_n1"], "split_n2": info["split_n2"], "chunk": info["chunk"],
                   "row_tile": info["row_tile"], "knobs": r["knobs"], "tuned": r["tuned"],
                   "tune_s": round(t_tune, 1)},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": round(tflops, 3),
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                     # against the FP32 vector peak without packed instructions,
                     # which this build does not use
                     "frac_unpacked_peak": round(tflops / FP32_VECTOR_UNPACKED_TFLOPS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_over_alg_bytes": None if traffic is None or by <= 0 else round(traffic / by, 2),
                     "avg_launch_ms": round(avg_ms, 5),
                     "flops_per_launch": round(fl),
                     "alg_bytes_per_launch": round(by),
                     "hbm_GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBS, 4),
                     "traffic_GBps": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1)},
        "mfma_roofline": mfma or None,
        # the whole step against both roofs: method flops 4P + 5 log2 N + 8 per
        # pol-sample; algorithmic bytes = input + dumps
        "step_roofline": {"alg_flops_per_pol_sample": round(step_flops_per_pol_sample(w), 2),
                          "TFLOPs": round(step_flops / step_s / 1e12, 3),
                          "alu_frac": round(step_flops / step_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
                          "alg_bytes_per_step": round(step_bytes),
                          "hbm_GBps": round(step_bytes / step_s / 1e9, 1),
                          "hbm_frac": round(step_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
                          "hbm_probe_copy_GBps": round(probe, 1),
                          "hbm_frac_of_probe": round(step_bytes / step_s / 1e9 / probe, 4),
                          "mfma_TFLOPs": round(step_mfma / step_s / 1e12, 2),
                          "mfma_frac": round(step_mfma / step_s / 1e12 / MFMA_FP16_PEAK_TFLOPS, 4)},
        "bandwidth_per_pol_GHz": round(value / n_pol, 3),
        "paper_style_Gbps": round(value / n_pol * 16, 1),
        "paths": {p: {"Gsamples_s": round(q["value"], 2), "ms_per_step": round(q["ms_per_step"], 4),
                      "max_rel_err_first_dump": None if "max_rel_err" not in q else float("%.3g" % q["max_rel_err"]),
                      "median_rel_err_first_dump": None if "median_rel_err" not in q
                      else float("%.3g" % q["median_rel_err"]),
                      "ms_per_step_median": round(q["ms_per_step_median"], 4),
                      "within_1e-5": None if "max_rel_err" not in q else bool(q["max_rel_err"] <= 1e-5),
                      "split_n2": q["info"]["split_n2"], "row_arith": q["info"]["row_arith"],
                      "knobs": q["knobs"], "tuned": q["tuned"],
                      "dominant": q["dominant"], "kernel_ms": q["kernel_ms"],
                      "launches_per_step": q["kernel_launches_per_step"]}
                  for p, q in paths.items()},
        "paper_context_Gsamples_s": {"pfb_max": 2.2, "direct_max": 2.8,
                                     "note": "GTX TITAN, PCIe copies included (paper Section 5)"},
        "gen_s": round(t_gen, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, host_blocks, args.cpu_spectra or w.get("cpu_spectra", 0))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + ["c5", "c2-host"])
    ap.add_argument("--depth", type=int, default=3, help="c2-host: device slots of the host stream")
    ap.add_argument("--mode", default=None, help="run one observing-mode preset (paper_1411_0436_amd.modes)")
    ap.add_argument("--cpu-spectra", type=int, default=0,
                    help="spectra of the stream the CPU oracle is timed on (0 = the workload's default)")
    ap.add_argument("--no-check", action="store_true", help="skip the first-dump check against the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default=None,
                    help="comma-separated precisions to time (fp32, fp16, fp16x2, mixed); "
                         "default: the workload's list")
    ap.add_argument("--sub-block", type=int, default=SUB_BLOCK,
                    help="c5: time samples per sub-band per block (a multiple of 2^19)")
    ap.add_argument("--split-n2", type=int, default=0)
    ap.add_argument("--tap-unroll", type=int, default=0, help="pre-filter tap loop (0 auto, 1 unrolled, 2 loop)")
    ap.add_argument("--col-pair", type=int, default=0, help="two-spectra column kernel (0 auto, 1 on, 2 off)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--row-tile", type=int, default=0, help="row-pass tile points (0 auto)")
    ap.add_argument("--no-tune", action="store_true",
                    help="plans with their built-in choices instead of the autotuner's")
    ap.add_argument("--c5-precision", default="fp32", choices=["fp32", "mixed"],
                    help="c5: precision of every sub-band")
    ap.add_argument("--blocks", type=int, default=0, help="override the workload's block count")
    ap.add_argument("--group-mb", type=int, default=0, help="bound on the two-pass intermediate (MiB)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py: this spectrometer runs on one GPU; --gpus %d is not supported "
              "(streams or sub-bands would shard across GPUs with no exchange)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_0436_amd import pfbspec as pf

    if args.mode:
        res = bench_mode(args)
        out = {"metric": "Gsamples/s PFB+FFT+integrate (dual-pol) at N=32K..512K; MFMA vs FP32 at 1e-5",
               "value": res["Gsamples_s"], "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": res["ms_per_block"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic (seeded int8 noise + tone, device-resident blocks)",
               "config": {"workload": "mode:" + args.mode}, "real_time_factor": res["real_time_factor"],
               "mode": res["mode"]}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "c2-host":
        res = bench_host_fed(args)
        # the PCIe-inclusive rate is reported beside, never as, the device-path value
        out = {"metric": "Gsamples/s PFB+FFT+integrate (dual-pol) at N=32K..512K; MFMA vs FP32 at 1e-5",
               "value": res["device_resident_Gsamples_s"], "unit": "Gsamples/s", "n_gpus": 1,
               "steps": args.steps, "warmup": 1, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32",
               "data": "synthetic (the c2 stream in page-locked host memory)",
               "config": {"workload": "c2-host", "N": 32768, "P": 8, "n_pol": 2, "n_int": 1024},
               "host_fed": res}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "c5":
        res, t_gen = bench_subbands(args)
        out = {"metric": "Gsamples/s PFB+FFT+integrate (dual-pol) at N=32K..512K; MFMA vs FP32 at 1e-5",
               "value": res["graph"]["Gsamples_s"], "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": res["graph"]["ms_per_block"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.c5_precision],
               "data": "synthetic (seeded int8 noise + one tone per sub-band, device-resident blocks)",
               "config": {"workload": "c5", "subbands": [list(x) for x in SUBBANDS], "block_samples": args.sub_block,
                          "precision": args.c5_precision, "chunk": args.chunk,
                          "launch": "batched form (front phase, row phase, tail per block) replayed from its "
                                    "HIP graph; 'batched' is the same three launches made directly"},
               "modes": res, "gen_s": round(t_gen, 1)}
        print(json.dumps(out), flush=True)
        return

    out = bench_stream(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
