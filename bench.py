"""Benchmark of the partitioned-convolution hot path on one MI355X.

A step is one audio block through the whole path (input spectrum, FDL
multiply-accumulate over every partition of every filter, inverse FFT and
overlap-save output) with the input block already resident in HBM.  Default
workload: 1 input -> 32 outputs, 480,000-tap (10 s) reverberant filters,
block = partition = 128 at 48 kHz, FP32 spectra.

Printed on one JSON line:
  value         audio seconds processed per wall second (x real-time) over
                the timed steps, device-resident blocks launched back to back;
  rtf           its inverse (processing time / audio time, < 1 is real time);
  latency       p50/p99/max of synchronous host-memory rta_process() calls
                (PCIe copies included) issued one every B/fs as an audio
                callback would, against the deadline B/fs; also back to back;
  roofline      algorithmic bytes per launch of the block kernel k_block
                (every spectrum row once, every delay-line slot once, the
                input and output blocks) / its mean duration from HIP events
                on the launch stream, vs 8 TB/s;
  cpu_baseline  the FP64 oracle (single-partition FFT overlap-save) timed on
                the host cores over the workload's whole signal (independent
                of --steps), with the GPU output's error against it.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "real-time factor + p99 block latency, 32 out × 10 s filters, B=128 @48kHz"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


class no_gc:
    """Python's cyclic garbage collector off inside a latency loop: a full
    collection triggered by the binding's small allocations would otherwise
    land inside a timed call (the library itself allocates nothing per
    block)."""

    def __enter__(self):
        gc.collect()
        gc.disable()

    def __exit__(self, *exc):
        gc.enable()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_04390_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, spectra: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"k_block_{workload}_{spectra}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"model": model, "nproc": nproc, "cpu_count": os.cpu_count()}


def cpu_baseline(wl, filt, x, max_channels: int, y_gpu=None, reps: int = 3):
    """Time the oracle's FFT overlap-save over the first `max_channels`
    outputs of the whole signal `x` (one warm-up, median of `reps` runs, one
    run only if a run takes more than 10 s); scale to the full job.  With
    y_gpu ([L][n] of the GPU's outputs for the same signal) also report the
    GPU's error against that oracle result."""
    import oracle
    L = wl.n_out
    nch = min(L, max_channels)
    sub = [row[:nch] for row in filt]
    threads = oracle.max_threads()
    oracle.fftols(x[:, :wl.block * 8], [[f[:wl.block] for f in row] for row in sub], wl.block * 8)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        y_ref = oracle.fftols(x, sub, x.shape[1])
        times.append(time.perf_counter() - t0)
        if times[-1] > 10.0:
            break
    dt = float(np.median(times))
    audio_s = x.shape[1] / wl.fs
    full_s = dt * L / nch
    # one thread: the oracle runs one output per thread, so one output alone
    # is the one-thread time per output
    one = [row[:1] for row in filt]
    t0 = time.perf_counter()
    oracle.fftols(x, one, x.shape[1])
    one_s = (time.perf_counter() - t0) * L
    taps_total = sum(len(f_) for row in filt for f_ in row if f_ is not None)
    cpu = host_cpu()
    res = {
        "value": audio_s / full_s,
        "unit": "x real-time (audio s / wall s)",
        "cores": min(threads, nch),
        "wall_s": full_s,
        "channel_filter_seconds_per_s": taps_total / wl.fs * audio_s / full_s,
        "one_thread": {"value": audio_s / one_s, "wall_s": one_s,
                       "speedup_on_cores": one_s / full_s},
        "kind": "oracle",
        "sample": (f"FP64 single-partition FFT overlap-save (the oracle as committed) over the "
                   f"workload's whole signal, {x.shape[1]} samples ({audio_s:.2f} s), for "
                   f"{nch} of {L} outputs on {min(threads, nch)} OpenMP threads (one per "
                   f"output at most); median of {len(times)} runs of {dt:.2f} s, scaled to "
                   f"{L} outputs; offline (one FFT per filter), no per-block latency"),
        "host": {**cpu, "omp_threads": threads},
    }
    if y_gpu is not None:
        err = oracle.error_db(y_gpu[:nch, :x.shape[1]], y_ref)
        res["gpu_error_db"] = {"max": float(err.max()), "mean": float(err.mean()),
                               "outputs": nch, "samples": int(x.shape[1]),
                               "vs": "relative RMS per output vs this oracle result, "
                                     "GPU output of the same whole signal"}
    return res


def read_probes(torch, rta, nbytes: int, grid: int, stream, reps: int = 20):
    """Attainable streaming-read bandwidth of k_mac's load pattern, at the
    spectra size (may be served partly by the 256 MB Infinity Cache) and at
    1 GiB (larger than it)."""
    out = {}
    for tag, size in (("spectra_size", nbytes), ("1GiB", 1 << 30)):
        buf = torch.ones(size // 4, dtype=torch.float32, device="cuda")
        sink = torch.empty(grid, dtype=torch.float32, device="cuda")
        for _ in range(3):
            rta.rta_probe_read(buf.data_ptr(), size, grid, sink.data_ptr(), stream.cuda_stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            rta.rta_probe_read(buf.data_ptr(), size, grid, sink.data_ptr(), stream.cuda_stream)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        out[tag] = {"bytes": size, "grid": grid, "us_median": 1e3 * float(np.median(ms)),
                    "gbs": size / (float(np.median(ms)) * 1e-3) / 1e9}
        del buf, sink
    return out


def copy_probe(mb: int, reps: int) -> None:
    """A plain copy kernel of known size (elementwise negation into a second
    buffer: reads and writes mb MiB each), for scaling the memory counters."""
    import torch
    n = mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "reps": reps}))


def serve_bench(args, torch, rta, workloads) -> dict:
    """Serving with continuous batching: 16 source slots -> 64 outputs, 12 s
    filters, block 64.  Sources arrive as a Poisson process and stay for
    exponentially distributed times; a control thread admits and releases
    them (admission by HBM arena and per-block bandwidth budget) while the
    main thread issues one synchronous host-memory block every B/fs."""
    import threading
    wl = workloads.config("serve")
    B, L, taps, fs = wl.block, wl.n_out, wl.lengths, float(wl.fs)
    spectra = args.spectra or wl.dtype
    scheme = None
    if args.scheme and args.scheme != "uniform":
        scheme = [tuple(int(v) for v in t.split("x")) for t in args.scheme.split(",")]
    n_blocks = int(args.serve_seconds * fs / B)
    period = B / fs
    rng = np.random.default_rng(wl.seed)
    arrivals, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / args.serve_rate)
        if t >= args.serve_seconds:
            break
        life = rng.exponential(args.serve_life)
        arrivals.append((int(t / period), int((t + life) / period), len(arrivals) % 4))
    log(f"serve: {len(arrivals)} arrivals over {args.serve_seconds} s, {n_blocks} blocks")
    pool = [workloads.reverb_filters(wl.seed + i, 1, L, taps, wl.rt60)[0] for i in range(4)]
    stream = torch.cuda.current_stream()
    probe = read_probes(torch, rta, 1 << 30, 1024, stream)["1GiB"]["gbs"]
    budget = period * probe * 1e9 * args.serve_budget_frac
    srv = rta.Server(wl.n_in, L, taps, B, fs=fs, scheme=scheme, spectra=spectra,
                     budget_bytes=budget)
    info0, _ = srv.query()
    log(f"arena {info0['arena_bytes'] / 1e9:.2f} GB, budget {budget / 1e9:.2f} GB/block")
    fb_taps = args.serve_feedback_taps
    if fb_taps:
        # feedback cancellation (Sec. III-A Eq. 3): paths from the 64
        # loudspeakers to the 16 microphone slots, weak enough to keep the
        # loop gain below one; same spectrum type as the synthesis (fused)
        paths = workloads.reverb_filters(wl.seed + 99, wl.n_in, L, fb_taps, 0.1)
        srv.set_feedback([[(0.002 * p).astype(np.float32) for p in row] for row in paths],
                         spectra=spectra)
        log(f"feedback: {L} -> {wl.n_in} x {fb_taps} taps, fused {srv.info()['feedback_fused']}")

    events = sorted([(a, 0, i) for i, (a, _, _) in enumerate(arrivals)] +
                    [(e, 1, i) for i, (_, e, _) in enumerate(arrivals)])
    state = {"block": 0, "done": False}
    slot_of, admit_ms, outcome = {}, [], {"admitted": 0, "capacity": 0, "memory": 0}

    def control():
        for blk, kind, i in events:
            while state["block"] < blk and not state["done"]:
                time.sleep(0.0002)
            if state["done"]:
                return
            if kind == 0:
                t0 = time.perf_counter()
                try:
                    slot_of[i] = srv.admit(pool[arrivals[i][2]])
                    admit_ms.append(1e3 * (time.perf_counter() - t0))
                    outcome["admitted"] += 1
                except rta.RtaError as e:
                    outcome["memory" if e.status == rta.RTA_E_NOMEM else "capacity"] += 1
            elif i in slot_of:
                srv.release(slot_of.pop(i))

    noise = workloads.white_noise(wl.seed + 1, wl.n_in, 256 * B)
    blocks = [np.ascontiguousarray(noise[:, k * B:(k + 1) * B]) for k in range(256)]
    out = np.empty((L, B), np.float32)
    for k in range(16):  # first use of the pinned buffers
        rta.rta_process(srv.ctx, blocks[k], out)
    srv.reset()
    th = threading.Thread(target=control, daemon=True)
    th.start()
    lat, live, mbpb = [], [], []
    gc.collect()
    gc.disable()
    nxt = time.perf_counter()
    for n in range(n_blocks):
        nxt += period
        state["block"] = n
        t0 = time.perf_counter()
        rta.rta_process(srv.ctx, blocks[n % 256], out)
        lat.append(time.perf_counter() - t0)
        if n % 50 == 0:
            inf, _ = srv.query()
            live.append(inf["live"])
            mbpb.append(inf["bytes_per_block"] / 1e6)
        if n % 3000 == 0:
            log(f"  block {n}: live {live[-1]}, {mbpb[-1]:.0f} MB/block")
        rem = nxt - time.perf_counter()
        if rem > 3e-4:
            time.sleep(rem - 2e-4)
        while time.perf_counter() < nxt:
            pass
    gc.enable()
    state["done"] = True
    th.join()
    info, _ = srv.query()
    srv.close()
    lat_us = np.array(lat) * 1e6
    deadline = rta.deadline_us(B, fs)
    p99 = float(np.percentile(lat_us, 99))
    return {
        "metric": "serving: p99 block latency under continuous batching, 16 slots x 64 out x 12 s, B=64",
        "value": p99, "unit": "us", "n_gpus": 1, "steps": n_blocks, "warmup": 16,
        "ms_per_step": float(np.mean(lat_us)) / 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if spectra == "fp32" else f"f32 (spectra {spectra})", "data": "synthetic",
        "config": {"workload": (f"serve: {wl.n_in} slots -> {L} out, {taps}-tap ({taps / fs:.0f} s) "
                                f"filters, block {B}, {spectra} spectra, "
                                f"{'uniform partitions' if scheme is None else args.scheme}; "
                                f"Poisson arrivals {args.serve_rate}/s, Exp({args.serve_life} s) "
                                f"lifetimes, {args.serve_seconds} s; feedback cancellation "
                                f"{L} -> {wl.n_in} x {fb_taps} taps" if fb_taps else
                                f"{'uniform partitions' if scheme is None else args.scheme}; "
                                f"Poisson arrivals {args.serve_rate}/s, Exp({args.serve_life} s) "
                                f"lifetimes, {args.serve_seconds} s; no feedback paths"),
                   "block": B, "n_in": wl.n_in, "n_out": L, "taps": taps, "spectra": spectra},
        "deadline_us": deadline,
        "latency": {"p50_us": float(np.percentile(lat_us, 50)), "p99_us": p99,
                    "max_us": float(lat_us.max()), "xruns": int(np.sum(lat_us > deadline)),
                    "mode": "rta_process paced every B/fs, host memory, PCIe included"},
        "serve": {"arrivals": len(arrivals), "admitted": outcome["admitted"],
                  "refused_capacity": outcome["capacity"], "refused_memory": outcome["memory"],
                  "live_mean": float(np.mean(live)), "live_max": int(np.max(live)),
                  "mb_per_block_mean": float(np.mean(mbpb)), "mb_per_block_max": float(np.max(mbpb)),
                  "budget_mb_per_block": budget / 1e6, "read_probe_gbs": probe,
                  "admit_ms_p50": float(np.percentile(admit_ms, 50)) if admit_ms else None,
                  "admit_ms_max": float(np.max(admit_ms)) if admit_ms else None,
                  "plan_swaps": info["plan_swaps"], "arena_gb": info["arena_bytes"] / 1e9},
    }


def host_stages(info) -> dict:
    """The library's own timing of rta_process's host-side stages."""
    n = max(1, info["host_calls"])
    names = ("input_copy", "launch", "wait", "output_copy")
    return {"calls": info["host_calls"],
            "max_us": dict(zip(names, info["host_max_us"])),
            "mean_us": {k: v / n for k, v in zip(names, info["host_sum_us"])},
            "slowest_call": info["host_slowest_call"], "slowest_us": info["host_slowest_us"],
            "waits_past_2ms": info["host_late_waits"]}


def sweep_point(torch, rta, workloads, B, L, seconds, fs, spectra, fb_seconds=None,
                steps=400, paced=300, seed=11, flags=0):
    """One point of the paper's sweeps (Sec. VI, Figs. 3-6): 1 input -> L
    outputs with `seconds`-long filters at block B; optionally feedback
    cancellation with one microphone and L feedback paths of fb_seconds.
    Returns mean device-path block time and paced host-path latency."""
    n_h = max(1, int(round(seconds * fs)))
    filt = workloads.reverb_filters(seed, 1, L, n_h, (6.0, 10.0), int(fs))
    cv = rta.Convolver(filt, B, fs=fs, spectra=spectra, flags=flags)
    if fb_seconds is not None:
        n_f = max(1, int(round(fb_seconds * fs)))
        fb = workloads.reverb_filters(seed + 1, 1, L, n_f, (0.3, 0.3), int(fs))
        cv.set_feedback([[(0.001 * f).astype(np.float32) for f in fb[0]]])
    x = workloads.white_noise(seed + 2, 1, 64 * B)
    xb = torch.from_numpy(x.reshape(1, 64, B).transpose(1, 0, 2).copy()).cuda()
    yb = torch.empty((64, L, B), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    launch = rta._lib.rta_process_device
    pin = [xb[i].data_ptr() for i in range(64)]
    pout = [yb[i].data_ptr() for i in range(64)]
    for i in range(64):
        launch(cv.ctx, pin[i], pout[i], sh)
    rta.rta_timing_enable(cv.ctx, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if launch(cv.ctx, pin[k % 64], pout[k % 64], sh) != 0:
            raise RuntimeError("rta_process_device failed")
    torch.cuda.synchronize()
    us = 1e6 * (time.perf_counter() - t0) / steps
    n_timed, kern_ms = rta.rta_timing_read(cv.ctx)
    rta.rta_timing_enable(cv.ctx, False)
    out = np.empty((L, B), np.float32)
    blocks = [np.ascontiguousarray(x[:, i * B:(i + 1) * B]) for i in range(64)]
    for i in range(16):
        rta.rta_process(cv.ctx, blocks[i], out)
    cv.reset()  # also restarts the library's host-stage counters
    lat = []
    period = B / fs
    paced = max(20, min(paced, int(2.0 / period)))  # at most about 2 s of audio
    with no_gc():
        nxt = time.perf_counter()
        for i in range(paced):
            nxt += period
            t = time.perf_counter()
            rta.rta_process(cv.ctx, blocks[i % 64], out)
            lat.append(time.perf_counter() - t)
            rem = nxt - time.perf_counter()
            if rem > 3e-4:
                time.sleep(rem - 2e-4)
            while time.perf_counter() < nxt:
                pass
    info = cv.info()
    cv.close()
    lat_us = np.array(lat) * 1e6
    deadline = rta.deadline_us(B, fs)
    return {"block": B, "n_out": L, "filter_s": seconds, "fb_filter_s": fb_seconds,
            "us_per_block": us, "kernel_us": 1e3 * kern_ms / max(1, n_timed),
            "x_real_time": (B / fs) / (us * 1e-6), "deadline_us": deadline,
            "paced_p50_us": float(np.percentile(lat_us, 50)),
            "paced_p99_us": float(np.percentile(lat_us, 99)),
            "paced_max_us": float(lat_us.max()), "paced_max_at": int(np.argmax(lat_us)),
            "paced_blocks": len(lat), "xruns": int(np.sum(lat_us > deadline)),
            "spectra_mb": info["spectra_bytes"] / 1e6, "fft_size": info["fft_size"],
            "feedback_fused": info["feedback_fused"], "host_stages": host_stages(info)}


def sweeps(args, torch, rta, workloads) -> dict:
    """The paper's four sweeps around its defaults (32 outputs, 10 s filters,
    B = 128, 48 kHz): block size, filter length, output channels, and the
    feedback-cancellation filter length."""
    fs = 48000.0
    spectra = args.spectra or "fp32"
    which = args.sweep.split(",")
    if "all" in which:
        which = ["block", "length", "outputs", "feedback", "nf3"]
    grid = {
        "block": [dict(B=b, L=32, seconds=10.0) for b in (16, 32, 64, 128, 256, 512, 1024, 2048, 4096)],
        "length": [dict(B=128, L=32, seconds=s) for s in (0.1, 0.5, 1.0, 2.0, 5.0, 10.0, 15.0, 20.0)],
        "outputs": [dict(B=128, L=l, seconds=10.0) for l in (1, 2, 4, 8, 16, 32, 64, 96, 120, 128)],
        "feedback": [dict(B=128, L=32, seconds=10.0, fb_seconds=s) for s in (0.1, 0.5, 1.0, 2.0, 5.0)],
        # Sec. V: n_f = 3B against 2B with feedback, from short filters (where
        # the saved transforms should pay) to long ones
        "nf3": [dict(B=128, L=32, seconds=s, fb_seconds=0.1, flags=f)
                for s in (0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0, 10.0) for f in (0, rta.RTA_FLAG_NF3)],
    }
    res = {}
    for name in which:
        pts = []
        for kw in grid[name]:
            pt = sweep_point(torch, rta, workloads, fs=fs, spectra=spectra, **kw)
            log(f"sweep {name}: {json.dumps(pt)}")
            pts.append(pt)
        res[name] = pts
    return {"sweeps": res, "spectra": spectra, "fs": fs,
            "defaults": "1 input -> 32 outputs, 10 s filters, B = 128"}


def graph_leg(args, torch, cv, info, xb, yb, direct_ms_per_step):
    """The same device-resident blocks through rta_graph_launch: runs of M
    block launches captured once (block index from the device counter),
    replayed back to back; compared with one rta_process_device call per
    block."""
    nph = info["n_phases"]
    M = -(-max(args.graph_blocks, nph) // nph) * nph
    M = min(M, xb.shape[0] // nph * nph)
    reps = max(1, args.steps // M)
    with cv.graph(xb[:M], yb[:M], M) as g:
        for _ in range(2):
            g.launch()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(reps):
            g.launch()
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    us = 1e6 * wall / (reps * M)
    log(f"graph replay: {reps} x {M} blocks: {us:.2f} us/block "
        f"(direct launches {1e3 * direct_ms_per_step:.2f} us/block)")
    return {"blocks_per_graph": M, "replays": reps, "us_per_block_wall": us,
            "us_per_block_events": 1e3 * ev0.elapsed_time(ev1) / (reps * M),
            "direct_us_per_block_wall": 1e3 * direct_ms_per_step,
            "mode": "hipGraph of M block launches (device block counter), replayed back to back"}


MALL_BYTES = 256 << 20  # MI355X Infinity Cache


def hbm_honest_leg(args, torch, rta, cv, info, make_ctx, xb, yb, bytes_per_launch):
    """The roofline of a workload whose spectra (16 MB to 1.5 x the 256 MB
    Infinity Cache) the cache could serve in part, measured where it cannot:
    n independent contexts with the same filters (separate copies of the
    spectra, together at least 1.5 x the cache) take blocks in turn on one
    stream, so each context's spectra were evicted by the others' since its
    previous block.  Per-block time from HIP events around the whole run
    (launch gaps included: an upper bound)."""
    sb = int(info["spectra_bytes"])
    if args.hbm_honest_contexts == 0 or sb >= int(1.5 * MALL_BYTES) or sb < (16 << 20):
        return None
    n = max(args.hbm_honest_contexts, -(-int(1.5 * MALL_BYTES) // sb))
    n = min(n, 8)
    ctxs = [cv] + [make_ctx() for _ in range(n - 1)]
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    launch = rta._lib.rta_process_device
    rounds = max(4, args.steps // n)
    nblk = xb.shape[0]
    pin = [xb[i % nblk].data_ptr() for i in range(rounds + 8)]
    pout = [yb[i % nblk].data_ptr() for i in range(rounds + 8)]
    for c in ctxs:
        c.reset()
    for i in range(8):  # warm-up
        for c in ctxs:
            if launch(c.ctx, pin[i], pout[i], sh) != 0:
                raise RuntimeError("rta_process_device failed")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(8, 8 + rounds):
        for c in ctxs:
            if launch(c.ctx, pin[i], pout[i], sh) != 0:
                raise RuntimeError("rta_process_device failed")
    ev1.record(stream)
    torch.cuda.synchronize()
    us = 1e3 * ev0.elapsed_time(ev1) / (rounds * n)
    for c in ctxs[1:]:
        c.close()
    cv.reset()
    achieved = bytes_per_launch / (us * 1e-6) / 1e9
    log(f"HBM-honest variant: {n} contexts, {n * sb / 1e6:.0f} MB of spectra in turn: {us:.2f} us/block, "
        f"{achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.3f} of peak)")
    return {"contexts": n, "working_set_bytes": n * sb, "blocks": rounds * n, "us_per_block_events": us,
            "achieved": achieved, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "mode": "n independent contexts (separate spectra copies, > the 256 MB Infinity Cache "
                    "together) taking blocks in turn on one stream; HIP events around the run"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="main")
    ap.add_argument("--spectra", default=None, choices=["fp32", "fp16", "bf16"],
                    help="spectra storage (default: the workload's)")
    ap.add_argument("--scheme", default=None,
                    help="partition scheme as size x count tiers, e.g. 128x15,1024x14,8192x0; "
                         "'uniform' forces one tier (default: the workload's)")
    ap.add_argument("--latency-blocks", type=int, default=2000)
    ap.add_argument("--paced-blocks", type=int, default=1000,
                    help="host blocks issued one every B/fs (real-time pacing)")
    ap.add_argument("--cpu-channels", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner first and use its scheme and tiling")
    ap.add_argument("--tune-cache", default=None,
                    help="with --autotune: JSON-lines tuning cache file (rta_autotune_cached)")
    ap.add_argument("--timing-every", type=int, default=16,
                    help="time spans of this many consecutive blocks with two HIP events each "
                         "(event packets on every block would slow the stream down)")
    ap.add_argument("--tile", default=None,
                    help="explicit tiling G:items:slices[:loads] (outputs per group, first-tier "
                         "items, bin slices per row, spectra loads 1 non-temporal / 2 ordinary); "
                         "0 keeps a default")
    ap.add_argument("--hbm-honest-contexts", type=int, default=3,
                    help="contexts for the cache-defeating roofline leg (spectra 16-384 MB only; 0 = off)")
    ap.add_argument("--graph-blocks", type=int, default=64,
                    help="also time graph replay of runs of this many block launches "
                         "(rounded up to the work-list period); 0 skips it")
    ap.add_argument("--sweep", default=None,
                    help="comma list of block,length,outputs,feedback,nf3 or 'all': the paper's "
                         "sweeps, and n_f = 3B against 2B with feedback")
    ap.add_argument("--serve", action="store_true",
                    help="serving with continuous batching (16 slots x 64 out x 12 s, B=64)")
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-rate", type=float, default=8.0, help="arrivals per second")
    ap.add_argument("--serve-life", type=float, default=2.0, help="mean source lifetime, s")
    ap.add_argument("--serve-feedback-taps", type=int, default=8192,
                    help="feedback paths 64 -> 16 of this many taps in the serving run (0: none)")
    ap.add_argument("--serve-budget-frac", type=float, default=0.5,
                    help="admission budget: this fraction of deadline x probed bandwidth")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the per-output sharding across GPUs is described in DESIGN.md but not built.",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb, max(1, args.steps))
        return 0

    from paper_2509_04390_amd import rta, workloads

    if args.serve:
        print(json.dumps(serve_bench(args, torch, rta, workloads)))
        return 0
    if args.sweep:
        print(json.dumps(sweeps(args, torch, rta, workloads)))
        return 0

    wl = workloads.config(args.workload)
    if args.spectra is None:
        args.spectra = wl.dtype
    scheme = wl.scheme
    if args.scheme == "uniform":
        scheme = None
    elif args.scheme:
        scheme = [tuple(int(v) for v in t.split("x")) for t in args.scheme.split(",")]
    B, Q, L, fs = wl.block, wl.n_in, wl.n_out, float(wl.fs)
    nblk = args.warmup + args.steps
    log(f"workload {wl.name}: Q={Q} L={L} taps={wl.lengths} B={B} spectra={args.spectra}")
    filt = wl.filters()
    wl_steps = workloads.Workload(**{**wl.__dict__, "n_blocks": max(nblk, wl.n_blocks)})
    x = wl_steps.signal_array()

    tuning, tuned = None, None
    if args.tile:
        parts = [int(v) for v in args.tile.split(":")]
        g_, it_, sl_ = parts[:3]
        ld_ = parts[3] if len(parts) > 3 else 0
        tuning = rta.make_tuning(outputs_per_group=g_, tail_items=it_, bin_slices=sl_,
                                 spectra_loads=ld_)
    if args.autotune:
        t0 = time.perf_counter()
        hit = False
        if args.tune_cache:
            tuning, chosen, us, hit = rta.rta_autotune_cached(
                args.tune_cache, fs, B, scheme, Q, L, filt, spectra=args.spectra, blocks=64)
        else:
            tuning, chosen, us = rta.rta_autotune(fs, B, scheme, Q, L, filt,
                                                  spectra=args.spectra, blocks=64)
        scheme = None if len(chosen) == 1 else chosen
        tuned = {"scheme": chosen, "outputs_per_group": tuning.outputs_per_group,
                 "tail_items": tuning.tail_items, "bin_slices": tuning.bin_slices,
                 "us_per_block": us, "from_cache": hit, "seconds": time.perf_counter() - t0}
        log(f"autotune: {tuned}")
    t0 = time.perf_counter()
    cv = rta.Convolver(filt, B, fs=fs, spectra=args.spectra, scheme=scheme, tuning=tuning)
    info = cv.info()
    log(f"created in {time.perf_counter() - t0:.2f} s: grid={info['grid']} "
        f"rows/item={info['rows_per_item']} G={info['outputs_per_group']} "
        f"spectra {info['spectra_bytes'] / 1e6:.1f} MB")

    # device-resident blocks [n][Q][B] and outputs [n][L][B]
    xb = torch.from_numpy(x[:, :nblk * B].reshape(Q, nblk, B).transpose(1, 0, 2).copy()).cuda()
    yb = torch.empty((nblk, L, B), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        cv.process_device(xb[i], yb[i], stream)
    torch.cuda.synchronize()

    # per-kernel HIP events recorded by the library on the launch stream;
    # device pointers are taken up front so the loop is one C call per block
    pin = [xb[i].data_ptr() for i in range(nblk)]
    pout = [yb[i].data_ptr() for i in range(nblk)]
    sh = stream.cuda_stream
    launch = rta._lib.rta_process_device
    # spans must fit inside the timed steps, or none would complete
    every = max(1, min(args.timing_every, args.steps))
    rta.rta_timing_enable(cv.ctx, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        i = args.warmup + k
        if launch(cv.ctx, pin[i], pout[i], sh) != 0:
            raise RuntimeError("rta_process_device failed")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_timed, kern_ms = rta.rta_timing_read(cv.ctx)
    rta.rta_timing_enable(cv.ctx, False)
    ms_per_step = 1e3 * wall / args.steps
    if n_timed > 0:
        kern_us = 1e3 * kern_ms / n_timed
        timing_how = (f"HIP events on the launch stream around spans of {every} back-to-back "
                      f"blocks inside the timed region ({n_timed} blocks): per-block time "
                      "including the gaps between launches, an upper bound on the kernel's")
    else:  # no complete span (cannot happen with every <= steps; kept as a guard)
        kern_us = 1e3 * ms_per_step
        timing_how = "wall clock per step (no event span completed): an upper bound"
    audio_per_step = B / fs
    value = audio_per_step / (ms_per_step / 1e3)
    log(f"timed {args.steps} steps: {ms_per_step * 1e3:.1f} us/step; {kern_us:.1f} us per block "
        f"in event-timed spans of {every} ({n_timed} blocks)")
    graph = graph_leg(args, torch, cv, info, xb, yb, ms_per_step) if args.graph_blocks else None
    probes = read_probes(torch, rta, int(info["spectra_bytes"]), info["grid"], stream)

    # synchronous host-memory blocks: per-block latency including PCIe (after
    # a few untimed calls: the first use of the pinned buffers is slow)
    cv.reset()
    lat = []
    out = np.empty((L, B), np.float32)
    for i in range(16 if args.latency_blocks or args.paced_blocks else 0):
        rta.rta_process(cv.ctx, np.ascontiguousarray(x[:, i * B:(i + 1) * B]), out)
    cv.reset()
    with no_gc():
        for i in range(args.latency_blocks):
            blk = np.ascontiguousarray(x[:, (i % nblk) * B:(i % nblk + 1) * B])
            t = time.perf_counter()
            rta.rta_process(cv.ctx, blk, out)
            lat.append(time.perf_counter() - t)
    lat_us = np.array(lat) * 1e6
    deadline = rta.deadline_us(B, fs)
    paced = None
    if args.paced_blocks:
        plat = []
        period = B / fs
        cv.reset()  # also restarts the library's host-stage counters
        with no_gc():
            nxt = time.perf_counter()
            for i in range(args.paced_blocks):
                nxt += period
                blk = np.ascontiguousarray(x[:, (i % nblk) * B:(i % nblk + 1) * B])
                t = time.perf_counter()
                rta.rta_process(cv.ctx, blk, out)
                plat.append(time.perf_counter() - t)
                while time.perf_counter() < nxt:
                    pass
        plat_us = np.array(plat) * 1e6
        paced = {"blocks": args.paced_blocks,
                 "mode": "rta_process paced every B/fs, host memory, PCIe included",
                 "p50_us": float(np.percentile(plat_us, 50)),
                 "p99_us": float(np.percentile(plat_us, 99)), "max_us": float(plat_us.max()),
                 "max_at_block": int(np.argmax(plat_us)),
                 "xruns": int(np.sum(plat_us > deadline)),
                 "host_stages": host_stages(cv.info())}

    bytes_per_launch = (info["h_bytes_per_block"] + info["x_bytes_per_block"]
                        + info["io_bytes_per_block"])
    achieved = bytes_per_launch / (kern_us * 1e-6) / 1e9
    traffic = measured_traffic(wl.name, args.spectra)
    # arithmetic per block: 8 real flops per complex multiply-accumulate, and
    # (reported apart) about 2.5 N log2 N per real N-point FFT for the Q
    # forward and L inverse transforms of each tier (2 P_t points; later tiers
    # once per P_t / B blocks)
    fft_flops = 0.0
    for t, P_t in enumerate(info["tier_size"]):
        N_t = 2 * P_t  # (3B points with n_f = 3B, where P = 3B/2)
        per_block = 1.0 if t == 0 else B / P_t  # the first tier's frame is every block
        fft_flops += (Q + L) * per_block * 2.5 * N_t * np.log2(N_t)
    cmac_flops = 8.0 * info["cmacs_per_block"]
    flops = {"cmac_per_block": cmac_flops, "fft_per_block": fft_flops,
             "cmac_gflops": cmac_flops / (kern_us * 1e3),
             "flops_per_byte": cmac_flops / bytes_per_launch,
             "note": "8 flops per complex multiply-accumulate; FFTs at 2.5 N log2 N per real "
                     "N-point transform (Q forward, L inverse per tier and frame)"}
    honest = hbm_honest_leg(args, torch, rta, cv, info,
                            lambda: rta.Convolver(filt, B, fs=fs, spectra=args.spectra, scheme=scheme,
                                                  tuning=tuning),
                            xb, yb, bytes_per_launch)
    cpu = None
    if not args.no_cpu_baseline:
        # the workload's whole signal, whatever --steps is: the GPU streams it
        # once more from a reset context, the oracle processes it in one go
        x_full = wl.signal_array()
        nb_full = x_full.shape[1] // B
        cv.reset()
        xf = torch.from_numpy(x_full[:, :nb_full * B].reshape(Q, nb_full, B)
                              .transpose(1, 0, 2).copy()).cuda()
        yf = torch.empty((nb_full, L, B), dtype=torch.float32, device="cuda")
        for i in range(nb_full):
            cv.process_device(xf[i], yf[i], stream)
        torch.cuda.synchronize()
        y_gpu = yf.permute(1, 0, 2).reshape(L, nb_full * B).cpu().numpy()
        del xf, yf
        log(f"timing the oracle on the host cores over {nb_full} blocks ...")
        cpu = cpu_baseline(wl, filt, x_full[:, :nb_full * B], args.cpu_channels, y_gpu)
        log(f"cpu baseline: {cpu['value']:.2f} x real time on {cpu['cores']} threads "
            f"({cpu['host']['model']}, nproc {cpu['host']['nproc']}; one thread "
            f"{cpu['one_thread']['value']:.2f} x, {cpu['one_thread']['speedup_on_cores']:.1f}x "
            f"speedup); GPU error {cpu['gpu_error_db']['max']:.1f} dB max")

    n_h = wl.max_len()
    lens = [int(np.asarray(f).size) for row in filt for f in row]
    taps_total = float(sum(lens))
    tiers = ("uniform partitions" if scheme is None else
             "tiers " + "/".join(f"{s_}x{c_ or 'rest'}" for s_, c_ in scheme))
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "x real-time (audio s / wall s)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.spectra == "fp32" else f"f32 (spectra {args.spectra})",
        "data": "synthetic",
        "config": {
            "workload": (f"{wl.name}: {Q} in -> {L} out, up to {n_h}-tap ({n_h / fs:.1f} s) "
                         f"exp-decayed Gaussian filters, block {B}, fs {int(fs)} Hz, "
                         f"{args.spectra} spectra, {tiers}"),
            "block": B, "n_in": Q, "n_out": L, "taps": n_h, "spectra": args.spectra,
            "tiers": [[int(a_), int(b_)] for a_, b_ in zip(info["tier_size"], info["tier_count"])],
            "phases": info["n_phases"],
            "tiling": {"outputs_per_group": info["outputs_per_group"], "grid": info["grid"],
                       "rows_per_item": info["rows_per_item"],
                       "spectra_loads": "non-temporal" if info["spectra_nontemporal"] else "ordinary"},
        },
        "rtf": (ms_per_step / 1e3) / audio_per_step,
        "channel_filter_seconds_per_s": taps_total / fs * value,
        "flops": flops,
        "deadline_us": deadline,
        "latency": paced,
        "latency_back_to_back": None if not len(lat_us) else {
            "blocks": args.latency_blocks,
            "mode": "back-to-back rta_process, host memory, PCIe included",
            "p50_us": float(np.percentile(lat_us, 50)),
            "p99_us": float(np.percentile(lat_us, 99)),
            "max_us": float(lat_us.max()),
            "max_at_block": int(np.argmax(lat_us)),
            "over_1ms": int(np.sum(lat_us > 1000.0)),
            "xruns": int(np.sum(lat_us > deadline))},
        "roofline": {
            "kernel": "k_block",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": bytes_per_launch,
            "kernel_us_mean": kern_us,
            "kernel_us_timing": timing_how,
        },
        "roofline_hbm_honest": honest,
        "read_probe": probes,
        "graph": graph,
        "autotune": tuned,
        "cpu_baseline": cpu,
    }
    cv.close()
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
