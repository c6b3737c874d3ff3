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
                the host cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
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


def cpu_baseline(wl, filt, x, max_channels: int):
    """Time the oracle's FFT overlap-save over the first `max_channels`
    outputs of the whole signal; scale to the full job."""
    import oracle
    L = wl.n_out
    nch = min(L, max_channels)
    sub = [row[:nch] for row in filt]
    oracle.fftols(x[:, :wl.block * 8], [[f[:wl.block] for f in row] for row in sub], wl.block * 8)
    t0 = time.perf_counter()
    oracle.fftols(x, sub, x.shape[1])
    dt = time.perf_counter() - t0
    audio_s = x.shape[1] / wl.fs
    full_s = dt * L / nch
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": audio_s / full_s,
        "unit": "x real-time (audio s / wall s)",
        "cores": min(threads, nch),
        "kind": "oracle",
        "sample": (f"FP64 single-partition FFT overlap-save over all {x.shape[1]} samples "
                   f"({audio_s:.2f} s) of {nch} of {L} outputs in {dt:.2f} s, scaled to {L} "
                   "outputs; offline (one FFT per filter), no per-block latency"),
    }


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


def main() -> int:
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
    args = ap.parse_args()

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
    if args.autotune:
        t0 = time.perf_counter()
        tuning, chosen, us = rta.rta_autotune(fs, B, scheme, Q, L, filt, spectra=args.spectra,
                                              blocks=64)
        scheme = None if len(chosen) == 1 else chosen
        tuned = {"scheme": chosen, "outputs_per_group": tuning.outputs_per_group,
                 "tail_items": tuning.tail_items, "us_per_block": us,
                 "seconds": time.perf_counter() - t0}
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
    rta.rta_timing_enable(cv.ctx, True)
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
    kern_us = 1e3 * kern_ms / max(1, n_timed)
    ms_per_step = 1e3 * wall / args.steps
    audio_per_step = B / fs
    value = audio_per_step / (ms_per_step / 1e3)
    log(f"timed {args.steps} steps: {ms_per_step * 1e3:.1f} us/step; k_block {kern_us:.1f} us "
        f"(mean of {n_timed})")
    probes = read_probes(torch, rta, int(info["spectra_bytes"]), info["grid"], stream)

    # synchronous host-memory blocks: per-block latency including PCIe (after
    # a few untimed calls: the first use of the pinned buffers is slow)
    cv.reset()
    lat = []
    out = np.empty((L, B), np.float32)
    for i in range(16):
        rta.rta_process(cv.ctx, np.ascontiguousarray(x[:, i * B:(i + 1) * B]), out)
    cv.reset()
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
                 "xruns": int(np.sum(plat_us > deadline))}

    bytes_per_launch = (info["h_bytes_per_block"] + info["x_bytes_per_block"]
                        + info["io_bytes_per_block"])
    achieved = bytes_per_launch / (kern_us * 1e-6) / 1e9
    traffic = measured_traffic(wl.name, args.spectra)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores ...")
        cpu = cpu_baseline(wl, filt, x[:, :wl.n_blocks * B], args.cpu_channels)

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
        },
        "rtf": (ms_per_step / 1e3) / audio_per_step,
        "channel_filter_seconds_per_s": taps_total / fs * value,
        "deadline_us": deadline,
        "latency": paced,
        "latency_back_to_back": {"blocks": args.latency_blocks,
                                 "mode": "back-to-back rta_process, host memory, PCIe included",
                                 "p50_us": float(np.percentile(lat_us, 50)),
                                 "p99_us": float(np.percentile(lat_us, 99)),
                                 "max_us": float(lat_us.max()),
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
        },
        "read_probe": probes,
        "autotune": tuned,
        "cpu_baseline": cpu,
    }
    cv.close()
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
