"""ctypes binding of librta (include/rta.h): argument marshalling only.

Every entry point keeps the C name.  All computation happens in the HIP
library; importing this module fails loudly when librta.so has not been built,
and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

# PyTorch-ROCm ships its own HIP runtime.  If librta.so were loaded first,
# a later `import torch` would bring a second HIP runtime into the process and
# the library's device calls would fail; importing torch first (when it is
# installed) makes librta.so bind to torch's runtime, so the process has one.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librta.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it first "
                      "(python -c 'import __graft_entry__ as g; g.build()')")
_lib = ctypes.CDLL(_LIB_PATH)

RTA_OK = 0
RTA_E_ARG = -1
RTA_E_NOMEM = -2
RTA_E_RANGE = -3
RTA_E_DEVICE = -4
RTA_E_STATE = -5
RTA_E_UNSUPPORTED = -6
RTA_E_CAPACITY = -7

RTA_SLOT_FREE, RTA_SLOT_JOINING, RTA_SLOT_LIVE, RTA_SLOT_LEAVING, RTA_SLOT_DRAINING = range(5)
SLOT_STATES = ("free", "joining", "live", "leaving", "draining")

RTA_FP32, RTA_FP16, RTA_BF16 = 0, 1, 2
DTYPES = {"fp32": RTA_FP32, "fp16": RTA_FP16, "bf16": RTA_BF16}

RTA_FLAG_SPIKE = 0x1
RTA_FLAG_NF3 = 0x2
RTA_MAX_TIERS = 8

EXPORTED = ("rta_create", "rta_process", "rta_process_device", "rta_reset",
            "rta_query", "rta_timing_enable", "rta_timing_read", "rta_probe_read",
            "rta_destroy", "rta_strerror", "rta_create_tuned", "rta_autotune",
            "rta_set_feedback", "rta_test_feedback_wait", "rta_serve_create", "rta_serve_admit",
            "rta_serve_admit_noalloc", "rta_serve_release", "rta_serve_query",
            "rta_graph_create", "rta_graph_launch", "rta_graph_destroy", "rta_autotune_cached")


class rta_scheme(ctypes.Structure):
    _fields_ = [("n_tiers", ctypes.c_int32),
                ("size", ctypes.POINTER(ctypes.c_int32)),
                ("count", ctypes.POINTER(ctypes.c_int32))]


class rta_info(ctypes.Structure):
    _fields_ = [("fs", ctypes.c_double),
                ("deadline_us", ctypes.c_double),
                ("block", ctypes.c_int32), ("n_in", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("n_tiers", ctypes.c_int32),
                ("spectra_dtype", ctypes.c_int32), ("n_phases", ctypes.c_int32),
                ("tier_size", ctypes.c_int32 * RTA_MAX_TIERS),
                ("tier_count", ctypes.c_int32 * RTA_MAX_TIERS),
                ("tier_offset", ctypes.c_int64 * RTA_MAX_TIERS),
                ("blocks_done", ctypes.c_int64),
                ("spectra_bytes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64),
                ("h_bytes_per_block", ctypes.c_double),
                ("x_bytes_per_block", ctypes.c_double),
                ("io_bytes_per_block", ctypes.c_double),
                ("cmacs_per_block", ctypes.c_double),
                ("tail_bytes_per_block", ctypes.c_double),
                ("grid", ctypes.c_int32),
                ("outputs_per_group", ctypes.c_int32),
                ("rows_per_item", ctypes.c_int32),
                ("poisoned", ctypes.c_int32),
                ("feedback_paths", ctypes.c_int32),
                ("feedback_fused", ctypes.c_int32),
                ("spectra_nontemporal", ctypes.c_int32),
                ("fft_size", ctypes.c_int32),
                ("host_calls", ctypes.c_int64),
                ("host_max_us", ctypes.c_double * 4),
                ("host_sum_us", ctypes.c_double * 4),
                ("host_slowest_call", ctypes.c_int64),
                ("host_slowest_us", ctypes.c_double),
                ("host_late_waits", ctypes.c_int64),
                ("bin_slices", ctypes.c_int32),
                ("max_group_slots", ctypes.c_int32)]


class rta_tuning(ctypes.Structure):
    _fields_ = [("outputs_per_group", ctypes.c_int32),
                ("tail_items", ctypes.c_int32),
                ("tail_rows", ctypes.c_int32),
                ("tier_rows", ctypes.c_int32),
                ("bin_slices", ctypes.c_int32),
                ("n_tiers", ctypes.c_int32),
                ("size", ctypes.c_int32 * RTA_MAX_TIERS),
                ("count", ctypes.c_int32 * RTA_MAX_TIERS),
                ("spectra_loads", ctypes.c_int32)]


class rta_serve_config(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("max_taps", ctypes.c_int64), ("arena_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_double)]


class rta_slot_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("start_block", ctypes.c_int64), ("stop_block", ctypes.c_int64),
                ("free_block", ctypes.c_int64), ("taps", ctypes.c_int64),
                ("bytes_per_block", ctypes.c_double)]


class rta_serve_info(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("live", ctypes.c_int32),
                ("draining", ctypes.c_int32), ("free_slots", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("arena_used_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_double), ("bytes_per_block", ctypes.c_double),
                ("admitted", ctypes.c_int64), ("rejected_slots", ctypes.c_int64),
                ("rejected_memory", ctypes.c_int64), ("rejected_budget", ctypes.c_int64),
                ("plan_swaps", ctypes.c_int64)]


_fp = ctypes.POINTER(ctypes.c_float)
_lib.rta_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, ctypes.c_int32,
                            ctypes.POINTER(rta_scheme), ctypes.c_int32, ctypes.c_int32,
                            ctypes.POINTER(_fp), ctypes.POINTER(ctypes.c_int64),
                            ctypes.c_int32, ctypes.c_uint32]
_lib.rta_create_tuned.argtypes = _lib.rta_create.argtypes + [ctypes.POINTER(rta_tuning)]
_lib.rta_autotune.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.POINTER(rta_scheme),
                              ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_fp),
                              ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, ctypes.c_uint32,
                              ctypes.c_int32, ctypes.POINTER(rta_tuning),
                              ctypes.POINTER(ctypes.c_double)]
_lib.rta_autotune_cached.argtypes = [ctypes.c_char_p] + _lib.rta_autotune.argtypes + [
    ctypes.POINTER(ctypes.c_int32)]
_lib.rta_process.argtypes = [ctypes.c_void_p, _fp, _fp]
_lib.rta_set_feedback.argtypes = [ctypes.c_void_p, ctypes.POINTER(_fp),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
_lib.rta_test_feedback_wait.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
_lib.rta_process_device.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
_lib.rta_graph_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_void_p)]
_lib.rta_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.rta_graph_destroy.argtypes = [ctypes.c_void_p]
_lib.rta_reset.argtypes = [ctypes.c_void_p]
_lib.rta_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(rta_info)]
_lib.rta_destroy.argtypes = [ctypes.c_void_p]
_lib.rta_timing_enable.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.rta_probe_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p]
_lib.rta_timing_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_double)]
_lib.rta_serve_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_double,
                                  ctypes.c_int32, ctypes.POINTER(rta_scheme),
                                  ctypes.POINTER(rta_serve_config), ctypes.c_int32,
                                  ctypes.c_uint32, ctypes.POINTER(rta_tuning)]
_lib.rta_serve_admit.argtypes = [ctypes.c_void_p, ctypes.POINTER(_fp),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
_lib.rta_serve_admit_noalloc.argtypes = _lib.rta_serve_admit.argtypes
_lib.rta_serve_release.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.rta_serve_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(rta_serve_info),
                                 ctypes.POINTER(rta_slot_info)]
_lib.rta_strerror.argtypes = [ctypes.c_int]
_lib.rta_strerror.restype = ctypes.c_char_p
for _f in ("rta_create", "rta_process", "rta_process_device", "rta_reset", "rta_query",
           "rta_timing_enable", "rta_timing_read", "rta_probe_read", "rta_destroy",
           "rta_create_tuned", "rta_autotune", "rta_set_feedback", "rta_test_feedback_wait",
           "rta_serve_create", "rta_serve_admit", "rta_serve_admit_noalloc", "rta_serve_release",
           "rta_serve_query"):
    getattr(_lib, _f).restype = ctypes.c_int


class RtaError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {rta_strerror(status)} ({status})")


def _check(status: int, where: str) -> None:
    if status != RTA_OK:
        raise RtaError(status, where)


def library_path() -> str:
    return _LIB_PATH


def deadline_us(block: int, fs: float) -> float:
    """Buffer latency B/fs in microseconds, the per-block budget (Sec. I)."""
    return 1e6 * block / fs


# ----------------------------------------------------------------------------
# C entry points under their own names
# ----------------------------------------------------------------------------

def rta_strerror(status: int) -> str:
    return _lib.rta_strerror(int(status)).decode()


def _marshal(filters, n_in, n_out, lengths, scheme):
    flat = _flatten(filters, n_in, n_out)
    keep = [np.ascontiguousarray(f, dtype=np.float32) if f is not None and len(f) else None
            for f in flat]
    ptrs = (_fp * len(keep))()
    lens = (ctypes.c_int64 * len(keep))()
    for i, f in enumerate(keep):
        ptrs[i] = f.ctypes.data_as(_fp) if f is not None else None
        lens[i] = 0 if f is None else f.size
    if lengths is not None:
        for i, n in enumerate(lengths):
            lens[i] = int(n)
    sch = None
    if scheme is not None:
        sizes = (ctypes.c_int32 * len(scheme))(*[int(s) for s, _ in scheme])
        counts = (ctypes.c_int32 * len(scheme))(*[int(c) for _, c in scheme])
        sch = rta_scheme(len(scheme), sizes, counts)
        sch._keep = (sizes, counts)
    return keep, ptrs, lens, sch


def make_tuning(outputs_per_group=0, tail_items=0, tail_rows=0, tier_rows=0,
                bin_slices=0, spectra_loads=0) -> rta_tuning:
    t = rta_tuning()
    t.outputs_per_group, t.tail_items = outputs_per_group, tail_items
    t.tail_rows, t.tier_rows, t.bin_slices = tail_rows, tier_rows, bin_slices
    t.spectra_loads = spectra_loads
    return t


def rta_create_tuned(fs: float, block: int, scheme, n_in: int, n_out: int, filters,
                     lengths=None, spectra="fp32", flags: int = 0, tuning=None):
    """filters: Q x L nested list of 1-D float32 arrays (None/empty = no path),
    or a flat length-Q*L list in [in][out] order.  scheme: None (UPOLS) or a
    sequence of (size, count) tiers.  tuning: rta_tuning or None.  Returns the
    opaque context handle."""
    keep, ptrs, lens, sch = _marshal(filters, n_in, n_out, lengths, scheme)
    dtype = DTYPES[spectra] if isinstance(spectra, str) else int(spectra)
    ctx = ctypes.c_void_p()
    st = _lib.rta_create_tuned(ctypes.byref(ctx), float(fs), int(block),
                               ctypes.byref(sch) if sch is not None else None,
                               int(n_in), int(n_out), ptrs, lens, dtype, int(flags),
                               ctypes.byref(tuning) if tuning is not None else None)
    _check(st, "rta_create_tuned")
    return ctx


def rta_create(fs: float, block: int, scheme, n_in: int, n_out: int, filters,
               lengths=None, spectra="fp32", flags: int = 0):
    """As rta_create_tuned with default tiling."""
    keep, ptrs, lens, sch = _marshal(filters, n_in, n_out, lengths, scheme)
    dtype = DTYPES[spectra] if isinstance(spectra, str) else int(spectra)
    ctx = ctypes.c_void_p()
    st = _lib.rta_create(ctypes.byref(ctx), float(fs), int(block),
                         ctypes.byref(sch) if sch is not None else None,
                         int(n_in), int(n_out), ptrs, lens, dtype, int(flags))
    _check(st, "rta_create")
    return ctx


def rta_autotune(fs: float, block: int, scheme, n_in: int, n_out: int, filters,
                 lengths=None, spectra="fp32", flags: int = 0, blocks: int = 64):
    """Returns (tuning, scheme [(size, count), ...], mean block time in us)."""
    keep, ptrs, lens, sch = _marshal(filters, n_in, n_out, lengths, scheme)
    dtype = DTYPES[spectra] if isinstance(spectra, str) else int(spectra)
    best = rta_tuning()
    us = ctypes.c_double()
    st = _lib.rta_autotune(float(fs), int(block), ctypes.byref(sch) if sch is not None else None,
                           int(n_in), int(n_out), ptrs, lens, dtype, int(flags), int(blocks),
                           ctypes.byref(best), ctypes.byref(us))
    _check(st, "rta_autotune")
    chosen = [(best.size[t], best.count[t]) for t in range(best.n_tiers)]
    return best, chosen, us.value


def rta_autotune_cached(cache_path: str, fs: float, block: int, scheme, n_in: int, n_out: int,
                        filters, lengths=None, spectra="fp32", flags: int = 0, blocks: int = 64):
    """rta_autotune behind a JSON-lines cache file.  Returns (tuning, scheme,
    mean block time in us, from_cache)."""
    keep, ptrs, lens, sch = _marshal(filters, n_in, n_out, lengths, scheme)
    dtype = DTYPES[spectra] if isinstance(spectra, str) else int(spectra)
    best = rta_tuning()
    us = ctypes.c_double()
    hit = ctypes.c_int32()
    st = _lib.rta_autotune_cached(os.fsencode(cache_path), float(fs), int(block),
                                  ctypes.byref(sch) if sch is not None else None,
                                  int(n_in), int(n_out), ptrs, lens, dtype, int(flags), int(blocks),
                                  ctypes.byref(best), ctypes.byref(us), ctypes.byref(hit))
    _check(st, "rta_autotune_cached")
    chosen = [(best.size[t], best.count[t]) for t in range(best.n_tiers)]
    return best, chosen, us.value, bool(hit.value)


def rta_process(ctx, inp: np.ndarray, out: np.ndarray) -> None:
    """inp: [n_in][block] float32 (C-contiguous); out: [n_out][block] float32."""
    assert inp.dtype == np.float32 and inp.flags.c_contiguous
    assert out.dtype == np.float32 and out.flags.c_contiguous
    _check(_lib.rta_process(ctx, inp.ctypes.data_as(_fp), out.ctypes.data_as(_fp)),
           "rta_process")


def rta_process_device(ctx, d_in: int, d_out: int, stream: int = 0) -> None:
    """Device pointers (ints, e.g. torch data_ptr()) and a hipStream_t handle."""
    _check(_lib.rta_process_device(ctx, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out),
                                   ctypes.c_void_p(stream or None)), "rta_process_device")


def rta_graph_create(ctx, d_in: int, d_out: int, n_blocks: int):
    """Device pointers of [n_blocks][n_in][block] and [n_blocks][n_out][block] FP32."""
    g = ctypes.c_void_p()
    _check(_lib.rta_graph_create(ctx, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out),
                                 int(n_blocks), ctypes.byref(g)), "rta_graph_create")
    return g


def rta_graph_launch(graph, stream: int = 0) -> None:
    _check(_lib.rta_graph_launch(graph, ctypes.c_void_p(stream or None)), "rta_graph_launch")


def rta_graph_destroy(graph) -> None:
    _check(_lib.rta_graph_destroy(graph), "rta_graph_destroy")


def rta_set_feedback(ctx, n_in: int, n_out: int, feedback, spectra="fp32") -> None:
    """feedback: n_in x n_out nested list of FP32 taps f_ql (output l to input
    q), None/empty = no path; feedback=None removes the paths."""
    if feedback is None:
        _check(_lib.rta_set_feedback(ctx, None, None, 0), "rta_set_feedback")
        return
    keep, ptrs, lens, _ = _marshal(feedback, n_in, n_out, None, None)
    dtype = DTYPES[spectra] if isinstance(spectra, str) else int(spectra)
    _check(_lib.rta_set_feedback(ctx, ptrs, lens, dtype), "rta_set_feedback")


def rta_test_feedback_wait(ctx, max_polls: int, never_ready: bool) -> None:
    """Bound the fused feedback wait (test aid for its failure path)."""
    _check(_lib.rta_test_feedback_wait(ctx, int(max_polls), 1 if never_ready else 0),
           "rta_test_feedback_wait")


def rta_reset(ctx) -> None:
    _check(_lib.rta_reset(ctx), "rta_reset")


def rta_query(ctx) -> dict:
    info = rta_info()
    _check(_lib.rta_query(ctx, ctypes.byref(info)), "rta_query")
    d = {}
    for name, _ in rta_info._fields_:
        v = getattr(info, name)
        if hasattr(v, "__len__"):
            v = list(v)[:info.n_tiers] if name.startswith("tier_") else list(v)
        d[name] = v
    return d


def rta_timing_enable(ctx, every) -> None:
    """every: record kernel events on every `every`-th block (True = 1,
    False/0 = off)."""
    _check(_lib.rta_timing_enable(ctx, int(every)), "rta_timing_enable")


def rta_timing_read(ctx):
    """(blocks, kernel_ms_total) since the last read."""
    n = ctypes.c_int64()
    a = ctypes.c_double()
    _check(_lib.rta_timing_read(ctx, ctypes.byref(n), ctypes.byref(a)), "rta_timing_read")
    return n.value, a.value


def rta_probe_read(d_buf: int, nbytes: int, grid: int, d_sink: int, stream: int = 0) -> None:
    """Launch the streaming-read probe (device pointers as ints)."""
    _check(_lib.rta_probe_read(ctypes.c_void_p(d_buf), int(nbytes), int(grid),
                               ctypes.c_void_p(d_sink), ctypes.c_void_p(stream or None)),
           "rta_probe_read")


def rta_serve_create(fs: float, block: int, scheme, n_slots: int, n_out: int, max_taps: int,
                     arena_bytes: int = 0, budget_bytes: float = 0.0, spectra="fp32",
                     flags: int = 0, tuning=None):
    """Serving context with n_slots source slots and n_out outputs."""
    _, _, _, sch = _marshal([None] * 1, 1, 1, None, scheme)
    cfg = rta_serve_config(int(n_slots), int(n_out), int(max_taps), int(arena_bytes),
                           float(budget_bytes))
    dtype = DTYPES[spectra] if isinstance(spectra, str) else int(spectra)
    ctx = ctypes.c_void_p()
    st = _lib.rta_serve_create(ctypes.byref(ctx), float(fs), int(block),
                               ctypes.byref(sch) if sch is not None else None,
                               ctypes.byref(cfg), dtype, int(flags),
                               ctypes.byref(tuning) if tuning is not None else None)
    _check(st, "rta_serve_create")
    return ctx


def rta_serve_admit(ctx, filters) -> int:
    """filters: n_out 1-D float32 arrays (None/empty = no path).  Returns the
    slot; raises RtaError (status RTA_E_CAPACITY / RTA_E_NOMEM) on refusal."""
    keep, ptrs, lens, _ = _marshal(list(filters), 1, len(filters), None, None)
    slot = ctypes.c_int32(-1)
    _check(_lib.rta_serve_admit(ctx, ptrs, lens, ctypes.byref(slot)), "rta_serve_admit")
    return slot.value


def rta_serve_admit_noalloc(ctx, filters) -> int:
    """rta_serve_admit without any device allocation (filters <= 2^20 taps)."""
    keep, ptrs, lens, _ = _marshal(list(filters), 1, len(filters), None, None)
    slot = ctypes.c_int32(-1)
    _check(_lib.rta_serve_admit_noalloc(ctx, ptrs, lens, ctypes.byref(slot)),
           "rta_serve_admit_noalloc")
    return slot.value


def rta_serve_release(ctx, slot: int) -> None:
    _check(_lib.rta_serve_release(ctx, int(slot)), "rta_serve_release")


def rta_serve_query(ctx, n_slots: Optional[int] = None):
    """(info dict, list of per-slot dicts or None)."""
    info = rta_serve_info()
    slots = (rta_slot_info * n_slots)() if n_slots else None
    _check(_lib.rta_serve_query(ctx, ctypes.byref(info), slots), "rta_serve_query")
    d = {name: getattr(info, name) for name, _ in rta_serve_info._fields_}
    per = None
    if slots is not None:
        per = []
        for sl in slots:
            e = {name: getattr(sl, name) for name, _ in rta_slot_info._fields_ if name != "pad"}
            e["state"] = SLOT_STATES[sl.state]
            per.append(e)
    return d, per


def rta_destroy(ctx) -> None:
    _check(_lib.rta_destroy(ctx), "rta_destroy")


def _flatten(filters, n_in: int, n_out: int) -> List:
    """Q x L nested lists -> flat [in][out] list; a flat list passes through."""
    if len(filters) == n_in and all(isinstance(r, (list, tuple)) for r in filters):
        flat = [f for row in filters for f in row]
    else:
        flat = list(filters)
    if len(flat) != n_in * n_out:
        raise ValueError(f"expected {n_in}x{n_out} filters, got {len(flat)}")
    return flat


# ----------------------------------------------------------------------------
# Convenience wrapper
# ----------------------------------------------------------------------------

class Convolver:
    """One context: ``process`` (host block), ``process_device`` (torch
    tensors on the current stream) and ``run`` (whole host signal)."""

    def __init__(self, filters, block: int, fs: float = 48000.0, scheme=None,
                 spectra="fp32", flags: int = 0, tuning=None):
        self.n_in = len(filters)
        self.n_out = len(filters[0])
        self.block = block
        self.ctx = None
        self.ctx = rta_create_tuned(fs, block, scheme, self.n_in, self.n_out, filters,
                                    spectra=spectra, flags=flags, tuning=tuning)

    def close(self):
        if self.ctx is not None:
            rta_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        return rta_query(self.ctx)

    def reset(self):
        rta_reset(self.ctx)

    def set_feedback(self, feedback, spectra="fp32"):
        """Estimated feedback paths f_ql (output l -> input q), Q x L nested."""
        rta_set_feedback(self.ctx, self.n_in, self.n_out, feedback, spectra)

    def process(self, block_in: np.ndarray) -> np.ndarray:
        out = np.empty((self.n_out, self.block), np.float32)
        rta_process(self.ctx, np.ascontiguousarray(block_in, dtype=np.float32), out)
        return out

    def process_device(self, d_in, d_out, stream=None) -> None:
        """d_in/d_out: contiguous float32 torch CUDA tensors."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        assert d_in.is_contiguous() and d_out.is_contiguous()
        assert d_in.dtype == torch.float32 and d_out.dtype == torch.float32
        assert d_in.numel() == self.n_in * self.block and d_out.numel() == self.n_out * self.block
        rta_process_device(self.ctx, d_in.data_ptr(), d_out.data_ptr(), stream.cuda_stream)

    def graph(self, d_in, d_out, n_blocks: int) -> "Graph":
        """Capture n_blocks block launches over device tensors (rta_graph_create)."""
        return Graph(self, d_in, d_out, n_blocks)

    def run(self, x: np.ndarray) -> np.ndarray:
        """Stream a whole host signal [n_in][n*block] through rta_process."""
        x = np.asarray(x, np.float32)
        nb = x.shape[1] // self.block
        y = np.empty((self.n_out, nb * self.block), np.float32)
        for b in range(nb):
            y[:, b * self.block:(b + 1) * self.block] = self.process(
                x[:, b * self.block:(b + 1) * self.block])
        return y

    def run_device(self, x: np.ndarray):
        """Stream a whole signal with device-resident blocks (torch tensors);
        returns the host output."""
        import torch
        x = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
        nb = x.shape[1] // self.block
        xb = x[:, :nb * self.block].reshape(self.n_in, nb, self.block).permute(1, 0, 2).contiguous()
        yb = torch.empty((nb, self.n_out, self.block), dtype=torch.float32, device="cuda")
        for b in range(nb):
            self.process_device(xb[b], yb[b])
        torch.cuda.synchronize()
        return yb.permute(1, 0, 2).reshape(self.n_out, nb * self.block).cpu().numpy()


class Graph:
    """A captured run of n_blocks block launches (rta_graph_create) over
    device tensors d_in [n_blocks][n_in][block] and d_out [n_blocks][n_out][block]."""

    def __init__(self, conv: "Convolver", d_in, d_out, n_blocks: int):
        import torch
        assert d_in.is_contiguous() and d_out.is_contiguous()
        assert d_in.dtype == torch.float32 and d_out.dtype == torch.float32
        assert d_in.numel() == n_blocks * conv.n_in * conv.block
        assert d_out.numel() == n_blocks * conv.n_out * conv.block
        self.conv, self.d_in, self.d_out, self.n_blocks = conv, d_in, d_out, n_blocks
        self.graph = rta_graph_create(conv.ctx, d_in.data_ptr(), d_out.data_ptr(), n_blocks)

    def launch(self, stream=None) -> None:
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        rta_graph_launch(self.graph, stream.cuda_stream)

    def close(self):
        if self.graph:
            rta_graph_destroy(self.graph)
            self.graph = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """A serving context: sources are admitted into slots and released while
    blocks stream; ``process`` takes [n_slots][block] input."""

    def __init__(self, n_slots: int, n_out: int, max_taps: int, block: int,
                 fs: float = 48000.0, scheme=None, spectra="fp32", flags: int = 0,
                 arena_bytes: int = 0, budget_bytes: float = 0.0, tuning=None):
        self.n_slots, self.n_out, self.block = n_slots, n_out, block
        self.ctx = None
        self.ctx = rta_serve_create(fs, block, scheme, n_slots, n_out, max_taps, arena_bytes,
                                    budget_bytes, spectra, flags, tuning)

    def close(self):
        if self.ctx is not None:
            rta_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, filters) -> int:
        return rta_serve_admit(self.ctx, filters)

    def admit_noalloc(self, filters) -> int:
        return rta_serve_admit_noalloc(self.ctx, filters)

    def set_feedback(self, feedback, spectra="fp32"):
        """Feedback paths f_ql from loudspeaker l to slot (microphone) q,
        n_slots x n_out nested; they stay with the slots."""
        rta_set_feedback(self.ctx, self.n_slots, self.n_out, feedback, spectra)

    def release(self, slot: int) -> None:
        rta_serve_release(self.ctx, slot)

    def query(self):
        return rta_serve_query(self.ctx, self.n_slots)

    def info(self) -> dict:
        return rta_query(self.ctx)

    def reset(self):
        rta_reset(self.ctx)

    def process(self, block_in: np.ndarray) -> np.ndarray:
        out = np.empty((self.n_out, self.block), np.float32)
        rta_process(self.ctx, np.ascontiguousarray(block_in, dtype=np.float32), out)
        return out
