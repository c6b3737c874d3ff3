"""Seeded synthetic workloads: reverberant FIR filters and input signals.

This module only draws random numbers and shapes arrays; it holds none of the
convolution arithmetic.  Tests, the benchmark and the oracle harness all take
their inputs from here, so the GPU library and the FP64 oracle see the very
same float32 arrays.

Filter model (the paper draws i.i.d. standard-normal filters, Sec. VI; here an
exponential decay is added so the filters look like room responses):

    h[n] = g[n] * exp(-6.91 * n / (RT60 * fs)),  g ~ N(0, 1),
    then h[d] += 1 with d ~ U{0, ..., delta_max-1}      (direct-sound tap)

6.91 = ln(1000): the envelope has fallen by 60 dB after RT60 seconds.
Draw order per generator: for each (q, l) in row-major [in][out] order the
RT60, then d, then the n_h Gaussian samples; inputs come from their own seed.
Everything is cast to float32 once.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

FS = 48000


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def reverb_filters(seed: int, n_in: int, n_out: int, lengths, rt60=(6.0, 10.0),
                   fs: int = FS, delta_max: int = 480) -> List[List[np.ndarray]]:
    """Q x L nested list of float32 filters.

    ``lengths`` is an int (all pairs), a length-Q sequence (per input) or a
    Q x L nested sequence; a length of 0 gives an empty filter (no path).
    ``rt60`` is a float (fixed) or a (lo, hi) uniform range drawn per pair.
    """
    rng = _rng(seed)
    filters: List[List[np.ndarray]] = []
    for q in range(n_in):
        row = []
        for l in range(n_out):
            if np.isscalar(lengths):
                n_h = int(lengths)
            elif np.isscalar(lengths[q]):
                n_h = int(lengths[q])
            else:
                n_h = int(lengths[q][l])
            r = float(rt60) if np.isscalar(rt60) else float(rng.uniform(rt60[0], rt60[1]))
            d = int(rng.integers(0, delta_max))
            g = rng.standard_normal(n_h)
            h = g * np.exp(-6.91 * np.arange(n_h) / (r * fs))
            if n_h > d:
                h[d] += 1.0
            row.append(h.astype(np.float32))
        filters.append(row)
    return filters


def white_noise(seed: int, n_in: int, n_samples: int, sigma: float = 0.1) -> np.ndarray:
    """[n_in][n_samples] float32 white Gaussian noise."""
    return (sigma * _rng(seed).standard_normal((n_in, n_samples))).astype(np.float32)


def log_sweep(n_in: int, n_samples: int, fs: int = FS, f0: float = 20.0,
              f1: float = 20000.0, amp: float = 0.1 * np.sqrt(2.0)) -> np.ndarray:
    """Exponential sine sweep f0 -> f1 over the whole signal, on every input."""
    t = np.arange(n_samples) / fs
    T = n_samples / fs
    k = np.log(f1 / f0)
    phase = 2 * np.pi * f0 * T / k * (np.exp(t * k / T) - 1.0)
    s = (amp * np.sin(phase)).astype(np.float32)
    return np.repeat(s[None, :], n_in, axis=0)


def uniform_lengths(seed: int, n_in: int, lo_s: float, hi_s: float, fs: int = FS) -> List[int]:
    """Per-source filter lengths round(U[lo, hi] * fs)."""
    rng = _rng(seed)
    return [int(round(rng.uniform(lo_s, hi_s) * fs)) for _ in range(n_in)]


@dataclass
class Workload:
    """A named, seeded problem: filters, input signal and block geometry."""
    name: str
    n_in: int
    n_out: int
    block: int
    lengths: object
    rt60: object
    n_blocks: int
    seed: int
    scheme: Optional[Sequence[Sequence[int]]] = None   # [(size, count), ...]
    dtype: str = "fp32"
    signal: str = "noise"
    fs: int = FS
    extra: dict = field(default_factory=dict)

    def filters(self):
        return reverb_filters(self.seed, self.n_in, self.n_out, self.lengths, self.rt60, self.fs)

    def max_len(self) -> int:
        if np.isscalar(self.lengths):
            return int(self.lengths)
        return int(max(np.max(np.asarray(x)) for x in self.lengths))

    def signal_array(self, flush: bool = False) -> np.ndarray:
        """Input [n_in][n_blocks*block]; with ``flush`` zero blocks are appended
        until the whole filter tail has been emitted."""
        n = self.n_blocks * self.block
        if self.signal == "sweep":
            x = log_sweep(self.n_in, n, self.fs)
        else:
            x = white_noise(self.seed + 1000, self.n_in, n)
        if flush:
            extra = -(-(self.max_len() - 1) // self.block) * self.block
            x = np.concatenate([x, np.zeros((self.n_in, extra), np.float32)], axis=1)
        return x


def config(name: str) -> Workload:
    """The workloads the method is measured on.

    small:  1 -> 1, 65,536 taps, RT60 2 s, block 256 (FFT 512), 100 blocks.
    main:   1 -> 32, 480,000 taps (10 s), RT60 U[6,10] s, block 128, 2,000 blocks.
    nupc:   4 sources -> 64 outputs, U[3,12] s per source, tiers 128/1024/8192.
    serve:  16 inputs -> 64 outputs, 12 s filters, block 64.
    target: 1 -> 64, 12 s filters, block 128.
    """
    if name == "small":
        return Workload("small", 1, 1, 256, 65536, 2.0, 100, seed=1)
    if name == "main":
        return Workload("main", 1, 32, 128, 480000, (6.0, 10.0), 2000, seed=2)
    if name == "nupc":
        lens = uniform_lengths(4, 4, 3.0, 12.0)
        return Workload("nupc", 4, 64, 128, lens, (6.0, 10.0), 2000, seed=4,
                        scheme=((128, 15), (1024, 14), (8192, 0)), dtype="fp16")
    if name == "serve":
        return Workload("serve", 16, 64, 64, 576000, (6.0, 10.0), 0, seed=5, dtype="fp16")
    if name == "target":
        return Workload("target", 1, 64, 128, 576000, (6.0, 10.0), 2000, seed=6)
    raise KeyError(name)
