"""FP64 CPU oracle for multichannel FIR convolution -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

It computes the plain definition of what the partitioned convolution must
produce (paper Sec. III-A Eq. 1-2: l_l = sum_q h_ql * m_q; Sec. III-B Eq. 4
for each (q,l) pair), in IEEE double, in two independent forms:

* ``direct`` / ``direct_at``: the convolution sum written out (Eq. 4 with
  0-based causal indices, summed over inputs as in Eq. 2);
* ``fftols``: one FFT overlap-save partition per filter (Eq. 5 applied to
  successive input segments; only wrap-free samples kept, Sec. IV step 3),
  with the oracle's own radix-2 FFT (``fft``);
* ``feedback_loop``: the auralization step with feedback cancellation
  (Sec. III-A Eq. 3, Sec. V), block-recursive, direct sums;
* ``serve_loop``: the same loop when sources join and leave microphone slots
  (each source with its own filter row, the feedback paths fixed per slot).

The C code lives in ``rta_oracle.c`` and is built with gcc by
``build_library()``.  Inputs: ``x`` is ``[Q][n_x]`` (any float array; it is
promoted to float64), ``filters`` is a Q x L nested list (row-major
[in][out], the matrix H of Eq. 1) of 1-D arrays, where ``None`` or an empty
array means "no path".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rta_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build_library() -> str:
    """Compile the oracle with gcc (OpenMP, FP64, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_library()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    i64 = ctypes.c_int64
    lib.orc_direct_range.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, dp,
                                     ip, i64, i64, dp]
    lib.orc_direct_at.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, dp, ip,
                                  ip, i64, dp]
    lib.orc_fft.argtypes = [dp, dp, i64, ctypes.c_int]
    lib.orc_feedback_loop.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, i64, dp, ip, dp, ip,
                                      dp, dp, dp]
    lib.orc_fftols.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, dp, ip,
                               i64, dp]
    lib.orc_max_threads.argtypes = []
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.orc_serve_loop.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, i64, i64,
                                   i32p, ip, ip, dp, ip, dp, ip, dp, dp, dp]
    for f in (lib.orc_direct_range, lib.orc_direct_at, lib.orc_fft,
              lib.orc_fftols, lib.orc_feedback_loop, lib.orc_max_threads, lib.orc_serve_loop):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _pack(x, filters):
    x = np.ascontiguousarray(np.atleast_2d(np.asarray(x, dtype=np.float64)))
    Q = len(filters)
    L = len(filters[0])
    if x.shape[0] != Q:
        raise ValueError(f"x has {x.shape[0]} channels, filters have {Q} inputs")
    lens = np.zeros(Q * L, dtype=np.int64)
    parts = []
    for q in range(Q):
        if len(filters[q]) != L:
            raise ValueError("filters must be a rectangular Q x L nested list")
        for l in range(L):
            f = filters[q][l]
            f = np.zeros(0) if f is None else np.asarray(f, dtype=np.float64).ravel()
            lens[q * L + l] = f.size
            parts.append(f)
    off = np.zeros(Q * L + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    h = np.ascontiguousarray(np.concatenate(parts) if off[-1] else np.zeros(1))
    return x, h, off, Q, L


def _check(status, name):
    if status != 0:
        raise RuntimeError(f"oracle {name} failed with status {status}")


def direct(x, filters, n0: int, n1: int) -> np.ndarray:
    """y[l, i] = y_l[n0 + i] for i in [0, n1-n0) -- the definition, Eq. 2/4."""
    x, h, off, Q, L = _pack(x, filters)
    y = np.zeros((L, n1 - n0), dtype=np.float64)
    _check(_load().orc_direct_range(Q, L, _dp(x), x.shape[1], _dp(h), _ip(off),
                                    n0, n1, _dp(y)), "direct")
    return y


def direct_at(x, filters, idx) -> np.ndarray:
    """y[l, i] = y_l[idx[i]] -- the definition at chosen output indices."""
    x, h, off, Q, L = _pack(x, filters)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    y = np.zeros((L, idx.size), dtype=np.float64)
    _check(_load().orc_direct_at(Q, L, _dp(x), x.shape[1], _dp(h), _ip(off),
                                 _ip(idx), idx.size, _dp(y)), "direct_at")
    return y


def fftols(x, filters, n_y: int) -> np.ndarray:
    """y[l, n] for n in [0, n_y) by single-partition FFT overlap-save (Eq. 5)."""
    x, h, off, Q, L = _pack(x, filters)
    y = np.zeros((L, n_y), dtype=np.float64)
    _check(_load().orc_fftols(Q, L, _dp(x), x.shape[1], _dp(h), _ip(off), n_y,
                              _dp(y)), "fftols")
    return y


def feedback_loop(m, synth, feedback, block: int):
    """Closed feedback-cancellation loop (Sec. III-A Eq. 3, Sec. V), block by
    block: mt = m - c delayed by one block, l = H^T * mt, c = F-hat * l.

    m: [P][N] microphone signals; synth: P x L nested filters h_pl (Eq. 1's
    H); feedback: P x L nested filters f_pl (Eq. 3's F-hat, loudspeaker l to
    microphone p).  Returns (l [L][N], c [P][N], mt [P][N])."""
    m, h, hoff, P, L = _pack(m, synth)
    _, f, foff, P2, L2 = _pack(m, feedback)
    if (P2, L2) != (P, L):
        raise ValueError("synthesis and feedback matrices must both be P x L")
    N = m.shape[1]
    l_out = np.zeros((L, N))
    c_out = np.zeros((P, N))
    mt = np.zeros((P, N))
    _check(_load().orc_feedback_loop(P, L, _dp(m), N, int(block), _dp(h), _ip(hoff), _dp(f),
                                     _ip(foff), _dp(l_out), _dp(c_out), _dp(mt)),
           "feedback_loop")
    return l_out, c_out, mt


def serve_loop(m, sources, feedback, block: int):
    """Feedback-cancellation loop with sources that join and leave microphone
    slots (a reading of Sec. III-A Eq. 1-3 and Sec. V; see rta_oracle.c).

    m: [Q][N] microphone signals, one row per slot; sources: list of
    (slot, first_block, end_block, filters) with `filters` a length-L list of
    1-D arrays (None/empty = no path), live during blocks
    [first_block, end_block); feedback: Q x L nested paths f_ql (loudspeaker
    l to slot q) or None.  Returns (l [L][N], c [Q][N], mt [Q][N])."""
    m = np.ascontiguousarray(np.atleast_2d(np.asarray(m, dtype=np.float64)))
    Q, N = m.shape
    if not sources:
        raise ValueError("at least one source is needed")
    L = len(sources[0][3])
    rows = [list(src[3]) for src in sources]
    _, h, hoff, S, L2 = _pack(np.zeros((len(rows), 1)), rows)
    if L2 != L:
        raise ValueError("every source needs L filters")
    if feedback is None:
        feedback = [[None] * L for _ in range(Q)]
    _, f, foff, Q2, L3 = _pack(m, feedback)
    if (Q2, L3) != (Q, L):
        raise ValueError("feedback must be Q x L")
    slot = np.ascontiguousarray([s[0] for s in sources], dtype=np.int32)
    a = np.ascontiguousarray([s[1] for s in sources], dtype=np.int64)
    b = np.ascontiguousarray([s[2] for s in sources], dtype=np.int64)
    l_out = np.zeros((L, N))
    c_out = np.zeros((Q, N))
    mt = np.zeros((Q, N))
    _check(_load().orc_serve_loop(Q, L, S, _dp(m), N, int(block),
                                  slot.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  _ip(a), _ip(b), _dp(h), _ip(hoff), _dp(f), _ip(foff),
                                  _dp(l_out), _dp(c_out), _dp(mt)), "serve_loop")
    return l_out, c_out, mt


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use in this process."""
    return int(_load().orc_max_threads())


def fft(z, inverse: bool = False) -> np.ndarray:
    """Unnormalized DFT with sign -1 (forward) or +1 (inverse, no 1/n)."""
    z = np.asarray(z, dtype=np.complex128)
    re = np.ascontiguousarray(z.real.copy())
    im = np.ascontiguousarray(z.imag.copy())
    _check(_load().orc_fft(_dp(re), _dp(im), re.size, 1 if inverse else -1), "fft")
    return re + 1j * im


def error_db(y_hat, y_ref, axis=-1) -> np.ndarray:
    """Relative RMS error in dB per channel: 20 log10(||y_hat-y|| / ||y||)."""
    y_hat = np.asarray(y_hat, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    num = np.sqrt(np.sum((y_hat - y_ref) ** 2, axis=axis))
    den = np.sqrt(np.sum(y_ref ** 2, axis=axis))
    with np.errstate(divide="ignore"):
        return 20.0 * np.log10(np.maximum(num, 1e-300) / den)
