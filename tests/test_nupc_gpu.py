"""GPU parity of non-uniform partitioned convolution (tiers of growing
partition size, later tiers delayed in the time domain) against the FP64
oracle.  The partition scheme only regroups the convolution sum, so every
scheme must reproduce the same output: FP32 spectra <= -100 dB relative RMS
per output, FP16 <= -60 dB."""
import numpy as np
import pytest

import oracle
from paper_2509_04390_amd import workloads

from test_parity_gpu import FP16_DB, FP32_DB, check_db, make_filters, padded_signal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rta():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2509_04390_amd import rta as mod
    return mod


def offsets(scheme):
    o, out = 0, []
    for size, count in scheme:
        out.append(o)
        o += size * count
    return out


# (B, scheme, lens[q][l], streamed blocks, flags)
SCHEMES = [
    # spread: tier 1 s = 7, r = 4 (3 blocks of multiply-accumulate), tier 2
    # s = 11, r = 16 (7 blocks)
    (16, [(16, 10), (64, 4), (256, 0)], [[3000, 700, 161]], 40, 0),
    # a later tier with more slack than one frame: spread capped at r - 1
    (16, [(16, 20), (64, 0)], [[2500, 321, 319]], 30, 0),
    # spike: each later-tier frame accumulated in a single block; both later
    # tiers at the least slack allowed (s = 5)
    (16, [(16, 8), (64, 3), (256, 0)], [[3000, 300]], 40, "spike"),
    # ragged MIMO: pairs ending in every tier, absent pairs, Q != L
    (32, [(32, 8), (128, 4), (512, 0)], [[4000, 0, 300], [150, 2500, 0]], 40, 0),
    # the standard scheme of block 128 (tiers 128 / 1024 / 8192)
    (128, [(128, 15), (1024, 14), (8192, 0)], [[20000, 17000]], 60, 0),
]


@pytest.mark.parametrize("case", range(len(SCHEMES)))
def test_nupc_fp32_matches_oracle_full_length(rta, case):
    B, scheme, lens, nb, flags = SCHEMES[case]
    Q, L = len(lens), len(lens[0])
    filt = make_filters(100 + case, lens)
    maxlen = max(max(r) for r in lens)
    x = padded_signal(200 + case, Q, nb, B, maxlen)
    say(f"nupc case {case}: B={B} scheme={scheme} lens={lens} samples={x.shape[1]}")
    fl = rta.RTA_FLAG_SPIKE if flags == "spike" else 0
    with rta.Convolver(filt, B, scheme=scheme, flags=fl) as cv:
        info = cv.info()
        assert info["n_tiers"] == len(scheme)
        assert info["tier_offset"] == offsets(scheme)
        y = cv.run(x)
    ref = oracle.direct(x, filt, 0, x.shape[1])
    check_db(y, ref, FP32_DB, f"nupc case {case}")


def test_nupc_device_path_equals_host_path(rta):
    B, scheme, lens, nb, _ = SCHEMES[0]
    filt = make_filters(300, lens)
    x = padded_signal(301, 1, nb, B, 3000)
    with rta.Convolver(filt, B, scheme=scheme) as cv:
        y1 = cv.run(x)
        cv.reset()
        y2 = cv.run_device(x)
    assert np.array_equal(y1, y2)


def test_delta_filters_around_tier_boundaries(rta):
    B = 16
    scheme = [(16, 8), (64, 3), (256, 0)]
    o1, o2 = offsets(scheme)[1:]
    delays = [o1 - 1, o1, o1 + 1, o1 + 63, o1 + 64, o2 - 1, o2, o2 + 1, o2 + 2 * 256 + 5]
    filt = [[np.eye(1, d + 1, d, dtype=np.float32)[0] for d in delays]]
    x = padded_signal(302, 1, 40, B, max(delays) + 1)
    with rta.Convolver(filt, B, scheme=scheme) as cv:
        y = cv.run(x)
    ref = np.zeros((len(delays), x.shape[1]))
    for l, d in enumerate(delays):
        ref[l, d:] = x[0, :x.shape[1] - d]
    check_db(y, ref, FP32_DB, "delta filters at tier boundaries")


def test_scheme_invariance_uniform_vs_nonuniform(rta):
    B = 32
    lens = [[6000, 4100]]
    filt = make_filters(303, lens)
    x = padded_signal(304, 1, 30, B, 6000)
    with rta.Convolver(filt, B) as cv:
        yu = cv.run(x)
    with rta.Convolver(filt, B, scheme=[(32, 12), (256, 0)]) as cv:
        yn = cv.run(x)
    err = oracle.error_db(yn, yu)
    say(f"  uniform vs non-uniform: {err.max():.1f} dB")
    assert np.all(err < FP32_DB)


def test_nupc_workload_fp16_sampled(rta):
    """4 sources -> 64 outputs, U[3,12] s filters per source, tiers
    128/1024/8192, FP16 spectra, 2,000 blocks of white noise."""
    wl = workloads.config("nupc")
    filt = wl.filters()
    x = wl.signal_array()
    say(f"nupc workload: lengths={wl.lengths} scheme={wl.scheme} blocks={wl.n_blocks}")
    with rta.Convolver(filt, wl.block, scheme=wl.scheme, spectra="fp16") as cv:
        info = cv.info()
        say(f"  spectra {info['spectra_bytes'] / 1e6:.1f} MB, phases {info['n_phases']}")
        y = cv.run_device(x)
    rng = np.random.default_rng(4)
    n = x.shape[1]
    idx = np.unique(np.r_[0, 127, 128, 1919, 1920, 16255, 16256, 16257, n - 1,
                          rng.integers(0, n, 60)])
    ref = oracle.direct_at(x, filt, idx)
    check_db(y[:, idx], ref, FP16_DB, "nupc workload fp16")


def test_nupc_workload_log_sweep_fp16_sampled(rta):
    """The same batched workload driven by an exponential sine sweep
    (20 Hz -> 20 kHz) on every source instead of noise."""
    wl = workloads.config("nupc")
    wl.signal = "sweep"
    filt = wl.filters()
    x = wl.signal_array()
    say(f"nupc workload, log-sine sweep: blocks={wl.n_blocks}")
    with rta.Convolver(filt, wl.block, scheme=wl.scheme, spectra="fp16") as cv:
        y = cv.run_device(x)
    rng = np.random.default_rng(5)
    n = x.shape[1]
    idx = np.unique(np.r_[0, 127, 128, 1919, 1920, 16255, 16256, 16257, n - 1,
                          rng.integers(0, n, 60)])
    ref = oracle.direct_at(x, filt, idx)
    check_db(y[:, idx], ref, FP16_DB, "nupc workload sweep fp16")
