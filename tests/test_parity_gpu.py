"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance: relative RMS error per output channel <= -100 dB for FP32 spectra
(1e-5), <= -60 dB for FP16 and <= -45 dB for BF16 spectra.  Small cases are
compared sample by sample over the whole output including the filter tail;
the full-size 1 -> 32 x 480,000-tap case is compared at sampled outputs that
the oracle evaluates one by one.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2509_04390_amd import workloads

pytestmark = pytest.mark.gpu

FP32_DB, FP16_DB, BF16_DB = -100.0, -60.0, -45.0


@pytest.fixture(scope="module")
def rta():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2509_04390_amd import rta as mod
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_filters(seed, lens, rt60=0.3):
    Q, L = len(lens), len(lens[0])
    filt = []
    for q in range(Q):
        row = []
        for l in range(L):
            n = lens[q][l]
            f = workloads.reverb_filters(seed * 1000 + q * L + l, 1, 1, max(n, 1), rt60)[0][0]
            row.append(f[:n] if n else None)
        filt.append(row)
    return filt


def padded_signal(seed, Q, n_blocks, B, max_len):
    x = workloads.white_noise(seed, Q, n_blocks * B)
    flush = -(-max(max_len - 1, 0) // B) * B
    return np.concatenate([x, np.zeros((Q, flush), np.float32)], axis=1)


def check_db(y, ref, limit, what):
    live = np.sum(ref ** 2, axis=1) > 0
    assert np.all(y[~live] == 0.0), f"{what}: outputs without a path must be zero"
    err = oracle.error_db(y[live], ref[live])
    say(f"  {what}: max error {err.max():.1f} dB over {live.sum()} outputs")
    assert np.all(err <= limit), f"{what}: {err} dB > {limit} dB"
    return err


CASES = [
    # (B, lens[q][l], streamed blocks)
    (16, [[1]], 6),
    (16, [[16]], 6),
    (16, [[17]], 6),
    (16, [[300, 0], [0, 77]], 20),
    (64, [[1000, 64, 0], [129, 700, 1]], 24),
    (128, [[5000, 128 * 7, 3], [1, 0, 4000], [2500, 130, 129]], 30),
    (256, [[65536 // 8, 256 * 20 + 1]], 12),
    (1024, [[10000], [3000]], 10),     # two bin slices per row
    (4096, [[20000, 9000]], 6),        # eight bin slices, 64 KB of LDS
]


@pytest.mark.parametrize("G", [1, 2, 4])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_upols_fp32_matches_oracle_full_length(rta, case, G):
    B, lens, nb = CASES[case]
    Q, L = len(lens), len(lens[0])
    filt = make_filters(case + 1, lens)
    maxlen = max(max(r) for r in lens)
    x = padded_signal(case + 50, Q, nb, B, maxlen)
    say(f"case {case}: B={B} Q={Q} L={L} lens={lens} G={G} samples={x.shape[1]}")
    # three partitions per work item: many items and partial slots even here
    with rta.Convolver(filt, B, tuning=rta.make_tuning(outputs_per_group=G, tail_rows=3)) as cv:
        y = cv.run(x)
    ref = oracle.direct(x, filt, 0, x.shape[1])
    check_db(y, ref, FP32_DB, f"B={B} G={G}")


@pytest.mark.parametrize("S", [2, 4, 8])
@pytest.mark.parametrize("case", [3, 4, 5, 6, 7])
def test_bin_sliced_items_match_oracle(rta, case, S):
    """First-tier items covering 1/S of each row's bins (more rows each, fewer
    partial slots per output group)."""
    B, lens, nb = CASES[case]
    Q, L = len(lens), len(lens[0])
    filt = make_filters(case + 1, lens)
    maxlen = max(max(r) for r in lens)
    x = padded_signal(case + 50, Q, nb, B, maxlen)
    say(f"case {case}: B={B} lens={lens} bin slices {S}")
    tun = rta.make_tuning(outputs_per_group=2, tail_rows=5, bin_slices=S)
    with rta.Convolver(filt, B, tuning=tun) as cv:
        y = cv.run(x)
        cv.reset()
        y2 = cv.run_device(x)
    assert np.array_equal(y, y2)
    ref = oracle.direct(x, filt, 0, x.shape[1])
    check_db(y, ref, FP32_DB, f"B={B} S={S}")


def test_device_path_equals_host_path_and_reruns_are_bitwise(rta):
    B, lens, nb = CASES[5]
    filt = make_filters(77, lens)
    x = padded_signal(78, len(lens), nb, B, 5000)
    with rta.Convolver(filt, B, tuning=rta.make_tuning(tail_rows=4)) as cv:
        say("host path")
        y1 = cv.run(x)
        cv.reset()
        say("device path")
        y2 = cv.run_device(x)
        cv.reset()
        y3 = cv.run(x)
        assert cv.info()["blocks_done"] == x.shape[1] // B
    assert np.array_equal(y1, y2)
    assert np.array_equal(y1, y3)


def test_block_shift_is_bitwise_invariant(rta):
    B = 64
    lens = [[3000, 200]]
    filt = make_filters(9, lens)
    x = padded_signal(10, 1, 20, B, 3000)
    xs = np.concatenate([np.zeros((1, B), np.float32), x], axis=1)
    with rta.Convolver(filt, B) as cv:
        y = cv.run(x)
        cv.reset()
        ys = cv.run(xs)
    assert np.all(ys[:, :B] == 0.0)
    assert np.array_equal(ys[:, B:], y)


def test_impulse_returns_the_filters(rta):
    B = 128
    lens = [[4000, 129, 128]]
    filt = make_filters(11, lens)
    x = np.zeros((1, 4096), np.float32)
    x[0, 0] = 1.0
    with rta.Convolver(filt, B) as cv:
        y = cv.run(x)
    ref = np.zeros((3, 4096))
    for l in range(3):
        ref[l, :lens[0][l]] = filt[0][l]
    check_db(y, ref, FP32_DB, "impulse")


def test_delta_filters_at_partition_boundaries(rta):
    B = 64
    delays = [0, 1, B - 1, B, B + 1, 5 * B - 1, 5 * B]
    filt = [[np.eye(1, d + 1, d, dtype=np.float32)[0] for d in delays]]
    x = padded_signal(12, 1, 12, B, max(delays) + 1)
    with rta.Convolver(filt, B) as cv:
        y = cv.run(x)
    ref = np.zeros((len(delays), x.shape[1]))
    for l, d in enumerate(delays):
        ref[l, d:] = x[0, :x.shape[1] - d]
    check_db(y, ref, FP32_DB, "delta filters")


@pytest.mark.parametrize("spectra,limit", [("fp16", FP16_DB), ("bf16", BF16_DB)])
def test_reduced_precision_spectra(rta, spectra, limit):
    wl = workloads.config("small")
    filt = wl.filters()
    x = wl.signal_array(flush=True)
    say(f"small config, {spectra} spectra, {x.shape[1]} samples")
    with rta.Convolver(filt, wl.block, spectra=spectra) as cv:
        y = cv.run_device(x)
    ref = oracle.fftols(x, filt, x.shape[1])
    check_db(y, ref, limit, spectra)


def test_fp16_overflow_is_reported(rta):
    big = [[np.full(256, 1000.0, np.float32)]]   # DC bin = 256000 > 65504
    with pytest.raises(rta.RtaError) as e:
        rta.Convolver(big, 256, spectra="fp16")
    assert e.value.status == rta.RTA_E_RANGE
    with rta.Convolver(big, 256, spectra="bf16"):
        pass


def test_small_config_fp32_streamed_and_tail(rta):
    wl = workloads.config("small")
    filt = wl.filters()
    x = wl.signal_array(flush=True)
    say(f"small config fp32: {x.shape[1]} samples")
    with rta.Convolver(filt, wl.block) as cv:
        y = cv.run(x)
        info = cv.info()
    assert info["tier_count"][0] == 65536 // 256
    ref = oracle.fftols(x, filt, x.shape[1])
    check_db(y, ref, FP32_DB, "small/fftols")
    idx = np.unique(np.r_[0, 255, 256, 25599, 25600, 65535, 65536, x.shape[1] - 1,
                          np.random.default_rng(0).integers(0, x.shape[1], 500)])
    refd = oracle.direct_at(x, filt, idx)
    check_db(y[:, idx], refd, FP32_DB, "small/direct")


@pytest.mark.parametrize("B,L,taps,spectra", [(128, 1, 200_000, "fp32"), (128, 4, 60_000, "fp32"),
                                                 (256, 1, 65_536, "fp32"), (64, 2, 40_000, "fp32"),
                                                 (128, 1, 200_000, "fp16"), (128, 2, 100_000, "bf16")])
def test_few_outputs_long_filters_slot_capped_plan(rta, B, L, taps, spectra):
    """Few outputs and long filters: the default plan caps the partial slots of
    an output group at what a head adds up from registers (16 per thread,
    256 / P threads per bin) and slices the rows' bins to keep items small.
    The caps and the output against the oracle, sample by sample."""
    lens = [[taps] * L]
    filt = make_filters(B + L, lens)
    n = -(-(taps + 4 * B) // B) * B  # past the filter length: every partition live
    x = workloads.white_noise(B + L + 7, 1, n)
    with rta.Convolver(filt, B, spectra=spectra) as cv:
        info = cv.info()
        y = cv.run_device(x)
    P = B  # n_f = 2B: P bins per row
    cap = 16 * (256 // P)
    say(f"B={B} L={L} taps={taps} {spectra}: rows/item {info['rows_per_item']}, bin slices "
        f"{info['bin_slices']}, slots per group {info['max_group_slots']} (cap {cap}), grid {info['grid']}")
    assert 0 < info["max_group_slots"] <= cap
    rng = np.random.default_rng(B + L)
    idx = np.unique(np.r_[0, B - 1, B, 2 * B, taps - 1, taps, n - B, n - 1, rng.integers(0, n, 300)])
    ref = oracle.direct_at(x, filt, idx)
    limit = {"fp32": FP32_DB, "fp16": FP16_DB, "bf16": BF16_DB}[spectra]
    check_db(y[:, idx], ref, limit, f"B={B} L={L} {spectra}")


@pytest.mark.parametrize("L,spectra,tuning_slices,want", [(32, "fp16", 0, 2), (40, "bf16", 0, 2),
                                                        (32, "fp32", 0, 1), (16, "fp16", 0, 1),
                                                        (32, "fp16", 1, 1), (32, "fp16", 4, 4)])
def test_tiling_default_slices_for_16bit(rta, L, spectra, tuning_slices, want):
    """Uniform partitions with 16-bit spectra and at least 32 outputs take two
    bin slices unless the caller sets them; FP32 spectra and fewer outputs keep
    one.  rta_info reports the layout, and the output matches the oracle."""
    B, taps = 128, 20_000
    filt = make_filters(L + 3, [[taps] * L])
    n = -(-(taps + 4 * B) // B) * B
    x = workloads.white_noise(L + 11, 1, n)
    tun = rta.make_tuning(bin_slices=tuning_slices) if tuning_slices else None
    with rta.Convolver(filt, B, spectra=spectra, tuning=tun) as cv:
        info = cv.info()
        y = cv.run_device(x)
    say(f"L={L} {spectra} slices asked {tuning_slices}: bin slices {info['bin_slices']}, "
        f"outputs per group {info['outputs_per_group']}, grid {info['grid']}")
    assert info["bin_slices"] == want
    rng = np.random.default_rng(L)
    idx = np.unique(np.r_[0, B - 1, B, taps - 1, taps, n - 1, rng.integers(0, n, 200)])
    ref = oracle.direct_at(x, filt, idx)
    limit = {"fp32": FP32_DB, "fp16": FP16_DB, "bf16": BF16_DB}[spectra]
    check_db(y[:, idx], ref, limit, f"L={L} {spectra} slices {info['bin_slices']}")


def test_main_config_full_size_sampled(rta):
    """1 input -> 32 outputs, 480,000-tap filters, block 128, 2,000 blocks."""
    wl = workloads.config("main")
    filt = wl.filters()
    x = wl.signal_array()
    say(f"main config: Q={wl.n_in} L={wl.n_out} taps={wl.lengths} blocks={wl.n_blocks}")
    with rta.Convolver(filt, wl.block) as cv:
        info = cv.info()
        assert info["tier_count"][0] == 3750
        y = cv.run_device(x)
    rng = np.random.default_rng(2)
    n = x.shape[1]
    idx = np.unique(np.r_[0, 1, 127, 128, n - 1, n - 128, rng.integers(0, n, 200)])
    ref = oracle.direct_at(x, filt, idx)
    check_db(y[:, idx], ref, FP32_DB, "main/direct")


def test_autotune_returns_a_tuning_that_matches_the_oracle(rta):
    B = 64
    lens = [[30000, 9000, 0], [12000, 30000, 500]]
    filt = make_filters(21, lens)
    tuning, scheme, us = rta.rta_autotune(48000.0, B, None, 2, 3, filt, blocks=16)
    say(f"autotune: scheme {scheme}, G={tuning.outputs_per_group}, "
        f"items={tuning.tail_items}, {us:.1f} us/block")
    assert scheme[0] == (B, scheme[0][1]) and us > 0
    x = padded_signal(22, 2, 40, B, 30000)
    with rta.Convolver(filt, B, scheme=scheme, tuning=tuning) as cv:
        y = cv.run(x)
    ref = oracle.fftols(x, filt, x.shape[1])
    check_db(y, ref, FP32_DB, "autotuned")


def test_block_timing_spans(rta):
    """rta_timing_enable(every): spans of `every` blocks, the first starting at
    the first block after the call; only complete spans are returned."""
    filt = make_filters(5, [[600, 100]])
    x = workloads.white_noise(6, 1, 64 * 40)
    with rta.Convolver(filt, 64) as cv:
        rta.rta_timing_enable(cv.ctx, 4)
        for b in range(18):                # spans 0-3, 4-7, 8-11, 12-15; 16-17 open
            cv.process(x[:, b * 64:(b + 1) * 64])
        n, ms = rta.rta_timing_read(cv.ctx)
        assert n == 16 and ms > 0.0
        rta.rta_timing_enable(cv.ctx, 1)   # block 18, 19, 20: one span each
        for b in range(18, 21):
            cv.process(x[:, b * 64:(b + 1) * 64])
        n, ms = rta.rta_timing_read(cv.ctx)
        assert n == 3 and ms > 0.0
        rta.rta_timing_enable(cv.ctx, 0)
        cv.process(x[:, 21 * 64:22 * 64])
        assert rta.rta_timing_read(cv.ctx) == (0, 0.0)
        rta.rta_timing_enable(cv.ctx, 4)   # from block 22: span 22-25; 26 open
        for b in range(22, 27):
            cv.process(x[:, b * 64:(b + 1) * 64])
        n, ms = rta.rta_timing_read(cv.ctx)
        assert n == 4 and ms > 0.0
        rta.rta_timing_enable(cv.ctx, 0)


@pytest.mark.parametrize("spectra,limit", [("fp16", FP16_DB), ("bf16", BF16_DB)])
def test_main_config_reduced_precision_sampled(rta, spectra, limit):
    """The main shape (1 -> 32 x 480,000 taps, block 128) with 16-bit spectra,
    streamed past the filter length so every partition meets input."""
    wl = workloads.config("main")
    filt = wl.filters()
    wl_long = workloads.Workload(**{**wl.__dict__, "n_blocks": 3800})
    x = wl_long.signal_array()
    say(f"main config {spectra}: {x.shape[1]} samples")
    with rta.Convolver(filt, wl.block, spectra=spectra) as cv:
        y = cv.run_device(x)
    rng = np.random.default_rng(3)
    n = x.shape[1]
    idx = np.unique(np.r_[0, 127, 128, 255, 479999, 480000, n - 1, rng.integers(0, n, 120)])
    ref = oracle.direct_at(x, filt, idx)
    check_db(y[:, idx], ref, limit, f"main/{spectra}")


@pytest.mark.parametrize("spectra,limit", [("fp32", FP32_DB), ("fp16", FP16_DB)])
def test_target_point_sampled(rta, spectra, limit):
    """1 -> 64 loudspeakers x 576,000-tap (12 s) filters at block 128, the
    launch configuration the benchmark times, streamed past the filter length
    (4,700 blocks) so every partition meets input; sampled outputs."""
    wl = workloads.config("target")
    filt = wl.filters()
    x = workloads.Workload(**{**wl.__dict__, "n_blocks": 4700}).signal_array()
    say(f"target point {spectra}: L={wl.n_out} taps={wl.lengths} samples={x.shape[1]}")
    with rta.Convolver(filt, wl.block, spectra=spectra) as cv:
        info = cv.info()
        assert info["tier_count"][0] == 4500
        y = cv.run_device(x)
    rng = np.random.default_rng(6)
    n = x.shape[1]
    idx = np.unique(np.r_[0, 1, 128, 575999, 576000, n - 1, rng.integers(0, n, 80),
                          rng.integers(576000, n, 40)])
    ref = oracle.direct_at(x, filt, idx)
    check_db(y[:, idx], ref, limit, f"target/{spectra}")


def test_host_stage_counters(rta):
    """rta_process times its host-side stages; rta_reset restarts the counts."""
    B = 64
    filt = make_filters(90, [[1000, 300]])
    x = padded_signal(91, 1, 12, B, 1000)
    with rta.Convolver(filt, B) as cv:
        cv.run(x)
        info = cv.info()
        n = x.shape[1] // B
        assert info["host_calls"] == n
        assert all(m >= 0 for m in info["host_max_us"]) and info["host_max_us"][2] > 0
        assert 0 <= info["host_slowest_call"] < n and info["host_slowest_us"] > 0
        assert sum(info["host_sum_us"]) <= n * info["host_slowest_us"] + 1e-6
        say(f"  host stages max us: {info['host_max_us']}, waits past 2 ms {info['host_late_waits']}")
        cv.reset()
        info = cv.info()
        assert info["host_calls"] == 0 and info["host_slowest_call"] == -1


def test_degenerate_contexts(rta):
    """Edge cases of the method: every path absent (outputs exactly zero),
    silence in (silence out, exactly), and a context that is created and
    destroyed without processing a block."""
    B = 32
    with rta.Convolver([[None, None], [None, None]], B) as cv:
        y = cv.run(workloads.white_noise(95, 2, 8 * B))
    assert y.shape == (2, 8 * B) and np.all(y == 0.0)
    filt = make_filters(96, [[700, 0, 90]])
    with rta.Convolver(filt, B) as cv:
        y = cv.run(np.zeros((1, 12 * B), np.float32))
        assert np.all(y == 0.0)
        assert cv.info()["blocks_done"] == 12
    rta.Convolver(filt, B).close()
