"""GPU parity of the n_f = 3 n_x variant (RTA_FLAG_NF3; Sec. V, last
paragraph): B-tap partitions with 3B-point transforms, and the feedback
convolution fed with the synthesis output spectra as they are (no inverse
then forward transform of y).  The variant only regroups the same sums, so
it must reproduce the FP64 oracle: plain synthesis (Sec. III-A Eq. 2)
against the direct sum, the closed loop (Eq. 3 and Sec. V) against the
oracle's block-recursive loop, within the same bounds as n_f = 2B."""
import numpy as np
import pytest

import oracle
from paper_2509_04390_amd import workloads

from test_parity_gpu import (BF16_DB, FP16_DB, FP32_DB, check_db, make_filters, padded_signal,
                             say)
from test_feedback_gpu import fused_bound, weak

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rta():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2509_04390_amd import rta as mod
    return mod


@pytest.mark.parametrize("B,spectra,limit", [(16, "fp32", FP32_DB), (64, "fp32", FP32_DB),
                                             (128, "fp32", FP32_DB), (256, "fp32", FP32_DB),
                                             (128, "fp16", FP16_DB), (64, "bf16", BF16_DB)])
def test_nf3_synthesis_matches_oracle(rta, B, spectra, limit):
    """Ragged MIMO (absent pairs, a filter shorter than one block, lengths
    that end mid-partition) streamed past the longest filter."""
    lens = [[3000, 0, 5 * B + 7], [B - 3, 2 * B, 4100]]
    filt = make_filters(700 + B, lens)
    x = padded_signal(701 + B, 2, 30, B, 4100)
    with rta.Convolver(filt, B, spectra=spectra, flags=rta.RTA_FLAG_NF3) as cv:
        info = cv.info()
        assert info["fft_size"] == 3 * B
        y = cv.run(x)
        cv.reset()
        y2 = cv.run_device(x)
    assert np.array_equal(y, y2)
    check_db(y, oracle.direct(x, filt, 0, x.shape[1]), limit, f"n_f=3B synthesis B={B} {spectra}")


def test_nf3_delta_filters_at_partition_boundaries(rta):
    """h = delta(n - d): y is x delayed by d, at d around the B-tap partition
    edges (a 3B-point transform with B-tap partitions must not alias)."""
    B = 32
    delays = [0, 1, B - 1, B, B + 1, 2 * B - 1, 2 * B, 3 * B - 1, 3 * B, 7 * B + 5]
    filt = [[np.eye(1, d + 1, d, dtype=np.float32)[0] for d in delays]]
    x = padded_signal(710, 1, 20, B, max(delays) + 1)
    with rta.Convolver(filt, B, flags=rta.RTA_FLAG_NF3) as cv:
        y = cv.run(x)
    ref = np.zeros((len(delays), x.shape[1]))
    for l, d in enumerate(delays):
        ref[l, d:] = x[0, :x.shape[1] - d]
    check_db(y, ref, FP32_DB, "n_f=3B delta filters")


@pytest.mark.parametrize("B", [32, 64])
def test_nf3_feedback_loop_matches_oracle(rta, B):
    P, L = 2, 3
    h = make_filters(720, [[3000, 1200, 0], [800, 2600, 300]])
    f = weak(make_filters(721, [[500, 300, 700], [0, 650, 200]]), 0.02)
    m = workloads.white_noise(722, P, 60 * B)
    say(f"n_f=3B feedback loop B={B}")
    with rta.Convolver(h, B, flags=rta.RTA_FLAG_NF3) as cv:
        cv.set_feedback(f)
        info = cv.info()
        assert info["feedback_fused"] == 1 and info["fft_size"] == 3 * B
        y = cv.run(m)
        cv.reset()
        y2 = cv.run_device(m)
    assert np.array_equal(y, y2)
    l_ref, _, _ = oracle.feedback_loop(m, h, f, B)
    check_db(y, l_ref, FP32_DB, f"n_f=3B feedback loop B={B}")


@pytest.mark.parametrize("spectra,limit", [("fp16", -60.0), ("bf16", -45.0)])
def test_nf3_feedback_with_16bit_spectra(rta, spectra, limit):
    B, P = 32, 2
    h = weak(make_filters(730, [[2500, 900, 0], [700, 2200, 400]]), 0.1)
    f = weak(make_filters(731, [[400, 250, 600], [0, 500, 150]]), 0.002)
    m = workloads.white_noise(732, P, 60 * B)
    with rta.Convolver(h, B, spectra=spectra, flags=rta.RTA_FLAG_NF3) as cv:
        cv.set_feedback(f, spectra=spectra)
        assert cv.info()["feedback_fused"] == 1
        y = cv.run(m)
    l_ref, c_ref, mt_ref = oracle.feedback_loop(m, h, f, B)
    bound, g = fused_bound(limit, c_ref, mt_ref)
    check_db(y, l_ref, bound, f"n_f=3B fused feedback {spectra}")


def test_nf3_64_loudspeakers_16_mics_8192_taps(rta):
    """16 microphones -> 64 loudspeakers, 8,192-tap feedback paths (64 ->
    16), block 64, streamed past the feedback length."""
    B, P, L = 64, 16, 64
    rng = np.random.default_rng(740)
    h = weak(make_filters(741, [[int(rng.integers(200, 1000)) for _ in range(L)] for _ in range(P)]),
             0.007)
    f = weak(make_filters(742, [[8192] * L for _ in range(P)], rt60=0.1), 0.002)
    nb = 8192 // B + 6
    m = workloads.white_noise(743, P, nb * B)
    with rta.Convolver(h, B, flags=rta.RTA_FLAG_NF3) as cv:
        cv.set_feedback(f)
        assert cv.info()["feedback_fused"] == 1
        y = cv.run_device(m)
    l_ref, _, _ = oracle.feedback_loop(m, h, f, B)
    check_db(y, l_ref, FP32_DB, "n_f=3B 64 -> 16 x 8192 feedback")


def test_nf3_matches_nf2_under_feedback(rta):
    """The two transform sizes give the same closed loop up to rounding."""
    B, P = 32, 1
    h = make_filters(750, [[1500, 900, 2000]])
    f = weak(make_filters(751, [[300, 200, 500]]), 0.03)
    m = workloads.white_noise(752, P, 50 * B)
    ys = []
    for flags in (0, rta.RTA_FLAG_NF3):
        with rta.Convolver(h, B, flags=flags) as cv:
            cv.set_feedback(f)
            ys.append(cv.run(m))
    err = oracle.error_db(ys[1], ys[0])
    say(f"  n_f=3B vs n_f=2B: {err.max():.1f} dB")
    assert np.all(err < FP32_DB)


def test_nf3_rejections(rta):
    B = 32
    h = make_filters(760, [[1000, 500]])
    with pytest.raises(rta.RtaError) as e:
        rta.Convolver(h, B, scheme=[(32, 12), (256, 0)], flags=rta.RTA_FLAG_NF3)
    assert e.value.status == rta.RTA_E_ARG
    with pytest.raises(rta.RtaError) as e:
        rta.Server(2, 2, 1000, B, flags=rta.RTA_FLAG_NF3)
    assert e.value.status == rta.RTA_E_UNSUPPORTED
    with rta.Convolver(h, B, flags=rta.RTA_FLAG_NF3) as cv:
        with pytest.raises(rta.RtaError) as e:
            cv.set_feedback(weak(make_filters(761, [[100, 100]]), 0.01), spectra="fp16")
        assert e.value.status == rta.RTA_E_UNSUPPORTED
        x = padded_signal(762, 1, 10, B, 1000)
        y = cv.run(x)   # the context is untouched by the refused call
    check_db(y, oracle.direct(x, h, 0, x.shape[1]), FP32_DB, "n_f=3B after a refused call")
