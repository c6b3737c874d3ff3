"""GPU parity of the feedback-cancellation loop (Sec. III-A Eq. 3, Sec. V)
against the FP64 oracle: block n's input is m_n - c_{n-1} with c = F * y,
y the context's own output.  FP32 spectra: <= -100 dB relative RMS."""
import numpy as np
import pytest

import oracle
from paper_2509_04390_amd import workloads

from test_parity_gpu import FP32_DB, check_db, make_filters, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rta():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2509_04390_amd import rta as mod
    return mod


def weak(filters, scale):
    return [[None if f is None else (f * scale).astype(np.float32) for f in row] for row in filters]


@pytest.mark.parametrize("B,scheme", [(32, None), (64, None), (32, [(32, 12), (256, 0)])])
def test_feedback_loop_matches_oracle(rta, B, scheme):
    P, L = 2, 3
    h = make_filters(40, [[3000, 1200, 0], [800, 2600, 300]])
    f = weak(make_filters(41, [[500, 300, 700], [0, 650, 200]]), 0.02)
    N = 60 * B
    m = workloads.white_noise(42, P, N)
    say(f"feedback loop B={B} scheme={scheme}")
    with rta.Convolver(h, B, scheme=scheme) as cv:
        cv.set_feedback(f)
        y = cv.run(m)
        cv.reset()
        y2 = cv.run_device(m)
    l_ref, c_ref, mt_ref = oracle.feedback_loop(m, h, f, B)
    check_db(y, l_ref, FP32_DB, f"feedback loop B={B}")
    assert np.array_equal(y, y2)


def test_feedback_cancels_a_matched_room(rta):
    """Microphones hear a source plus the loudspeakers through paths F one block
    late (simulated on the host, block by block); with the estimate equal to F
    the loudspeakers carry only the synthesized source: y = H^T * s."""
    B, P, L = 64, 1, 4
    h = make_filters(43, [[4000, 2500, 3000, 1000]])
    f = weak(make_filters(44, [[900, 700, 1200, 400]]), 0.02)
    nb = 80
    s = workloads.white_noise(45, P, nb * B)
    y = np.zeros((L, nb * B), np.float32)
    with rta.Convolver(h, B) as cv:
        cv.set_feedback(f)
        for n in range(nb):
            fb = np.zeros((P, B))
            if n > 0:   # room: F * y, block n-1
                t0 = (n - 1) * B
                for p in range(P):
                    for l in range(L):
                        full = np.convolve(y[l, :t0 + B].astype(np.float64), f[p][l])
                        fb[p] += full[t0:t0 + B]
            m_n = (s[:, n * B:(n + 1) * B] + fb).astype(np.float32)
            y[:, n * B:(n + 1) * B] = cv.process(m_n)
    want = oracle.direct(s, h, 0, nb * B)
    check_db(y, want, FP32_DB, "matched room")


def test_feedback_removed_restores_plain_synthesis(rta):
    B = 32
    h = make_filters(46, [[2000, 500]])
    f = weak(make_filters(47, [[300, 300]]), 0.05)
    m = workloads.white_noise(48, 1, 40 * B)
    with rta.Convolver(h, B) as cv:
        cv.set_feedback(f)
        cv.set_feedback(None)
        y = cv.run(m)
    check_db(y, oracle.direct(m, h, 0, m.shape[1]), FP32_DB, "feedback removed")


@pytest.mark.parametrize("fb_spectra,spectra_db", [("fp16", -60.0), ("bf16", -45.0)])
def test_feedback_in_a_separate_launch(rta, fb_spectra, spectra_db):
    """Feedback spectra of another storage type than the synthesis spectra: the
    feedback convolution runs as its own launch after each block instead of
    inside the synthesis launch.  The estimate c carries the storage type's
    relative error; it reaches the output through m - c, so the bound is that
    error scaled by rms(c) / rms(m - c) (both from the oracle)."""
    B, P, L = 32, 2, 3
    h = make_filters(50, [[2500, 900, 0], [700, 2200, 400]])
    # weak paths: the bound below ignores the loop's own amplification of
    # the estimate's rounding error, which grows with the loop gain
    f = weak(make_filters(51, [[400, 250, 600], [0, 500, 150]]), 0.004)
    m = workloads.white_noise(52, P, 50 * B)
    with rta.Convolver(h, B) as cv:
        cv.set_feedback(f, spectra=fb_spectra)
        y = cv.run(m)
    l_ref, c_ref, mt_ref = oracle.feedback_loop(m, h, f, B)
    gain = np.sqrt(np.mean(c_ref ** 2, axis=1) / np.mean(mt_ref ** 2, axis=1)).max()
    limit = spectra_db + 20.0 * np.log10(max(1.0, gain))
    say(f"  |c| / |m - c| = {gain:.2f}: bound {limit:.1f} dB")
    check_db(y, l_ref, limit, f"feedback in its own launch ({fb_spectra})")


def test_fused_feedback_with_many_microphones_and_long_paths(rta):
    """16 microphones x 8 loudspeakers, feedback paths longer than the synthesis
    filters, non-uniform synthesis tiers: the fused loop against the oracle."""
    B = 64
    rng = np.random.default_rng(53)
    hl = [[int(rng.integers(0, 3000)) for _ in range(8)] for _ in range(16)]
    fl = [[int(rng.integers(0, 4000)) for _ in range(8)] for _ in range(16)]
    h = make_filters(54, hl)
    f = weak(make_filters(55, fl), 0.005)
    m = workloads.white_noise(56, 16, 40 * B)
    with rta.Convolver(h, B, scheme=[(64, 12), (512, 0)]) as cv:
        cv.set_feedback(f)
        y = cv.run(m)
        cv.reset()
        y2 = cv.run_device(m)
    assert np.array_equal(y, y2)
    l_ref, _, _ = oracle.feedback_loop(m, h, f, B)
    check_db(y, l_ref, FP32_DB, "fused feedback 16 mics")


def fused_bound(limit, c_ref, mt_ref):
    """Output error bound with 16-bit synthesis and feedback spectra: the
    synthesis spectra carry a relative error d, and so does the estimate c,
    which reaches the output through m - c; the two are independent, so the
    bound is d * sqrt(1 + g^2), g = rms(c) / rms(m - c) (from the oracle)."""
    g = np.sqrt(np.mean(c_ref ** 2, axis=1) / np.mean(mt_ref ** 2, axis=1)).max()
    return limit + 10.0 * np.log10(1.0 + g * g), g


@pytest.mark.parametrize("spectra,limit", [("fp16", -60.0), ("bf16", -45.0)])
def test_fused_feedback_with_16bit_spectra(rta, spectra, limit):
    """Synthesis and feedback spectra both 16-bit: the feedback convolution
    runs inside the synthesis launch (the fused 16-bit kernels)."""
    B, P, L = 32, 2, 3
    # scales keep the loop gain |F H| well below 1 (|c| / |m - c| about 0.15)
    h = weak(make_filters(60, [[2500, 900, 0], [700, 2200, 400]]), 0.1)
    f = weak(make_filters(61, [[400, 250, 600], [0, 500, 150]]), 0.002)
    m = workloads.white_noise(62, P, 60 * B)
    with rta.Convolver(h, B, spectra=spectra) as cv:
        cv.set_feedback(f, spectra=spectra)
        info = cv.info()
        assert info["feedback_paths"] == 1 and info["feedback_fused"] == 1
        y = cv.run(m)
        cv.reset()
        y2 = cv.run_device(m)
    assert np.array_equal(y, y2)
    l_ref, c_ref, mt_ref = oracle.feedback_loop(m, h, f, B)
    bound, g = fused_bound(limit, c_ref, mt_ref)
    say(f"  {spectra}: |c| / |m - c| = {g:.3f}, bound {bound:.1f} dB")
    check_db(y, l_ref, bound, f"fused feedback {spectra}")


@pytest.mark.parametrize("spectra,limit", [("fp32", FP32_DB), ("fp16", -60.0)])
def test_fused_feedback_64_loudspeakers_16_mics_8192_taps(rta, spectra, limit):
    """16 microphones -> 64 loudspeakers, feedback paths of 8,192 taps
    (64 -> 16), block 64, streamed past the feedback length so every feedback
    partition meets signal; the fused loop against the oracle loop."""
    B, P, L = 64, 16, 64
    rng = np.random.default_rng(63)
    # scales keep the loop gain well below 1 (|c| / |m - c| about 0.17)
    h = weak(make_filters(64, [[int(rng.integers(200, 1000)) for _ in range(L)] for _ in range(P)]),
             0.007)
    f = weak(make_filters(65, [[8192] * L for _ in range(P)], rt60=0.1), 0.002)
    nb = 8192 // B + 6
    m = workloads.white_noise(66, P, nb * B)
    say(f"fused feedback {spectra}: {P} mics x {L} loudspeakers, 8192-tap paths, {nb} blocks")
    with rta.Convolver(h, B, spectra=spectra) as cv:
        cv.set_feedback(f, spectra=spectra)
        assert cv.info()["feedback_fused"] == 1
        y = cv.run_device(m)
    l_ref, c_ref, mt_ref = oracle.feedback_loop(m, h, f, B)
    bound, g = fused_bound(limit, c_ref, mt_ref)
    say(f"  |c| / |m - c| = {g:.3f}, bound {bound:.1f} dB")
    check_db(y, l_ref, bound, f"64 -> 16 x 8192 feedback {spectra}")


def test_feedback_wait_that_gives_up_fails_the_block(rta):
    """The synthesis workgroups' wait for the feedback estimate is bounded;
    forced to give up (an unreachable count, checked from the host), every
    kernel still finishes, the block reports RTA_E_DEVICE and the context is
    poisoned."""
    B = 32
    h = make_filters(67, [[500, 300]])
    f = weak(make_filters(68, [[200, 100]]), 0.01)
    m = workloads.white_noise(69, 1, 4 * B)
    cv = rta.Convolver(h, B)
    cv.set_feedback(f)
    assert cv.info()["feedback_fused"] == 1
    cv.process(m[:, :B])                       # a normal block first
    rta.rta_test_feedback_wait(cv.ctx, 64, True)
    with pytest.raises(rta.RtaError) as e:
        cv.process(m[:, B:2 * B])
    assert e.value.status == rta.RTA_E_DEVICE
    with pytest.raises(rta.RtaError) as e:
        cv.process(m[:, 2 * B:3 * B])
    assert e.value.status == rta.RTA_E_DEVICE
    with pytest.raises(rta.RtaError):
        cv.info()
    cv.close()
    # the device path reports it at the next call
    import torch
    cv = rta.Convolver(h, B)
    cv.set_feedback(f)
    rta.rta_test_feedback_wait(cv.ctx, 64, True)
    xi = torch.from_numpy(m[:, :B].copy()).cuda()
    yo = torch.empty((2, B), dtype=torch.float32, device="cuda")
    cv.process_device(xi, yo)
    torch.cuda.synchronize()
    with pytest.raises(rta.RtaError) as e:
        cv.process_device(xi, yo)
    assert e.value.status == rta.RTA_E_DEVICE
    cv.close()


def test_matched_room_does_not_drift_over_60_seconds(rta):
    """60 s of the closed loop at the cfg5 shape: 16 microphones, 64
    loudspeakers, 8,192-tap paths, block 64 (45,000 blocks).  The room is a
    second context with the true paths F (64 -> 16) whose output for block n
    reaches the microphones in block n + 1; the canceller holds F^ = F, so
    the loudspeakers must carry H^T * s alone (Sec. III-A Eq. 1-3), at the
    end of the minute as at its start: FP32 bound at late samples, checked
    by direct sums."""
    B, P, L = 64, 16, 64
    nb = 60 * 48000 // B
    rng = np.random.default_rng(770)
    h = weak(make_filters(771, [[int(rng.integers(200, 1000)) for _ in range(L)] for _ in range(P)]),
             0.007)
    f = weak(make_filters(772, [[8192] * L for _ in range(P)], rt60=0.1), 0.002)
    room_filters = [[f[q][l] for q in range(P)] for l in range(L)]  # 64 inputs -> 16 outputs
    s = workloads.white_noise(773, P, nb * B)
    y = np.empty((L, nb * B), np.float32)
    with rta.Convolver(h, B) as cv, rta.Convolver(room_filters, B) as room:
        cv.set_feedback(f)
        assert cv.info()["feedback_fused"] == 1
        heard = np.zeros((P, B), np.float32)
        for n in range(nb):
            m = s[:, n * B:(n + 1) * B] + heard
            yn = cv.process(m)
            y[:, n * B:(n + 1) * B] = yn
            heard = room.process(yn)
    for what, lo, hi in (("first 5 s", 8192, 5 * 48000), ("last 5 s", nb * B - 5 * 48000, nb * B)):
        idx = np.unique(rng.integers(lo, hi, 200))
        ref = oracle.direct_at(s, h, idx)
        check_db(y[:, idx], ref, FP32_DB, f"matched room, {what}")
