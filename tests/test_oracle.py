"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test names the passage it pins and what a plausible slip would break:
closed forms (exact rational sums, geometric series, DFT pairs), invariants
(linearity, time shift, superposition over inputs), special cases that reduce
to library routines (numpy.convolve, numpy.fft), and the agreement of the two
independent oracle forms (direct sum vs FFT overlap-save).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------------------
# FFT (Eq. 5 uses an n_f-point FFT; the oracle's own radix-2 transform)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 1024])
def test_fft_shifted_impulse_is_a_pure_phase(n):
    # DFT pair: delta[m - s]  <->  exp(-2 pi i k s / n) for every k.
    k = np.arange(n)
    for s in sorted({0, min(1, n - 1), n // 3, n - 1}):
        z = np.zeros(n, complex)
        z[s] = 1.0
        want = np.exp(-2j * np.pi * ((k * s) % n) / n)   # phase reduced exactly
        got = oracle.fft(z)
        assert np.max(np.abs(got - want)) < 1e-13 * max(1, np.log2(n))


@pytest.mark.parametrize("n", [8, 512])
def test_fft_complex_exponential_is_a_single_bin(n):
    # DFT pair: exp(+2 pi i m j / n)  <->  n * delta[k - m].
    j = np.arange(n)
    for m in (0, 1, n // 2, n - 3):
        got = oracle.fft(np.exp(2j * np.pi * m * j / n))
        want = np.zeros(n, complex)
        want[m] = n
        assert np.max(np.abs(got - want)) < 1e-10


@pytest.mark.parametrize("n", [2, 16, 4096])
def test_fft_matches_numpy_both_directions(n):
    z = rng(n).standard_normal(n) + 1j * rng(n + 1).standard_normal(n)
    f = oracle.fft(z)
    assert np.max(np.abs(f - np.fft.fft(z))) < 1e-12 * n
    b = oracle.fft(z, inverse=True)
    assert np.max(np.abs(b - n * np.fft.ifft(z))) < 1e-12 * n


def test_fft_roundtrip_and_parseval():
    n = 2048
    z = rng(3).standard_normal(n) + 1j * rng(4).standard_normal(n)
    f = oracle.fft(z)
    assert abs(np.sum(np.abs(f) ** 2) / n - np.sum(np.abs(z) ** 2)) < 1e-9 * n
    back = oracle.fft(f, inverse=True) / n
    assert np.max(np.abs(back - z)) < 1e-13


def test_fft_rejects_non_power_of_two():
    with pytest.raises(RuntimeError):
        oracle.fft(np.zeros(12))


# ----------------------------------------------------------------------------
# Direct form (Eq. 4 per pair, Eq. 2 over inputs)
# ----------------------------------------------------------------------------

def test_impulse_input_returns_each_filter_exactly():
    # x = delta[n]  =>  y_l = h_{0l} (no rounding: one nonzero product by 1.0)
    r = rng(10)
    lens = [1, 7, 300]
    filt = [[r.standard_normal(n).astype(np.float32) for n in lens]]
    x = np.zeros((1, 400), np.float32)
    x[0, 0] = 1.0
    y = oracle.direct(x, filt, 0, 420)
    for l, n in enumerate(lens):
        assert np.array_equal(y[l, :n], filt[0][l].astype(np.float64))
        assert np.all(y[l, n:] == 0.0)


@pytest.mark.parametrize("d", [0, 1, 127, 128, 129, 479])
def test_delta_filter_delays_the_input_exactly(d):
    # h = delta[n - d]  =>  y[n] = x[n - d]   (Sec. III-B: causal FIR, no extra delay)
    x = rng(d).standard_normal((1, 700)).astype(np.float32)
    h = np.zeros(d + 1, np.float32)
    h[d] = 1.0
    y = oracle.direct(x, [[h]], 0, 800)[0]
    want = np.zeros(800)
    want[d:d + 700] = x[0, :800 - d] if d + 700 > 800 else x[0]
    assert np.array_equal(y, want)


def test_geometric_filter_and_input_match_exact_rational_sum():
    # h[j] = a^j (j < Lh), x[n] = b^n (n < Nx): every value is a dyadic or
    # small-integer rational exactly representable in double, so the
    # convolution sum has an exact value computed here with Fractions from
    # the geometric-series closed form:
    #   y[n] = b^n * sum_{j=j0}^{j1} (a/b)^j
    #        = b^n * ((a/b)^j0 - (a/b)^(j1+1)) / (1 - a/b)
    a, b = Fraction(3, 4), Fraction(-1, 2)
    Lh, Nx = 30, 25
    h = np.array([float(a ** j) for j in range(Lh)])
    x = np.array([[float(b ** n) for n in range(Nx)]])
    y = oracle.direct(x, [[h]], 0, Lh + Nx - 1)[0]
    r = a / b
    for n in range(Lh + Nx - 1):
        j0, j1 = max(0, n - (Nx - 1)), min(n, Lh - 1)
        exact = b ** n * (r ** j0 - r ** (j1 + 1)) / (1 - r)
        assert abs(y[n] - float(exact)) <= 4e-16 * max(1.0, abs(float(exact)))


def test_constant_input_gives_the_step_response():
    # x[n] = 1 for n < Nx  =>  y[n] = sum_{j <= n} h[j] while n < Nx.
    h = rng(11).standard_normal(500)
    x = np.ones((1, 800))
    y = oracle.direct(x, [[h]], 0, 800)[0]
    step = np.cumsum(h)
    want = np.concatenate([step, np.full(300, step[-1])])
    assert np.max(np.abs(y - want)) < 1e-12


def test_sinusoid_in_steady_state_follows_the_frequency_response():
    # x[n] = cos(w n); for n >= Lh-1 the output is Re{H(e^{iw}) e^{iwn}} with
    # H the DTFT of h.  For h[j] = a^j, H = (1 - (a e^{-iw})^Lh)/(1 - a e^{-iw}).
    a, Lh, w = 0.97, 200, 2 * np.pi * 0.0371
    h = a ** np.arange(Lh)
    n = np.arange(600)
    y = oracle.direct(np.cos(w * n)[None, :], [[h]], 0, 600)[0]
    z = a * np.exp(-1j * w)
    H = (1 - z ** Lh) / (1 - z)
    ss = np.real(H * np.exp(1j * w * n))
    assert np.max(np.abs(y[Lh - 1:] - ss[Lh - 1:])) < 1e-11


def test_siso_matches_numpy_convolve_full_length():
    r = rng(12)
    for nx, nh in [(1, 1), (5, 300), (300, 5), (1000, 777)]:
        x = r.standard_normal(nx)
        h = r.standard_normal(nh)
        y = oracle.direct(x[None, :], [[h]], 0, nx + nh - 1)[0]
        assert np.max(np.abs(y - np.convolve(x, h))) < 1e-11


def test_mimo_is_the_sum_over_inputs_of_pairwise_convolutions():
    # Eq. 2: l_l = sum_q h_ql * m_q with H indexed [q][l].  Q != L, every pair
    # a different length and one pair absent, so a transposed H, a wrong pair
    # offset or a dropped input all change the result.
    r = rng(13)
    Q, L, nx = 3, 2, 400
    lens = [[50, 0], [123, 7], [1, 260]]
    filt = [[r.standard_normal(lens[q][l]) for l in range(L)] for q in range(Q)]
    x = r.standard_normal((Q, nx))
    n_y = nx + 260 - 1
    y = oracle.direct(x, filt, 0, n_y)
    for l in range(L):
        want = np.zeros(n_y)
        for q in range(Q):
            if lens[q][l]:
                c = np.convolve(x[q], filt[q][l])
                want[:c.size] += c
        assert np.max(np.abs(y[l] - want)) < 1e-11


def test_linearity_and_block_aligned_time_shift():
    r = rng(14)
    h = r.standard_normal(333)
    x1, x2 = r.standard_normal((1, 600)), r.standard_normal((1, 600))
    y1 = oracle.direct(x1, [[h]], 0, 900)
    y2 = oracle.direct(x2, [[h]], 0, 900)
    y12 = oracle.direct(2.5 * x1 - 0.75 * x2, [[h]], 0, 900)
    assert np.max(np.abs(y12 - (2.5 * y1 - 0.75 * y2))) < 1e-11
    s = 77
    xs = np.concatenate([np.zeros((1, s)), x1], axis=1)
    ys = oracle.direct(xs, [[h]], 0, 900 + s)
    assert np.array_equal(ys[:, s:], y1)
    assert np.all(ys[:, :s] == 0.0)


def test_direct_at_agrees_with_the_range_form():
    r = rng(15)
    filt = [[r.standard_normal(90), r.standard_normal(40)]]
    x = r.standard_normal((1, 256))
    full = oracle.direct(x, filt, 0, 400)
    idx = np.array([0, 1, 89, 90, 255, 256, 344, 399])
    assert np.array_equal(oracle.direct_at(x, filt, idx), full[:, idx])
    part = oracle.direct(x, filt, 100, 200)
    assert np.array_equal(part, full[:, 100:200])


# ----------------------------------------------------------------------------
# FFT overlap-save form (Eq. 5, OLS keeps the wrap-free samples)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("Q,L,nx,maxlen", [(1, 1, 50, 1), (1, 3, 2000, 97),
                                             (2, 3, 3000, 1000), (3, 1, 5000, 4096)])
def test_fftols_agrees_with_direct_to_fp64_rounding(Q, L, nx, maxlen):
    # Several segments (n_y >> hop) and ragged lengths exercise the hop,
    # the discard and the window start; -240 dB is ~1e-12 relative RMS.
    r = rng(Q * 100 + L)
    lens = r.integers(1, maxlen + 1, size=(Q, L))
    lens[0, 0] = maxlen
    filt = [[r.standard_normal(lens[q][l]) for l in range(L)] for q in range(Q)]
    x = r.standard_normal((Q, nx))
    n_y = nx + maxlen - 1
    yd = oracle.direct(x, filt, 0, n_y)
    yf = oracle.fftols(x, filt, n_y)
    assert np.max(oracle.error_db(yf, yd)) < -240


def test_fftols_with_absent_paths_and_zero_history():
    r = rng(16)
    filt = [[None, r.standard_normal(64)], [r.standard_normal(10), None]]
    x = r.standard_normal((2, 300))
    yd = oracle.direct(x, filt, 0, 400)
    yf = oracle.fftols(x, filt, 400)
    assert np.max(np.abs(yf - yd)) < 1e-12


def test_error_db_definition():
    y = np.array([[3.0, 4.0]])
    assert oracle.error_db(y * (1 + 1e-5), y)[0] == pytest.approx(-100.0, abs=1e-6)


# ----------------------------------------------------------------------------
# Feedback-cancellation loop (Sec. III-A Eq. 3, Sec. V): mt = m - c delayed by
# one block, l = H^T * mt, c = F-hat * l
# ----------------------------------------------------------------------------

def _rand_filters(r, P, L, n, scale=0.3):
    return [[r.standard_normal(n) * scale for _ in range(L)] for _ in range(P)]


def test_feedback_loop_without_feedback_is_plain_synthesis():
    r = rng(30)
    P, L, N, B = 2, 3, 700, 16
    h = _rand_filters(r, P, L, 90)
    zero = [[np.zeros(5) for _ in range(L)] for _ in range(P)]
    m = r.standard_normal((P, N))
    l, c, mt = oracle.feedback_loop(m, h, zero, B)
    assert np.all(c == 0.0) and np.array_equal(mt, m)
    for j in range(L):
        want = sum(np.convolve(m[p], h[p][j])[:N] for p in range(P))
        assert np.max(np.abs(l[j] - want)) < 1e-11


def test_feedback_loop_gain_feedback_is_a_block_comb():
    # H = delta, F-hat = a delta: mt[t] = m[t] - a mt[t - B], so an impulse
    # gives mt[kB] = (-a)^k (exact: a = 1/2) and zero elsewhere.
    B, a, N = 4, 0.5, 64
    m = np.zeros((1, N))
    m[0, 0] = 1.0
    l, c, mt = oracle.feedback_loop(m, [[np.array([1.0])]], [[np.array([a])]], B)
    want = np.zeros(N)
    want[::B] = (-a) ** np.arange(N // B)
    assert np.array_equal(mt[0], want)
    assert np.array_equal(l[0], want)
    assert np.array_equal(c[0], a * want)


def test_feedback_loop_cancels_a_matched_room_exactly():
    # Simulated room: the microphones hear the source s plus the loudspeaker
    # signals through paths F, one block late.  With F-hat = F the loop removes
    # them: mt = s and l = H^T * s.
    r = rng(31)
    P, L, N, B = 2, 3, 600, 8
    # weak feedback paths keep the loop stable, as real ones are
    h = _rand_filters(r, P, L, 50)
    f = _rand_filters(r, P, L, 30, scale=0.01)
    s = r.standard_normal((P, N))
    l_star = np.array([sum(np.convolve(s[p], h[p][j])[:N] for p in range(P)) for j in range(L)])
    fb = np.array([sum(np.convolve(l_star[j], f[p][j])[:N] for j in range(L)) for p in range(P)])
    m = s.copy()
    m[:, B:] += fb[:, :N - B]
    l, c, mt = oracle.feedback_loop(m, h, f, B)
    assert np.max(np.abs(mt - s)) < 1e-10
    assert np.max(np.abs(l - l_star)) < 1e-10


def test_feedback_loop_is_linear_and_block_causal():
    r = rng(32)
    P, L, N, B = 1, 2, 400, 32
    h = _rand_filters(r, P, L, 70)
    f = _rand_filters(r, P, L, 40, scale=0.01)
    m1, m2 = r.standard_normal((P, N)), r.standard_normal((P, N))
    l1 = oracle.feedback_loop(m1, h, f, B)[0]
    l2 = oracle.feedback_loop(m2, h, f, B)[0]
    l12 = oracle.feedback_loop(1.5 * m1 - 0.25 * m2, h, f, B)[0]
    assert np.max(np.abs(l12 - (1.5 * l1 - 0.25 * l2))) < 1e-10
    m3 = m1.copy()
    m3[:, 5 * B:] = r.standard_normal((P, N - 5 * B))
    l3 = oracle.feedback_loop(m3, h, f, B)[0]
    assert np.array_equal(l3[:, :5 * B], l1[:, :5 * B])
    assert not np.allclose(l3[:, 5 * B:], l1[:, 5 * B:])


# ----------------------------------------------------------------------------
# Serving loop: the feedback loop when sources join and leave microphone
# slots (reading of Sec. III-A Eq. 1-3 and Sec. V for changing talkers)
# ----------------------------------------------------------------------------

def test_serve_loop_with_every_slot_always_live_is_the_feedback_loop():
    # one source per slot, live throughout, carrying that slot's filter row:
    # the plain loop (itself pinned above)
    r = rng(40)
    P, L, N, B = 3, 2, 480, 16
    h = _rand_filters(r, P, L, 60)
    f = _rand_filters(r, P, L, 25, scale=0.01)
    m = r.standard_normal((P, N))
    srcs = [(p, 0, N // B, h[p]) for p in range(P)]
    got = oracle.serve_loop(m, srcs, f, B)
    want = oracle.feedback_loop(m, h, f, B)
    for g, w in zip(got, want):
        assert np.max(np.abs(g - w)) < 1e-12


def test_serve_loop_without_feedback_is_each_source_over_its_live_blocks():
    # no feedback paths: each source's filters applied to its slot's signal
    # cut to its live blocks (numpy.convolve), summed; a source that left
    # keeps ringing through its own filters
    r = rng(41)
    Q, L, N, B = 2, 3, 640, 16
    m = r.standard_normal((Q, N))
    srcs = [(0, 2, 15, [r.standard_normal(70) for _ in range(L)]),
            (1, 0, 40, [r.standard_normal(33), None, r.standard_normal(90)]),
            (0, 22, 31, [None, r.standard_normal(120), r.standard_normal(5)])]
    l, c, mt = oracle.serve_loop(m, srcs, None, B)
    assert np.all(c == 0.0)
    want = np.zeros((L, N))
    for q, a, b, row in srcs:
        x = np.zeros(N)
        x[a * B:b * B] = m[q, a * B:b * B]
        for j in range(L):
            if row[j] is not None:
                want[j] += np.convolve(x, row[j])[:N]
    assert np.max(np.abs(l - want)) < 1e-11
    # slot 0 is dead in blocks [15, 22) and [31, 40): its input reads as zero
    assert np.all(mt[0, 15 * B:22 * B] == 0.0) and np.all(mt[0, 31 * B:] == 0.0)
    assert np.array_equal(mt[1], m[1])


def test_serve_loop_gain_feedback_comb_stops_with_the_source():
    # H = delta, F-hat = a delta, one source live in blocks [3, 7): an impulse
    # at its first sample gives mt[(3 + k) B] = (-a)^k while it is live, then
    # silence; the loudspeaker carries mt (delta filter)
    B, a, N = 4, 0.5, 48
    m = np.zeros((1, N))
    m[0, 3 * B] = 1.0
    m[0, 9 * B] = 7.0           # after the source left: ignored
    l, c, mt = oracle.serve_loop(m, [(0, 3, 7, [np.array([1.0])])], [[np.array([a])]], B)
    want = np.zeros(N)
    for k in range(4):
        want[(3 + k) * B] = (-a) ** k
    assert np.array_equal(mt[0], want)
    assert np.array_equal(l[0], want)
    assert np.array_equal(c[0], a * want)


def test_serve_loop_ignores_a_slot_signal_while_no_source_is_live():
    r = rng(42)
    Q, L, N, B = 2, 2, 320, 16
    m = r.standard_normal((Q, N))
    f = _rand_filters(r, Q, L, 20, scale=0.02)
    srcs = [(0, 0, 6, [r.standard_normal(40) for _ in range(L)]),
            (1, 4, 20, [r.standard_normal(30) for _ in range(L)]),
            (0, 12, 20, [r.standard_normal(25) for _ in range(L)])]
    base = oracle.serve_loop(m, srcs, f, B)
    m2 = m.copy()
    m2[0, 6 * B:12 * B] = 1e6 * r.standard_normal(6 * B)   # slot 0 dead there
    m2[1, :4 * B] = -3.0                                     # slot 1 dead there
    other = oracle.serve_loop(m2, srcs, f, B)
    for g, w in zip(other, base):
        assert np.array_equal(g, w)
