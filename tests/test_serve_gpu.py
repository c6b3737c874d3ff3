"""GPU parity of serving with continuous batching: sources are admitted into
slots and released while blocks stream, and the outputs must equal the plain
MIMO convolution (Sec. III-A Eq. 2) of every source's signal over the blocks
it was live, with its filters (the FP64 oracle; FP32 spectra <= -100 dB
relative RMS per output, FP16 <= -60 dB).  Rows of slots that are not live
carry NaN, which must never reach the output."""
import numpy as np
import pytest

import oracle
from paper_2509_04390_amd import workloads

from test_parity_gpu import FP16_DB, FP32_DB, check_db, make_filters, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rta():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2509_04390_amd import rta as mod
    return mod


def run_scenario(rta, srv, sources, events, n_blocks, retry=()):
    """sources: name -> (filters [L], signal [N]); events: block -> list of
    ("admit" | "release", name).  Names in `retry` whose admission is refused
    for capacity are tried again at every later block.  Returns the output
    [L][n_blocks * B] and name -> [slot, start, stop]."""
    B, Q, L = srv.block, srv.n_slots, srv.n_out
    y = np.empty((L, n_blocks * B), np.float32)
    slot_of, rec, waiting, refused = {}, {}, [], 0
    for n in range(n_blocks):
        todo = [("admit", w) for w in waiting] + list(events.get(n, []))
        waiting = []
        for ev, name in todo:
            if ev == "admit":
                try:
                    q = srv.admit(sources[name][0])
                except rta.RtaError as e:
                    assert e.status == rta.RTA_E_CAPACITY and name in retry, e
                    waiting.append(name)
                    refused += 1
                    continue
                slot_of[name] = q
                rec[name] = [q, n, None]
            else:
                srv.release(slot_of.pop(name))
                rec[name][2] = n
        blk = np.full((Q, B), np.nan, np.float32)
        for name, q in slot_of.items():
            blk[q] = sources[name][1][n * B:(n + 1) * B]
        y[:, n * B:(n + 1) * B] = srv.process(blk)
        if any(ev for ev in todo):
            # the library agrees on when each source started and stopped
            _, slots = srv.query()
            for name, (q, start, stop) in rec.items():
                if name in slot_of and slots[q]["state"] in ("live", "draining"):
                    assert slots[q]["start_block"] == start, (name, slots[q])
                if stop is not None and stop == n and slots[q]["state"] == "draining":
                    assert slots[q]["stop_block"] == stop, (name, slots[q])
    assert not waiting, f"never admitted: {waiting}"
    return y, rec, refused


def reference(sources, rec, L, B, N):
    names = sorted(rec)
    x = np.zeros((len(names), N), np.float32)
    filt = []
    for i, name in enumerate(names):
        _, start, stop = rec[name]
        stop = N // B if stop is None else stop
        x[i, start * B:stop * B] = sources[name][1][start * B:stop * B]
        filt.append(list(sources[name][0]))
    return oracle.direct(x, filt, 0, N)


def make_sources(seed, lens, N):
    """name -> (filters [L] with lengths lens[name], white-noise signal [N])."""
    out = {}
    for i, name in enumerate(sorted(lens)):
        f = make_filters(seed + i, [lens[name]])[0]
        out[name] = (f, workloads.white_noise(seed + 100 + i, 1, N)[0])
    return out


LENS = {"A": [1500, 300, 0, 2000], "B": [900, 2000, 1200, 64],
        "C": [2000, 2000, 2000, 2000], "D": [100, 1700, 33, 700]}


@pytest.mark.parametrize("B,scheme", [(32, None), (32, [(32, 12), (256, 0)]),
                                      (16, [(16, 8), (64, 3), (256, 0)])])
def test_admit_release_and_slot_reuse_match_oracle(rta, B, scheme):
    """Three slots: A, B, C fill them; D is refused until A, released at block
    10, has drained, then takes A's slot; B and D leave before the end."""
    L, max_taps = 4, 2000
    n_blocks = 260 if B == 16 else 200
    N = n_blocks * B
    src = make_sources(60, LENS, N)
    events = {0: [("admit", "A")], 3: [("admit", "B")], 6: [("admit", "C")],
              8: [("admit", "D")], 10: [("release", "A")], 120: [("release", "B")],
              150: [("release", "D")]}
    say(f"serve B={B} scheme={scheme}")
    with rta.Server(3, L, max_taps, B, scheme=scheme) as srv:
        y, rec, refused = run_scenario(rta, srv, src, events, n_blocks, retry=("D",))
        info, slots = srv.query()
    say(f"  {rec}, refused {refused}, swaps {info['plan_swaps']}")
    assert rec["D"][0] == rec["A"][0], "D must reuse A's slot"
    assert refused > 0 and info["rejected_slots"] == refused
    assert info["admitted"] == 4
    ref = reference(src, rec, L, B, N)
    check_db(y, ref, FP32_DB, f"serving B={B} scheme={scheme}")


def test_mix_equals_sum_of_alone_runs(rta):
    B, L = 32, 4
    n_blocks = 120
    N = n_blocks * B
    src = make_sources(70, {k: LENS[k] for k in ("A", "B")}, N)
    ev_a = {2: [("admit", "A")], 50: [("release", "A")]}
    ev_b = {7: [("admit", "B")], 90: [("release", "B")]}
    mix_ev = {2: [("admit", "A")], 7: [("admit", "B")], 50: [("release", "A")],
              90: [("release", "B")]}
    outs = []
    for ev in (ev_a, ev_b, mix_ev):
        with rta.Server(2, L, 2000, B, scheme=[(32, 12), (256, 0)]) as srv:
            outs.append(run_scenario(rta, srv, src, ev, n_blocks)[0])
    err = oracle.error_db(outs[2], outs[0].astype(np.float64) + outs[1])
    say(f"  mix vs sum of alone runs: {err.max():.1f} dB")
    assert np.all(err <= FP32_DB)


def test_admission_control(rta):
    B, L, max_taps = 32, 4, 4000
    long_f = make_filters(80, [[max_taps] * L])[0]
    short_f = make_filters(81, [[200] * L])[0]
    # arena for a little more than one max_taps source on every output
    per_src = L * (-(-max_taps // B)) * B * 8
    with rta.Server(4, L, max_taps, B, arena_bytes=int(per_src * 1.5)) as srv:
        info, _ = srv.query()
        assert info["arena_bytes"] >= per_src
        q0 = srv.admit(long_f)
        with pytest.raises(rta.RtaError) as e:
            srv.admit(long_f)
        assert e.value.status == rta.RTA_E_NOMEM
        q1 = srv.admit(short_f)          # still fits
        assert q1 != q0
        info, slots = srv.query()
        assert info["rejected_memory"] == 1 and info["admitted"] == 2
        assert info["arena_used_bytes"] == sum(
            L * (-(-n // B)) * B * 8 for n in (max_taps, 200))
        with pytest.raises(rta.RtaError) as e:   # over the maximum length
            srv.admit([np.zeros(max_taps + 1, np.float32)] + [None] * (L - 1))
        assert e.value.status == rta.RTA_E_ARG
    # bandwidth budget: room for one long source per block, not two
    with rta.Server(4, L, max_taps, B) as probe:
        probe.admit(long_f)
        one = probe.query()[0]["bytes_per_block"]
    with rta.Server(4, L, max_taps, B, budget_bytes=one * 1.5) as srv:
        srv.admit(long_f)
        with pytest.raises(rta.RtaError) as e:
            srv.admit(long_f)
        assert e.value.status == rta.RTA_E_CAPACITY
        srv.admit(short_f)
        info, _ = srv.query()
        assert info["rejected_budget"] == 1 and info["bytes_per_block"] <= one * 1.5
    # slots
    with rta.Server(1, L, max_taps, B) as srv:
        srv.admit(short_f)
        with pytest.raises(rta.RtaError) as e:
            srv.admit(short_f)
        assert e.value.status == rta.RTA_E_CAPACITY
        with pytest.raises(rta.RtaError) as e:
            srv.release(0) or srv.release(0)  # second release: not live
        assert e.value.status == rta.RTA_E_STATE


def test_reset_keeps_live_sources_and_frees_released(rta):
    B, L = 32, 4
    n_blocks = 100
    N = n_blocks * B
    src = make_sources(90, {k: LENS[k] for k in ("A", "B")}, N)
    with rta.Server(2, L, 2000, B) as srv:
        y1, rec1, _ = run_scenario(rta, srv, src, {0: [("admit", "A")], 0 + 1: [("admit", "B")],
                                                  20: [("release", "B")]}, n_blocks)
        srv.reset()
        info, slots = srv.query()
        assert info["live"] == 1 and info["free_slots"] == 1
        qa = rec1["A"][0]
        assert slots[qa]["state"] == "live" and slots[qa]["start_block"] == 0
        # after the reset A is live from block 0 again, with zero history
        blk_src = {"A": src["A"]}
        y2 = np.empty((L, N), np.float32)
        for n in range(n_blocks):
            blk = np.full((2, B), np.nan, np.float32)
            blk[qa] = blk_src["A"][1][n * B:(n + 1) * B]
            y2[:, n * B:(n + 1) * B] = srv.process(blk)
    ref = reference(blk_src, {"A": [qa, 0, None]}, L, B, N)
    check_db(y2, ref, FP32_DB, "serving after reset")


def test_serve_workload_fp16_sampled(rta):
    """16 slots -> 64 outputs, 12 s filters, block 64, FP16 spectra: three
    sources join at different blocks and one leaves; sampled outputs against
    the oracle."""
    wl = workloads.config("serve")
    B, L, taps = wl.block, wl.n_out, wl.lengths
    n_blocks = 400
    N = n_blocks * B
    src = {}
    for i, name in enumerate("XYZ"):
        f = workloads.reverb_filters(wl.seed + i, 1, L, taps, wl.rt60)[0]
        src[name] = (f, workloads.white_noise(wl.seed + 50 + i, 1, N)[0])
    events = {0: [("admit", "X")], 37: [("admit", "Y")], 101: [("admit", "Z")],
              250: [("release", "X")]}
    say(f"serve workload: 16 slots x {L} outputs, {taps} taps, B={B}, fp16")
    with rta.Server(16, L, taps, B, spectra="fp16") as srv:
        y, rec, _ = run_scenario(rta, srv, src, events, n_blocks)
        info, _ = srv.query()
        say(f"  arena {info['arena_bytes'] / 1e9:.2f} GB, used {info['arena_used_bytes'] / 1e9:.2f} GB,"
            f" {info['bytes_per_block'] / 1e6:.1f} MB/block")
    rng = np.random.default_rng(5)
    idx = np.unique(np.r_[0, 63, 64, 37 * B - 1, 37 * B, 101 * B, 250 * B - 1, 250 * B,
                          250 * B + 1, N - 1, rng.integers(0, N, 40)])
    names = sorted(rec)
    x = np.zeros((len(names), N), np.float32)
    for i, name in enumerate(names):
        _, start, stop = rec[name]
        stop = n_blocks if stop is None else stop
        x[i, start * B:stop * B] = src[name][1][start * B:stop * B]
    ref = oracle.direct_at(x, [list(src[n][0]) for n in names], idx)
    check_db(y[:, idx], ref, FP16_DB, "serve workload fp16")


def weak(filters, scale):
    return [None if f is None else (f * scale).astype(np.float32) for f in filters]


@pytest.mark.parametrize("B,scheme,spectra,limit", [
    (32, None, "fp32", FP32_DB),
    (16, [(16, 8), (64, 3), (256, 0)], "fp32", FP32_DB),
    (32, None, "fp16", FP16_DB)])
def test_serving_with_feedback_cancellation_matches_oracle(rta, B, scheme, spectra, limit):
    """Feedback paths fixed per slot (microphone) on a serving context: sources
    join and leave while each slot's input is its microphone minus the
    previous block's estimate, and zero while no source is live in it.
    Against the oracle's serving loop (FP64, block-recursive)."""
    L, max_taps, n_slots = 4, 2000, 3
    n_blocks = 200
    N = n_blocks * B
    src = make_sources(80, LENS, N)
    src = {k: (weak(v[0], 0.1), v[1]) for k, v in src.items()}
    rng = np.random.default_rng(81)
    fb = [[(0.001 * rng.standard_normal(300) * np.exp(-np.arange(300) / 80.0)).astype(np.float32)
           for _ in range(L)] for _ in range(n_slots)]
    events = {0: [("admit", "A")], 3: [("admit", "B")], 6: [("admit", "C")],
              8: [("admit", "D")], 10: [("release", "A")], 120: [("release", "B")],
              150: [("release", "D")]}
    say(f"serve + feedback B={B} scheme={scheme} {spectra}")
    with rta.Server(n_slots, L, max_taps, B, scheme=scheme, spectra=spectra) as srv:
        srv.set_feedback(fb, spectra=spectra)
        info = srv.info()
        assert info["feedback_paths"] == 1 and info["feedback_fused"] == 1
        y, rec, refused = run_scenario(rta, srv, src, events, n_blocks, retry=("D",))
    m = np.zeros((n_slots, N), np.float32)
    sources = []
    for name, (q, start, stop) in sorted(rec.items()):
        stop = n_blocks if stop is None else stop
        m[q, start * B:stop * B] = src[name][1][start * B:stop * B]
        sources.append((q, start, stop, src[name][0]))
    l_ref, c_ref, mt_ref = oracle.serve_loop(m, sources, fb, B)
    live = np.sum(mt_ref ** 2, axis=1) > 0
    g = np.sqrt(np.sum(c_ref[live] ** 2, axis=1) / np.sum(mt_ref[live] ** 2, axis=1)).max()
    bound = limit + 10.0 * np.log10(1.0 + g * g)
    say(f"  {rec}; |c| / |m - c| = {g:.3f}, bound {bound:.1f} dB")
    assert g > 0.01, "the feedback estimate must matter"
    check_db(y, l_ref, bound, f"serving + feedback B={B} {spectra}")
