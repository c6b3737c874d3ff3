"""Graph replay (rta_graph_create / rta_graph_launch) and the tuning cache
(rta_autotune_cached) on the GPU.  A replayed run of blocks must give the
same output, bit for bit, as the same blocks launched one at a time with
rta_process_device (Sec. IV's per-block steps, unchanged), and both must
match the FP64 oracle (Sec. III-A Eq. 2) within the FP32 bound."""
import numpy as np
import pytest

import oracle

from test_parity_gpu import FP32_DB, check_db, make_filters, padded_signal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rta():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2509_04390_amd import rta as mod
    return mod


def blocks_of(x, B):
    import torch
    Q, n = x.shape
    nb = n // B
    return torch.from_numpy(np.ascontiguousarray(
        x[:, :nb * B].reshape(Q, nb, B).transpose(1, 0, 2))).cuda()


def to_signal(yb):
    nb, L, B = yb.shape
    return yb.permute(1, 0, 2).reshape(L, nb * B).cpu().numpy()


def direct(cv, xb):
    import torch
    yb = torch.empty((xb.shape[0], cv.n_out, cv.block), dtype=torch.float32, device="cuda")
    for b in range(xb.shape[0]):
        cv.process_device(xb[b], yb[b])
    torch.cuda.synchronize()
    return yb


# (name, B, scheme, lens[q][l], feedback gain or None, flags)
CASES = [
    ("uniform Q=2 L=3", 32, None, [[3000, 1200, 0], [800, 2600, 300]], None, 0),
    ("nupc 16/64/256", 16, [(16, 8), (64, 3), (256, 0)], [[3000, 700, 161]], None, 0),
    ("uniform + fused feedback", 32, None, [[2500, 900, 1700], [1300, 0, 2100]], 0.02, 0),
    ("n_f=3B + fused feedback", 32, None, [[2500, 900, 1700], [1300, 0, 2100]], 0.02, 2),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_graph_replay_equals_direct_launches(rta, case):
    import torch
    name, B, scheme, lens, fb_gain, flags = CASES[case]
    Q, L = len(lens), len(lens[0])
    filt = make_filters(500 + case, lens)
    say(f"graph case {name}: B={B} scheme={scheme}")
    with rta.Convolver(filt, B, scheme=scheme, flags=flags) as cv:
        if fb_gain is not None:
            fb = make_filters(512, [[500, 300, 700], [0, 650, 200]])
            fb = [[None if f is None else (f * fb_gain).astype(np.float32) for f in row]
                  for row in fb]
            cv.set_feedback(fb)
            assert cv.info()["feedback_fused"] == 1
        nph = cv.info()["n_phases"]
        M = nph if nph >= 8 else 8 * nph
        # replay, replay, nph direct blocks, replay, replay, then direct to the end
        nb_total = 4 * M + nph + 3 * M
        x = padded_signal(520 + case, Q, nb_total, B, 0)
        xb = blocks_of(x, B)
        ref = direct(cv, xb)
        cv.reset()
        gin = torch.empty((M, Q, B), dtype=torch.float32, device="cuda")
        gout = torch.empty((M, L, B), dtype=torch.float32, device="cuda")
        yb = torch.empty_like(ref)
        with cv.graph(gin, gout, M) as g:
            pos = 0
            plan = ["g", "g", "d", "g", "g", "rest"]
            for step in plan:
                if step == "g":
                    gin.copy_(xb[pos:pos + M])
                    g.launch()
                    yb[pos:pos + M].copy_(gout)
                    torch.cuda.synchronize()
                    got, want = yb[pos:pos + M], ref[pos:pos + M]
                    assert torch.equal(got, want), f"{name}: replay at block {pos} differs"
                    pos += M
                elif step == "d":
                    for b in range(pos, pos + nph):
                        cv.process_device(xb[b], yb[b])
                    pos += nph
                else:
                    for b in range(pos, nb_total):
                        cv.process_device(xb[b], yb[b])
                    pos = nb_total
            torch.cuda.synchronize()
        assert torch.equal(yb, ref), f"{name}: graph + direct run differs from direct launches"
        assert cv.info()["blocks_done"] == nb_total
    y = to_signal(yb)
    if fb_gain is None:
        ref_y = oracle.direct(x, filt, 0, x.shape[1])
    else:
        ref_y = oracle.feedback_loop(x, filt, fb, B)[0]
    check_db(y, ref_y, FP32_DB, f"graph {name}")


def test_graph_launch_checks_phase_and_configuration(rta):
    import torch
    B, scheme, lens = 16, [(16, 8), (64, 3), (256, 0)], [[3000, 700]]
    filt = make_filters(530, lens)
    with rta.Convolver(filt, B, scheme=scheme) as cv:
        nph = cv.info()["n_phases"]
        gin = torch.zeros((nph, 1, B), dtype=torch.float32, device="cuda")
        gout = torch.empty((nph, 2, B), dtype=torch.float32, device="cuda")
        with pytest.raises(rta.RtaError) as e:
            rta.rta_graph_create(cv.ctx, gin.data_ptr(), gout.data_ptr(), nph + 1)
        assert e.value.status == rta.RTA_E_ARG
        with cv.graph(gin, gout, nph) as g:
            cv.process_device(gin[0], gout[0])  # one block: out of phase
            with pytest.raises(rta.RtaError) as e:
                g.launch()
            assert e.value.status == rta.RTA_E_STATE
            for b in range(1, nph):
                cv.process_device(gin[b], gout[b])
            g.launch()  # back in phase
            torch.cuda.synchronize()
            cv.set_feedback([[np.ones(10, np.float32)] * 2])  # reconfigures the launches
            with pytest.raises(rta.RtaError) as e:
                g.launch()
            assert e.value.status == rta.RTA_E_STATE


def test_autotune_cache_round_trip(rta, tmp_path):
    B = 64
    lens = [[4000, 2500]]
    filt = make_filters(540, lens)
    path = str(tmp_path / "tuning.jsonl")
    t1, s1, us1, hit1 = rta.rta_autotune_cached(path, 48000.0, B, None, 1, 2, filt, blocks=8)
    assert not hit1 and us1 > 0
    t2, s2, us2, hit2 = rta.rta_autotune_cached(path, 48000.0, B, None, 1, 2, filt, blocks=8)
    assert hit2 and s2 == s1 and abs(us2 - us1) < 1e-3
    for f in ("outputs_per_group", "tail_items", "tail_rows", "tier_rows", "bin_slices"):
        assert getattr(t1, f) == getattr(t2, f), f
    with open(path) as fh:
        assert len(fh.readlines()) == 1
    say(f"  cached tuning: scheme {s2}, G={t2.outputs_per_group}, {us2:.1f} us")
    x = padded_signal(541, 1, 20, B, 4000)
    with rta.Convolver(filt, B, scheme=None if len(s2) == 1 else s2, tuning=t2) as cv:
        y = cv.run(x)
    check_db(y, oracle.direct(x, filt, 0, x.shape[1]), FP32_DB, "cached tuning")
