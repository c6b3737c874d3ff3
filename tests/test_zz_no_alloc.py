"""rta_serve_admit_noalloc (the admission that allocates no device memory,
staging its spectra build in the library's fixed device array) against
rta_serve_admit: two admissions in a row, the second with shorter filters,
into two identical serving contexts fed the same blocks -- the outputs must
be bit-identical, and both must match the FP64 oracle (FP32 spectra,
<= -100 dB relative RMS per output)."""
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


@pytest.mark.parametrize("B,scheme", [(32, None), (16, [(16, 8), (64, 3), (256, 0)])])
def test_noalloc_admission_matches_the_allocating_one(rta, B, scheme):
    L, max_taps, n_slots, n_blocks = 4, 3000, 2, 120
    N = n_blocks * B
    fa = make_filters(90, [[3000, 1200, 0, 2500]])[0]
    fb = make_filters(91, [[700, 300, 64, 0]])[0]           # the smaller second input
    xa = workloads.white_noise(92, 1, N)[0]
    xb = workloads.white_noise(93, 1, N)[0]
    outs = []
    for noalloc in (False, True):
        with rta.Server(n_slots, L, max_taps, B, scheme=scheme) as srv:
            admit = srv.admit_noalloc if noalloc else srv.admit
            y = np.empty((L, N), np.float32)
            qa = qb = None
            for n in range(n_blocks):
                if n == 0:
                    qa = admit(fa)
                if n == 20:
                    qb = admit(fb)
                if n == 70:
                    srv.release(qa)
                blk = np.full((n_slots, B), np.nan, np.float32)
                if n < 70:
                    blk[qa] = xa[n * B:(n + 1) * B]
                if n >= 20:
                    blk[qb] = xb[n * B:(n + 1) * B]
                y[:, n * B:(n + 1) * B] = srv.process(blk)
        say(f"  B={B} scheme={scheme} noalloc={noalloc}: slots {qa}, {qb}")
        outs.append(y)
    assert np.array_equal(outs[0], outs[1]), "noalloc admission changed the output"
    x = np.zeros((2, N), np.float32)
    x[0, :70 * B] = xa[:70 * B]
    x[1, 20 * B:] = xb[20 * B:]
    ref = oracle.direct(x, [fa, fb], 0, N)
    check_db(outs[1], ref, FP32_DB, f"noalloc admissions B={B}")


def test_noalloc_admission_rejects_filters_beyond_its_array(rta):
    big = 1 << 20
    with rta.Server(1, 1, big + 1, 1024) as srv:
        with pytest.raises(rta.RtaError) as e:
            srv.admit_noalloc([np.zeros(big + 1, np.float32)])
        assert e.value.status == rta.RTA_E_ARG
        q = srv.admit_noalloc([np.ones(big, np.float32) * 1e-3])   # at the limit
        assert q == 0
