"""The benchmark run exactly as it is invoked for the record (one GPU, 20
timed steps after 5 warm-up steps), in-process: it must print one JSON line
with a positive roofline fraction, the cache-defeating roofline leg, and a
CPU baseline whose comparison of the GPU output against the oracle meets the
FP32 bound."""
import json

import pytest

pytestmark = pytest.mark.gpu


def test_bench_with_the_recording_arguments(capsys):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import bench
    rc = bench.main(["--gpus", "1", "--steps", "20", "--warmup", "5",
                     "--paced-blocks", "50", "--latency-blocks", "50"])
    assert rc == 0
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    res = json.loads(lines[0])
    print(json.dumps({k: res[k] for k in ("value", "ms_per_step", "roofline")}), flush=True)
    assert res["steps"] == 20 and res["warmup"] == 5 and res["n_gpus"] == 1
    assert res["value"] > 1.0
    assert res["roofline"]["frac"] > 0.0
    assert res["roofline"]["achieved"] > 0.0
    # the cache-defeating leg: main's 123 MB of FP32 spectra need 4 contexts
    # (1.5 x the 256 MB Infinity Cache), and can only be slower per block
    honest = res["roofline_hbm_honest"]
    assert honest["contexts"] >= 3 and honest["working_set_bytes"] >= 1.5 * (256 << 20)
    assert 0.0 < honest["frac"] <= res["roofline"]["frac"] * 1.05
    cpu = res["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["value"] > 0
    assert cpu["wall_s"] > 0 and cpu["channel_filter_seconds_per_s"] > 0
    assert 0 < cpu["one_thread"]["value"] <= cpu["value"] * 1.5
    assert cpu["gpu_error_db"]["max"] <= -100.0
    assert cpu["gpu_error_db"]["samples"] == 2000 * 128
