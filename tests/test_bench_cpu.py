"""Host-side behaviour of the benchmark that needs no GPU."""
import bench


def test_bench_refuses_more_than_one_gpu():
    assert bench.main(["--gpus", "2"]) == 2


def test_host_cpu_reports_model_and_cores():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and isinstance(h["model"], str)
