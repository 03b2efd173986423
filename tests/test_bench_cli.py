"""bench.py's command-line contract (CPU): more than one GPU is refused with
a message, and the serving schedule is a fixed function of its seed."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_serve_schedule_is_seeded_and_shaped():
    import bench
    a = bench.serve_schedule(bench.SERVE)
    b = bench.serve_schedule(bench.SERVE)
    assert a == b and len(a) == 128
    assert all(q["N"] in (4000, 8000, 12000, 16000, 20000) for q in a)
    assert all(30 <= q["nev"] <= 150 and q["nex"] == int(0.4 * q["nev"] + 0.5) for q in a)
    t = [q["t"] for q in a]
    assert t[0] == 0.0 and all(x <= y for x, y in zip(t, t[1:]))
    # mean gap close to 1/4 s (Poisson at 4 per second)
    assert 0.15 < t[-1] / (len(t) - 1) < 0.35


def _info(**kw):
    base = dict(filter_flops=0.0, t_filter_kernels=0.0, filter_launches=0, t_filter=1.0,
                matvecs_filter=0, matvecs_filter_fp32=0, t_filter32_kernels=0.0,
                filter32_launches=0, gemm_time=0.0, gemm_flops=0.0, gemm_launches=0,
                t_shadow=0.0, t_lanczos=0.1, t_qr=0.1, t_rr=0.1, t_resid=0.1, t_total=1.5,
                lanczos_flops=1.0, lanczos_bytes=1.0, filter_bytes=1.0, qr_flops=1.0,
                qr_bytes=1.0, rr_flops=1.0, rr_bytes=1.0, resid_flops=1.0, resid_bytes=1.0)
    base.update(kw)
    return base


def test_kernel_roofline_reports_the_dominant_kernel_and_gates_traffic():
    import bench
    N = 24000
    unit = 8.0 * N * N
    # FP64 launches dominate: achieved = flops / summed launch time.
    i64 = _info(gemm_time=2.0, gemm_flops=unit * 20000, gemm_launches=200,
                matvecs_filter=20000, filter_flops=unit * 20000, t_filter_kernels=2.0)
    S, roof, phase, phases, a64, a32 = bench.kernel_roofline([i64], N, "planted24k")
    assert roof["kernel"].startswith("k_filter ") and roof["unit"] == "TFLOP/s"
    assert abs(roof["achieved"] - unit * 20000 / 2.0 / 1e12) < 1e-9
    assert abs(roof["frac"] - roof["achieved"] / bench.FP64_PEAK_TFLOPS) < 1e-12
    assert roof["avg_launch_ms"] == 10.0
    # The committed planted N = 24000 record matches the kernel sources, so
    # its traffic is reported; an unprofiled workload reports none.
    assert roof["traffic"] is not None and roof["traffic"] > 16.0 * N * N
    assert bench.kernel_roofline([i64], N, "no-such-workload")[1]["traffic"] is None
    # FP32 launches dominate.
    i32 = _info(gemm_time=1.0, gemm_flops=unit * 100, gemm_launches=10,
                matvecs_filter=30000, matvecs_filter_fp32=25000, t_filter32_kernels=3.0,
                filter32_launches=300, filter_flops=unit * 30000, t_filter_kernels=1.0)
    roof32 = bench.kernel_roofline([i32], N, "planted24k")[1]
    assert roof32["kernel"].startswith("k_filter32") and roof32["peak"] == bench.FP32_PEAK_TFLOPS
    assert abs(roof32["achieved"] - unit * 25000 / 3.0 / 1e12) < 1e-9
    assert roof32["traffic"] is None          # no FP32 record for that workload


def test_serve_roofline_is_flops_over_the_makespan():
    import bench

    class R:
        def __init__(self, info):
            self.info = info
    info = dict(gemm_flops=4e15, gemm_time=100.0, gemm_launches=50, matvecs_filter_fp32=0,
                t_filter32_kernels=0.0, filter32_launches=0)
    done = [({"N": 8000}, R(info), 0.0), ({"N": 4000}, R(info), 0.0)]
    roof = bench.serve_roofline(done, makespan=100.0)
    assert roof["kernel"].startswith("k_filter ")
    assert abs(roof["achieved"] - 8e15 / 100.0 / 1e12) < 1e-9
    assert abs(roof["per_launch_tflops_while_sharing"] - 8e15 / 200.0 / 1e12) < 1e-9
    assert roof["launches"] == 100


def test_cpu_baseline_is_marked_extrapolated_with_fit_points():
    """The oracle timed on a bounded sample: a value scaled past the sample
    says so, and carries the three measured fit points and their exponent."""
    import bench
    w = dict(kind="dk", N=24000, nev=20, std=0.02, decay=200.0)
    out = bench.cpu_baseline(w, 0, budget_s=0.3)
    assert out["kind"] == "oracle" and out["extrapolated"] is True
    pts = out["fit_points_n_s"]
    assert len(pts) == 3 and pts[0][0] < pts[1][0] < pts[2][0] < 24000
    assert all(t > 0 for _, t in pts)
    n_s, t_s = pts[-1]
    assert abs(out["value"] - t_s * (24000 / n_s) ** 3) <= 1e-9 * out["value"]
    assert 1.0 < out["fit_exponent"] < 4.5
    assert "not measured" in out["sample"]
