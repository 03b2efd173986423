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
