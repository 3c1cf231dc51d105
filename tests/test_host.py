"""Host-side logic that needs no GPU: the benchmark's command-line contract
and the closure's input standardisation."""
import json
import os
import subprocess
import sys

import numpy as np

from paper_2102_12559_amd import closure

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_standardize_floors_constant_features():
    rng = np.random.default_rng(0)
    X = np.stack([rng.normal(1.0, 0.1, 1000), np.full(1000, 1.0),
                  1e-9 * rng.normal(size=1000)], axis=1)
    Y = rng.normal(size=(1000, 2))
    xm, xs, ym, ys = closure.standardize(X, Y)
    assert abs(xs[0] - 0.1) < 0.01
    assert xs[1] == closure.XSTD_FLOOR and xs[2] == closure.XSTD_FLOOR
    # a change of 1e-3 in a feature that never varied in training stays bounded
    z = np.clip((np.array([1.0, 1.0 + 1e-3, 1e-3]) - xm) / xs, -closure.XCLIP, closure.XCLIP)
    assert np.all(np.abs(z) <= closure.XCLIP)


def test_init_params_glorot_range():
    p = closure.init_params(10, 64, 27, seed=3)
    F, H, O = 10, 64, 27
    w1 = p[:F * H]
    assert np.max(np.abs(w1)) <= np.sqrt(6.0 / (F + H)) + 1e-7
    b1 = p[F * H:F * H + H]
    assert np.all(b1 == 0)
    assert p.size == F * H + H + H * H + H + H * O + O


def test_profile_period_is_coprime_with_the_criterion_period():
    import bench
    for steps in (100, 200, 400, 2000, 20000):
        p = bench.profile_every(steps)
        assert p >= 1
        if p > 1:
            assert p % 2 == 1 and p % 5 != 0   # coprime with 20
        assert steps // p >= 15 or p == 1   # enough sampled steps


def test_roofline_of_takes_the_dominant_stream_collide_class():
    import bench
    prof = {
        "ghost_fill": dict(launches=10, ms=5.0, bytes=0.0, cells=0.0),
        "stream_collide_low": dict(launches=10, ms=2.0, bytes=10 * 72e6, cells=1e7),
        "stream_collide_high": dict(launches=10, ms=3.0, bytes=10 * 288e5, cells=1e5),
        "band_convert": dict(launches=10, ms=1.0, bytes=0.0, cells=0.0),
    }
    r = bench.roofline_of(prof, "no-such-workload")
    assert r["kernel"] == "stream_collide_high"          # largest stream-collide time
    assert abs(r["avg_launch_us"] - 300.0) < 1e-9
    assert abs(r["achieved"] - 288e5 / 300e-6 / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4
    assert r["traffic"] is None                          # no counter summary for it



def test_traffic_summary_attaches_by_launch_class(tmp_path, monkeypatch):
    """A counter summary holds one entry per launch class; it is attached only
    to the class it measured and only while the kernel sources hash to the
    value it was taken on."""
    import bench
    prof_dir = tmp_path / "profiles"
    prof_dir.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h-now")
    d = {"kernel_source_hash": "h-now",
         "launches": {"stream_collide_low": {"kernel": "k", "hbm_bytes_per_launch": 123}}}
    (prof_dir / "traffic_w.json").write_text(json.dumps(d))
    assert bench.traffic_for("w", "stream_collide_low") == 123
    assert bench.traffic_for("w", "stream_collide_high") is None
    assert bench.traffic_for("other", "stream_collide_low") is None
    d["kernel_source_hash"] = "h-then"
    (prof_dir / "traffic_w.json").write_text(json.dumps(d))
    assert bench.traffic_for("w", "stream_collide_low") is None
