"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte
counts it divides by, and the rule that counter traffic is reported only for
the kernel sources and launch it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_count_each_array_once():
    """The compulsory bytes of one pass, whatever kernels it runs in: 4 B per
    follower id; per user row_ptr 4 and, in FP64, z, c, μ, 1/den, s_new (8 B
    each) — the factored pass's 4M + 44N — or the weighted pass's 12M + 28N."""
    n, m = 1000, 20000
    assert bench.algorithmic_bytes("step64", n, m) == 4 * m + 44 * n
    for k in ("part64", "band64", "bins64"):  # the gather kernel(s) carry the pass's bytes
        assert bench.algorithmic_bytes(k, n, m) == bench.algorithmic_bytes("step64", n, m)
    assert bench.algorithmic_bytes("step64_w", n, m) == 12 * m + 28 * n
    assert bench.algorithmic_bytes("final64", n, m) == 4 * m + (4 + 4 * 8) * n
    assert bench.algorithmic_bytes("step32", n, m) == 4 * m + 32 * n
    assert bench.algorithmic_bytes("band32", n, m) < bench.algorithmic_bytes("band64", n, m)
    assert bench.algorithmic_bytes("bins32", n, m) == bench.algorithmic_bytes("step32", n, m)


def test_batched_bytes_read_the_pattern_once():
    """One pass over K scenarios reads col and row_ptr once and, per user and
    scenario, five FP64 (step) or five FP32 (correction) vectors."""
    n, m, k = 1000, 20000, 64
    assert bench.batched_bytes("scen64", n, m, 1) == bench.algorithmic_bytes("step64", n, m)
    assert bench.batched_bytes("scen32", n, m, k) == 4 * m + 4 * n + 20 * k * n
    assert bench.batched_bytes("scen64", n, m, k) - bench.batched_bytes("scen64", n, m, k - 1) == 40 * n


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    h = bench.source_hash()
    rec = {"source_hash": h, "kernel": "k_slices<4>",
           "algorithmic_bytes": 123, "hbm_bytes_per_launch": 456.0}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_part64_wl.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.traffic_from_profile("part64", "wl", "k_slices<4>", 123) == 456.0
    assert bench.traffic_from_profile("part64", "wl", "k_slices<5>", 123) is None
    assert bench.traffic_from_profile("part64", "wl", "k_slices<4>", 124) is None
    assert bench.traffic_from_profile("part64", "other", "k_slices<4>", 123) is None
    (prof / "traffic_part64_wl.json").write_text(json.dumps(dict(rec, source_hash="0" * 16)))
    assert bench.traffic_from_profile("part64", "wl", "k_slices<4>", 123) is None


def test_bench_descriptions_match_the_generator():
    """The workload text bench.py prints in `config` states the generator's
    own parameters (sizes, degree, exponent, activity spread, tolerance)."""
    import synth
    for name, text in bench.DESCRIPTIONS.items():
        w = synth.WORKLOADS[name]
        if w.get("kind") == "multi":
            assert f"{w['n_graphs']} directed Chung-Lu graphs" in text
            assert f"[{w['n_lo']:,}, {w['n_hi']:,}]" in text
        else:
            assert f"N={w['n']:,}" in text, name
        assert f"mean degree {w['mean_degree']}" in text, name
        assert f"exponent {w['gamma']}" in text, name
        sig = f"{w['sigma']:g}" if w["sigma"] != int(w["sigma"]) else f"{int(w['sigma'])}"
        assert f"LogNormal(0,{sig})" in text, name
        assert f"tol {w['tol']:.0e}".replace("e-0", "e-") in text, name
        if "d_max" in w:
            assert f"max followers {w['d_max']:,}" in text
        if "scenarios" in w:
            assert text.startswith(f"{w['scenarios']} activity scenarios")
