"""Host logic of bench.py (no GPU): the crossover-thickness interpolation, the algorithmic FLOP
counts the roofline divides by, the guard that drops the counter-measured traffic once the
kernel sources change, and the refusal of runs on more than one GPU."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_tau_star_is_exact_for_a_power_law(bench):
    # an analog rate a(tau) = A tau^-p is a straight line in log-log coordinates, so the
    # interpolation between measured points must return the exact crossing tau* = (A / r)^(1/p)
    A, pw = 3.0e9, 1.7
    table = {str(int(t)): A * t ** -pw for t in (1, 10, 100, 300, 1000)}
    for r in (A * 50.0 ** -pw, A * 200.0 ** -pw, A * 777.0 ** -pw):
        want = (A / r) ** (1.0 / pw)
        assert bench.tau_star(r, table) == pytest.approx(want, rel=1e-12)


def test_tau_star_range_ends(bench):
    table = {"1": 1e9, "10": 5e8, "100": 1e8}
    assert bench.tau_star(2e9, table) == 1.0          # faster than the walk everywhere
    assert bench.tau_star(1e7, table) is None         # slower over the whole range
    assert bench.tau_star(5e8, table) == pytest.approx(10.0, rel=1e-12)


def test_flop_counts(bench):
    # 2 (10 H + 3 H^2 + 5 H) per evaluation of the plain network
    assert bench.flops_per_sample(512, 1) == 1_588_224
    assert bench.flops_per_sample(256, 1) == 400_896
    assert bench.flops_per_sample(512, 16) == 16 * 1_588_224
    # residual network: input layer over 17 features, embedding 32 over 12, three blocks of an
    # H x H map and two 32 -> H modulation maps, output layer
    H, E = 512, 32
    want = 2 * (H * 17 + E * 12 + 3 * (H * H + 2 * H * E) + 5 * H)
    assert bench.film_flops_per_sample(512, 1) == want == 1_792_768


def test_traffic_is_dropped_when_the_sources_change(bench, tmp_path, monkeypatch):
    good = tmp_path / "good.md"
    good.write_text(f"traffic_source_sha256: {bench.kernel_source_hash()}\ntraffic_bytes_per_launch: 123.5\n")
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_source_sha256: " + "0" * 64 + "\ntraffic_bytes_per_launch: 123.5\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(good))
    assert bench.measured_traffic() == 123.5
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
