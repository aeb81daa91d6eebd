"""Host-side logic of bench.py: the committed counter summary is reported
as roofline traffic only for the kernel, grid and sources it was taken on."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
import pytest  # noqa: E402


def _summary():
    kv = {}
    for line in open(bench.TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_summary_matches_sources():
    kv = _summary()
    if kv["source_sha256_16"] != bench.smoother_source_hash():
        assert bench.measured_traffic(kv["kernel"], float(kv["algorithmic_bytes_per_launch"])) is None
        pytest.skip("smoother sources changed since the counters were taken (traffic reported as null)")
    alg = float(kv["algorithmic_bytes_per_launch"])
    t = bench.measured_traffic(kv["kernel"], alg)
    assert t == float(kv["hbm_bytes_per_launch"])
    assert 0.9 * alg <= t <= 1.5 * alg


def test_traffic_not_reported_for_other_grid_or_kernel():
    kv = _summary()
    if kv["source_sha256_16"] != bench.smoother_source_hash():
        pytest.skip("smoother sources changed since the counters were taken")
    alg = float(kv["algorithmic_bytes_per_launch"])
    assert bench.measured_traffic(kv["kernel"], alg * 8) is None
    assert bench.measured_traffic("some other kernel", alg) is None


def test_oracle_leg_runs_on_the_host():
    """The CPU-baseline legs run in child processes that never touch the
    GPU; at a tiny size both legs solve and report their core count."""
    import json
    import subprocess
    for kind, threads in (("vcycle", "1"), ("cg", "2")):
        env = dict(os.environ, OMP_NUM_THREADS=threads, MG_ORACLE_NATIVE="1")
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-leg", kind, "--n", "16"],
                           env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr
        leg = json.loads(r.stdout.strip().splitlines()[-1])
        assert leg["cores"] == int(threads) and leg["rel_res"] <= 1e-10 and leg["value"] > 0
