"""Host-side pieces of bench.py: the counter side of the roofline point and the
lookup of committed counter summaries by kernel source hash (no GPU)."""
import glob
import os
import re

import pytest

import bench


def test_traffic_point_without_counters():
    assert bench.traffic_point(None, 1.0) == {"traffic_gbps": None, "traffic_frac": None}
    assert bench.traffic_point(1e9, 0.0) == {"traffic_gbps": None, "traffic_frac": None}


def test_traffic_point_rate_and_fraction():
    # 8 GB per 1 ms launch is 8 TB/s: the whole of the 8 TB/s peak
    p = bench.traffic_point(8e9, 1.0)
    assert p["traffic_gbps"] == pytest.approx(8000.0)
    assert p["traffic_frac"] == pytest.approx(1.0)
    p = bench.traffic_point(2e9, 2.0)
    assert p["traffic_gbps"] == pytest.approx(1000.0)
    assert p["traffic_frac"] == pytest.approx(0.125)


def _summaries():
    out = []
    for path in sorted(glob.glob(os.path.join(bench.ROOT, "profiles", "*_counters.md"))):
        m = re.match(r"(k_[a-z_]+)_(.+)_counters\.md$", os.path.basename(path))
        if m:
            out.append((path, m.group(1), m.group(2)))
    return out


@pytest.mark.parametrize("path,kernel,workload", _summaries())
def test_counter_summaries_are_read_only_on_their_own_sources(path, kernel, workload):
    text = open(path).read()
    h = re.search(r"kernel_source_hash:\s*(\w+)", text).group(1)
    v = float(re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text).group(1))
    assert v > 0
    assert bench.read_traffic(kernel, workload, h) == pytest.approx(v)
    assert bench.read_traffic(kernel, workload, "0" * 16) is None
    assert bench.read_traffic(kernel, workload + "-absent", h) is None


@pytest.mark.parametrize("path,kernel,workload", _summaries())
def test_counter_summaries_are_read_only_at_their_batch_width(path, kernel, workload):
    text = open(path).read()
    m = re.search(r"--batch-width (\d+)", text)
    if not m:
        pytest.skip("summary of a kernel without batches")
    h = re.search(r"kernel_source_hash:\s*(\w+)", text).group(1)
    w = int(m.group(1))
    assert bench.read_traffic(kernel, workload, h, w) is not None
    assert bench.read_traffic(kernel, workload, h, 2 * w) is None


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused_before_any_device_work(argv, env):
    import subprocess
    import sys
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), *argv],
                       capture_output=True, text=True, env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
