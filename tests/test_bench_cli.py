"""bench.py's host-side contract, on the CPU: it measures one GPU and says so
for any other count before touching a device, and the HBM traffic it attaches
to its roofline comes only from counter runs of the current kernel source in
the launch shape that was timed."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [0, 2, 8])
def test_refuses_other_gpu_counts(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_traffic_lookup_needs_the_current_source_and_the_timed_shape(tmp_path):
    entries = [{"variant": 2, "proposals_per_launch": 81920, "bytes_per_launch": 1.5e11},
               {"variant": 1, "proposals_per_launch": 81920, "bytes_per_launch": 1.4e11}]
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"source_hash": bench.kernel_source_hash(), "entries": entries}))
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"source_hash": "0" * 16, "entries": entries}))
    assert bench.measured_traffic(81920, 2, name=str(good)) == 1.5e11
    assert bench.measured_traffic(81920, 1, name=str(good)) == 1.4e11
    assert bench.measured_traffic(81920, 0, name=str(good)) is None        # variant not measured
    assert bench.measured_traffic(131072, 2, name=str(good)) is None       # other launch shape
    assert bench.measured_traffic(81920, 2, name=str(stale)) is None       # kernel changed since
    assert bench.measured_traffic(81920, 2, name=str(tmp_path / "missing.json")) is None


def test_committed_traffic_entries_add_up():
    """Each entry's bytes are the scaled counters of the timed launch (the
    last dispatch of its runs): FETCH_SIZE and WRITE_SIZE in KiB, times 1024
    and the calibration factor of a plain copy of known size (stored rounded
    to five digits, hence the tolerance)."""
    with open(os.path.join(ROOT, "profiles", "sampler_team_ferro64_traffic.json")) as fh:
        d = json.load(fh)
    assert d["entries"]
    for e in d["entries"]:
        fs = e.get("fetch_scale", d["fetch_scale"])
        ws = e.get("write_scale", d["write_scale"])
        assert e["fetch_bytes"] == pytest.approx(e["fetch_kib_raw"][-1] * 1024 * fs, rel=1e-4)
        assert e["write_bytes"] == pytest.approx(e["write_kib_raw"][-1] * 1024 * ws, rel=1e-4)
        assert e["bytes_per_launch"] == pytest.approx(e["fetch_bytes"] + e["write_bytes"], rel=1e-12)
        assert e["proposals_per_launch"] == 4096 * e["mh_steps_per_launch"]
