"""Host-side checks of the benchmark's command line (no GPU needed): a
request for more than one GPU ends with a message and exit status 2 before
anything touches a device, and the profile-record helpers read the
committed records."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_records_parse():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("tracking_c3_traffic.md", "tracking_c3_read_requests.md"):
        path = os.path.join(ROOT, "profiles", name)
        rec = [ln for ln in open(path) if ln.startswith("record: ")]
        assert len(rec) == 1, name
        data = json.loads(rec[0][len("record: "):])
        assert data["workload"] == "C3" and len(data["source_sha256"]) == 64
    assert len(bench.kernel_source_hash()) == 64
