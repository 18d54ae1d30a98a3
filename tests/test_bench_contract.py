"""Host-side checks of the benchmark's command line: it runs on one GPU only
and says so in its one JSON line when asked for more."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_bench_traffic_records_name_existing_sources():
    """Every measured-traffic record names a kernel source of the package (the
    bench reports a record's traffic only while that source's hash matches)."""
    sys.path.insert(0, ROOT)
    import bench
    for rec in bench.MEASURED_TRAFFIC.values():
        assert os.path.isfile(os.path.join(ROOT, "paper_1712_05384_amd", "csrc", rec["source"]))
        assert len(rec["sha256_16"]) == 16 and rec["bytes_per_launch"] > 0
