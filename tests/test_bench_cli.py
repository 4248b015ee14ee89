"""Host-side checks of bench.py's command line (no GPU needed): it refuses more than one GPU with a
message (everything here runs on one GPU), refuses the three-part BF16 split outside the batch
workload, and the roofline's profile figures are tied to the layer kernel's sources."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("n", ["2", "8"])
def test_more_than_one_gpu_is_refused(n):
    r = run_bench("--gpus", n)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bf16x3_outside_the_batch_is_refused():
    r = run_bench("--prec", "bf16x3")
    assert r.returncode == 2 and "batch1024" in r.stderr


def test_profile_figures_follow_the_kernel_sources():
    """The bench line quotes the committed rocprofv3 figures only while the layer kernel's sources
    are the ones they were taken from (the summaries record the SHA-256 of those sources)."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_08523_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    for path, tag, get in ((bench.COUNTER_SUMMARY, "traffic_json", bench.measured_traffic),
                           (bench.TRACE_SUMMARY, "trace_json", bench.measured_profile),
                           (bench.SQ_SUMMARY, "sq_json", bench.measured_pipe_busy)):
        line = next(l for l in open(path) if l.startswith(tag + ":"))
        rec = json.loads(line.split(":", 1)[1])
        if rec["source_sha256"] == h.hexdigest():
            assert get() is not None, path
        else:
            assert get() is None, path
