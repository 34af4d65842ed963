"""Host-side logic of bench.py: the traffic figure is taken from a committed profile only
while that profile was taken on the current kernel sources, and more than one GPU is
refused before anything touches a device."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
D1 = "a" * 64
D2 = "b" * 64


def test_traffic_taken_only_at_the_recorded_digest():
    text = (f"# k\n\nsources sha256: {D1}  (...)\n  HBM bytes per dispatch (gemm_pupil_kernel): 123456\n"
            f"  trace average us (gemm_pupil_kernel): 861.25\n")
    assert bench.traffic_from_summary(text, "gemm_pupil_kernel", D1) == 123456
    assert bench.traffic_from_summary(text, "gemm_image_kernel", D1) is None
    assert bench.traffic_from_summary(text, "gemm_pupil_kernel", D2) is None
    assert bench.summary_field(text, "trace average us", "gemm_pupil_kernel", D1) == 861.25
    assert bench.summary_field(text, "trace average us", "gemm_pupil_kernel", D2) is None
    assert bench.traffic_from_summary(text.replace("HBM bytes per dispatch", "bytes"), "gemm_pupil_kernel", D1) is None
    assert bench.traffic_from_summary("no digest here", "gemm_pupil_kernel", D1) is None


def test_sources_digest_is_stable_and_hex():
    d = bench.sources_digest()
    assert d == bench.sources_digest()
    assert len(d) == 64 and all(c in "0123456789abcdef" for c in d)


def test_missing_profile_gives_no_traffic():
    assert bench.profiled_traffic("no_such_summary.txt", "gemm_pupil_kernel") is None
    assert bench.profiled_average("no_such_summary.txt", "gemm_pupil_kernel") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.lstrip().startswith("{")
