"""Host-side contract of bench.py (CPU only): the one-GPU guard, and the
HBM-traffic figures it reports for the dominant Jacobi kernels, which must
belong to the kernel source in the tree."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_files_match_the_kernel_source():
    """The counter-derived traffic of each Jacobi kernel is reported only while
    the source it was measured on is the one in the tree; the committed files
    are that measurement (so the bench line carries a traffic figure), with a
    fetch and a write part of the size the kernels' algorithmic bytes imply
    (the pair kernel reads 32 m 8 bytes per pair, ~48 MB per launch on the
    headline workload, and writes 8 KB per pair)."""
    for kernel in ("jacobi_pair", "jacobi_rotate"):
        path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{bench.WORKLOAD}.txt")
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        src = open(os.path.join(ROOT, fields["source"]), "rb").read()
        assert fields["source_sha256"] == hashlib.sha256(src).hexdigest(), kernel
        t = bench.measured_traffic(kernel)
        assert t == float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])
    pair = bench.measured_traffic("jacobi_pair")
    assert 30e6 < pair < 60e6
