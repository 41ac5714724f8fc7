"""The in/out index's host build and lookup (the same header the kernels
include, compiled for the host) against brute-force membership: the
address's position among the union's boundaries (Algorithm 1's in/out mark
over the whole prefix list is membership in the union of the prefixes)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_inout_index_host_lookup_vs_brute_force():
    tmp = tempfile.mkdtemp(prefix="sinet_io_")
    try:
        exe = os.path.join(tmp, "check")
        r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-I",
                            os.path.join(ROOT, "paper_2106_12863_amd", "csrc"),
                            os.path.join(ROOT, "tests", "inout_index_check.cpp"), "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout[-2000:]
        assert "bad 0" in r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
