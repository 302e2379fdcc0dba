"""bench.py's command-line contract and its link to the committed profiles
(no GPU needed)."""

import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("workload,source", [
    ("erk5_u5_nx8192_nt65536_m8_fp32relax", "relax_kernels.h"),
    ("erk3_u3_nx4096_nt16384_m8_fcycle", "relax_kernels.h"),
    ("sdirk3_u3_nx2048_nt8192_m16_2level", "sdirk_pf_kernels.h"),
    ("erk3_u3_inflow_nx4096_nt16384_m8_vcycle", "bounded_kernels.h"),
])
def test_committed_counters_match_the_kernel_sources(workload, source):
    # the HBM byte counters in profiles/ were taken from the current kernel
    # source (else bench.py reports traffic as null)
    import bench
    src = os.path.join(ROOT, "paper_1910_03726_amd", "csrc", source)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    text = open(os.path.join(ROOT, "profiles", f"{workload}_hbm_counters.txt")).read()
    assert f"kernel source ({source}) sha256[:16]: {sha}" in text
    t = bench.measured_traffic(workload, source)
    assert t is not None and 1e7 < t < 1e10
    # and a mismatching source gives no traffic
    assert bench.measured_traffic(workload, "spectral.hip") is None
