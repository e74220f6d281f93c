"""CPU check of the adjoint building blocks (paper_2603_12185_amd/csrc/cf_adjoint.h):
every vector-Jacobian product of the free-body step (prediction, correction and
integration, one contact's facet impulses and wrench for condim 1/3/4/6, sphere
pair and plane-point geometry with body-pose adjoints), instantiated in float64
on the host, against central differences of its own forward piece."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "adjoint_host.hip")


def test_adjoint_pieces_match_central_differences(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "adjoint_host")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", SRC, "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
