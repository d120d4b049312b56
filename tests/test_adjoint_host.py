"""CPU check of the library's per-site reverse-mode functions: each
vector-Jacobian product (molecular field, stress, Beris-Edwards rate,
collision) against central finite differences of the library's own forward
functions, compiled for the host (no GPU needed)."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_per_site_vjps_match_finite_differences():
    src = os.path.join(ROOT, "tests", "native", "adjoint_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "adjoint_check")
        subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
                        "-I" + os.path.join(ROOT, "include"), src, "-o", exe], check=True,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
