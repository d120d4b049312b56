"""CPU check of the arithmetic of the float form with stochastic rounding,
compiled for the host from the library's per-site header (no GPU needed):
the stochastic rounding of the Q update is unbiased and moves a Q whose
increments lie below half a unit in the last place, the per-site uniform
numbers are uniform, and the bulk part of the molecular field (Eq. 4) is
its exact value for the float Q rounded once."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stochastic_rounding_arithmetic():
    src = os.path.join(ROOT, "tests", "native", "sr_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sr_check")
        subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                        "-ffp-contract=on", "-I" + os.path.join(ROOT, "include"), src, "-o", exe], check=True,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
