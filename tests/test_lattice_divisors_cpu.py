"""The kernels decode a lattice index into block coordinates with a
multiply-shift in place of two integer divisions (Lattice::div_m in
tsdf_internal.hpp).  A host program built from the same header checks it
against integer division for every lattice extent up to 70 000 blocks and
for large ones, over indices up to 2^31 - 1."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multiply_shift_equals_division(tmp_path):
    exe = tmp_path / "lattice_div"
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2311_00626_amd", "csrc"),
                    os.path.join(ROOT, "tests", "lattice_div_driver.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    n = int(out.stdout.split()[0])
    assert n > 8_000_000 and out.stdout.split()[2] == "0", out.stdout
