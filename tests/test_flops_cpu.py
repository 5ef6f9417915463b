"""Operation count of the interior-face fluxes, RTLBFS and TLBFS (compiled for
the host from the GPU library's own source with a counting number type).
These counts are the per-face part of the algorithmic flops per cell-update
used for the ALU roofline.  Multiplications by the compile-time lattice
components +-1 are counted as written (the compiler folds them)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXPECTED = {"2d_plain": 407, "2d_dev": 428, "3d_plain": 840, "3d_dev": 871,
            "tlbfs_2d_plain": 414, "tlbfs_2d_dev": 533, "tlbfs_3d_plain": 953, "tlbfs_3d_dev": 1188,
            # one interior face of a body-fitted mesh: frame rotation and tangential shift of both
            # sides, the flux, the rotation back and the area weighting
            "curv_2d_plain": 523, "curv_2d_dev": 545, "curv_tlbfs_2d_plain": 530, "curv_tlbfs_2d_dev": 650}


@pytest.fixture(scope="module")
def counts(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("flops") / "flop_count")
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_2202_13449_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "flop_count.hip"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.strip().splitlines():
        name, a, m, d = line.split()
        res[name] = (int(a), int(m), int(d))
    return res


def test_face_flux_operation_counts(counts):
    for name, total in EXPECTED.items():
        a, m, d = counts[name]
        assert d == 1  # one division per face: 1 / rho*
        assert a + m + d == total, (name, a, m, d)
