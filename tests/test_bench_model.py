"""Host-side checks of the benchmark's byte model and command line (no GPU).

The algorithmic bytes per extended site are recounted here from the field
contents of one application of D (Sec. 2.3): input and output spinors (4
spins x 3 colours complex = 24 reals each), the four hopping links of the
site (3 x 3 complex = 18 reals each) and the two 6 x 6 Hermitian Pauli
blocks (36 reals each); FP16+scale adds one fp32 scale per spinor site.
With the mirror-fused link reads of a C* lattice only the physical half's
links are read (Sec. 2.1: the mirror links are their complex conjugates).
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

REAL_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_bytes_per_site(prec):
    spinors = 2 * 24
    links = 4 * 18
    pauli = 2 * 36
    want = (spinors + links + pauli) * REAL_BYTES[prec] + (2 * 4 if prec == 2 else 0)
    assert bench.BYTES_PER_SITE[prec] == want
    # no mirror fusion without the LDS-staged kernel, or without bit 64
    for choice in (1, 17, 49, 64 | 1):
        assert bench.site_bytes(prec, choice) == want
    # mirror-fused: half of the link bytes
    for choice in (64 | 16 | 1, 64 | 32 | 16 | 2):
        assert bench.site_bytes(prec, choice) == want - links * REAL_BYTES[prec] // 2


def test_fp64_headline_bytes():
    assert bench.site_bytes(0, 113) * 4194304 == 1248 * 4194304


def test_kernel_name():
    assert bench.kernel_name(0, 0) == "dirac_kernel (not tuned)"
    assert bench.kernel_name(2, 0) == "dirac_kernel<0, 0, 2>"
    assert bench.kernel_name(49, 0) == "dirac_lds_kernel<0, 0, 1, true>"
    assert bench.kernel_name(113, 1) == "dirac_lds_kernel<1, 0, 1, true> (mirror-fused links)"
    assert bench.kernel_name(241, 2) == "dirac_wave_kernel<2, 0, 1, true> (mirror-fused links)"


def test_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
