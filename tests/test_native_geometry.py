"""CPU check of the HIP library's site-index maths (the native order used by
every kernel) against the oracle's neighbour tables: decode/encode is a
bijection onto [0, V) that keeps the parity halves, and the neighbours with
their fermion signs match the extended-lattice geometry of Sec. 2.1 (period
2L1 in direction 1, shifted C* boundaries, antiperiodic or open time)."""

import os
import subprocess

import numpy as np
import pytest

from oracle import Lattice

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("geom") / "geom_harness")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1710_08839_amd", "csrc"),
           os.path.join(HERE, "native", "geom_harness.cpp"), "-o", exe]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        pytest.fail("compiling the geometry harness failed:\n" + p.stderr)
    return exe


@pytest.mark.parametrize("dims,cstar,tbc,block", [
    ((4, 4, 4, 4), 0, 0, (2, 2, 2, 2)),
    ((8, 4, 4, 4), 3, 0, (4, 4, 4, 4)),
    ((4, 4, 4, 4), 3, 1, (2, 2, 2, 2)),
    ((6, 4, 4, 2), 2, 1, (2, 2, 2, 2)),
    ((4, 6, 4, 4), 1, 0, (2, 6, 2, 4)),
    ((8, 8, 8, 8), 0, 0, (4, 4, 4, 4)),
])
def test_native_geometry(harness, dims, cstar, tbc, block):
    args = [str(v) for v in (*dims, cstar, tbc, *block)]
    p = subprocess.run([harness] + args, capture_output=True, text=True)
    assert p.returncode == 0, p.stdout[-500:]
    rows = np.array([list(map(int, ln.split())) for ln in p.stdout.strip().splitlines()])
    lat = Lattice(dims, cstar=cstar, time_bc=tbc)
    assert rows.shape == (lat.V, 17)
    native = rows[:, 0]
    assert sorted(native) == list(range(lat.V))
    # even sites first
    assert np.all((native < lat.V // 2) == (lat.parity == 0))
    for mu in range(4):
        fw, fs = rows[:, 1 + 4 * mu], rows[:, 2 + 4 * mu]
        bw, bs = rows[:, 3 + 4 * mu], rows[:, 4 + 4 * mu]
        assert np.array_equal(fw, lat.fwd[mu])
        assert np.array_equal(bw, lat.bwd[mu])
        assert np.array_equal(fs, lat.sign[mu].astype(int))
        assert np.array_equal(bs, lat.bsign[mu].astype(int))


def test_generic_hop_matches_projections(tmp_path):
    """The direction-generic hop used where lanes of one wavefront hop in
    different directions equals the per-direction projections (1 -+ g_mu);
    and the multiply-shift division by the run length of the block-major
    field layout equals integer division."""
    exe = str(tmp_path / "hop_harness")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1710_08839_amd", "csrc"),
           os.path.join(HERE, "native", "hop_harness.cpp"), "-o", exe]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    worst, scale, bad = float(out[0]), float(out[1]), int(out[2])
    assert scale > 1.0
    assert worst < 1e-12 * scale
    # the multiply-shift division of the block-major field layout is exact
    assert bad == 0
