"""Pins of the block-local SAP oracle (oracle/solvers.py: block_solve_at,
sap_cycle_block_at), which the full-size GPU test uses on lattices too large
to build the whole operator, against the whole-lattice Schwarz procedure it
restates (BlockOperator, sap): on a lattice small enough to build the whole
operator, one SAP cycle on blocks of both colours, including blocks whose
faces cross the C* and time boundaries, agrees to rounding."""

import numpy as np
import pytest

from oracle import Lattice
from oracle import dirac as od
from oracle import fields as of
from oracle import solvers as osv
from paper_1710_08839_amd import synth


@pytest.mark.parametrize("time_bc", [0, 2], ids=["antiperiodic", "sf"])
def test_sap_cycle_block_at_matches_whole_lattice(time_bc):
    dims = (8, 8, 8, 8)
    lat = Lattice(dims, cstar=3, time_bc=time_bc)
    u, a = synth.gauge_field(dims, 11, 0.3, 0.15)
    ue, ae = of.extend_gauge(lat, u, a)
    kappa, q, csw = 0.13, -1 / 3, 1.5
    op = od.build_operator(lat, ue, ae, kappa, q=q, csw=csw, csw_u1=1.0)
    blocks = osv.Blocks(lat, (4, 4, 4, 4))
    assert blocks.check_colouring()
    r = synth.gaussian_source(synth.rng_from_seed(9), lat.V)
    ref = osv.sap(op, blocks, r, ncy=1, nmr=3)
    # block 0: colour 0 at the time boundary and the C* wraps in x2, x3;
    # block 1: colour 1, its x3 faces across the shifted C* boundary and its
    # x0 face across the time boundary
    for b, colour in ((0, 0), (1, 1)):
        sites, v = osv.sap_cycle_block_at(lat, ue, ae, blocks, r, b, 3, kappa, q, csw, 1.0)
        assert blocks.colour[sites[0]] == colour
        assert od.norm(v - ref[sites]) <= 1e-12 * od.norm(ref[sites])
