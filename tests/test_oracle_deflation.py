"""Pins of the deflation oracle (oracle/deflation.py) against what the
mathematics fixes: block orthonormality and the Gram-Schmidt order, the
nearest-neighbour structure of the little operator, the projector
identities, the exact limit in which the subspace is the whole space (M_dfl =
D^-1, FGCR converges in one step), SAP-smoothed inverse iteration moving the
fields toward the low modes, and deflated solves that agree with the plain
SAP solver's solution.  How many iterations deflation saves is a measured
property, not a pin (on 8x4^3 C*, kappa 0.1365, 2^4 blocks, Ns = 12 and ten
inverse-iteration steps the oracle's FGCR needs 26 instead of 43)."""

import numpy as np
import pytest

from oracle import Lattice
from oracle import deflation as odf
from oracle import dirac as od
from oracle import fields as of
from oracle import solvers as osv
from oracle.dense import dense_matrix
from paper_1710_08839_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _op(dims, cstar, kappa, seed, eps=0.3, q=-1 / 3, csw=1.5):
    lat = Lattice(dims, cstar=cstar)
    u, a = synth.gauge_field(dims, seed, eps, 0.15)
    ue, ae = of.extend_gauge(lat, u, a)
    return lat, od.build_operator(lat, ue, ae, kappa, q=q, csw=csw, csw_u1=1.0)


def _fields(lat, ns, seed):
    rng = synth.rng_from_seed(seed)
    return np.array([synth.gaussian_source(rng, lat.V) for _ in range(ns)])


def rel(a, b):
    return od.norm(a - b) / od.norm(b)


@pytest.fixture(scope="module")
def small():
    lat, op = _op((4, 4, 4, 4), 1, 0.128, 31)
    blocks = osv.Blocks(lat, (2, 2, 2, 2))
    assert blocks.check_colouring()
    psi = odf.deflation_fields(op, blocks, _fields(lat, 4, 41), ninv=2, ncy=2, nmr=3)
    phi = odf.block_orthonormalise(blocks, psi)
    return lat, op, blocks, psi, phi, odf.Deflation(op, blocks, phi)


def test_block_orthonormal_in_gram_schmidt_order(small):
    lat, op, blocks, psi, phi, _ = small
    ns = len(phi)
    for b in range(blocks.n_blocks):
        on = blocks.block_id == b
        v = phi[:, on].reshape(ns, -1)
        assert np.max(np.abs(v.conj() @ v.T - np.eye(ns))) < 1e-13
        w = psi[:, on].reshape(ns, -1)
        for l in range(ns):
            # theta psi_l lies in span(phi_0..phi_l) but not in span(phi_0..phi_{l-1})
            c = v[:l + 1].conj() @ w[l]
            assert np.linalg.norm(w[l] - c @ v[:l + 1]) < 1e-12 * np.linalg.norm(w[l])
            if l:
                c = v[:l].conj() @ w[l]
                assert np.linalg.norm(w[l] - c @ v[:l]) > 1e-3 * np.linalg.norm(w[l])


def test_little_operator_is_nearest_neighbour(small):
    lat, op, blocks, psi, phi, dfl = small
    ns, nb = len(phi), blocks.n_blocks
    # block adjacency from the lattice's own neighbour tables (C* shifts included)
    adj = np.eye(nb, dtype=bool)
    for mu in range(4):
        adj[blocks.block_id, blocks.block_id[lat.fwd[mu]]] = True
        adj[blocks.block_id, blocks.block_id[lat.bwd[mu]]] = True
    mag = np.abs(dfl.a).reshape(nb, ns, nb, ns).max(axis=(1, 3))
    assert np.all(mag[~adj] == 0)
    assert np.all(mag[adj] > 1e-3)


def test_projector_identities(small):
    lat, op, blocks, psi, phi, dfl = small
    rng = np.random.default_rng(3)
    c = rng.standard_normal((blocks.n_blocks, len(phi))) + 1j * rng.standard_normal((blocks.n_blocks, len(phi)))
    dv = op.apply(odf.prolong(blocks, phi, c))
    # P_L D V = 0, V^dag P_L = 0, P_L^2 = P_L
    assert od.norm(dfl.project_left(dv)) < 1e-12 * od.norm(dv)
    r = synth.gaussian_source(synth.rng_from_seed(5), lat.V)
    pr = dfl.project_left(r)
    assert np.max(np.abs(odf.restrict(blocks, phi, pr))) < 1e-12 * od.norm(r)
    assert rel(dfl.project_left(pr), pr) < 1e-12
    # V^dag V = 1 on coefficient vectors
    assert np.max(np.abs(odf.restrict(blocks, phi, odf.prolong(blocks, phi, c)) - c)) < 1e-12


def test_whole_space_gives_the_inverse():
    """Ns = 12 x block volume: S is the whole space, V A^-1 V^dag = D^-1, so
    M_dfl r = D^-1 r and FGCR converges in one step."""
    lat, op = _op((4, 2, 2, 2), 0, 0.13, 37, eps=0.5)
    blocks = osv.Blocks(lat, (2, 2, 2, 2))
    ns = 12 * 16
    phi = odf.block_orthonormalise(blocks, _fields(lat, ns, 43))
    dfl = odf.Deflation(op, blocks, phi)
    d = dense_matrix(op.apply, lat.V)
    r = synth.gaussian_source(synth.rng_from_seed(6), lat.V)
    exact = np.linalg.solve(d, r.reshape(-1)).reshape(r.shape)
    assert rel(dfl.coarse(r), exact) < 1e-10
    assert rel(dfl.precond(r, 2, 3), exact) < 1e-10
    x, it = osv.fgcr(op.apply, lambda v: dfl.precond(v, 2, 3), r, 1e-10, nkv=4)
    assert it == 1 and rel(x, exact) < 1e-10


def test_deflation_fields_approach_low_modes(small):
    """SAP-smoothed inverse iteration moves the fields toward the low modes of
    D: |D psi| / |psi| falls well below that of the random start."""
    lat, op, blocks, psi, phi, _ = small
    start = _fields(lat, len(psi), 41)
    for p0, p in zip(start, psi):
        assert od.norm(op.apply(p)) / od.norm(p) < 0.5 * od.norm(op.apply(p0)) / od.norm(p0)


def test_deflated_solve_matches_sap_solve(small):
    lat, op, blocks, psi, phi, dfl = small
    eta = synth.gaussian_source(synth.rng_from_seed(7), lat.V)
    x, it = odf.dfl_solve(dfl, eta, 1e-12, ncy=2, nmr=3, nkv=8)
    assert od.norm(eta - op.apply(x)) <= 1e-12 * od.norm(eta)
    bops = (osv.BlockOperator(op, blocks, 0), osv.BlockOperator(op, blocks, 1))
    y, _ = osv.fgcr(op.apply, lambda v: osv.sap(op, blocks, v, 2, 3, bops), eta, 1e-13, nkv=8)
    assert rel(x, y) < 1e-10
