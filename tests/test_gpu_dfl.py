"""GPU parity of the local deflation (qxd_dfl_setup, QXD_SOLVER_DFL_SAP_GCR)
against the deflation oracle (oracle/deflation.py): the basis built from the
same start fields, the little operator assembled from the library's own
basis, the deflated preconditioner, and deflated solves checked with the
oracle's D."""

import numpy as np
import pytest

from gpu_common import Case, rel, to_dev, to_host
from oracle import deflation as odf
from oracle import dirac as od
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

NS, NINV, NCY, NMR = 6, 2, 2, 3


@pytest.fixture(scope="module")
def ctx():
    from paper_1710_08839_amd import qxd
    return qxd.Context(0)


@pytest.fixture(scope="module")
def case(ctx):
    # 8 x (2*8) x 8 x 8 C* lattice, 4^4 blocks: 32 blocks, every count even
    return Case(ctx, (8, 8, 8, 8), cstar=1, q=-1 / 3, kappa=0.128, csw=1.5, eps=0.3, seed=61)


@pytest.fixture(scope="module")
def setup(case):
    """The library's subspace from given start fields, and the oracle's from
    the same ones."""
    import torch
    c = case
    starts = np.stack([c.source(700 + k) for k in range(NS)])
    c.field.dfl_setup(c.quark, ns=NS, ninv=NINV, ncy=NCY, nmr=NMR, little_tol=1e-12, init=to_dev(starts))
    out = torch.empty((1, c.V, 4, 3), dtype=torch.complex128, device="cuda")
    basis = []
    for k in range(NS):
        c.field.dfl_basis(c.quark, k, out)
        torch.cuda.synchronize()
        basis.append(to_host(out)[0])
    blocks = osv.Blocks(c.lat, (4, 4, 4, 4))
    ref = odf.block_orthonormalise(blocks, odf.deflation_fields(c.op, blocks, starts, NINV, NCY, NMR))
    return np.array(basis), ref, blocks


def test_basis_matches_oracle(case, setup):
    basis, ref, blocks = setup
    for k in range(NS):
        assert rel(basis[k], ref[k]) < 2e-4, k
    # block-orthonormal to the FP32 storage
    for b in range(blocks.n_blocks):
        on = blocks.block_id == b
        v = basis[:, on].reshape(NS, -1)
        assert np.max(np.abs(v.conj() @ v.T - np.eye(NS))) < 2e-6


def test_little_operator_matches_oracle(case, setup):
    """A from the library equals V^dag D V computed by the oracle on the
    library's own basis (FP64 assembly from the FP32-stored basis)."""
    c = case
    basis, _, blocks = setup
    a, nbr = c.field.dfl_little(c.quark)
    nb = blocks.n_blocks
    assert a.shape == (nb, 9, NS, NS)
    dense = np.zeros((nb * NS, nb * NS), dtype=complex)
    for b in range(nb):
        assert nbr[b, 0] == b
        for d in range(9):
            n = nbr[b, d]
            dense[b * NS:(b + 1) * NS, n * NS:(n + 1) * NS] += a[b, d]
    # the slots' neighbours are the blocks across the faces
    lat = c.lat
    for mu in range(4):
        for s, nxt in ((0, lat.fwd[mu]), (1, lat.bwd[mu])):
            face = {}
            for x in range(lat.V):
                if blocks.block_id[nxt[x]] != blocks.block_id[x]:
                    face[blocks.block_id[x]] = blocks.block_id[nxt[x]]
            for b, n in face.items():
                assert nbr[b, 1 + 2 * mu + s] == n, (b, mu, s)
    ref = odf.little_operator(c.op, blocks, basis)
    assert np.max(np.abs(dense - ref)) < 1e-12 * np.max(np.abs(ref))


def test_precond_matches_oracle(case, setup):
    """M_dfl r with the little system solved to 1e-12: FP32 storage of the
    vectors (D and the Schwarz preconditioner at FP32 accuracy)."""
    import torch
    c = case
    basis, _, blocks = setup
    dfl = odf.Deflation(c.op, blocks, basis)
    r = c.source(901)
    y = torch.empty_like(to_dev(r))
    c.field.dfl_precond(c.quark, to_dev(r), y, little_tol=1e-12, ncy=NCY, nmr=NMR)
    torch.cuda.synchronize()
    expect = dfl.precond(r, NCY, NMR)
    assert rel(to_host(y), expect) < 5e-5
    # the coarse part alone: with the Schwarz part removed by r = D V c
    # (P_L r = 0) M_dfl r = V c
    coef = np.random.default_rng(4).standard_normal((blocks.n_blocks, NS)) * (1 + 0.5j)
    vc = odf.prolong(blocks, basis, coef)
    r2 = c.op.apply(vc)
    c.field.dfl_precond(c.quark, to_dev(r2), y, little_tol=1e-12, ncy=NCY, nmr=NMR)
    torch.cuda.synchronize()
    assert rel(to_host(y), vc) < 5e-5


@pytest.mark.parametrize("little_tol", [0.2, 1e-12], ids=["fp16-matrices", "fp32-matrices"])
def test_precond_repeatable(case, setup, little_tol):
    """Repeated applications of the deflated preconditioner to one vector
    agree bit for bit (fixed-order reductions; the little GCR's stopping
    step is decided on the same residual norms); with the default loose
    little tolerance the little solve reads the FP16 copies of the little
    matrices, with a tight one the FP32 copies."""
    import torch
    c = case
    r = to_dev(c.source(903))
    outs = []
    for _ in range(3):
        y = torch.empty_like(r)
        c.field.dfl_precond(c.quark, r, y, little_tol=little_tol, ncy=NCY, nmr=NMR)
        torch.cuda.synchronize()
        outs.append(to_host(y))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.all(np.isfinite(outs[0]))


@pytest.mark.parametrize("little_tol", [0.2, 1e-12], ids=["fp16-matrices", "fp32-matrices"])
def test_precond_of_zero(case, setup, little_tol):
    """M_dfl 0 = 0 exactly: the little GCR's steps on a zero residual change
    nothing (no division by a zero norm), the step queued past convergence
    included, and the preconditioner leaves no stale values behind."""
    import torch
    c = case
    y = torch.full_like(to_dev(c.source(904)), 7.0)
    c.field.dfl_precond(c.quark, torch.zeros_like(y), y, little_tol=little_tol, ncy=NCY, nmr=NMR)
    torch.cuda.synchronize()
    assert not torch.any(y != 0).item()


@pytest.mark.parametrize("nkv", [8, 32])
def test_deflated_solve(case, setup, nkv):
    import torch
    from paper_1710_08839_amd import qxd
    c = case
    eta = np.stack([c.source(910 + r) for r in range(2)])
    psi = torch.empty_like(to_dev(eta))
    s = qxd.solver(kind=qxd.DFL_SAP_GCR, tol=1e-10, nkv=nkv, ncy=NCY, nmr=NMR, inner_prec=qxd.F32)
    st, info = c.field.solve(c.quark, s, to_dev(eta), psi, nrhs=2)
    assert st == 0
    ph = to_host(psi)
    for r in range(2):
        assert od.norm(eta[r] - c.op.apply(ph[r])) / od.norm(eta[r]) <= 1.05e-10, r
        assert info[r].true_resid <= 1e-10 and info[r].inner_iters > 0


def test_random_start_fields(ctx):
    """Start fields from the library's own generator: the basis is
    block-orthonormal and the deflated solve converges; ns 4 on 2^4 blocks."""
    import torch
    from paper_1710_08839_amd import qxd
    c = Case(ctx, (4, 4, 4, 4), cstar=3, q=2 / 3, kappa=0.126, csw=1.2, seed=67, block=(2, 2, 2, 2))
    c.field.dfl_setup(c.quark, ns=4, ninv=3, ncy=2, nmr=3, seed=12345)
    out = torch.empty((1, c.V, 4, 3), dtype=torch.complex128, device="cuda")
    blocks = osv.Blocks(c.lat, (2, 2, 2, 2))
    basis = []
    for k in range(4):
        c.field.dfl_basis(c.quark, k, out)
        torch.cuda.synchronize()
        basis.append(to_host(out)[0])
    basis = np.array(basis)
    for b in range(blocks.n_blocks):
        v = basis[:, blocks.block_id == b].reshape(4, -1)
        assert np.max(np.abs(v.conj() @ v.T - np.eye(4))) < 2e-6
    eta = c.source(77)
    psi = torch.empty_like(to_dev(eta))
    st, info = c.field.solve(c.quark, qxd.solver(kind=qxd.DFL_SAP_GCR, tol=1e-10, nkv=8, ncy=2, nmr=3),
                             to_dev(eta), psi)
    assert st == 0
    assert od.norm(eta - c.op.apply(to_host(psi))) / od.norm(eta) <= 1.05e-10


@pytest.mark.parametrize("tbc, cf, cfp", [(1, 1.0, 1.0), (2, 1.25, 1.0), (3, 1.1, 0.85)],
                         ids=["open", "sf", "open-sf"])
def test_time_boundaries(ctx, tbc, cf, cfp):
    """Open, SF and open-SF time boundaries: the little operator the library
    assembles from its boundary-aware D equals V^dag D V computed by the
    oracle on the library's basis, and the deflated solve reaches the
    tolerance measured with the oracle's D."""
    import torch
    from paper_1710_08839_amd import qxd
    c = Case(ctx, (8, 8, 8, 8), cstar=1, time_bc=tbc, q=-1 / 3, kappa=0.128, csw=1.5, eps=0.3, seed=80 + tbc,
             cF=cf, cF_prime=cfp)
    ns = 4
    c.field.dfl_setup(c.quark, ns=ns, ninv=3, ncy=2, nmr=3, seed=4242)
    out = torch.empty((1, c.V, 4, 3), dtype=torch.complex128, device="cuda")
    basis = []
    for k in range(ns):
        c.field.dfl_basis(c.quark, k, out)
        torch.cuda.synchronize()
        basis.append(to_host(out)[0])
    basis = np.array(basis)
    blocks = osv.Blocks(c.lat, (4, 4, 4, 4))
    a, nbr = c.field.dfl_little(c.quark)
    nb = blocks.n_blocks
    dense = np.zeros((nb * ns, nb * ns), dtype=complex)
    for b in range(nb):
        for d in range(9):
            dense[b * ns:(b + 1) * ns, nbr[b, d] * ns:(nbr[b, d] + 1) * ns] += a[b, d]
    ref = odf.little_operator(c.op, blocks, basis)
    assert np.max(np.abs(dense - ref)) < 1e-12 * np.max(np.abs(ref))
    eta = c.source(78)
    psi = torch.empty_like(to_dev(eta))
    st, info = c.field.solve(c.quark, qxd.solver(kind=qxd.DFL_SAP_GCR, tol=1e-10, nkv=8, ncy=2, nmr=3),
                             to_dev(eta), psi)
    assert st == 0
    assert od.norm(eta - c.op.apply(to_host(psi))) / od.norm(eta) <= 1.05e-10


@pytest.mark.parametrize("ns", [1, 32], ids=["ns1", "ns32"])
def test_smallest_and_largest_subspace(ctx, ns):
    """The extreme subspace sizes (1 and the maximum 32 vectors per block) on
    a 4^4 C* lattice with 2^4 blocks (192 components per block): the basis is
    block-orthonormal, the little operator equals the oracle's V^dag D V on
    the library's basis, and the deflated solve reaches the tolerance."""
    import torch
    from paper_1710_08839_amd import qxd
    c = Case(ctx, (4, 4, 4, 4), cstar=1, q=-1 / 3, kappa=0.126, csw=1.3, seed=90 + ns, block=(2, 2, 2, 2))
    c.field.dfl_setup(c.quark, ns=ns, ninv=2, ncy=2, nmr=3, seed=7)
    out = torch.empty((1, c.V, 4, 3), dtype=torch.complex128, device="cuda")
    basis = []
    for k in range(ns):
        c.field.dfl_basis(c.quark, k, out)
        torch.cuda.synchronize()
        basis.append(to_host(out)[0])
    basis = np.array(basis)
    blocks = osv.Blocks(c.lat, (2, 2, 2, 2))
    for b in range(blocks.n_blocks):
        v = basis[:, blocks.block_id == b].reshape(ns, -1)
        assert np.max(np.abs(v.conj() @ v.T - np.eye(ns))) < 1e-5
    a, nbr = c.field.dfl_little(c.quark)
    nb = blocks.n_blocks
    dense = np.zeros((nb * ns, nb * ns), dtype=complex)
    for b in range(nb):
        for d in range(9):
            dense[b * ns:(b + 1) * ns, nbr[b, d] * ns:(nbr[b, d] + 1) * ns] += a[b, d]
    ref = odf.little_operator(c.op, blocks, basis)
    assert np.max(np.abs(dense - ref)) < 1e-12 * np.max(np.abs(ref))
    eta = c.source(91)
    psi = torch.empty_like(to_dev(eta))
    st, info = c.field.solve(c.quark, qxd.solver(kind=qxd.DFL_SAP_GCR, tol=1e-10, nkv=8, ncy=2, nmr=3),
                             to_dev(eta), psi)
    assert st == 0
    assert od.norm(eta - c.op.apply(to_host(psi))) / od.norm(eta) <= 1.05e-10


def test_dfl_errors(case):
    import torch
    from paper_1710_08839_amd import qxd
    c = case
    eta = to_dev(c.source(5))
    psi = torch.empty_like(eta)
    other = qxd.quark(0.127, -1 / 3, 1.5, 1.0)  # no subspace for this quark
    with pytest.raises(qxd.QxdError):
        c.field.solve(other, qxd.solver(kind=qxd.DFL_SAP_GCR), eta, psi)
    with pytest.raises(qxd.QxdError):
        c.field.solve(c.quark, qxd.solver(kind=qxd.DFL_SAP_GCR, inner_prec=qxd.F16S), eta, psi)
    with pytest.raises(qxd.QxdError):
        c.field.dfl_setup(c.quark, ns=33)
    with pytest.raises(qxd.QxdError):
        c.field.dfl_basis(other, 0, psi)
