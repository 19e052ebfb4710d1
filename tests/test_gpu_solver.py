"""GPU solvers against the FP64 oracle.

* SAP preconditioner: M_SAP rho from the library equals the oracle's step-by-
  step Schwarz procedure (same blocks, colours, cycles and MR steps) to the
  precision bar (1e-12 FP64, 1e-5 FP32, 1e-2 FP16/BF16 storage).
* Solves: every solve reaches a true FP64 residual |eta - D psi| / |eta| <=
  1e-10, where D is the oracle's operator applied to the GPU's solution, and
  the solution agrees with the oracle's even-odd solve to within the residual
  bound times the condition number.
"""

import numpy as np
import pytest

from gpu_common import Case, rel, to_dev, to_host
from oracle import dirac as od
from oracle import solvers as osv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1710_08839_amd import qxd
    return qxd.Context(0)


@pytest.fixture(scope="module")
def cstar_case(ctx):
    # 8 x (2*8) x 8 x 8 extended sites, 4^4 blocks: 2 x 4 x 2 x 2 blocks,
    # L1 / b1 = 2 (even) as the shifted C* boundaries require for colouring
    return Case(ctx, (8, 8, 8, 8), cstar=3, q=-1 / 3, kappa=0.1365, csw=1.9, eps=0.25, seed=20171003)


@pytest.fixture(scope="module")
def open_case(ctx):
    # as cstar_case with an open time boundary: the links across x0 = T-1 -> 0
    # are absent in the block solves, the face updates and the Dirac operator
    return Case(ctx, (8, 8, 8, 8), cstar=3, time_bc=1, q=-1 / 3, kappa=0.1365, csw=1.9, eps=0.25,
                seed=20171004)


@pytest.fixture(scope="module")
def sf_case(ctx):
    # Schroedinger-functional time boundary: the slice x0 = 0 is fixed, dD_b
    # with c_F = 1.25 on x0 = 1 and T-1
    return Case(ctx, (8, 8, 8, 8), cstar=3, time_bc=2, q=-1 / 3, kappa=0.1365, csw=1.9, eps=0.25,
                seed=20171005, cF=1.25)


@pytest.fixture(scope="module")
def osf_case(ctx):
    # open-SF: SF at x0 = 0 (c_F on x0 = 1), open at x0 = T-1 (c_F')
    return Case(ctx, (8, 8, 8, 8), cstar=1, time_bc=3, q=2 / 3, kappa=0.13, csw=1.7, eps=0.25,
                seed=20171006, cF=1.1, cF_prime=0.85)


@pytest.fixture(scope="module")
def periodic_case(ctx):
    return Case(ctx, (8, 8, 8, 8), cstar=0, u1=False, kappa=0.124, csw=1.0, eps=0.3, seed=20171000)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5), (2, 1e-2), (3, 1e-2)],
                         ids=["f64", "f32", "f16s", "bf16"])
@pytest.mark.parametrize("ncy,nmr", [(1, 0), (1, 1), (2, 4)])
@pytest.mark.parametrize("which", ["cstar_case", "open_case", "sf_case", "osf_case"],
                         ids=["antiperiodic", "open", "sf", "open-sf"])
def test_sap_matches_oracle(request, which, prec, tol, ncy, nmr):
    import torch
    c = request.getfixturevalue(which)
    blocks = osv.Blocks(c.lat, (4, 4, 4, 4))
    assert blocks.check_colouring()
    rho = c.source(31)
    ref = osv.sap(c.op, blocks, rho, ncy=ncy, nmr=nmr)
    out = torch.empty_like(to_dev(rho))
    c.field.sap_apply(c.quark, prec, ncy, nmr, to_dev(rho), out)
    torch.cuda.synchronize()
    assert rel(to_host(out), ref) < tol


def test_sap_periodic(periodic_case):
    import torch
    c = periodic_case
    blocks = osv.Blocks(c.lat, (4, 4, 4, 4))
    rho = c.source(32)
    ref = osv.sap(c.op, blocks, rho, ncy=3, nmr=4)
    out = torch.empty_like(to_dev(rho))
    c.field.sap_apply(c.quark, 0, 3, 4, to_dev(rho), out)
    torch.cuda.synchronize()
    assert rel(to_host(out), ref) < 1e-12


def _check_solution(c, eta, psi, ref=None):
    res = od.norm(eta - c.op.apply(psi)) / od.norm(eta)
    assert res <= 1.05e-10, res
    if ref is not None:
        assert rel(psi, ref) < 1e-7


def test_eo_gcr_f64(periodic_case):
    import torch
    from paper_1710_08839_amd import qxd
    c = periodic_case
    eta = c.source(1000)
    psi = torch.empty_like(to_dev(eta))
    st, info = c.field.solve(c.quark, qxd.solver(kind=qxd.EO_GCR, tol=1e-10, nkv=16), to_dev(eta), psi)
    assert st == 0 and info[0].true_resid <= 1e-10
    ref, _ = osv.solve_eo(c.op, eta, 1e-12)
    _check_solution(c, eta, to_host(psi), ref)


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["f64", "f32", "f16s", "bf16"])
@pytest.mark.parametrize("which", ["cstar_case", "open_case", "sf_case", "osf_case"],
                         ids=["antiperiodic", "open", "sf", "open-sf"])
def test_sap_gcr(request, which, prec):
    import torch
    from paper_1710_08839_amd import qxd
    c = request.getfixturevalue(which)
    eta = c.source(1001)
    psi = torch.empty_like(to_dev(eta))
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, ncy=4, nmr=4, inner_prec=prec)
    st, info = c.field.solve(c.quark, s, to_dev(eta), psi)
    assert st == 0, info[0].status
    assert info[0].true_resid <= 1e-10
    _check_solution(c, eta, to_host(psi))


@pytest.mark.parametrize("which", ["open_case", "sf_case", "osf_case"], ids=["open", "sf", "open-sf"])
def test_eo_gcr_time_boundaries(request, which):
    """Plain FP64 even-odd GCR with the open, SF and open-SF time boundaries."""
    import torch
    from paper_1710_08839_amd import qxd
    c = request.getfixturevalue(which)
    eta = c.source(1005)
    psi = torch.empty_like(to_dev(eta))
    st, info = c.field.solve(c.quark, qxd.solver(kind=qxd.EO_GCR, tol=1e-10, nkv=32), to_dev(eta), psi)
    assert st == 0 and info[0].true_resid <= 1e-10
    _check_solution(c, eta, to_host(psi))


_FGCR_REF = {}


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5), (2, 1e-2), (3, 1e-2)],
                         ids=["f64", "f32", "f16s", "bf16"])
@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("passes", [1, 2], ids=["cgs", "cgs2"])
def test_fgcr_steps_match_oracle(cstar_case, prec, tol, k, passes):
    """The iterate after k flexible-GCR steps (SAP preconditioner, one outer
    defect-correction step) equals the oracle's k-step FGCR on the same source
    to the bar of the inner precision: the per-step error of the mixed-
    precision solver against FP64.  The library orthogonalises by one
    classical Gram-Schmidt pass with FP64 sums (or two, the second against the
    stored vectors with its coefficients added to the first), the oracle by
    modified Gram-Schmidt with normalised vectors; they agree in exact
    arithmetic."""
    import torch
    from paper_1710_08839_amd import qxd
    c = cstar_case
    eta = c.source(1003)
    if k not in _FGCR_REF:
        blocks = osv.Blocks(c.lat, (4, 4, 4, 4))
        en = od.norm(eta)
        ref, it = osv.fgcr(c.op.apply, lambda r: osv.sap(c.op, blocks, r, ncy=2, nmr=4), eta / en, 1e-14,
                           nkv=8, maxiter=k)
        assert it == k
        _FGCR_REF[k] = en * ref
    ref = _FGCR_REF[k]
    psi = torch.empty_like(to_dev(eta))
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-14, maxiter=k, nkv=8, ncy=2, nmr=4, inner_prec=prec,
                   inner_tol=1e-14, max_outer=1)
    qxd.set_gs_passes(passes)
    try:
        st, info = c.field.solve(c.quark, s, to_dev(eta), psi, check=False)
    finally:
        qxd.set_gs_passes(1)
    assert st == -3 and info[0].inner_iters == k and info[0].outer_iters == 1
    err = rel(to_host(psi), ref)
    assert err < tol, err


def test_solve_with_guess_and_point_source(cstar_case):
    import torch
    from paper_1710_08839_amd import qxd, synth
    c = cstar_case
    eta = synth.point_source(c.V, 0, 2, 1)
    psi = torch.empty_like(to_dev(eta))
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, inner_prec=qxd.F32)
    st, _ = c.field.solve(c.quark, s, to_dev(eta), psi)
    assert st == 0
    _check_solution(c, eta, to_host(psi))
    # restarting from the solution needs no further work
    st, info = c.field.solve(c.quark, s, to_dev(eta), psi, use_guess=True)
    assert st == 0 and info[0].outer_iters == 0
    _check_solution(c, eta, to_host(psi))


def test_solve_errors(cstar_case):
    import torch
    from paper_1710_08839_amd import qxd
    c = cstar_case
    eta = c.source(5)
    eta[3, 1, 1] = np.nan
    psi = torch.empty_like(to_dev(eta))
    st, _ = c.field.solve(c.quark, qxd.solver(), to_dev(eta), psi, check=False)
    assert st == -4  # EFLOAT
    eta = c.source(6)
    st, info = c.field.solve(c.quark, qxd.solver(kind=qxd.EO_GCR, maxiter=2), to_dev(eta), psi, check=False)
    assert st == -3 and info[0].inner_iters <= 3  # ENOCONV, best iterate written
    bad = qxd.quark(0.13, 0.25, 1.0, 1.0)  # q / q_el not an integer
    with pytest.raises(qxd.QxdError):
        c.field.solve(bad, qxd.solver(), to_dev(eta), psi)
    for passes in (0, 3):
        with pytest.raises(qxd.QxdError):
            qxd.set_gs_passes(passes)
