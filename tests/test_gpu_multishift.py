"""GPU parity of the twisted-mass even-odd operators, the theta-periodic
boundary phases, the multi-shift CG and rational functions of D^dag D^
against the FP64 oracle (oracle/rational.py, oracle/fields.py), which the CPU
suite pins against dense linear algebra, the paper's Table 2 and closed forms.

Bars: operators 1e-12 (FP64), 1e-5 (FP32), 1e-2 (FP16/BF16 storage); solves
reach their FP64 residual; the multi-shift iterate after k steps equals the
oracle's k-step iterate (same recurrences, FP64) to 1e-11.
"""

import numpy as np
import pytest

from gpu_common import Case, rel, to_dev, to_host
from oracle import dirac as od
from oracle import fields as of
from oracle import rational as orat
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2, 3: 1e-2}
MU = 0.07


@pytest.fixture(scope="module")
def ctx():
    from paper_1710_08839_amd import qxd
    return qxd.Context(0)


@pytest.fixture(scope="module")
def small(ctx):
    # 4 x (2*4) x 4 x 4 C* lattice, open time, 2^4 blocks
    c = Case(ctx, (4, 4, 4, 4), cstar=3, time_bc=1, q=-1 / 3, kappa=0.13, csw=1.9, seed=61, block=(2, 2, 2, 2))
    return c


@pytest.fixture(scope="module")
def periodic(ctx):
    return Case(ctx, (8, 8, 8, 8), cstar=0, u1=True, q=2 / 3, kappa=0.125, csw=1.5, seed=62)


def _even(case, x):
    return case.op.restrict(x, case.lat.even)


def _g5(v):
    return np.einsum("st,...xtc->...xsc", od.GAMMA5, v)


def _quark(case, mu=0.0, theta=(0, 0, 0, 0)):
    from paper_1710_08839_amd import qxd
    q = case.quark
    return qxd.quark(q.kappa, q.q, q.csw, q.csw_u1, mu, theta)


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["f64", "f32", "f16s", "bf16"])
@pytest.mark.parametrize("which", ["small", "periodic"])
def test_twisted_schur_operators(request, which, prec):
    """D^ + i mu g5, its adjoint and the normal operator D^dag D^ + mu^2."""
    import torch
    from paper_1710_08839_amd import qxd
    c = request.getfixturevalue(which)
    x = c.source(71)
    xe = _even(c, x)
    q = _quark(c, MU)
    refs = {qxd.OP_DHAT: c.op.apply_schur(xe) + 1j * MU * _g5(xe),
            qxd.OP_DHAT_DAG: orat.schur_dagger(c.op, xe) - 1j * MU * _g5(xe),
            qxd.OP_NORMAL: orat.NormalOperator(c.op, MU).apply(xe)}
    for op, ref in refs.items():
        y = torch.empty_like(to_dev(x))
        c.field.apply(q, op, prec, to_dev(x), y)
        torch.cuda.synchronize()
        tol = TOL[prec] * (3 if op == qxd.OP_NORMAL and prec >= 2 else 1)
        assert rel(to_host(y), ref) < tol, (op, rel(to_host(y), ref))


THETAS = [(0, dict(dims=(8, 4, 4, 4), cstar=0, time_bc=0), (0.3, -0.8, 1.3, 0.45)),
          (1, dict(dims=(8, 4, 4, 4), cstar=1, time_bc=0), (-0.6, 0.0, 0.9, 2.1)),
          (2, dict(dims=(8, 4, 4, 4), cstar=2, time_bc=1), (0.0, 0.0, 0.0, -1.7))]


@pytest.mark.parametrize("k", range(len(THETAS)), ids=[f"cstar{t[1]['cstar']}" for t in THETAS])
def test_theta_phases(ctx, k):
    """D with fermion boundary phases against the oracle in every storage,
    autotuned and with the mirror-fused link reads (C*: the mirror half's
    phase is the conjugate, so reading it at the physical partner stays
    exact); a SAP-GCR and an even-odd GCR solve reach 1e-10 in the oracle's D."""
    import torch
    from paper_1710_08839_amd import qxd
    _, kw, theta = THETAS[k]
    c = Case(ctx, q=2 / 3, kappa=0.128, csw=1.7, seed=80 + k, block=(2, 2, 2, 2), **kw)
    ue, ae = of.extend_gauge(c.lat, c.u, c.a)
    op = od.build_operator(c.lat, ue, ae, 0.128, q=2 / 3, csw=1.7, theta=theta)
    q = qxd.quark(0.128, 2 / 3, 1.7, 1.0, 0.0, theta)
    x = c.source(81)
    ref = op.apply(x)
    assert rel(ref, c.op.apply(x)) > 1e-3  # the phases matter
    try:
        for choice in (0, 113):
            qxd.set_dirac_variant(choice)
            for prec in (0, 1, 2, 3):
                y = torch.empty_like(to_dev(x))
                c.field.apply(q, qxd.OP_D, prec, to_dev(x), y)
                torch.cuda.synchronize()
                assert rel(to_host(y), ref) < TOL[prec], (choice, prec)
    finally:
        qxd.set_dirac_variant(0)
    for s in (qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, ncy=3, nmr=4, inner_prec=qxd.F32),
              qxd.solver(kind=qxd.EO_GCR, tol=1e-10, nkv=32)):
        psi = torch.empty_like(to_dev(x))
        st, info = c.field.solve(q, s, to_dev(x), psi)
        assert st == 0
        assert od.norm(x - op.apply(to_host(psi))) / od.norm(x) <= 1.05e-10
    c.field.release()


def test_theta_rejected(small):
    from paper_1710_08839_amd import qxd
    import torch
    x = to_dev(small.source(1))
    y = torch.empty_like(x)
    for theta in ((0, 0.2, 0, 0), (0, 0, 0, 0.3), (0.1, 0, 0, 0)):  # C* directions; open time
        with pytest.raises(qxd.QxdError):
            small.field.apply(_quark(small, 0.0, theta), qxd.OP_D, 0, x, y)


SHIFTS = [0.0, 4e-3, 0.03, 0.25, 2.0]


@pytest.mark.parametrize("k", [1, 4, 15])
def test_multishift_steps_match_oracle(small, k):
    """After k iterations every shifted iterate equals the oracle's."""
    import torch
    c = small
    x = c.source(91)
    X = orat.NormalOperator(c.op, MU)
    ref, it, _ = orat.multishift_cg(X.apply, _even(c, x), SHIFTS, 1e-30, maxiter=k)
    assert it == k
    psi = torch.empty((len(SHIFTS),) + x.shape, dtype=torch.complex128, device="cuda")
    st, info = c.field.multishift(_quark(c, MU), SHIFTS, to_dev(x), psi, tol=1e-14, maxiter=k, check=False)
    assert st == -3 and all(i.inner_iters == k for i in info)
    ph = to_host(psi)
    for j in range(len(SHIFTS)):
        assert rel(ph[j], ref[j]) < 1e-11, (j, rel(ph[j], ref[j]))


@pytest.mark.parametrize("which", ["small", "periodic"])
def test_multishift_converges(request, which):
    import torch
    c = request.getfixturevalue(which)
    x = c.source(92)
    b = _even(c, x)
    X = orat.NormalOperator(c.op, MU)
    psi = torch.empty((len(SHIFTS),) + x.shape, dtype=torch.complex128, device="cuda")
    st, info = c.field.multishift(_quark(c, MU), SHIFTS, to_dev(x), psi, tol=1e-10)
    assert st == 0
    ph = to_host(psi)
    its = [i.inner_iters for i in info]
    assert its == sorted(its, reverse=True)
    for j, s in enumerate(SHIFTS):
        r = od.norm(b - X.apply(ph[j]) - s * ph[j]) / od.norm(b)
        assert r <= 1.05e-10 and info[j].true_resid <= 1.05e-10, (j, r)
        assert np.all(ph[j][c.lat.odd] == 0)


def _table2():
    rows = [ln.split() for ln in open(__file__.replace("test_gpu_multishift.py", "golden/rational_qcd2.txt"))
            if ln.strip() and not ln.startswith("#")]
    return np.array([float(r[1]) for r in rows]), np.array([float(r[2]) for r in rows])


def test_rational_functions(small):
    """Table 2's R (A from its minimax normalisation), its frequency-splitting
    factor P_2 and a twisted-mass Hasenbusch ratio, against the oracle's
    rational application.  Runs after the tests above built the operator with
    another twisted mass: an operator is shared by quarks that differ only in
    mu, and each call must use its own quark's mu."""
    import torch
    c = small
    x = c.source(93)
    b = _even(c, x)
    nu, mu = _table2()
    cases = [(0.0, 0.1734, nu, mu), (0.0, 1.0, nu[7:8], mu[7:8]), (0.0, 1.0, [0.5], [0.05])]
    for muq, A, n_, m_ in cases:
        rat = orat.Rational(A, n_, m_)
        ref = orat.rational_apply(orat.NormalOperator(c.op, muq).apply, rat, b, 1e-13)
        out = torch.empty_like(to_dev(x))
        st, info = c.field.rational(_quark(c, muq), A, n_, m_, to_dev(x), out, tol=1e-11)
        assert st == 0 and len(info) == len(m_)
        assert rel(to_host(out), ref) < 1e-8, (len(m_), rel(to_host(out), ref))
        assert np.all(to_host(out)[c.lat.odd] == 0)


def test_twisted_mass_is_per_call(small):
    """Two quarks that differ only in the twisted mass share one cached
    operator; each application uses its own mu (in either order)."""
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    x = c.source(95)
    xe = _even(c, x)
    for mu in (0.3, 0.0, 0.11):
        y = torch.empty_like(to_dev(x))
        c.field.apply(_quark(c, mu), qxd.OP_NORMAL, 0, to_dev(x), y)
        torch.cuda.synchronize()
        assert rel(to_host(y), orat.NormalOperator(c.op, mu).apply(xe)) < 1e-12, mu
