"""Multi-shift conjugate gradient on the even-odd normal operator, and rational
functions of that operator (FP64 reference; test infrastructure only).

Sec. 2.4 of the paper: the pseudofermion action uses a rational function of
D^dag D^ (D^ the even-odd Schur complement),
    R = A prod_{j=1}^N (D^dag D^ + nu_j^2) / (D^dag D^ + mu_j^2),
approximating (D^dag D^ + muhat^2)^(-1/4), written as a product of
frequency-splitting factors P_k that each hold the zeros and poles of one
index range.  The twisted-mass regulator muhat^2 (Sec. 2.4) and the
twisted-mass Hasenbusch factors (D^dag D^ + mu_a^2) / (D^dag D^ + mu_b^2) of
the QCD1 action (Appendix A) are rational functions of the same operator.
Every pole is a shifted system (D^dag D^ + sigma) x = b, which the paper's
multi-shift conjugate gradient (feature list of Sec. 2; Table 2 and the
QCD+QED runs of Appendix B) solves for all shifts in one Krylov space.

  schur_dagger(op, psi_e)   D^dag psi_e, from the adjoints of the pieces of
                            D^ = D_ee - D_eo D_oo^-1 D_oe
  NormalOperator            X = D^dag D^ + mu^2 on even-site spinors (mu: a
                            twisted mass; X is Hermitian positive definite)
  multishift_cg             (X + sigma_j) x_j = b for every shift sigma_j,
                            the collinear-residual recurrences written out
                            step by step (Jegerlehner's shifted CG)
  Rational                  A prod (t + nu_j^2)/(t + mu_j^2): value, partial
                            fractions, frequency-splitting factors
  rational_apply            R(X) b through the partial fractions and the
                            multi-shift CG

Vectors are spinor arrays [V, 4, 3] complex128 whose odd sites are zero.
"""

import numpy as np

from .dirac import EYE4, GAMMA, dot, norm


# --------------------------------------------------------------------------
# the adjoint of the Schur complement and the normal operator
# --------------------------------------------------------------------------
def _hop_dagger(op, psi):
    """H^dag psi for the hopping part H of D: the adjoint of
    H psi(x) = -1/2 sum_mu [(1-g_mu) W(x,mu) psi(x+mu) + (1+g_mu) W(x-mu,mu)^dag psi(x-mu)]
    (gamma_mu Hermitian) is
    H^dag psi(y) = -1/2 sum_mu [(1-g_mu) W(y-mu,mu)^dag psi(y-mu) + (1+g_mu) W(y,mu) psi(y+mu)],
    with the boundary factors of the same links."""
    lat = op.lat
    out = np.zeros_like(psi)
    for mu in range(4):
        bw = psi[..., lat.bwd[mu], :, :] * lat.bsign[mu][:, None, None]
        bw = np.einsum("xab,...xsb->...xsa", op.wd[lat.bwd[mu], mu], bw)
        out += np.einsum("st,...xtc->...xsc", EYE4 - GAMMA[mu], bw)
        fw = psi[..., lat.fwd[mu], :, :] * lat.sign[mu][:, None, None]
        fw = np.einsum("xab,...xsb->...xsa", op.w[:, mu], fw)
        out += np.einsum("st,...xtc->...xsc", EYE4 + GAMMA[mu], fw)
    return -0.5 * out


def _block_dagger(blocks, psi, sites):
    """out(x) = B(x)^dag psi(x) on the listed sites (zero elsewhere); blocks
    [len(sites), 12, 12] on spin (x) colour."""
    b = np.conj(np.swapaxes(blocks, -1, -2))
    out = np.zeros_like(psi)
    v = psi[..., sites, :, :]
    flat = v.reshape(v.shape[:-2] + (12,))
    out[..., sites, :, :] = np.einsum("xij,...xj->...xi", b, flat).reshape(v.shape)
    return out


def schur_dagger(op, psi_e):
    """D^dag psi_e = D_ee^dag psi_e - D_oe^dag D_oo^-dag D_eo^dag psi_e."""
    lat = op.lat
    even, odd = lat.even, lat.odd
    x = op.restrict(psi_e, even)
    t = op.restrict(_hop_dagger(op, x), odd)          # D_eo^dag x (odd sites)
    u = _block_dagger(op.pauli_inv_odd(), t, odd)      # D_oo^-dag t
    v = op.restrict(_hop_dagger(op, u), even)          # D_oe^dag u (even sites)
    return _block_dagger(op.pauli[even], x, even) - v


class NormalOperator:
    """X = D^dag D^ + mu^2 on even-site vectors (mu: twisted mass)."""

    def __init__(self, op, mu=0.0):
        self.op = op
        self.mu2 = float(mu) ** 2

    def apply(self, psi_e):
        return schur_dagger(self.op, self.op.apply_schur(psi_e)) + self.mu2 * psi_e


# --------------------------------------------------------------------------
# multi-shift CG
# --------------------------------------------------------------------------
def multishift_cg(apply_x, b, shifts, tol, maxiter=100000, history=None):
    """Solve (X + sigma_j) x_j = b for every shift with one CG Krylov space.

    CG on X + sigma_0 (sigma_0 the smallest shift) generates residuals r_k and
    directions p_k; the residual of shift j is collinear, r_k^j = zeta_k^j r_k,
    with zeta from the three-term recurrence
        zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1}
                     / (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + s a_k)),
    s = sigma_j - sigma_0, zeta_0 = zeta_{-1} = 1, a_{-1} = 1, b_{-1} = 0; then
        a_k^j = a_k zeta_{k+1} / zeta_k,   b_k^j = b_k (zeta_{k+1} / zeta_k)^2,
        x^j += a_k^j p_k^j,   p_{k+1}^j = zeta_{k+1} r_{k+1} + b_k^j p_k^j.
    Shift j stops once |zeta^j r| <= tol |b|.  Returns ([x_j], iterations,
    [iterations of shift j])."""
    shifts = np.asarray(shifts, dtype=float)
    n = len(shifts)
    s0 = float(np.min(shifts))
    ds = shifts - s0
    bn = norm(b)
    xs = [np.zeros_like(b) for _ in range(n)]
    ps = [b.copy() for _ in range(n)]
    zeta = np.ones(n)
    zeta_old = np.ones(n)
    active = np.ones(n, dtype=bool)
    its = np.zeros(n, dtype=int)
    r = b.copy()
    p = b.copy()
    rr = np.real(dot(r, r))
    a_old, b_old = 1.0, 0.0
    it = 0
    while it < maxiter and np.any(active):
        q = apply_x(p) + s0 * p
        a = rr / np.real(dot(p, q))
        zeta_new = zeta.copy()
        for j in np.nonzero(active)[0]:
            den = a * b_old * (zeta_old[j] - zeta[j]) + zeta_old[j] * a_old * (1.0 + ds[j] * a)
            zeta_new[j] = zeta[j] * zeta_old[j] * a_old / den
            xs[j] = xs[j] + (a * zeta_new[j] / zeta[j]) * ps[j]
        r = r - a * q
        rr_new = np.real(dot(r, r))
        beta = rr_new / rr
        for j in np.nonzero(active)[0]:
            ps[j] = zeta_new[j] * r + beta * (zeta_new[j] / zeta[j]) ** 2 * ps[j]
            its[j] = it + 1
        p = r + beta * p
        zeta_old, zeta = zeta, zeta_new
        a_old, b_old, rr = a, beta, rr_new
        it += 1
        res = np.abs(zeta) * np.sqrt(rr)
        if history is not None:
            history.append(res / bn)
        active &= res > tol * bn
    return xs, it, its


def cg(apply_a, b, tol, maxiter=100000):
    """Plain conjugate gradient on a Hermitian positive definite A."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.real(dot(r, r))
    bn = norm(b)
    it = 0
    while np.sqrt(rr) > tol * bn and it < maxiter:
        q = apply_a(p)
        a = rr / np.real(dot(p, q))
        x = x + a * p
        r = r - a * q
        rr_new = np.real(dot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


# --------------------------------------------------------------------------
# rational functions of X
# --------------------------------------------------------------------------
class Rational:
    """R(t) = A prod_j (t + nu_j^2) / (t + mu_j^2)."""

    def __init__(self, A, nu, mu):
        self.A = float(A)
        self.nu = np.asarray(nu, dtype=float)
        self.mu = np.asarray(mu, dtype=float)
        if self.nu.shape != self.mu.shape:
            raise ValueError("as many zeros as poles")

    def __call__(self, t):
        t = np.asarray(t, dtype=float)[..., None]
        return self.A * np.prod((t + self.nu ** 2) / (t + self.mu ** 2), axis=-1)

    def partial_fractions(self):
        """rho_j with R(t) = A (1 + sum_j rho_j / (t + mu_j^2)): the residue of
        prod_k (t + nu_k^2) / (t + mu_k^2) at t = -mu_j^2."""
        a, bb = self.nu ** 2, self.mu ** 2
        rho = np.empty(len(bb))
        for j in range(len(bb)):
            num = np.prod(a - bb[j])
            den = np.prod(np.delete(bb, j) - bb[j])
            rho[j] = num / den
        return rho

    def factors(self, bounds):
        """Frequency-splitting factors P_k (A = 1) holding the zero/pole
        indices [bounds[k], bounds[k+1])."""
        return [Rational(1.0, self.nu[s:e], self.mu[s:e]) for s, e in zip(bounds[:-1], bounds[1:])]


def rational_apply(apply_x, rat, b, tol, maxiter=100000):
    """R(X) b = A (b + sum_j rho_j (X + mu_j^2)^-1 b)."""
    xs, _, _ = multishift_cg(apply_x, b, rat.mu ** 2, tol, maxiter)
    rho = rat.partial_fractions()
    out = b.copy()
    for j, x in enumerate(xs):
        out = out + rho[j] * x
    return rat.A * out
