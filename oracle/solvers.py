"""Solvers for the Dirac equation D psi = eta (FP64 reference).

The paper names the solvers it inherits (abstract; Sec. 2: "the locally-
deflated SAP-preconditioned GCR solver") but does not print their steps.  The
steps below follow the standard literature the paper builds on (Luscher's
Schwarz-preconditioned GCR); every choice is a stated reading:

  gcr          restarted GCR with stored (p_k, A p_k) and modified Gram-Schmidt.
  mr_steps     nmr minimal-residual steps: t = A s, alpha = (t,s)/(t,t),
               v += alpha s, s -= alpha t.
  sap_colour   one colour of the Schwarz alternating procedure: on every block
               of that colour the even-odd block problem is solved
               approximately by MR on the block Schur operator with Dirichlet
               faces; psi and the residual are updated.
  sap          ncy cycles over the two colours, starting from psi = 0.
  fgcr         flexible GCR, right-preconditioned by M (SAP), Gram-Schmidt on
               chi_k = D phi_k, coefficients by back-substitution.
  defect_correction
               outer loop x += s * inner(r / s), r = eta - D x, until
               |r| / |eta| <= tol.

Vectors are spinor arrays [V, 4, 3] complex128; inner products are
(a, b) = sum conj(a) b.
"""

import numpy as np

from .dirac import dot, norm


# --------------------------------------------------------------------------
# restarted GCR
# --------------------------------------------------------------------------
def gcr(apply_a, b, tol, nkv=16, maxiter=10000, x0=None, history=None):
    """Solve A x = b to |b - A x| <= tol |b|; returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = norm(b)
    r = b - apply_a(x)
    it = 0
    while it < maxiter:
        ps, qs = [], []
        for _k in range(nkv):
            p = r.copy()
            q = apply_a(p)
            for pl, ql in zip(ps, qs):
                beta = dot(ql, q)
                q = q - beta * ql
                p = p - beta * pl
            nq = norm(q)
            q /= nq
            p /= nq
            alpha = dot(q, r)
            x = x + alpha * p
            r = r - alpha * q
            ps.append(p)
            qs.append(q)
            it += 1
            rn = norm(r)
            if history is not None:
                history.append(rn / bn)
            if rn <= tol * bn or it >= maxiter:
                break
        r = b - apply_a(x)
        if norm(r) <= tol * bn:
            return x, it
    return x, it


def solve_eo(op, eta, tol, nkv=16, maxiter=10000):
    """Even-odd solve: D^ psi_e = eta^_e by GCR, then reconstruct psi_o.

    The GCR tolerance is tightened until the residual of the full system,
    |eta - D psi| / |eta|, meets tol.
    """
    eta_hat = op.eo_prepare(eta)
    en = norm(eta)
    t = tol
    psi_e = None
    total = 0
    for _ in range(6):
        psi_e, it = gcr(op.apply_schur, eta_hat, t * en / max(norm(eta_hat), 1e-300),
                        nkv=nkv, maxiter=maxiter, x0=psi_e)
        total += it
        psi = op.eo_reconstruct(psi_e, eta)
        if norm(eta - op.apply(psi)) <= tol * en:
            return psi, total
        t *= 0.1
    return psi, total


# --------------------------------------------------------------------------
# Schwarz alternating procedure
# --------------------------------------------------------------------------
class Blocks:
    """Block decomposition of the extended lattice and its two colours."""

    def __init__(self, lat, bs):
        self.lat = lat
        self.bs = tuple(bs)
        nb = []
        for mu in range(4):
            if lat.ext[mu] % bs[mu] or bs[mu] % 2:
                raise ValueError("block sizes must be even and divide the extents")
            nb.append(lat.ext[mu] // bs[mu])
        self.nb = tuple(nb)
        bc = lat.coords // np.array(bs)
        self.block_id = ((bc[:, 0] * nb[1] + bc[:, 1]) * nb[2] + bc[:, 2]) * nb[3] + bc[:, 3]
        self.n_blocks = nb[0] * nb[1] * nb[2] * nb[3]
        self.colour = bc.sum(axis=1) % 2

    def check_colouring(self):
        """No two blocks of one colour share a face (else SAP would race)."""
        lat = self.lat
        for mu in range(4):
            nbid = self.block_id[lat.fwd[mu]]
            cross = nbid != self.block_id
            if np.any(self.colour[lat.fwd[mu]][cross] == self.colour[cross]):
                return False
        return True


class BlockOperator:
    """D_Lambda on all blocks of one colour at once: D with the hops that leave
    a block dropped (Dirichlet faces), restricted to that colour's sites."""

    def __init__(self, op, blocks, colour):
        self.op = op
        self.blocks = blocks
        lat = op.lat
        self.sel = np.nonzero(blocks.colour == colour)[0]
        self.mask = np.zeros(lat.V, dtype=bool)
        self.mask[self.sel] = True
        bid = blocks.block_id
        # hop factors: link (x,mu) kept iff x and x+mu lie in the same block
        same = np.stack([bid[lat.fwd[mu]] == bid for mu in range(4)])
        self.fsign = lat.sign * same
        self.bsign = np.stack([self.fsign[mu, lat.bwd[mu]] for mu in range(4)])
        self.sel_e = np.nonzero(self.mask & (lat.parity == 0))[0]
        self.sel_o = np.nonzero(self.mask & (lat.parity == 1))[0]
        self.pinv_o = np.linalg.inv(op.pauli[self.sel_o])

    def hop(self, psi):
        from .dirac import EYE4, GAMMA
        lat, op = self.op.lat, self.op
        out = np.zeros_like(psi)
        for mu in range(4):
            fw = psi[lat.fwd[mu]] * self.fsign[mu][:, None, None]
            fw = np.einsum("xab,xsb->xsa", op.w[:, mu], fw)
            out += np.einsum("st,xtc->xsc", EYE4 - GAMMA[mu], fw)
            bw = psi[lat.bwd[mu]] * self.bsign[mu][:, None, None]
            bw = np.einsum("xab,xsb->xsa", op.wd[lat.bwd[mu], mu], bw)
            out += np.einsum("st,xtc->xsc", EYE4 + GAMMA[mu], bw)
        out = -0.5 * out
        out[~self.mask] = 0
        return out

    def _on(self, psi, sites):
        out = np.zeros_like(psi)
        out[sites] = psi[sites]
        return out

    def apply(self, psi):
        out = self.op.apply_pauli(psi) + self.hop(psi)
        out[~self.mask] = 0
        return out

    def oo_inv(self, psi):
        out = np.zeros_like(psi)
        out[self.sel_o] = np.einsum("xij,xj->xi", self.pinv_o,
                                    psi[self.sel_o].reshape(-1, 12)).reshape(-1, 4, 3)
        return out

    def schur(self, s_e):
        """D^_Lambda s_e = D_ee s_e - D_eo D_oo^-1 D_oe s_e on every block."""
        dee = self._on(self.op.apply_pauli(s_e), self.sel_e)
        u = self.oo_inv(self._on(self.hop(self._on(s_e, self.sel_e)), self.sel_o))
        return dee - self._on(self.hop(u), self.sel_e)

    def block_dot(self, a, b):
        """Per-block inner products (a, b)_Lambda, indexed by block id."""
        v = np.sum(np.conj(a) * b, axis=(1, 2))
        return np.bincount(self.blocks.block_id, weights=v.real, minlength=self.blocks.n_blocks) \
            + 1j * np.bincount(self.blocks.block_id, weights=v.imag, minlength=self.blocks.n_blocks)

    def mr_steps(self, rho_e, nmr):
        """nmr MR steps on D^_Lambda v_e = rho_e per block; returns (v_e, s)."""
        bid = self.blocks.block_id
        v = np.zeros_like(rho_e)
        s = rho_e.copy()
        for _ in range(nmr):
            t = self.schur(s)
            ts = self.block_dot(t, s)
            tt = self.block_dot(t, t).real
            alpha = np.where(tt > 0, ts / np.where(tt > 0, tt, 1.0), 0.0)
            a_site = alpha[bid][:, None, None]
            v = v + a_site * s
            s = s - a_site * t
        return v, s

    def solve(self, r, nmr):
        """Approximate D_Lambda^-1 r on every block of the colour (even-odd MR)."""
        r_e = self._on(r, self.sel_e)
        r_o = self._on(r, self.sel_o)
        rho_e = r_e - self._on(self.hop(self.oo_inv(r_o)), self.sel_e)
        v_e, _ = self.mr_steps(rho_e, nmr)
        v_o = self.oo_inv(r_o - self._on(self.hop(v_e), self.sel_o))
        return v_e + v_o


def sap_colour(op, blocks, colour, psi, r, nmr, bop=None):
    """One colour of SAP: psi += v, r -= D v with v the block solutions."""
    bop = bop or BlockOperator(op, blocks, colour)
    v = bop.solve(r, nmr)
    return psi + v, r - op.apply(v)


def sap(op, blocks, rho, ncy, nmr, bops=None):
    """M_SAP rho: ncy cycles of (black, white) block solves from psi = 0."""
    bops = bops or (BlockOperator(op, blocks, 0), BlockOperator(op, blocks, 1))
    psi = np.zeros_like(rho)
    r = rho.copy()
    for _ in range(ncy):
        for c in (0, 1):
            psi, r = sap_colour(op, blocks, c, psi, r, nmr, bops[c])
    return psi


# --------------------------------------------------------------------------
# single blocks of lattices too large to build the whole operator
# --------------------------------------------------------------------------
def block_solve_at(lat, u_ext, a_ext, sites, r, nmr, kappa, q=0.0, csw=0.0, csw_u1=1.0, q_el=1.0 / 6.0):
    """BlockOperator.solve for one block from the site formula: D_Lambda (D
    on the block's sites with every hop that leaves the block dropped) as a
    dense matrix over the block, built from the Pauli term at those sites and
    the links between them, then the same even-odd MR steps.  sites: the
    block's sites, r: the residual on them [n, 4, 3].  Returns v [n, 4, 3]."""
    from .dirac import EYE4, GAMMA
    from .fields import charge_hat, pauli_term
    sites = np.asarray(sites)
    n = len(sites)
    pos = {int(x): i for i, x in enumerate(sites)}
    qhat = charge_hat(q, q_el) if a_ext is not None else 0
    p = pauli_term(lat, u_ext, a_ext, kappa, q if a_ext is not None else 0.0, csw, csw_u1, q_el, sites)
    d = np.zeros((n, 12, n, 12), dtype=complex)
    for i in range(n):
        d[i, :, i, :] = p[i]

    def link(x, mu):
        w = u_ext[x, mu]
        return w * np.exp(1j * qhat * a_ext[x, mu]) if qhat else w

    for i, x in enumerate(sites):
        for mu in range(4):
            yf, yb = int(lat.fwd[mu][x]), int(lat.bwd[mu][x])
            if yf in pos and not lat.frozen[x]:
                d[i, :, pos[yf], :] += -0.5 * lat.sign[mu][x] * np.kron(EYE4 - GAMMA[mu], link(x, mu))
            if yb in pos and not lat.frozen[yb]:
                d[i, :, pos[yb], :] += -0.5 * lat.bsign[mu][x] * np.kron(EYE4 + GAMMA[mu],
                                                                         np.conj(link(yb, mu)).T)
    d = d.reshape(12 * n, 12 * n)
    par = lat.parity[sites]
    ie = (12 * np.nonzero(par == 0)[0][:, None] + np.arange(12)).reshape(-1)
    io = (12 * np.nonzero(par == 1)[0][:, None] + np.arange(12)).reshape(-1)
    dee, deo, doe = d[np.ix_(ie, ie)], d[np.ix_(ie, io)], d[np.ix_(io, ie)]
    doo_inv = np.linalg.inv(d[np.ix_(io, io)])
    rf = r.reshape(-1)
    r_e, r_o = rf[ie], rf[io]
    rho_e = r_e - deo @ (doo_inv @ r_o)
    v_e = np.zeros_like(rho_e)
    s_e = rho_e.copy()
    for _ in range(nmr):
        t = dee @ s_e - deo @ (doo_inv @ (doe @ s_e))
        tt = np.real(np.vdot(t, t))
        alpha = np.vdot(t, s_e) / tt if tt > 0 else 0.0
        v_e = v_e + alpha * s_e
        s_e = s_e - alpha * t
    v = np.zeros(12 * n, dtype=complex)
    v[ie] = v_e
    v[io] = doo_inv @ (r_o - doe @ v_e)
    return v.reshape(n, 4, 3)


def sap_cycle_block_at(lat, u_ext, a_ext, blocks, r, b, nmr, kappa, q=0.0, csw=0.0, csw_u1=1.0, q_el=1.0 / 6.0):
    """M_SAP r after one cycle (ncy = 1, from psi = 0), on the sites of block
    b only, from the site formula: a colour-0 block holds its block solve of
    r; a colour-1 block the block solve of r - D v0, where v0 holds the block
    solves of r on the colour-0 blocks next to it (the only ones D v0 reaches
    it from).  r: the residual on the whole lattice [V, 4, 3].  Returns
    (sites of b, M_SAP r on them)."""
    from .dirac import apply_at_sites
    bid = blocks.block_id
    sites = np.nonzero(bid == b)[0]
    if blocks.colour[sites[0]] == 0:
        return sites, block_solve_at(lat, u_ext, a_ext, sites, r[sites], nmr, kappa, q, csw, csw_u1, q_el)
    nbrs = set()
    for mu in range(4):
        for nb in (lat.fwd[mu][sites], lat.bwd[mu][sites]):
            nbrs.update(int(c) for c in np.unique(bid[nb]) if c != b)
    v0 = np.zeros_like(r)
    for c in sorted(nbrs):
        sc = np.nonzero(bid == c)[0]
        v0[sc] = block_solve_at(lat, u_ext, a_ext, sc, r[sc], nmr, kappa, q, csw, csw_u1, q_el)
    rb = r[sites] - apply_at_sites(lat, u_ext, a_ext, v0, sites, kappa, q, csw, csw_u1, q_el)
    return sites, block_solve_at(lat, u_ext, a_ext, sites, rb, nmr, kappa, q, csw, csw_u1, q_el)


# --------------------------------------------------------------------------
# flexible GCR with a variable right preconditioner
# --------------------------------------------------------------------------
def fgcr(apply_d, precond, b, tol, nkv=16, maxiter=1000, history=None):
    """Solve D x = b with x = sum beta_k phi_k, phi_k = M rho_k.

    Per cycle: chi_k = D phi_k is orthogonalised against chi_0..k-1
    (a_lk = (chi_l, chi_k)), normalised (b_k = |chi_k|), c_k = (chi_k, rho_k),
    rho_{k+1} = rho_k - c_k chi_k.  At the end of the cycle the upper
    triangular system (diagonal b, off-diagonal a) is solved for beta with
    right-hand side c and x += sum beta_k phi_k; the next cycle restarts from
    rho = b - D x.
    """
    x = np.zeros_like(b)
    bn = norm(b)
    rho = b.copy()
    it = 0
    while it < maxiter:
        phis, chis = [], []
        a = np.zeros((nkv, nkv), dtype=complex)
        bk = np.zeros(nkv)
        c = np.zeros(nkv, dtype=complex)
        k_used = 0
        done = False
        for k in range(nkv):
            phi = precond(rho)
            chi = apply_d(phi)
            for l in range(k):
                a[l, k] = dot(chis[l], chi)
                chi = chi - a[l, k] * chis[l]
            bk[k] = norm(chi)
            chi = chi / bk[k]
            c[k] = dot(chi, rho)
            rho = rho - c[k] * chi
            phis.append(phi)
            chis.append(chi)
            k_used = k + 1
            it += 1
            rn = norm(rho)
            if history is not None:
                history.append(rn / bn)
            if rn <= tol * bn or it >= maxiter:
                done = True
                break
        beta = np.zeros(k_used, dtype=complex)
        for k in range(k_used - 1, -1, -1):
            s = c[k] - sum(a[k, j] * beta[j] for j in range(k + 1, k_used))
            beta[k] = s / bk[k]
        for k in range(k_used):
            x = x + beta[k] * phis[k]
        rho = b - apply_d(x)
        if done and norm(rho) <= tol * bn:
            break
    return x, it


def defect_correction(apply_d, inner_solve, eta, tol, max_outer=100, history=None):
    """x += s * inner(r / s) with r = eta - D x and s = |r| until |r| <= tol |eta|."""
    x = np.zeros_like(eta)
    r = eta.copy()
    en = norm(eta)
    outer = 0
    while norm(r) > tol * en and outer < max_outer:
        s = norm(r)
        delta = inner_solve(r / s)
        x = x + s * delta
        r = eta - apply_d(x)
        outer += 1
        if history is not None:
            history.append(norm(r) / en)
    return x, outer
