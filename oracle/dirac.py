"""Wilson-clover Dirac operator and its even-odd Schur complement.

Paper Sec. 2.3: D = m0 + Dw + dD_sw + dD_b (dD_b: fields.boundary_term), with
    Dw = sum_mu (1/2) { gamma_mu (nabla_mu + nabla*_mu) - nabla*_mu nabla_mu },
    nabla_mu psi(x)  = W(x,mu) psi(x+mu) - psi(x),
    nabla*_mu psi(x) = psi(x) - W(x-mu,mu)^dag psi(x-mu).
For unitary W this expands to the site formula used here,
    (D psi)(x) = P(x) psi(x)
               - 1/2 sum_mu [ (1 - gamma_mu) W(x,mu) psi(x+mu)
                            + (1 + gamma_mu) W(x-mu,mu)^dag psi(x-mu) ],
with P(x) = 4 + m0 + dD_sw(x) the Pauli term; hops across the time boundary
carry the fermion sign (-1 antiperiodic, 0 open).

Paper Sec. 2.4: even-odd blocks D_ee, D_eo, D_oe, D_oo with the standard
site parity, and the Schur complement D^ = D_ee - D_eo D_oo^-1 D_oe.

Gamma matrices: chiral basis, 2x2 blocks with Pauli matrices s_k,
    gamma_0 = [[0, -1], [-1, 0]],  gamma_k = [[0, -i s_k], [i s_k, 0]],
so that gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1, 1, -1, -1) and
the charge-conjugation matrix C = gamma_0 gamma_2 is real with C^T = -C,
C^dag = C^-1, C gamma_mu C^-1 = -gamma_mu^T (Sec. 2.1).

Spinor layout: psi[..., V, 4, 3] complex128 (spin outer, colour inner).
"""

import numpy as np

_S = [np.array([[0, 1], [1, 0]], dtype=complex),
      np.array([[0, -1j], [1j, 0]], dtype=complex),
      np.array([[1, 0], [0, -1]], dtype=complex)]
_I2 = np.eye(2, dtype=complex)
_Z2 = np.zeros((2, 2), dtype=complex)

GAMMA = [np.block([[_Z2, -_I2], [-_I2, _Z2]])] + [
    np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in _S]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
CMAT = GAMMA[0] @ GAMMA[2]
EYE4 = np.eye(4, dtype=complex)


def sigma_munu(mu, nu):
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


class DiracOperator:
    """D on one gauge field for one quark flavour (FP64, plain definition)."""

    def __init__(self, lat, w, pauli):
        self.lat = lat
        self.w = w                      # [V, 4, 3, 3] hopping links U z^qhat
        self.wd = np.conj(np.swapaxes(w, -1, -2))
        self.pauli = pauli              # [V, 12, 12]
        self._pinv_odd = None

    # -- pieces -----------------------------------------------------------
    def hop(self, psi):
        """H psi = -1/2 sum_mu [(1-g_mu) W psi(x+mu) + (1+g_mu) W^dag(x-mu) psi(x-mu)]."""
        lat = self.lat
        out = np.zeros_like(psi)
        for mu in range(4):
            fw = psi[..., lat.fwd[mu], :, :] * lat.sign[mu][:, None, None]
            fw = np.einsum("xab,...xsb->...xsa", self.w[:, mu], fw)
            out += np.einsum("st,...xtc->...xsc", EYE4 - GAMMA[mu], fw)
            bw = psi[..., lat.bwd[mu], :, :] * lat.bsign[mu][:, None, None]
            bw = np.einsum("xab,...xsb->...xsa", self.wd[lat.bwd[mu], mu], bw)
            out += np.einsum("st,...xtc->...xsc", EYE4 + GAMMA[mu], bw)
        return -0.5 * out

    def apply_pauli(self, psi, sites=None):
        p = self.pauli if sites is None else self.pauli[sites]
        shp = psi.shape
        flat = psi.reshape(shp[:-2] + (12,))
        return np.einsum("xij,...xj->...xi", p, flat).reshape(shp)

    def apply(self, psi):
        """(D psi) on all of the extended lattice."""
        return self.apply_pauli(psi) + self.hop(psi)

    def apply_g5(self, psi):
        return np.einsum("st,...xtc->...xsc", GAMMA5, psi)

    # -- even-odd ---------------------------------------------------------
    def pauli_inv_odd(self):
        if self._pinv_odd is None:
            self._pinv_odd = np.linalg.inv(self.pauli[self.lat.odd])
        return self._pinv_odd

    def restrict(self, psi, sites):
        out = np.zeros_like(psi)
        out[..., sites, :, :] = psi[..., sites, :, :]
        return out

    def apply_oo_inv(self, psi):
        """D_oo^-1 on the odd sites (zero on even sites)."""
        out = np.zeros_like(psi)
        odd = self.lat.odd
        shp = psi[..., odd, :, :].shape
        flat = psi[..., odd, :, :].reshape(shp[:-2] + (12,))
        out[..., odd, :, :] = np.einsum("xij,...xj->...xi", self.pauli_inv_odd(), flat).reshape(shp)
        return out

    def d_oe(self, psi_e):
        """D_oe psi_e: hops from even to odd sites (result on odd sites)."""
        return self.restrict(self.hop(self.restrict(psi_e, self.lat.even)), self.lat.odd)

    def d_eo(self, psi_o):
        return self.restrict(self.hop(self.restrict(psi_o, self.lat.odd)), self.lat.even)

    def apply_schur(self, psi_e):
        """D^ psi_e = D_ee psi_e - D_eo D_oo^-1 D_oe psi_e (even sites)."""
        even = self.lat.even
        dee = self.restrict(self.apply_pauli(self.restrict(psi_e, even)), even)
        return dee - self.d_eo(self.apply_oo_inv(self.d_oe(psi_e)))

    def eo_prepare(self, eta):
        """eta^_e = eta_e - D_eo D_oo^-1 eta_o."""
        return self.restrict(eta, self.lat.even) - self.d_eo(self.apply_oo_inv(eta))

    def eo_reconstruct(self, psi_e, eta):
        """psi = psi_e + D_oo^-1 (eta_o - D_oe psi_e)."""
        odd_part = self.apply_oo_inv(self.restrict(eta, self.lat.odd) - self.d_oe(psi_e))
        return self.restrict(psi_e, self.lat.even) + odd_part


def build_operator(lat, u_ext, a_ext, kappa, q=0.0, csw=0.0, csw_u1=1.0, q_el=1.0 / 6.0, theta=None):
    """D for one flavour from extended-lattice U, A (a_ext may be None);
    theta: fermion boundary phases (fields.theta_phases)."""
    from .fields import charge_hat, hopping_links, pauli_term
    qhat = charge_hat(q, q_el) if a_ext is not None else 0
    a = a_ext if a_ext is not None else np.zeros((lat.V, 4))
    w = hopping_links(lat, u_ext, a, qhat, theta)
    p = pauli_term(lat, u_ext, a_ext, kappa, q if a_ext is not None else 0.0, csw, csw_u1, q_el)
    return DiracOperator(lat, w, p)


def apply_at_sites(lat, u_ext, a_ext, psi, sites, kappa, q=0.0, csw=0.0, csw_u1=1.0, q_el=1.0 / 6.0):
    """(D psi)(x) at the listed sites only, by the same site formula, for
    lattices too large to build the whole operator (no boundary phases)."""
    from .fields import charge_hat, pauli_term
    sites = np.asarray(sites)
    qhat = charge_hat(q, q_el) if a_ext is not None else 0
    p = pauli_term(lat, u_ext, a_ext, kappa, q if a_ext is not None else 0.0, csw, csw_u1, q_el, sites)
    out = np.einsum("xij,xj->xi", p, psi[sites].reshape(-1, 12)).reshape(-1, 4, 3)
    acc = np.zeros_like(out)
    for mu in range(4):
        yf = lat.fwd[mu][sites]
        yb = lat.bwd[mu][sites]
        live_f = (~lat.frozen[sites]).astype(float)[:, None, None]
        live_b = (~lat.frozen[yb]).astype(float)[:, None, None]
        wf = live_f * u_ext[sites, mu] * (np.exp(1j * qhat * a_ext[sites, mu])[:, None, None] if qhat else 1.0)
        wb = live_b * u_ext[yb, mu] * (np.exp(1j * qhat * a_ext[yb, mu])[:, None, None] if qhat else 1.0)
        fw = np.einsum("xab,xsb->xsa", wf, psi[yf]) * lat.sign[mu][sites][:, None, None]
        bw = np.einsum("xba,xsb->xsa", np.conj(wb), psi[yb]) * lat.bsign[mu][sites][:, None, None]
        acc += np.einsum("st,xtc->xsc", EYE4 - GAMMA[mu], fw)
        acc += np.einsum("st,xtc->xsc", EYE4 + GAMMA[mu], bw)
    return out - 0.5 * acc


def schur_at_sites(lat, u_ext, a_ext, psi, sites, kappa, q=0.0, csw=0.0, csw_u1=1.0, q_el=1.0 / 6.0):
    """(D^ psi_e)(x) = (D_ee psi_e - D_eo D_oo^-1 D_oe psi_e)(x) at the listed
    even sites only (the odd entries of psi are not used), by the site
    formula, for lattices too large to build the whole operator: D_oe psi_e
    on the odd neighbours of the sites, D_oo^-1 there from the Pauli term at
    those sites, then D_eo of the result at the sites."""
    from .fields import pauli_term
    sites = np.asarray(sites)
    if np.any(lat.parity[sites] != 0):
        raise ValueError("schur_at_sites takes even sites")
    qq = q if a_ext is not None else 0.0
    pe = psi.copy()
    pe[lat.parity == 1] = 0
    odd = np.unique(np.concatenate([lat.fwd[mu][sites] for mu in range(4)] + [lat.bwd[mu][sites] for mu in range(4)]))
    # D psi_e on odd sites is D_oe psi_e (the Pauli term meets zeros there)
    z = apply_at_sites(lat, u_ext, a_ext, pe, odd, kappa, qq, csw, csw_u1, q_el).reshape(-1, 12)
    p_o = pauli_term(lat, u_ext, a_ext, kappa, qq, csw, csw_u1, q_el, odd)
    t = np.zeros_like(psi)
    t[odd] = np.linalg.solve(p_o, z[..., None])[..., 0].reshape(-1, 4, 3)
    # D t on the even sites is D_eo t (t vanishes on even sites)
    dt = apply_at_sites(lat, u_ext, a_ext, t, sites, kappa, qq, csw, csw_u1, q_el)
    p_e = pauli_term(lat, u_ext, a_ext, kappa, qq, csw, csw_u1, q_el, sites)
    return np.einsum("xij,xj->xi", p_e, pe[sites].reshape(-1, 12)).reshape(-1, 4, 3) - dt


def normal_at_sites(lat, u_ext, a_ext, psi, sites, kappa, q=0.0, csw=0.0, csw_u1=1.0, q_el=1.0 / 6.0, mu=0.0):
    """(X psi_e)(x) with X = D^dag D^ + mu^2 at the listed even sites only, by
    the site formula (D^dag = g5 D^ g5 on even sites): D^ psi_e on the even
    sites two hops around them, then D^ of g5 times that at the sites."""
    sites = np.asarray(sites)
    odd = np.unique(np.concatenate([lat.fwd[m][sites] for m in range(4)] + [lat.bwd[m][sites] for m in range(4)]))
    near = np.unique(np.concatenate([sites] + [lat.fwd[m][odd] for m in range(4)] + [lat.bwd[m][odd] for m in range(4)]))
    y = np.zeros_like(psi)
    y[near] = schur_at_sites(lat, u_ext, a_ext, psi, near, kappa, q, csw, csw_u1, q_el)
    g5y = np.einsum("st,xtc->xsc", GAMMA5, y)
    out = np.einsum("st,xtc->xsc", GAMMA5,
                    schur_at_sites(lat, u_ext, a_ext, g5y, sites, kappa, q, csw, csw_u1, q_el))
    return out + mu * mu * psi[sites]


def dot(a, b):
    """(a, b) = sum conj(a) b over everything."""
    return np.vdot(a, b)


def norm(a):
    return np.sqrt(np.real(np.vdot(a, a)))
