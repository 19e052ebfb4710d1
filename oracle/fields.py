"""Gauge fields on the extended lattice, clover field tensors, Pauli term.

Orbifold (Sec. 2.1, eq. "orbi:gauge"): on the mirror lattice the gauge field
is the charge conjugate of the physical one, U(x + L1 e1, mu) = U(x, mu)^*
and A(x + L1 e1, mu) = -A(x, mu).

Hopping links (Sec. 2.3): the covariant derivatives carry
W(x, mu) = U(x, mu) z(x, mu)^qhat with z = exp(iA) and the integer charge
qhat = q / q_el.

Clover (Sec. 2.3): the SU(3) field tensor is the clover average of the
Luscher-Sint-Sommer-Weisz paper cited there,
    F(x) = (Q_munu(x) - Q_numu(x)) / 8,
with Q_munu the sum of the four plaquette leaves in the (mu, nu) plane that
start and end at x, all with the same orientation (no trace subtraction).  The
U(1) tensor is the paper's explicit formula
    Ahat_munu(x) = i/(4 q_el) Im{ z_munu(x) + z_munu(x-mu) + z_munu(x-nu)
                                  + z_munu(x-mu-nu) }.
With open time boundaries, links crossing x0 = T-1 -> 0 do not exist and the
leaves that contain one are dropped.

Pauli term: P(x) = (4 + m0) + c_sw sum_{mu,nu} (i/4) sigma_munu F_munu
                   + q c_sw^U(1) sum_{mu,nu} (i/4) sigma_munu Ahat_munu,
with m0 = 1/(2 kappa) - 4 and sigma_munu = (i/2)[gamma_mu, gamma_nu].
"""

import numpy as np

from .dirac import sigma_munu

PLANES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def dagger(m):
    return np.conj(np.swapaxes(m, -1, -2))


def extend_gauge(lat, u_phs, a_phs=None):
    """Extended-lattice fields from physical ones via the orbifold constraint."""
    u = np.empty((lat.V, 4, 3, 3), dtype=np.complex128)
    a = np.zeros((lat.V, 4), dtype=np.float64)
    ph = lat.phys_index()
    u[ph] = u_phs
    if a_phs is not None:
        a[ph] = a_phs
    if lat.cstar:
        mi = lat.mirror(ph)
        u[mi] = np.conj(u_phs)
        if a_phs is not None:
            a[mi] = -a_phs
    return u, a


def charge_hat(q, q_el):
    qh = q / q_el
    r = round(qh)
    if abs(qh - r) > 1e-9:
        raise ValueError("q / q_el must be an integer")
    return int(r)


def theta_phases(lat, theta):
    """Fermion boundary phases [V, 4] (Sec. 2 feature list: theta-periodic
    fermions in periodic space directions).  psi(x + L_mu e_mu) = e^{i theta_mu}
    psi(x) is realised as the factor e^{i theta_mu} on every link (x, mu) whose
    forward hop crosses the boundary of direction mu.  Reading for C* lattices:
    on the mirror half the phase is conjugated, e^{-i theta_mu}, as the
    orbifold constraint conjugates every U(1) field there (Sec. 2.1); this
    keeps D[U,z] T = T D[U*,z*] and the antisymmetry of C T D (Sec. 2.4).
    theta_0 multiplies the antiperiodic sign of the time hop; it must vanish
    with open time, and theta_k must vanish in C* directions (direction 1 is
    C* whenever any is)."""
    ph = np.ones((lat.V, 4), dtype=np.complex128)
    if theta is None:
        return ph
    theta = np.asarray(theta, dtype=float)
    for mu in range(4):
        if theta[mu] == 0.0:
            continue
        if (mu == 0 and lat.time_bc != 0) or (mu >= 1 and mu in lat.cstar_dirs):
            raise ValueError(f"theta_{mu} must be 0 for this boundary condition")
        cross = lat.coords[:, mu] == lat.ext[mu] - 1
        sgn = np.where(lat.is_phys, 1.0, -1.0)
        ph[cross, mu] = np.exp(1j * theta[mu] * sgn[cross])
    return ph


def hopping_links(lat, u, a, qhat, theta=None):
    """W(x, mu) = U(x, mu) exp(i qhat A(x, mu)), times the fermion boundary
    phase of theta_phases on the links that cross a boundary.  With SF or
    open-SF time boundaries the links of the fixed slice x0 = 0 carry no hop
    (the fermion field vanishes there), so that slice is decoupled."""
    w = u * (np.exp(1j * qhat * a) * theta_phases(lat, theta))[:, :, None, None]
    if lat.frozen.any():
        w = w.copy()
        w[lat.frozen] = 0.0
    return w


def _existing(lat):
    """1 for links that exist in the gauge field, 0 for the links an open time
    end cuts (open and open-SF; with SF the links into x0 = T exist)."""
    return lat.link_exists  # [4, V]


def su3_field_tensor(lat, u, sites=None):
    """F[plane, x, 3, 3] for the six planes mu < nu (anti-Hermitian), at all
    sites or at the listed ones."""
    ex = _existing(lat)
    x = np.arange(lat.V) if sites is None else np.asarray(sites)

    def U(y, mu):
        return u[y, mu] * ex[mu][y][:, None, None]

    def Ud(y, mu):
        return dagger(U(y, mu))

    f = np.empty((6, len(x), 3, 3), dtype=np.complex128)
    for p, (mu, nu) in enumerate(PLANES):
        xpm = lat.fwd[mu][x]
        xpn = lat.fwd[nu][x]
        xmm = lat.bwd[mu][x]
        xmn = lat.bwd[nu][x]
        xmm_pn = lat.fwd[nu][xmm]     # x - mu + nu
        xmm_mn = lat.bwd[nu][xmm]     # x - mu - nu
        xpm_mn = lat.fwd[mu][xmn]     # x + mu - nu
        q = (_chain([U(x, mu), U(xpm, nu), Ud(xpn, mu), Ud(x, nu)])
             + _chain([U(x, nu), Ud(xmm_pn, mu), Ud(xmm, nu), U(xmm, mu)])
             + _chain([Ud(xmm, mu), Ud(xmm_mn, nu), U(xmm_mn, mu), U(xmn, nu)])
             + _chain([Ud(xmn, nu), U(xmn, mu), U(xpm_mn, nu), Ud(x, mu)]))
        f[p] = (q - dagger(q)) / 8.0
    return f


def _chain(ms):
    r = ms[0]
    for m in ms[1:]:
        r = r @ m
    return r


def u1_field_tensor(lat, a, q_el, sites=None):
    """Ahat[plane, x] for mu < nu, the paper's formula (purely imaginary)."""
    ex = _existing(lat)
    x = np.arange(lat.V) if sites is None else np.asarray(sites)

    def z(y, mu):
        return np.exp(1j * a[y, mu]) * ex[mu][y]

    def zmn(y, mu, nu):
        return z(y, mu) * z(lat.fwd[mu][y], nu) * np.conj(z(lat.fwd[nu][y], mu)) * np.conj(z(y, nu))

    ah = np.empty((6, len(x)), dtype=np.complex128)
    for p, (mu, nu) in enumerate(PLANES):
        xmm = lat.bwd[mu][x]
        xmn = lat.bwd[nu][x]
        s = zmn(x, mu, nu) + zmn(xmm, mu, nu) + zmn(xmn, mu, nu) + zmn(lat.bwd[nu][xmm], mu, nu)
        ah[p] = 1j / (4.0 * q_el) * np.imag(s)
    return ah


def boundary_term(lat, sites=None):
    """The coefficient of dD_b per site (Sec. 2.3): with open time (c_F - 1) on
    x0 = 0 and T-1; with SF (c_F - 1) on x0 = 1 and T-1; with open-SF
    (c_F - 1) on x0 = 1 and (c_F' - 1) on x0 = T-1; zero with periodic time."""
    x0 = lat.coords[:, 0] if sites is None else lat.coords[np.asarray(sites), 0]
    t = lat.phys[0]
    d = np.zeros(len(x0))
    if lat.time_bc == 1:
        d[(x0 == 0) | (x0 == t - 1)] = lat.cF - 1.0
    elif lat.time_bc == 2:
        d[(x0 == 1) | (x0 == t - 1)] = lat.cF - 1.0
    elif lat.time_bc == 3:
        d[x0 == 1] = lat.cF - 1.0
        d[x0 == t - 1] = lat.cF_prime - 1.0
    return d


def pauli_term(lat, u, a, kappa, q, csw, csw_u1, q_el, sites=None):
    """P[x, 12, 12] on spin (x) colour, index s*3 + c (all or listed sites):
    4 + m0 + dD_sw + dD_b, and the identity on the fixed slice of SF and
    open-SF time boundaries."""
    p = _pauli_bulk(lat, u, a, kappa, q, csw, csw_u1, q_el, sites)
    p += boundary_term(lat, sites)[:, None, None] * np.eye(12)
    fz = lat.frozen if sites is None else lat.frozen[np.asarray(sites)]
    p[fz] = np.eye(12)
    return p


def _pauli_bulk(lat, u, a, kappa, q, csw, csw_u1, q_el, sites=None):
    m0 = 1.0 / (2.0 * kappa) - 4.0
    f = su3_field_tensor(lat, u, sites)
    n = f.shape[1]
    p = np.zeros((n, 12, 12), dtype=np.complex128)
    p += (4.0 + m0) * np.eye(12)
    eye3 = np.eye(3)
    if a is not None and q != 0.0:
        ah = u1_field_tensor(lat, a, q_el, sites)
    else:
        ah = None
    for k, (mu, nu) in enumerate(PLANES):
        # sum over both orders (mu,nu), (nu,mu) of (i/4) sigma F = (i/2) sigma F for mu<nu
        s = 0.5j * sigma_munu(mu, nu)
        p += csw * np.einsum("st,xab->xsatb", s, f[k]).reshape(n, 12, 12)
        if ah is not None:
            p += q * csw_u1 * np.einsum("st,x,ab->xsatb", s, ah[k], eye3).reshape(n, 12, 12)
    return p
