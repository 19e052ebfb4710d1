"""Seeded synthetic inputs shared by the FP64 oracle tests and the GPU path.

This module only draws random numbers and shapes them into the input arrays
the library accepts: SU(3) and U(1) link fields on the physical lattice, and
quark sources on the extended lattice.  It contains none of the Dirac
operator's arithmetic, no geometry beyond array sizes, and no C* orbifold
construction (the mirror half of the gauge field is built by the library and,
independently, by the oracle).

Layouts (all host numpy arrays, C order):
  * SU(3) links  U[V_phs, 4, 3, 3] complex128, U[x, mu, a, b] = row a, col b.
  * U(1) angles  A[V_phs, 4] float64 in [-pi, pi).
  * spinors      psi[V_ext, 4, 3] complex128 (spin index outer, colour inner).
Sites are lexicographic with x0 slowest and x3 fastest; on the physical
lattice the extent of direction 1 is L1, on the extended lattice it is 2*L1
under C* boundary conditions.

Draw order (fixed, so that a seed identifies an input bit for bit):
  links: G = N(0,1) real parts for all [V_phs,4,3,3] entries, then the
  imaginary parts; angles: one N(0, sigma) per [V_phs,4]; Gaussian source:
  real parts for all [V_ext,4,3], then imaginary parts.
"""

import numpy as np


def rng_from_seed(seed):
    return np.random.Generator(np.random.PCG64(seed))


def su3_links(rng, n_sites, eps, chunk=1 << 18):
    """SU(3) links U = GramSchmidt(1 + i*eps*H), H = (G + G^dag)/2.

    G has independent N(0,1) real and imaginary parts.  The rows of M are
    orthonormalised and the third row is replaced by conj(row1 x row2), which
    makes U special unitary and U ~ exp(i*eps*H) for small eps.
    """
    out = np.empty((n_sites, 4, 3, 3), dtype=np.complex128)
    re = rng.standard_normal((n_sites, 4, 3, 3))
    im = rng.standard_normal((n_sites, 4, 3, 3))
    for s in range(0, n_sites, chunk):
        e = min(n_sites, s + chunk)
        g = re[s:e] + 1j * im[s:e]
        h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
        m = np.eye(3) + 1j * eps * h
        r0 = m[..., 0, :]
        r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
        r1 = m[..., 1, :]
        r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
        r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
        r2 = np.conj(np.cross(r0, r1))
        out[s:e, :, 0, :] = r0
        out[s:e, :, 1, :] = r1
        out[s:e, :, 2, :] = r2
    return out


def u1_angles(rng, n_sites, sigma):
    """U(1) gauge potential A ~ N(0, sigma) per link, wrapped to [-pi, pi)."""
    a = rng.normal(0.0, sigma, size=(n_sites, 4))
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def gaussian_source(rng, n_sites):
    """Spinor with independent N(0,1) real and imaginary parts."""
    re = rng.standard_normal((n_sites, 4, 3))
    im = rng.standard_normal((n_sites, 4, 3))
    return re + 1j * im


def point_source(n_sites, site, spin, colour):
    eta = np.zeros((n_sites, 4, 3), dtype=np.complex128)
    eta[site, spin, colour] = 1.0
    return eta


def phys_volume(dims):
    t, l1, l2, l3 = dims
    return t * l1 * l2 * l3


def ext_volume(dims, cstar):
    t, l1, l2, l3 = dims
    return t * (2 * l1 if cstar else l1) * l2 * l3


def gauge_field(dims, seed, eps, sigma=None):
    """(U, A) on the physical lattice; A is None for SU(3)-only fields."""
    rng = rng_from_seed(seed)
    v = phys_volume(dims)
    u = su3_links(rng, v, eps)
    a = u1_angles(rng, v, sigma) if sigma is not None else None
    return u, a


def source(dims, cstar, seed):
    return gaussian_source(rng_from_seed(seed), ext_volume(dims, cstar))
