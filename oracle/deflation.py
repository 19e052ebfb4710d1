"""Local deflation of the SAP-preconditioned GCR solver (FP64 reference; test
infrastructure only).

The paper's solver for the expensive pseudofermion factors is the locally
deflated SAP-GCR it inherits from openQCD (abstract; Sec. 2 feature list;
Appendix A, where it serves every twisted mass but the largest; Table 2, rows
8-14), built on the local coherence of the low modes of D (Luscher 2007, cited
in the feature list).  The paper does not print its steps; they are taken
from that published method, and every choice below is a reading:

  deflation_fields  Ns global fields psi_l, random on input, each refined by
                    ninv steps of approximate inverse iteration,
                    psi <- M_sap psi / |M_sap psi|, with the Schwarz
                    preconditioner (ncy, nmr) as the approximate inverse of D.
  Basis             the block-restricted fields theta_Lambda psi_l (theta the
                    restriction to the SAP block Lambda), orthonormalised block
                    by block by modified Gram-Schmidt in the order l = 0 ..
                    Ns-1.  The deflation subspace S = span{phi_{Lambda,k}} has
                    dimension Ns x (number of blocks); V is the isometry from
                    coefficient vectors c[Lambda, k] to fields,
                    V c = sum_{Lambda,k} c[Lambda, k] phi_{Lambda,k}.
  little_operator   A = V^dag D V, the Dirac operator on S: the entry
                    ((Lambda, k), (Lambda', l)) is (phi_{Lambda,k},
                    D phi_{Lambda',l}); it vanishes unless Lambda' is Lambda
                    or one of its neighbours (D couples nearest neighbours).
  deflated_precond  M_dfl r = V A^-1 V^dag r + M_sap (r - D V A^-1 V^dag r):
                    the solution on S first, then the Schwarz preconditioner
                    on the residual that remains.  With
                    P_L = 1 - D V A^-1 V^dag this is V A^-1 V^dag + M_sap P_L.
  dfl_solve         defect correction around FGCR right-preconditioned by
                    M_dfl, as for the SAP solver.

If S is the whole space (Ns = 12 x block volume), V is unitary, V A^-1 V^dag =
D^-1 and M_dfl = D^-1 exactly; the tests pin the chain on that limit.

Fields are spinor arrays [V, 4, 3] complex128; a basis is an array
[Ns, V, 4, 3] whose k-th field holds phi_{Lambda,k} on every block Lambda;
coefficient vectors are arrays [n_blocks, Ns] complex128.
"""

import numpy as np

from .dirac import norm
from .solvers import BlockOperator, defect_correction, fgcr, sap


# --------------------------------------------------------------------------
# the deflation subspace
# --------------------------------------------------------------------------
def block_dots(blocks, a, b):
    """(a, b)_Lambda for every block, indexed by block id."""
    v = np.sum(np.conj(a) * b, axis=(-2, -1))
    return np.bincount(blocks.block_id, weights=v.real, minlength=blocks.n_blocks) \
        + 1j * np.bincount(blocks.block_id, weights=v.imag, minlength=blocks.n_blocks)


def deflation_fields(op, blocks, psi0, ninv, ncy, nmr):
    """The Ns global fields after ninv SAP-smoothed inverse-iteration steps
    from the given start fields psi0 [Ns, V, 4, 3]."""
    bops = (BlockOperator(op, blocks, 0), BlockOperator(op, blocks, 1))
    out = []
    for psi in psi0:
        psi = psi / norm(psi)
        for _ in range(ninv):
            psi = sap(op, blocks, psi, ncy, nmr, bops)
            psi = psi / norm(psi)
        out.append(psi)
    return np.array(out)


def block_orthonormalise(blocks, fields):
    """phi_{Lambda,k}: on every block, modified Gram-Schmidt of the restricted
    fields theta_Lambda psi_l in the order l = 0 .. Ns-1."""
    bid = blocks.block_id
    phi = fields.copy()
    for k in range(len(phi)):
        for j in range(k):
            c = block_dots(blocks, phi[j], phi[k])
            phi[k] = phi[k] - c[bid][:, None, None] * phi[j]
        n = np.sqrt(block_dots(blocks, phi[k], phi[k]).real)
        if np.any(n == 0):
            raise ValueError("a restricted deflation field vanishes on some block")
        phi[k] = phi[k] / n[bid][:, None, None]
    return phi


# --------------------------------------------------------------------------
# V, V^dag and the little operator
# --------------------------------------------------------------------------
def restrict(blocks, phi, r):
    """V^dag r: c[Lambda, k] = (phi_{Lambda,k}, r)_Lambda."""
    return np.stack([block_dots(blocks, p, r) for p in phi], axis=1)


def prolong(blocks, phi, c):
    """V c = sum_{Lambda,k} c[Lambda, k] phi_{Lambda,k}."""
    bid = blocks.block_id
    out = np.zeros(phi.shape[1:], dtype=complex)
    for k in range(len(phi)):
        out += c[bid, k][:, None, None] * phi[k]
    return out


def little_operator(op, blocks, phi):
    """A = V^dag D V as a dense matrix over the index (Lambda, k) ->
    Lambda * Ns + k, column by column: column (Lambda', l) is V^dag D of the
    single basis vector phi_{Lambda',l}."""
    ns, nb = len(phi), blocks.n_blocks
    a = np.zeros((nb * ns, nb * ns), dtype=complex)
    bid = blocks.block_id
    for lb in range(nb):
        on = (bid == lb)[:, None, None]
        for l in range(ns):
            col = restrict(blocks, phi, op.apply(phi[l] * on))
            a[:, lb * ns + l] = col.reshape(-1)
    return a


class Deflation:
    """The deflation subspace of one operator with its little operator; the
    little system is solved exactly (dense LU)."""

    def __init__(self, op, blocks, phi):
        self.op, self.blocks, self.phi = op, blocks, phi
        self.ns = len(phi)
        self.a = little_operator(op, blocks, phi)

    def coarse(self, r):
        """V A^-1 V^dag r."""
        c = restrict(self.blocks, self.phi, r).reshape(-1)
        y = np.linalg.solve(self.a, c).reshape(self.blocks.n_blocks, self.ns)
        return prolong(self.blocks, self.phi, y)

    def project_left(self, r):
        """P_L r = r - D V A^-1 V^dag r."""
        return r - self.op.apply(self.coarse(r))

    def precond(self, r, ncy, nmr, bops=None):
        """M_dfl r = V A^-1 V^dag r + M_sap (r - D V A^-1 V^dag r)."""
        u = self.coarse(r)
        return u + sap(self.op, self.blocks, r - self.op.apply(u), ncy, nmr, bops)


def dfl_solve(dfl, eta, tol, ncy, nmr, nkv=16, inner_tol=1e-14, maxiter=1000, history=None):
    """Defect correction around FGCR(M_dfl); returns (psi, total FGCR
    iterations)."""
    bops = (BlockOperator(dfl.op, dfl.blocks, 0), BlockOperator(dfl.op, dfl.blocks, 1))
    its = []

    def inner(r):
        x, it = fgcr(dfl.op.apply, lambda v: dfl.precond(v, ncy, nmr, bops), r, inner_tol, nkv=nkv,
                     maxiter=maxiter, history=history)
        its.append(it)
        return x

    psi, _ = defect_correction(dfl.op.apply, inner, eta, tol)
    return psi, sum(its)
