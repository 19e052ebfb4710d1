"""Extended lattice, C* shifted boundary conditions and neighbour tables.

Paper Sec. 2.1: with C* boundary conditions in direction 1 (and possibly 2
and 3) the code simulates the extended lattice L0 x 2L1 x L2 x L3, whose
second half in direction 1 is the mirror lattice.  All fields are periodic
with period 2L1 in direction 1 (eq. "periodic"); a C* direction k = 2, 3 is
realised by shifted boundary conditions: a step across x_k = L_k - 1 -> 0
also moves x1 by L1 (eq. "shifted", Fig. 1).

Time (Sec. 2 feature list: open, SF, open-SF, periodic; Sec. 2.3: the
boundary improvement term dD_b):
  time_bc = 0  periodic gauge field, antiperiodic fermions;
  time_bc = 1  open: the hop across x0 = T-1 -> 0 is absent;
  time_bc = 2  Schroedinger functional (SF): the fermion field is fixed to zero
               on the boundary slice x0 = 0 (stored as a slice whose rows and
               columns of D are the identity), the hop across x0 = T-1 -> 0 is
               absent;
  time_bc = 3  open-SF: SF at x0 = 0, open at x0 = T-1.
The improvement coefficients cF (and cF_prime at the open end of open-SF)
enter dD_b (fields.pauli_term).

Site index: ((x0*N1 + x1)*L2 + x2)*L3 + x3 with N1 = 2L1 under C*, else L1.
"""

import numpy as np


class Lattice:
    def __init__(self, dims, cstar=0, time_bc=0, cF=1.0, cF_prime=1.0):
        dims = tuple(int(d) for d in dims)
        if len(dims) != 4:
            raise ValueError("dims must be (T, L1, L2, L3)")
        if cstar not in (0, 1, 2, 3):
            raise ValueError("cstar must be 0..3")
        if time_bc not in (0, 1, 2, 3):
            raise ValueError("time_bc must be 0 (antiperiodic), 1 (open), 2 (SF) or 3 (open-SF)")
        self.phys = dims
        self.cstar = cstar
        self.time_bc = time_bc
        self.cF = float(cF)
        self.cF_prime = float(cF_prime)
        t, l1, l2, l3 = dims
        self.L1 = l1
        n1 = 2 * l1 if cstar else l1
        self.ext = (t, n1, l2, l3)
        self.V = t * n1 * l2 * l3
        self.Vphs = t * l1 * l2 * l3
        # C* directions: cstar=1 -> {1}, 2 -> {1,2}, 3 -> {1,2,3}
        self.cstar_dirs = set(range(1, cstar + 1))

        idx = np.arange(self.V)
        x3 = idx % l3
        x2 = (idx // l3) % l2
        x1 = (idx // (l3 * l2)) % n1
        x0 = idx // (l3 * l2 * n1)
        self.coords = np.stack([x0, x1, x2, x3], axis=1)
        self.parity = (x0 + x1 + x2 + x3) % 2

        self.fwd = np.empty((4, self.V), dtype=np.int64)
        self.sign = np.ones((4, self.V), dtype=np.float64)  # sign of link (x, mu)
        for mu in range(4):
            y = self.coords.copy()
            y[:, mu] += 1
            wrap = y[:, mu] == self.ext[mu]
            y[wrap, mu] = 0
            if mu == 0:
                self.sign[0, wrap] = -1.0 if time_bc == 0 else 0.0
            elif mu in (2, 3) and mu in self.cstar_dirs:
                # shifted boundary: x + L_k e_k is identified with x + L1 e_1
                y[wrap, 1] = (y[wrap, 1] + l1) % n1
            self.fwd[mu] = self.index(y)
        self.bwd = np.empty_like(self.fwd)
        for mu in range(4):
            self.bwd[mu, self.fwd[mu]] = idx
        # the sign of the hop x -> x - mu belongs to the link (x - mu, mu)
        self.bsign = np.stack([self.sign[mu, self.bwd[mu]] for mu in range(4)])

        # SF and open-SF: the slice x0 = 0 is the fixed (zero) boundary field
        self.frozen = (self.coords[:, 0] == 0) if time_bc in (2, 3) else np.zeros(self.V, dtype=bool)
        # links that exist in the gauge field: the time links across
        # x0 = T-1 -> 0 are absent at an open end (open, open-SF); with SF
        # they connect the bulk to the boundary at x0 = T
        self.link_exists = np.ones((4, self.V))
        if time_bc in (1, 3):
            self.link_exists[0, self.coords[:, 0] == t - 1] = 0.0

        self.even = np.nonzero(self.parity == 0)[0]
        self.odd = np.nonzero(self.parity == 1)[0]
        self.is_phys = self.coords[:, 1] < l1

    def index(self, c):
        t, n1, l2, l3 = self.ext
        c = np.asarray(c)
        return ((c[..., 0] * n1 + c[..., 1]) * l2 + c[..., 2]) * l3 + c[..., 3]

    def mirror(self, idx=None):
        """x -> x + L1 e_1 (mod 2L1): the translation T of eq. "translation"."""
        if not self.cstar:
            raise ValueError("no mirror lattice without C* boundary conditions")
        c = self.coords.copy() if idx is None else self.coords[idx].copy()
        c[..., 1] = (c[..., 1] + self.L1) % self.ext[1]
        return self.index(c)

    def phys_index(self):
        """Extended-lattice index of every physical site, in physical lex order."""
        return np.nonzero(self.is_phys)[0]
