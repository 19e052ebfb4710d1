"""Shared helpers of the GPU parity tests: build the same synthetic field for
the oracle (numpy, FP64) and the HIP library, and move spinors around."""

import numpy as np

from oracle import Lattice
from oracle import dirac as od
from oracle import fields as of
from paper_1710_08839_amd import synth


class Case:
    """One gauge field and quark on both sides."""

    def __init__(self, ctx, dims, cstar=0, time_bc=0, eps=0.3, sigma=0.15, kappa=0.124, q=2 / 3,
                 csw=1.0, csw_u1=1.0, seed=1, block=(4, 4, 4, 4), u1=True, cF=1.0, cF_prime=1.0):
        from paper_1710_08839_amd import qxd
        self.dims, self.cstar, self.time_bc = dims, cstar, time_bc
        self.lat = Lattice(dims, cstar=cstar, time_bc=time_bc, cF=cF, cF_prime=cF_prime)
        self.u, self.a = synth.gauge_field(dims, seed, eps, sigma if u1 else None)
        ue, ae = of.extend_gauge(self.lat, self.u, self.a)
        self.op = od.build_operator(self.lat, ue, ae if u1 else None, kappa, q=q, csw=csw, csw_u1=csw_u1)
        self.field = qxd.Field(ctx, dims, self.u, self.a, cstar=cstar, time_bc=time_bc, block=block, cF=cF,
                               cF_prime=cF_prime)
        self.quark = qxd.quark(kappa, q, csw, csw_u1)
        self.V = self.lat.V
        assert self.field.volume == self.V

    def source(self, seed):
        return synth.gaussian_source(synth.rng_from_seed(seed), self.V)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def to_host(t):
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
