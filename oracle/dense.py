"""Dense-matrix tools for tiny lattices (brute force for the pins).

dense_matrix(apply, V): the 12V x 12V matrix of a linear operator on spinors,
built column by column by applying it to unit vectors.
"""

import numpy as np


def dense_matrix(apply, n_sites, batch=768):
    n = 12 * n_sites
    m = np.empty((n, n), dtype=np.complex128)
    for s in range(0, n, batch):
        e = min(n, s + batch)
        basis = np.zeros((e - s, n), dtype=np.complex128)
        basis[np.arange(e - s), np.arange(s, e)] = 1.0
        cols = apply(basis.reshape(e - s, n_sites, 4, 3)).reshape(e - s, n)
        m[:, s:e] = cols.T
    return m


def site_dofs(sites):
    """Row/column indices of all 12 components of the given sites."""
    sites = np.asarray(sites)
    return (sites[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)
