"""Truncation at the middle cut of the two-site block, by definition.

DMRG keeps the D states of largest weight in the reduced density matrix of
one side of the cut (Sec. "Numerical procedure": fixed D or fixed truncation
error; Sec. "Error sources": the error is controlled by D).  On the explicit
Fock-space wavefunction the weights are the squared Schmidt values of the
bipartition (sites 0..k | sites k+1..n-1): an SVD of the reshaped vector.
With SU(2) symmetry every multiplet of spin S_a appears as 2S_a+1 equal
Schmidt values for a singlet state, so a multiplet's weight is their sum.
"""
from __future__ import annotations

import numpy as np

from .mps_fock import Embedding


def schmidt_values(mps, layout, psi):
    """Schmidt values (descending) of the two-site wavefunction across the
    middle cut, from its Fock-space expansion at M = S."""
    emb = Embedding(mps, layout)
    phi = emb.expand(psi).reshape(emb.nr, 4, 4, emb.nl)  # [right, site k+1, site k, left]
    # left part: (site k, left) ; right part: (right, site k+1)
    mat = phi.transpose(2, 3, 0, 1).reshape(4 * emb.nl, emb.nr * 4)
    return np.linalg.svd(mat, compute_uv=False)


def discarded_weight(values, keep):
    w = np.sort(np.asarray(values) ** 2)[::-1]
    return float(w[keep:].sum() / w.sum())
