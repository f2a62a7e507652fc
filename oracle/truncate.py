"""Truncation at the middle cut of the two-site block, by definition.

DMRG keeps the D states of largest weight in the reduced density matrix of
one side of the cut (Sec. "Numerical procedure": fixed D or fixed truncation
error; Sec. "Error sources": the error is controlled by D).  On the explicit
Fock-space wavefunction the weights are the squared Schmidt values of the
bipartition (sites 0..k | sites k+1..n-1): an SVD of the reshaped vector.
With SU(2) symmetry every multiplet of spin S_a appears as 2S_a+1 equal
Schmidt values for a singlet state, so a multiplet's weight is their sum.

Dynamic block state selection (Sec. "Numerical procedure": the number of
kept states follows from a fixed truncation error rather than a fixed D)
keeps the fewest multiplets, largest weights first, whose discarded weight is
at most eps_tr of the total, within [d_min, d_max].
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


def multiplet_weights(values, rel_tol=1e-9):
    """Group the Schmidt values of a singlet state into SU(2) multiplets: a run
    of 2S+1 equal values is one multiplet of spin S with weight the sum of
    their squares.  Returns (weights, two_s), weights descending; values
    below rel_tol of the largest are dropped (the cut's null space).  The
    grouping relies on distinct multiplets having distinct weights, which
    holds for random wavefunctions."""
    v = np.sort(np.asarray(values, dtype=np.float64))[::-1]
    v = v[v > rel_tol * v[0]]
    weights, two_s = [], []
    i = 0
    while i < v.size:
        j = i + 1
        while j < v.size and abs(v[j] - v[i]) <= rel_tol * v[i]:
            j += 1
        weights.append(float((v[i:j] ** 2).sum()))
        two_s.append(j - i - 1)
        i = j
    # a multiplet's weight is (2S+1) v^2, so value order is not weight order
    order = np.argsort(-np.array(weights), kind="stable")
    return np.array(weights)[order], np.array(two_s)[order]


def dbss_keep(weights, eps_tr, d_min, d_max):
    """Number of multiplets kept: the smallest m such that the weights beyond
    the m largest sum to at most eps_tr of the total, then clamped to
    [d_min, d_max] and to the number of multiplets.  eps_tr = 0 keeps
    min(d_max, count)."""
    w = np.sort(np.asarray(weights, dtype=np.float64))[::-1]
    count = w.size
    if eps_tr <= 0.0:
        return min(d_max, count)
    total = w.sum()
    m = count
    # tail[m] = weight discarded when m multiplets are kept
    tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])
    for cand in range(1, count + 1):
        if tail[cand] <= eps_tr * total:
            m = cand
            break
    return min(d_max, max(m, min(d_min, count)))
