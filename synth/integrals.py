"""Seeded molecular-like integrals h_pq and g_pqrs = (pq|rs) (chemists' notation).

The paper's molecules and their integrals are not available, so these recipes
stand in for them (Sec. "Preparation of benchmark systems"): a linear-chain
pi-system like the PAH series, and block-structured iron-sulfur-like integrals.
Every g is built in density-fitting form g_pqrs = sum_L B^L_pq B^L_rs with each
B^L symmetric, which makes g 8-fold symmetric and positive semidefinite as a
(pq),(rs) matrix before the explicit on-site / exchange overrides.

Draw order is fixed (numpy default_rng / PCG64): off-diagonal h first (upper
triangle, row-major), then B (per L, upper triangle including the diagonal,
row-major), then any override draws.  "N(mu, sigma)" means standard deviation
sigma.
"""
from __future__ import annotations

import numpy as np


def _sym_from_triu(n, vals, k):
    m = np.zeros((n, n))
    iu = np.triu_indices(n, k)
    m[iu] = vals
    m = m + np.triu(m, 1).T
    return m


def _g_from_b(b):
    nb = b.shape[0]
    n = b.shape[1]
    bm = b.reshape(nb, n * n)
    return (bm.T @ bm).reshape(n, n, n, n)


def chain_linear_h(n, rng, sigma=0.05):
    """Diagonal linearly spaced -2..+1 Eh, off-diagonals N(0, sigma) symmetrised."""
    h = _sym_from_triu(n, rng.normal(0.0, sigma, n * (n - 1) // 2), 1)
    h[np.diag_indices(n)] = -2.0 + 3.0 * np.arange(n) / max(n - 1, 1)
    return h


def small_cas(n, seed, naux=None, b_sigma=0.3):
    """Small-CAS recipe: linear h diagonal, random B (entries N(0, 0.3))."""
    rng = np.random.default_rng(seed)
    naux = 32 if naux is None else naux
    h = chain_linear_h(n, rng)
    b = np.stack([_sym_from_triu(n, v, 0) for v in rng.normal(0.0, b_sigma, (naux, n * (n + 1) // 2))])
    return h, _g_from_b(b), b


def huckel_chain(n, seed, naux=None, b_scale=0.3, decay=4.0):
    """Hueckel-like chain: on-site 0, nearest-neighbour hopping -1 Eh, further
    neighbours N(0, 0.02); B^L_pq = b_scale * exp(-|p-q|/decay) * z, z ~ N(0,1)."""
    h, b = huckel_chain_hb(n, seed, naux, b_scale, decay)
    return h, _g_from_b(b), b


def embedded_cas(n_core=48, n_act=24, n_virt=48, seed=3, naux=None, shift=2.0):
    """Orbital-gradient workload: the Hueckel-chain recipe over
    n = n_core + n_act + n_virt orbitals (naux = 3n density-fitting vectors),
    with the core diagonal of h shifted by -shift and the virtual diagonal by
    +shift Eh.  Returns (h, B); the four-index g is not formed."""
    n = n_core + n_act + n_virt
    h, b = huckel_chain_hb(n, seed, naux)
    idx = np.arange(n)
    h[idx[:n_core], idx[:n_core]] -= shift
    v = idx[n_core + n_act:]
    h[v, v] += shift
    return h, b


def huckel_chain_hb(n, seed, naux=None, b_scale=0.3, decay=4.0):
    """h and B of ``huckel_chain`` (same draws, g not formed)."""
    rng = np.random.default_rng(seed)
    naux = 3 * n if naux is None else naux
    h = _sym_from_triu(n, rng.normal(0.0, 0.02, n * (n - 1) // 2), 1)
    idx = np.arange(n)
    h[idx, idx] = 0.0
    h[idx[:-1], idx[:-1] + 1] = -1.0
    h[idx[:-1] + 1, idx[:-1]] = -1.0
    dist = np.abs(idx[:, None] - idx[None, :])
    env = b_scale * np.exp(-dist / decay)
    b = np.stack([_sym_from_triu(n, v, 0) for v in rng.normal(0.0, 1.0, (naux, n * (n + 1) // 2))]) * env
    return h, b


FES_LAYOUT = (("L", 6), ("d", 8), ("L", 12), ("d", 8), ("L", 12), ("d", 8), ("L", 12), ("d", 8), ("L", 8))


def iron_sulfur_like(seed, layout=FES_LAYOUT):
    """Fe-S-like chain: four blocks of 8 d-like orbitals separated by ligand
    orbitals.  Base is the Hueckel chain recipe (naux = 3n); then in each d block
    g_pppp += U(0.6, 0.9) and for p != q the exchange-type elements
    g_pqpq = g_pqqp = g_qppq = g_qpqp += K_pq ~ U(0.05, 0.1); finally every
    nearest-neighbour hop that touches a ligand orbital becomes N(-0.3, 0.05)."""
    kinds = "".join(k * m for k, m in layout)
    n = len(kinds)
    h, g, b = huckel_chain(n, seed)
    rng = np.random.default_rng(seed + 7919)
    pos = 0
    for kind, m in layout:
        if kind == "d":
            blk = np.arange(pos, pos + m)
            for p in blk:
                g[p, p, p, p] += rng.uniform(0.6, 0.9)
            for i, p in enumerate(blk):
                for q in blk[i + 1:]:
                    kx = rng.uniform(0.05, 0.1)
                    g[p, q, p, q] += kx
                    g[p, q, q, p] += kx
                    g[q, p, p, q] += kx
                    g[q, p, q, p] += kx
        pos += m
    for p in range(n - 1):
        if kinds[p] == "L" or kinds[p + 1] == "L":
            t = rng.normal(-0.3, 0.05)
            h[p, p + 1] = t
            h[p + 1, p] = t
    return h, g, b


def hubbard_dimer(t=1.0, u=3.0):
    """Two-site Hubbard model written as integrals: h_01 = -t, g_pppp = U."""
    h = np.array([[0.0, -t], [-t, 0.0]])
    g = np.zeros((2, 2, 2, 2))
    g[0, 0, 0, 0] = u
    g[1, 1, 1, 1] = u
    return h, g
