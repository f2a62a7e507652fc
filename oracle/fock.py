"""Determinant (Fock) space, the ab-initio Hamiltonian, S^2 and brute-force FCI.

Spin-orbital P = 2p + sigma (sigma = 0 up, 1 down), orbital-major in chain
order with up before down.  A determinant is the integer whose bit P is the
occupation of P, and stands for prod_{P ascending} (a+_P)^{n_P} |0>.  So
a_Q |n> = (-1)^{#occupied P < Q} |n - e_Q>, and a+_P likewise.  A full
Fock-space vector of n orbitals is indexed by this integer directly.

Hamiltonian (Sec. "Complete active space SCF"; the printed two-electron term is
read with the standard pairing and the factor 1/2, see the readings list):

    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) sum_{s,t} a+_{p s} a+_{r t} a_{s t} a_{q s}

with E_pq = sum_s a+_{p s} a_{q s}.  Using the anticommutation relations,
sum_{st} a+_ps a+_rt a_st a_qs = E_pq E_rs - delta_qr E_ps, which is how it is
applied here (the standard direct-CI form); ``jw_hamiltonian`` builds the same
operator literally from Jordan-Wigner matrices for tiny n as a cross-check.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def sector_dets(n, n_up, n_dn):
    """Sorted determinants with n_up up and n_dn down electrons in n orbitals."""
    ups = [sum(1 << (2 * p) for p in c) for c in itertools.combinations(range(n), n_up)]
    dns = [sum(1 << (2 * p + 1) for p in c) for c in itertools.combinations(range(n), n_dn)]
    d = np.array([u | v for u in ups for v in dns], dtype=np.int64)
    d.sort()
    return d


def _popcount_below(d, pos):
    return np.bitwise_count(d & np.int64((1 << pos) - 1)).astype(np.int64)


def excitation(src, P, Q, dst):
    """Sparse matrix of a+_P a_Q mapping span(src) -> span(dst) (both sorted)."""
    has_q = (src >> Q) & 1 == 1
    d1 = src ^ np.int64(1 << Q)
    ok = has_q & (((d1 >> P) & 1) == 0)
    cols = np.nonzero(ok)[0]
    d1 = d1[cols]
    sgn = _popcount_below(src[cols], Q) + _popcount_below(d1, P)
    d2 = d1 | np.int64(1 << P)
    rows = np.searchsorted(dst, d2)
    inb = rows < len(dst)
    rows, cols, sgn, d2 = rows[inb], cols[inb], sgn[inb], d2[inb]
    hit = dst[rows] == d2
    vals = np.where(sgn[hit] % 2 == 0, 1.0, -1.0)
    return sp.csr_matrix((vals, (rows[hit], cols[hit])), shape=(len(dst), len(src)))


def epq_matrices(n, dets):
    """E_pq = sum_sigma a+_{p sigma} a_{q sigma} on span(dets), all p, q."""
    return [[excitation(dets, 2 * p, 2 * q, dets) + excitation(dets, 2 * p + 1, 2 * q + 1, dets)
             for q in range(n)] for p in range(n)]


def hamiltonian_sparse(h, g, dets, e=None):
    """H on span(dets) as a sparse matrix (direct-CI form E E - delta E)."""
    n = h.shape[0]
    e = epq_matrices(n, dets) if e is None else e
    t = h - 0.5 * np.einsum("prrq->pq", g)
    dim = len(dets)
    hm = sp.csr_matrix((dim, dim))
    for p in range(n):
        for q in range(n):
            if t[p, q] != 0.0:
                hm = hm + t[p, q] * e[p][q]
    for r in range(n):
        for s in range(n):
            gpq = sp.csr_matrix((dim, dim))
            for p in range(n):
                for q in range(n):
                    if g[p, q, r, s] != 0.0:
                        gpq = gpq + g[p, q, r, s] * e[p][q]
            hm = hm + 0.5 * (gpq @ e[r][s])
    return hm.tocsr()


def apply_h(h, g, dets, v, e=None):
    """H v for v on span(dets), matrix-free: D_rs = E_rs v, W_pq = sum g_pqrs D_rs,
    H v = sum_pq E_pq (t_pq v + W_pq / 2)."""
    n = h.shape[0]
    e = epq_matrices(n, dets) if e is None else e
    t = h - 0.5 * np.einsum("prrq->pq", g)
    dmat = np.stack([e[r][s] @ v for r in range(n) for s in range(n)])
    w = g.reshape(n * n, n * n) @ dmat
    out = np.zeros_like(v)
    for p in range(n):
        for q in range(n):
            out += e[p][q] @ (t[p, q] * v + 0.5 * w[p * n + q])
    return out


def s2_matrix(n, n_elec, two_m):
    """S^2 = S- S+ + Sz^2 + Sz on the (N, M) determinant sector, and the dets."""
    n_up = (n_elec + two_m) // 2
    n_dn = n_elec - n_up
    d0 = sector_dets(n, n_up, n_dn)
    dim = len(d0)
    sz = two_m / 2.0
    m = sp.identity(dim, format="csr") * (sz * sz + sz)
    if n_dn > 0 and n_up < n:
        d1 = sector_dets(n, n_up + 1, n_dn - 1)
        splus = sum(excitation(d0, 2 * p, 2 * p + 1, d1) for p in range(n))
        sminus = sum(excitation(d1, 2 * p + 1, 2 * p, d0) for p in range(n))
        m = m + sminus @ splus
    return m.tocsr(), d0


def fci_spectrum(h, g, n_elec, two_s):
    """All eigenvalues of H restricted to total spin S (brute force, dense).

    Works in the M = S determinant sector, projects onto the S^2 = S(S+1)
    eigenspace, and diagonalises H there."""
    n = h.shape[0]
    s2, dets = s2_matrix(n, n_elec, two_s)
    w, u = np.linalg.eigh(s2.toarray())
    target = two_s / 2.0 * (two_s / 2.0 + 1.0)
    basis = u[:, np.abs(w - target) < 1e-8]
    hm = hamiltonian_sparse(h, g, dets)
    hs = basis.T @ (hm @ basis)
    return np.linalg.eigvalsh(0.5 * (hs + hs.T))


# ---- literal Jordan-Wigner construction, tiny n only (cross-check) ------------------

def jw_annihilators(n):
    """Dense 4^n x 4^n matrices of a_P (P = 2p + sigma) on the full Fock space."""
    dim = 1 << (2 * n)
    idx = np.arange(dim, dtype=np.int64)
    ops = []
    for P in range(2 * n):
        has = (idx >> P) & 1 == 1
        src = idx[has]
        dst = src ^ (1 << P)
        sgn = np.where(np.bitwise_count(src & ((1 << P) - 1)) % 2 == 0, 1.0, -1.0)
        a = np.zeros((dim, dim))
        a[dst, src] = sgn
        ops.append(a)
    return ops


def jw_hamiltonian(h, g):
    """H built literally: sum h_pq a+_ps a_qs + 1/2 sum g_pqrs a+_ps a+_rt a_st a_qs."""
    n = h.shape[0]
    a = jw_annihilators(n)
    ad = [x.T for x in a]
    dim = a[0].shape[0]
    hm = np.zeros((dim, dim))
    for p in range(n):
        for q in range(n):
            for s in range(2):
                hm += h[p, q] * ad[2 * p + s] @ a[2 * q + s]
    for p, q, r, s_ in itertools.product(range(n), repeat=4):
        if g[p, q, r, s_] == 0.0:
            continue
        for s in range(2):
            for t in range(2):
                hm += 0.5 * g[p, q, r, s_] * ad[2 * p + s] @ ad[2 * r + t] @ a[2 * s_ + t] @ a[2 * q + s]
    return hm
