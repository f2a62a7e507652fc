"""CAS-SCF energy as a function of an orbital rotation, and its gradient, by
definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Complete active space SCF": the DMRG-SCF macro-iteration alternates a
DMRG solve (reduced density matrices at fixed orbitals) with an orbital step
that lowers the energy at fixed density matrices by a rotation of the
orbitals.  Reading (the paper gives no formulas for this step):

* the rotation is U = exp(-K), K antisymmetric with K_pq = kappa_pq (p > q)
  and K_qp = -kappa_pq; integrals transform as h(kappa) = U^T h U and, in
  density-fitting form (pq|rs) = sum_L B^L_pq B^L_rs, as B^L(kappa) =
  U^T B^L U;
* orbitals are ordered core (doubly occupied), active, virtual, and at fixed
  spin-summed RDMs of the active space, gamma~_tu = <sum_s a+_ts a_us> and
  Gamma~_tuvw = <sum_st a+_ts a+_ut a_vt a_ws>,

    E(kappa) = 2 sum_i h_ii + sum_ij [2 (ii|jj) - (ij|ji)]
               + sum_tu F^c_tu gamma~_tu + 1/2 sum_tuvw (tu|vw) Gamma~_tvwu,
    F^c_pq  = h_pq + sum_i [2 (pq|ii) - (pi|iq)]

  (i, j core; t, u, v, w active; integrals at kappa).

Two routes to the gradient dE/dkappa_pq (p > q), independent of each other:
``gradient_fd`` differentiates ``energy`` by central differences, and
``generalized_fock_gradient`` is the closed form at kappa = 0,
2 (F_pq - F_qp) with F_pq = sum_r D_pr h_qr + sum_rst P_prst (qr|st) built
from the full-space one- and two-body density matrices D and P.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def kappa_matrix(kappa_lower):
    """K from kappa (n x n; only the strictly lower triangle is read)."""
    k = np.tril(np.asarray(kappa_lower, dtype=np.float64), -1)
    return k - k.T


def rotation(kappa_lower):
    return expm(-kappa_matrix(kappa_lower))


def transform(h, B, kappa_lower):
    u = rotation(kappa_lower)
    return u.T @ h @ u, np.einsum("pa,Lpq,qb->Lab", u, B, u, optimize=True)


def energy_from_integrals(h, B, gamma, Gamma, n_core, n_act):
    c = slice(0, n_core)
    a = slice(n_core, n_core + n_act)
    g_ccaa = np.einsum("Lij,Lkl->ijkl", B[:, c, c], B[:, c, c])
    e = 2.0 * np.trace(h[c, c])
    e += 2.0 * np.einsum("iijj->", g_ccaa) - np.einsum("ijji->", g_ccaa)
    # F^c over the active block
    j_core = np.einsum("Ltu,Lii->tu", B[:, a, a], B[:, c, c])
    k_core = np.einsum("Lti,Liu->tu", B[:, a, c], B[:, c, a])
    fc = h[a, a] + 2.0 * j_core - k_core
    e += np.einsum("tu,tu->", fc, gamma)
    g_aaaa = np.einsum("Ltu,Lvw->tuvw", B[:, a, a], B[:, a, a])
    e += 0.5 * np.einsum("tuvw,tvwu->", g_aaaa, Gamma)
    return float(e)


def energy(h, B, kappa_lower, gamma, Gamma, n_core, n_act):
    hk, bk = transform(h, B, kappa_lower)
    return energy_from_integrals(hk, bk, gamma, Gamma, n_core, n_act)


def gradient_fd(h, B, kappa_lower, gamma, Gamma, n_core, n_act, step=1e-5, pairs=None):
    """Central differences of ``energy`` in kappa_pq for p > q (all pairs, or
    the given list); returns the antisymmetric matrix G with G_pq = dE/dkappa_pq."""
    n = h.shape[0]
    k0 = np.tril(np.asarray(kappa_lower, dtype=np.float64), -1)
    grad = np.zeros((n, n))
    todo = pairs if pairs is not None else [(p, q) for p in range(n) for q in range(p)]
    for p, q in todo:
        kp = k0.copy()
        kp[p, q] += step
        km = k0.copy()
        km[p, q] -= step
        d = (energy(h, B, kp, gamma, Gamma, n_core, n_act) - energy(h, B, km, gamma, Gamma, n_core, n_act)) / (2 * step)
        grad[p, q] = d
        grad[q, p] = -d
    return grad


def full_density_matrices(gamma, Gamma, n_core, n_act, n):
    """D and P (E = sum D_pq h_pq + 1/2 sum P_pqrs (pq|rs)) over all n orbitals:
    the doubly occupied core, the active RDMs, zero on the virtuals."""
    c = range(n_core)
    a0 = n_core
    D = np.zeros((n, n))
    P = np.zeros((n, n, n, n))
    for i in c:
        D[i, i] = 2.0
    D[a0:a0 + n_act, a0:a0 + n_act] = gamma
    for i in c:
        for j in c:
            P[i, i, j, j] += 4.0
            P[i, j, j, i] -= 2.0
    for t in range(n_act):
        for u in range(n_act):
            for i in c:
                P[a0 + t, a0 + u, i, i] += 2.0 * gamma[t, u]
                P[i, i, a0 + t, a0 + u] += 2.0 * gamma[t, u]
                P[a0 + t, i, i, a0 + u] -= gamma[t, u]
                P[i, a0 + u, a0 + t, i] -= gamma[t, u]
    # active: 1/2 sum (tu|vw) Gamma~_tvwu  ->  P_tuvw = Gamma~_tvwu
    P[a0:a0 + n_act, a0:a0 + n_act, a0:a0 + n_act, a0:a0 + n_act] = np.einsum("tvwu->tuvw", Gamma)
    return D, P


def generalized_fock_gradient(h, B, gamma, Gamma, n_core, n_act):
    """dE/dkappa at kappa = 0: G_pq = 2 (F_pq - F_qp), F_pq = sum_r D_pr h_qr +
    sum_rst P_prst (qr|st)."""
    n = h.shape[0]
    D, P = full_density_matrices(gamma, Gamma, n_core, n_act, n)
    g = np.einsum("Lpq,Lrs->pqrs", B, B)
    F = D @ h.T + np.einsum("prst,qrst->pq", P, g)
    G = 2.0 * (F - F.T)
    return np.tril(G, -1) - np.tril(G, -1).T
