"""Exact identities of the two-site effective Hamiltonian that hold at any size.

Both the oracle's pins and the GPU tests at the full workload sizes use them.
They involve no part of either implementation: only the Hamiltonian's
definition (Sec. "Complete active space SCF") and the MPS's variational space.

* Integral shifts.  With h' = h + alpha*1 and (pq|rs)' = (pq|rs) +
  beta*delta_pq*delta_rs the Hamiltonian gains alpha*N + beta*N(N-1)/2, a
  constant on the fixed-N space the MPS spans, so
  H'_eff psi = H_eff psi + (alpha*N + beta*N(N-1)/2) psi.
  With the integrals of S^2 added (gamma*S^2; they are not 8-fold symmetric,
  so only the oracle, which takes any g, is checked with them) the shift is
  gamma*S(S+1).
* Orbital sign gauge.  Replacing a_p by -a_p for p in a set F changes h_pq by
  s_p s_q and (pq|rs) by s_p s_q s_r s_s (s = -1 on F), and every state by the
  sign (-1)^(occupation of F).  On the MPS this is a sign on the singly
  occupied (sigma = 1) blocks of the site tensors of F; on the two-site
  coefficients of sites k, k+1 in F it is the sign P on their sigma = 1
  sub-blocks.  Then H'_eff = P H_eff P exactly.
"""
from __future__ import annotations

import copy

import numpy as np


def shift_integrals(h, g, alpha, beta):
    n = h.shape[0]
    h2 = h + alpha * np.eye(n)
    g2 = g.copy()
    for p in range(n):
        for r in range(n):
            g2[p, p, r, r] += beta
    return h2, g2


def shift_value(n_elec, two_s, alpha, beta, gamma=0.0):
    s = two_s / 2.0
    return alpha * n_elec + beta * n_elec * (n_elec - 1) / 2.0 + gamma * s * (s + 1.0)


def s2_integrals(n):
    """(h, g) with sum h_pq E_pq + 1/2 sum g_pqrs sum_st a+_ps a+_rt a_st a_qs = S^2,
    from S^2 = 3/4 N - 1/2 sum_pq e~_pqpq - 1/4 sum_pq e~_pqqp with
    e~_abcd = sum_st a+_as a+_bt a_ct a_ds."""
    h = 0.75 * np.eye(n)
    g = np.zeros((n, n, n, n))
    for p in range(n):
        for q in range(n):
            g[p, q, q, p] -= 1.0
            g[p, p, q, q] -= 0.5
    return h, g


def gauge_integrals(h, g, flips):
    s = np.ones(h.shape[0])
    s[list(flips)] = -1.0
    return h * np.outer(s, s), g * np.einsum("p,q,r,s->pqrs", s, s, s, s)


def gauge_mps(mps, flips):
    """The MPS with a_p -> -a_p for p in flips (sites outside the two-site block)."""
    out = copy.deepcopy(mps)
    for j in range(out.k):
        if j in flips:
            out.A[j] = [(a, s, b, -blk if s == 1 else blk) for (a, s, b, blk) in out.A[j]]
    for j in range(out.k + 2, out.n):
        if j in flips:
            out.B[j] = [(a, s, b, -blk if s == 1 else blk) for (a, s, b, blk) in out.B[j]]
    return out


def gauge_psi(psi, layout, k, flips):
    """P psi: sign on the sigma1 = 1 rows if k is flipped and on the sigma2 = 1
    columns if k+1 is flipped."""
    out = np.array(psi, dtype=np.float64, copy=True)
    for b in layout:
        blk = out[b["offset"]:b["offset"] + b["nrows"] * b["ncols"]].reshape(b["nrows"], b["ncols"])
        if k in flips:
            for (_, s1, r0, dl) in b["rows"]:
                if s1 == 1:
                    blk[r0:r0 + dl, :] *= -1.0
        if k + 1 in flips:
            for (s2, _, c0, dr) in b["cols"]:
                if s2 == 1:
                    blk[:, c0:c0 + dr] *= -1.0
    return out


def transformed(h, g, mps, alpha, beta, flips):
    """Integrals and MPS of the combined shift and gauge: returns (h', g', mps')
    with H'_eff = P (H_eff + c) P, c = shift_value(N, 2S, alpha, beta)."""
    h2, g2 = shift_integrals(h, g, alpha, beta)
    h2, g2 = gauge_integrals(h2, g2, flips)
    return h2, g2, gauge_mps(mps, flips)
