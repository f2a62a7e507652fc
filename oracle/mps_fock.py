"""Expansion of an SU(2) matrix product state into M-resolved Fock-space vectors.

This is the definition of the multiplet basis (Sec. "Conservation of the total
spin"; MPS form of Sec. "Tensor network states"): every block state is built by
coupling one site at a time with Clebsch-Gordan coefficients, and the two-site
space is embedded into the full Fock space by the linear map V.  Fock indices
follow ``oracle.fock``: site j occupies bits 2j (up) and 2j+1 (down), so
appending a site to the right of a block multiplies its local index by 4^j.

Local multiplet states: sigma=0 -> |0>; sigma=1 -> |1/2, +1/2> = a+_up|0>,
|1/2, -1/2> = a+_dn|0>; sigma=2 -> a+_up a+_dn |0>.  Local Fock index =
n_up + 2 n_dn.
"""
from __future__ import annotations

import numpy as np

from .cg import cg

LOCAL = ((0, 0), (1, 1), (2, 0))


def local_index(sigma, m2):
    if sigma == 0:
        return 0
    if sigma == 2:
        return 3
    return 1 if m2 == 1 else 2


def mlist(s2):
    return [s2 - 2 * i for i in range(s2 + 1)]


def left_block_vectors(mps, b):
    """{il: U} for left bond b; U has shape (D_l, 2S_l+1, 4^b), axis 1 runs over
    M = S, S-1, ..., -S."""
    cur = {0: np.ones((1, 1, 1))}
    for j in range(b):
        lb, ab = mps.left_bonds[j], mps.left_bonds[j + 1]
        nxt = {ia: np.zeros((da, sa + 1, 4, 4 ** j)) for ia, (na, sa, da) in enumerate(ab)}
        for il, s, ia, blk in mps.A[j]:
            sl, ss, sa = lb[il][1], LOCAL[s][1], ab[ia][1]
            for iml, ml in enumerate(mlist(sl)):
                for ms in mlist(ss):
                    ma = ml + ms
                    if abs(ma) > sa:
                        continue
                    c = cg(sl, ml, ss, ms, sa, ma)
                    if c == 0.0:
                        continue
                    ima = (sa - ma) // 2
                    nxt[ia][:, ima, local_index(s, ms), :] += c * (blk.T @ cur[il][:, iml, :])
        cur = {ia: v.reshape(v.shape[0], v.shape[1], -1) for ia, v in nxt.items()}
    return cur


def right_block_vectors(mps, b):
    """{ic: U} for right bond b (sites b..n-1); U has shape (D_c, 2S_c+1, 4^(n-b)),
    Fock index = local(site b) + 4 * (index of the rest)."""
    n = mps.n
    cur = {0: np.ones((1, 1, 1))}
    for j in range(n - 1, b - 1, -1):
        cb, rb = mps.right_bonds[j], mps.right_bonds[j + 1]
        width = 4 ** (n - j - 1)
        nxt = {ic: np.zeros((dc, sc + 1, width, 4)) for ic, (nc, sc, dc) in enumerate(cb)}
        for ic, s, ir, blk in mps.B[j]:
            ss, sr, sc = LOCAL[s][1], rb[ir][1], cb[ic][1]
            for ms in mlist(ss):
                for imr, mr in enumerate(mlist(sr)):
                    mc = ms + mr
                    if abs(mc) > sc:
                        continue
                    c = cg(ss, ms, sr, mr, sc, mc)
                    if c == 0.0:
                        continue
                    imc = (sc - mc) // 2
                    nxt[ic][:, imc, :, local_index(s, ms)] += c * (blk @ cur[ir][:, imr, :])
        cur = {ic: v.reshape(v.shape[0], v.shape[1], -1) for ic, v in nxt.items()}
    return cur


def _terms(mps, blk):
    """All (row sub-block, col sub-block, M-components, coefficient) of one
    super-block at total M = S."""
    k = mps.k
    lb, rb = mps.left_bonds[k], mps.right_bonds[k + 2]
    two_s = mps.two_s
    sa, sc = blk["a"][1], blk["c"][1]
    for (il, s1, r0, dl) in blk["rows"]:
        sl, ss1 = lb[il][1], LOCAL[s1][1]
        for (s2, ir, c0, dr) in blk["cols"]:
            ss2, sr = LOCAL[s2][1], rb[ir][1]
            for ma in mlist(sa):
                mc = two_s - ma
                if abs(mc) > sc:
                    continue
                c_out = cg(sa, ma, sc, mc, two_s, two_s)
                if c_out == 0.0:
                    continue
                for iml, ml in enumerate(mlist(sl)):
                    m1 = ma - ml
                    if abs(m1) > ss1 or (ss1 - m1) % 2:
                        continue
                    c_l = cg(sl, ml, ss1, m1, sa, ma)
                    if c_l == 0.0:
                        continue
                    for imr, mr in enumerate(mlist(sr)):
                        m2 = mc - mr
                        if abs(m2) > ss2 or (ss2 - m2) % 2:
                            continue
                        c_r = cg(ss2, m2, sr, mr, sc, mc)
                        if c_r == 0.0:
                            continue
                        yield (il, s1, r0, dl, s2, ir, c0, dr, iml, m1, imr, m2, c_out * c_l * c_r)


class Embedding:
    """The map V from the reduced two-site coordinates (super-block layout) to
    the full Fock space at M = S, and its transpose."""

    def __init__(self, mps, layout):
        self.mps, self.layout = mps, layout
        k = mps.k
        self.UL = left_block_vectors(mps, k)
        self.UR = right_block_vectors(mps, k + 2)
        self.nl, self.nr = 4 ** k, 4 ** (mps.n - k - 2)
        self.terms = [list(_terms(mps, blk)) for blk in layout]

    def expand(self, psi):
        phi = np.zeros((self.nr, 4, 4, self.nl))
        for blk, terms in zip(self.layout, self.terms):
            mat = psi[blk["offset"]: blk["offset"] + blk["nrows"] * blk["ncols"]].reshape(blk["nrows"], blk["ncols"])
            for (il, s1, r0, dl, s2, ir, c0, dr, iml, m1, imr, m2, coef) in terms:
                sub = mat[r0:r0 + dl, c0:c0 + dr]
                phi[:, local_index(s2, m2), local_index(s1, m1), :] += coef * (
                    self.UR[ir][:, imr, :].T @ sub.T @ self.UL[il][:, iml, :])
        return phi.reshape(-1)

    def project(self, phi_flat, out_len):
        phi = phi_flat.reshape(self.nr, 4, 4, self.nl)
        out = np.zeros(out_len)
        for blk, terms in zip(self.layout, self.terms):
            mat = np.zeros((blk["nrows"], blk["ncols"]))
            for (il, s1, r0, dl, s2, ir, c0, dr, iml, m1, imr, m2, coef) in terms:
                sl = phi[:, local_index(s2, m2), local_index(s1, m1), :]
                mat[r0:r0 + dl, c0:c0 + dr] += coef * (self.UL[il][:, iml, :] @ sl.T @ self.UR[ir][:, imr, :].T)
            out[blk["offset"]: blk["offset"] + mat.size] = mat.ravel()
        return out
