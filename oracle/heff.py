"""The two-site effective Hamiltonian by its definition.

DMRG minimises the energy over MPS (Sec. "Tensor network states and density
matrix renormalization group"); at the two-site block (k, k+1) the variational
space is the image of V (``oracle.mps_fock.Embedding``), and the Davidson
matrix-vector product is the projected Hamiltonian

    H_eff psi = V^T H V psi,

with H the ab-initio Hamiltonian on the full determinant space (``oracle.fock``).
No environments, complementary operators or recoupling coefficients are used.
Practical for n <= 12 orbitals.
"""
from __future__ import annotations

import numpy as np

from . import fock
from .mps_fock import Embedding


class HeffDefinition:
    def __init__(self, h, g, mps, layout, e_core=0.0):
        self.h, self.g, self.e_core = h, g, e_core
        self.emb = Embedding(mps, layout)
        n = mps.n
        n_up = (mps.n_elec + mps.two_s) // 2
        self.dets = fock.sector_dets(n, n_up, mps.n_elec - n_up)
        self.e = fock.epq_matrices(n, self.dets)
        self.size = sum(b["nrows"] * b["ncols"] for b in layout)

    def apply(self, psi):
        full = self.emb.expand(psi)
        v = full[self.dets]
        hv = fock.apply_h(self.h, self.g, self.dets, v, self.e) + self.e_core * v
        out = np.zeros_like(full)
        out[self.dets] = hv
        return self.emb.project(out, self.size)

    def dense(self):
        """H_eff as a dense matrix, column by column (small cases only)."""
        cols = [self.apply(np.eye(1, self.size, i).ravel()) for i in range(self.size)]
        return np.stack(cols, axis=1)

    def isometry_defect(self, nprobe=8, seed=0):
        """max |<V x, V y> - <x, y>| over random probes (V must be an isometry)."""
        rng = np.random.default_rng(seed)
        xs = [rng.normal(size=self.size) for _ in range(nprobe)]
        vx = [self.emb.expand(x) for x in xs]
        err = 0.0
        for i in range(nprobe):
            for j in range(nprobe):
                err = max(err, abs(vx[i] @ vx[j] - xs[i] @ xs[j]))
        return err


def hpsi(h, g, mps, layout, psi, e_core=0.0):
    return HeffDefinition(h, g, mps, layout, e_core).apply(psi)
