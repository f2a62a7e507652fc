"""Active-space reduced density matrices of a CAS-CI state from the oracle's
explicit determinant space (test helper; the RDMs feed the orbital-gradient
checks)."""
import numpy as np

from oracle import fock


def cas_ci_rdms(h, g, n, n_core, n_act, n_elec_act, seed):
    """Active-space RDMs of the lowest singlet CAS-CI state (core doubly occupied,
    virtuals empty), from explicit Jordan-Wigner operators on the active space,
    and the energy <Psi|H|Psi> of the same state evaluated on the full
    determinant space."""
    ncor = n_core
    a = slice(ncor, ncor + n_act)
    # effective active Hamiltonian is not needed: diagonalise H on the CAS space directly
    nu = ncor + n_elec_act // 2
    dets = fock.sector_dets(n, nu, nu)
    core_mask = sum(3 << (2 * i) for i in range(ncor))
    virt_mask = sum(3 << (2 * p) for p in range(ncor + n_act, n))
    cas = [i for i, d in enumerate(dets) if (d & core_mask) == core_mask and (d & virt_mask) == 0]
    hm = fock.hamiltonian_sparse(h, g, dets).toarray()[np.ix_(cas, cas)]
    w, v = np.linalg.eigh(hm)
    s2, d0 = fock.s2_matrix(n, 2 * nu, 0)
    s2c = s2.toarray()[np.ix_(cas, cas)]
    # lowest singlet
    for j in range(len(w)):
        if abs(v[:, j] @ s2c @ v[:, j]) < 1e-8:
            break
    psi_full = np.zeros(1 << (2 * n))
    psi_full[np.asarray(dets)[cas]] = v[:, j]
    # RDMs from literal operators on the full Fock space
    ops = fock.jw_annihilators(n)
    ad = [x.T for x in ops]
    gam = np.zeros((n_act, n_act))
    Gam = np.zeros((n_act,) * 4)
    for t in range(n_act):
        for u in range(n_act):
            for s in range(2):
                gam[t, u] += psi_full @ (ad[2 * (ncor + t) + s] @ (ops[2 * (ncor + u) + s] @ psi_full))
    for t in range(n_act):
        for u in range(n_act):
            for vv in range(n_act):
                for ww in range(n_act):
                    val = 0.0
                    for s in range(2):
                        for r in range(2):
                            x = ops[2 * (ncor + ww) + s] @ psi_full
                            x = ops[2 * (ncor + vv) + r] @ x
                            x = ad[2 * (ncor + u) + r] @ x
                            x = ad[2 * (ncor + t) + s] @ x
                            val += psi_full @ x
                    Gam[t, u, vv, ww] = val
    return gam, Gam, float(w[j])
