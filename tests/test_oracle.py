"""Pins of the FP64 CPU oracle against facts fixed outside it: a library routine
(sympy's Clebsch-Gordan), closed forms, a literal Jordan-Wigner construction,
brute-force FCI spectra, operator identities and a determinant count the paper
prints.  None of these re-type the oracle's own formulas."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fock, heff
from oracle.cg import cg
from oracle.mps_fock import Embedding
from casci import cas_ci_rdms
from synth.integrals import hubbard_dimer, small_cas
from synth.mps import LOCAL, SU2MPS, full_counts, psi_layout, random_mps, random_psi

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_cg_matches_sympy():
    from sympy import Rational
    from sympy.physics.wigner import clebsch_gordan
    worst = 0.0
    for j1, j2 in [(1, 1), (2, 1), (3, 2), (4, 3), (6, 5), (8, 1)]:
        for J in range(abs(j1 - j2), j1 + j2 + 1, 2):
            for m1 in range(-j1, j1 + 1, 2):
                for m2 in range(-j2, j2 + 1, 2):
                    if abs(m1 + m2) > J:
                        continue
                    ref = float(clebsch_gordan(Rational(j1, 2), Rational(j2, 2), Rational(J, 2),
                                               Rational(m1, 2), Rational(m2, 2), Rational(m1 + m2, 2)))
                    worst = max(worst, abs(ref - cg(j1, m1, j2, m2, J, m1 + m2)))
    assert worst < 1e-14


def test_hubbard_dimer_closed_form():
    h, g = hubbard_dimer(1.0, 3.0)
    e0 = fock.fci_spectrum(h, g, 2, 0)[0]
    closed = (3.0 - math.sqrt(9.0 + 16.0)) / 2.0
    assert abs(e0 - closed) < 1e-12
    assert abs(e0 - GOLDEN["hubbard_dimer_t1_u3_ground_energy"]["value"]) < 1e-12


@pytest.mark.parametrize("n_up,n_dn", [(2, 1), (1, 1), (3, 2)])
def test_direct_ci_equals_literal_jordan_wigner(n_up, n_dn):
    h, g, _ = small_cas(3, 11)
    full = fock.jw_hamiltonian(h, g)
    d = fock.sector_dets(3, n_up, n_dn)
    assert np.abs(full[np.ix_(d, d)] - fock.hamiltonian_sparse(h, g, d).toarray()).max() < 1e-12
    v = np.random.default_rng(0).normal(size=len(d))
    assert np.abs(fock.apply_h(h, g, d, v) - full[np.ix_(d, d)] @ v).max() < 1e-12


def test_noninteracting_limit():
    h, g, _ = small_cas(6, 3)
    g = np.zeros_like(g)
    e0 = fock.fci_spectrum(h, g, 6, 0)[0]
    eps = np.linalg.eigvalsh(h)
    assert abs(e0 - 2.0 * eps[:3].sum()) < 1e-12


def test_singlet_count_and_s2_identity():
    # number of S=0 states of CAS(8,8) equals the Weyl-Paldus count (1764)
    h, g, _ = small_cas(8, 0)
    assert len(fock.fci_spectrum(h, g, 8, 0)) == full_counts(8)[(8, 0)] == 1764
    # S^2 = 3/4 N - 1/2 sum_pq e_pqqp... checked as <S^2> from explicit spin operators
    s2, dets = fock.s2_matrix(4, 4, 0)
    w = np.linalg.eigvalsh(s2.toarray())
    allowed = {0.0, 2.0, 6.0}
    assert all(min(abs(x - a) for a in allowed) < 1e-10 for x in w)


def _path_mps(path2):
    """MPS with one multiplet per bond following the doubled-spin path, the
    last two sites forming the two-site block (all sites singly occupied)."""
    n = len(path2)
    k = n - 2
    left = [[(0, 0, 1)]] + [[(b + 1, path2[b], 1)] for b in range(k)]
    mps = SU2MPS(n=n, n_elec=n, two_s=path2[-1], k=k, left_bonds=left, right_bonds={n: [(0, 0, 1)]})
    for j in range(k):
        mps.A.append([(0, 1, 0, np.ones((1, 1)))])
    lay = psi_layout(left[k], mps.right_bonds[n], n, path2[-1])
    psi = np.zeros(sum(b["nrows"] * b["ncols"] for b in lay))
    for b in lay:
        if b["a"] == (n - 1, path2[-2]) and b["c"] == (1, 1):
            for (il, s1, r0, dl) in b["rows"]:
                for (s2, ir, c0, dr) in b["cols"]:
                    if s1 == 1 and s2 == 1:
                        psi[b["offset"] + r0 * b["ncols"] + c0] = 1.0
    return mps, lay, psi


def test_leading_csf_has_252_determinants():
    # two S=5/2 fragments of five open shells each, coupled to a singlet
    path = [1, 2, 3, 4, 5, 4, 3, 2, 1, 0]
    mps, lay, psi = _path_mps(path)
    full = Embedding(mps, lay).expand(psi)
    nz = np.count_nonzero(np.abs(full) > 1e-12)
    assert nz == GOLDEN["leading_csf_determinants"]["value"]
    assert abs(np.linalg.norm(full) - 1.0) < 1e-12
    s2, dets = fock.s2_matrix(10, 10, 0)
    v = full[dets]
    assert np.abs(s2 @ v).max() < 1e-12


@pytest.mark.parametrize("n,nel,two_s,d", [(6, 6, 0, 16), (7, 7, 1, 16), (6, 6, 2, 16), (8, 8, 0, 12)])
def test_mps_expansion_is_isometric_spin_eigenstate(n, nel, two_s, d):
    mps = random_mps(n, nel, two_s, d, k=n // 2 - 1, seed=5)
    psi, lay = random_psi(mps, seed=6)
    he = heff.HeffDefinition(*small_cas(n, 1)[:2], mps, lay)
    assert he.isometry_defect() < 1e-11
    full = he.emb.expand(psi)
    s2, dets = fock.s2_matrix(n, nel, two_s)
    v = full[dets]
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    s = two_s / 2.0
    assert np.abs(s2 @ v - s * (s + 1) * v).max() < 1e-11


@pytest.mark.parametrize("n,nel,two_s", [(6, 6, 0), (7, 7, 1), (6, 6, 2)])
def test_heff_spectrum_equals_fci_when_two_site_space_is_complete(n, nel, two_s):
    h, g, _ = small_cas(n, 2)
    mps = random_mps(n, nel, two_s, 10 ** 6, k=n // 2 - 1, seed=3)
    psi, lay = random_psi(mps)
    hd = heff.HeffDefinition(h, g, mps, lay).dense()
    assert np.abs(hd - hd.T).max() < 1e-11
    ev = np.linalg.eigvalsh(0.5 * (hd + hd.T))
    ref = fock.fci_spectrum(h, g, nel, two_s)
    assert len(ev) == len(ref)
    assert np.abs(ev - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_heff_spectrum_cas88_centre_equals_singlet_fci():
    h, g, _ = small_cas(8, 0)
    mps = random_mps(8, 8, 0, 64, k=3, seed=0)
    psi, lay = random_psi(mps)
    hd = heff.HeffDefinition(h, g, mps, lay).dense()
    ev = np.linalg.eigvalsh(0.5 * (hd + hd.T))
    ref = fock.fci_spectrum(h, g, 8, 0)
    assert np.abs(ev - ref).max() < 1e-10 * np.abs(ref).max()


def test_heff_truncated_is_hermitian_and_variational():
    h, g, _ = small_cas(8, 4)
    mps = random_mps(8, 8, 0, 6, k=3, seed=8)
    psi, lay = random_psi(mps)
    he = heff.HeffDefinition(h, g, mps, lay)
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=he.size), rng.normal(size=he.size)
    assert abs(x @ he.apply(y) - he.apply(x) @ y) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(y) * 100
    hd = he.dense()
    e_min = np.linalg.eigvalsh(0.5 * (hd + hd.T))[0]
    assert e_min >= fock.fci_spectrum(h, g, 8, 0)[0] - 1e-10


def test_leading_csf_middle_cut_has_six_equal_schmidt_values():
    # two S=5/2 fragments coupled to a singlet: sum_M (-1)^(5/2-M)/sqrt(6) |5/2 M>|5/2 -M>
    from oracle import truncate as otr
    path = [1, 2, 3, 4, 5, 4, 3, 2, 1, 0]
    mps, lay, psi = _path_mps(path)
    # cut between sites 8 and 9 of this MPS: the right part is one doublet, so
    # the Schmidt values are those of |S=1/2 (x) 1/2 -> 0>: two equal values
    sv = otr.schmidt_values(mps, lay, psi)
    nz = sv[sv > 1e-12]
    assert len(nz) == 2 and np.allclose(nz, 1 / np.sqrt(2))
    # full Fock-space SVD across the 5|5 cut of the same state
    from oracle.mps_fock import Embedding
    full = Embedding(mps, lay).expand(psi)
    mat = full.reshape(4 ** 5, 4 ** 5)  # index = left(sites 0..4) + 4^5 * right(sites 5..9)
    s = np.linalg.svd(mat.T, compute_uv=False)
    nz = s[s > 1e-12]
    assert len(nz) == 6 and np.allclose(nz, 1 / np.sqrt(6))
    # the same run of six equal values is one S=5/2 multiplet of weight 1
    from oracle import truncate as otr2
    w, s2 = otr2.multiplet_weights(s)
    assert s2.tolist() == [5] and abs(w[0] - 1.0) < 1e-12


def test_multiplet_grouping_recovers_a_constructed_spectrum():
    # multiplets (weight, 2S) expanded to 2S+1 Schmidt values sqrt(w/(2S+1))
    # each, shuffled, with a null space of zeros and rounding-level noise
    from oracle import truncate as otr
    mult = [(0.41, 0), (0.22, 2), (0.17, 1), (0.09, 4), (0.06, 0), (0.03, 3), (0.02, 2)]
    vals = []
    for wt, ts in mult:
        vals += [np.sqrt(wt / (ts + 1))] * (ts + 1)
    vals = np.array(vals + [0.0] * 7 + [1e-17] * 3)
    np.random.default_rng(0).shuffle(vals)
    w, s2 = otr.multiplet_weights(vals)
    assert np.allclose(w, [m[0] for m in mult], rtol=0, atol=1e-15)
    assert s2.tolist() == [m[1] for m in mult]


def test_dbss_keep_worked_example():
    # weights 0.6, 0.25, 0.1, 0.04, 0.01 (total 1): keeping 3 discards 0.05,
    # keeping 4 discards 0.01, keeping 2 discards 0.15
    from oracle import truncate as otr
    w = [0.04, 0.6, 0.01, 0.25, 0.1]  # order must not matter
    assert otr.dbss_keep(w, 0.0501, 0, 100) == 3
    assert otr.dbss_keep(w, 0.0499, 0, 100) == 4
    assert otr.dbss_keep(w, 0.0099, 0, 100) == 5
    assert otr.dbss_keep(w, 0.1501, 0, 100) == 2
    assert otr.dbss_keep(w, 0.1499, 0, 100) == 3
    assert otr.dbss_keep(w, 0.9, 0, 100) == 1     # never below one multiplet
    assert otr.dbss_keep(w, 0.0501, 4, 100) == 4  # d_min raises
    assert otr.dbss_keep(w, 0.0501, 0, 2) == 2    # d_max caps
    assert otr.dbss_keep(w, 0.0501, 9, 9) == 5    # capped by the count
    assert otr.dbss_keep(w, 0.0, 0, 4) == 4       # eps 0: fixed D
    assert otr.dbss_keep(w, 0.0, 0, 100) == 5


# ---- exact identities at any size (tests/identities.py), pinned on the oracle ---------

@pytest.mark.parametrize("n,ne,ts,d,k,seed", [(6, 6, 0, 16, 2, 2), (7, 7, 1, 16, 2, 3), (6, 6, 2, 16, 2, 4),
                                              (8, 7, 1, 20, 3, 5)])
def test_oracle_integral_shift_identities(n, ne, ts, d, k, seed):
    import identities as ident
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    y = heff.hpsi(h, g, mps, lay, psi)
    alpha, beta, gamma = 0.37, -0.21, 0.53
    h2, g2 = ident.shift_integrals(h, g, alpha, beta)
    hs, gs = ident.s2_integrals(n)
    y2 = heff.hpsi(h2 + gamma * hs, g2 + gamma * gs, mps, lay, psi)
    c = ident.shift_value(ne, ts, alpha, beta, gamma)
    assert np.abs(y2 - y - c * psi).max() < 1e-10 * np.abs(y).max()
    # a wrong S^2 factor, or a dropped beta term, would not pass
    assert np.abs(y2 - y - (c + 0.01) * psi).max() > 1e-3


def test_s2_integrals_reproduce_the_spin_operator():
    import identities as ident
    n = 3
    hs, gs = ident.s2_integrals(n)
    for n_up, n_dn in [(2, 1), (1, 1), (2, 2), (3, 1)]:
        d = fock.sector_dets(n, n_up, n_dn)
        hm = fock.hamiltonian_sparse(hs, gs, d).toarray()
        s2, d0 = fock.s2_matrix(n, n_up + n_dn, n_up - n_dn)
        assert np.array_equal(np.asarray(d0), np.asarray(d))
        assert np.abs(hm - s2.toarray()).max() < 1e-12


@pytest.mark.parametrize("flips", [(0,), (3,), (4,), (1, 3, 6), (2, 5, 7)])
def test_oracle_sign_gauge_identity(flips):
    import identities as ident
    n, ne, ts, d, k, seed = 8, 8, 0, 20, 3, 9
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    y = heff.hpsi(h, g, mps, lay, psi)
    h2, g2, mps2 = ident.transformed(h, g, mps, 0.0, 0.0, set(flips))
    y2 = heff.hpsi(h2, g2, mps2, lay, ident.gauge_psi(psi, lay, k, set(flips)))
    assert np.abs(ident.gauge_psi(y2, lay, k, set(flips)) - y).max() < 1e-10 * np.abs(y).max()
    # the transformed integrals alone (old MPS) give a different operator
    y3 = heff.hpsi(h2, g2, mps, lay, ident.gauge_psi(psi, lay, k, set(flips)))
    if any(f not in (k, k + 1) for f in flips):
        assert np.abs(ident.gauge_psi(y3, lay, k, set(flips)) - y).max() > 1e-6


def test_rdm1_spin0_coupling_factor():
    """[f+_p f_q]^0 built from Clebsch-Gordan coefficients on Fock space equals
    -E_pq/sqrt(2) (Sec. "Conservation of the total spin", the coupled 1-RDM):
    f+ = (a+_up, a+_dn) and f = (a_dn, -a_up) as rank-1/2 tensors."""
    n = 3
    a = fock.jw_annihilators(n)
    ad = [x.T for x in a]
    factor = GOLDEN["rdm1_coupled_factor"]["value"]
    for p in range(n):
        for q in range(n):
            fdag = {1: ad[2 * p], -1: ad[2 * p + 1]}   # m = +1/2, -1/2 (twice m)
            f = {1: a[2 * q + 1], -1: -a[2 * q]}
            coupled = sum(cg(1, m, 1, -m, 0, 0) * fdag[m] @ f[-m] for m in (1, -1))
            epq = ad[2 * p] @ a[2 * q] + ad[2 * p + 1] @ a[2 * q + 1]
            assert np.abs(coupled - factor * epq).max() < 1e-14
    assert abs(factor + 1.0 / math.sqrt(2.0)) < 1e-15


def test_discarded_weight_is_the_truncation_residual():
    """Eckart-Young: keeping the top-m Schmidt vectors leaves
    |M - P_m M|_F^2 / |M|_F^2, computed here from the eigenvectors of M M^T."""
    from oracle.truncate import discarded_weight
    rng = np.random.default_rng(5)
    m = rng.normal(size=(12, 9))
    vals = np.linalg.svd(m, compute_uv=False)
    w, u = np.linalg.eigh(m @ m.T)
    u = u[:, np.argsort(-w)]
    for keep in (0, 1, 4, 9):
        pm = u[:, :keep] @ (u[:, :keep].T @ m)
        ref = np.linalg.norm(m - pm) ** 2 / np.linalg.norm(m) ** 2
        assert abs(discarded_weight(vals, keep) - ref) < 1e-12
    # worked example: values 0.8 and 0.6 (in either order), keep one
    assert abs(discarded_weight([0.6, 0.8], 1) - 0.36) < 1e-15


# ---- orbital rotation energy and gradient (oracle/orbital.py) ----------------------------

def test_orbital_energy_at_zero_rotation_is_the_cas_ci_energy():
    from oracle import orbital
    n, n_core, n_act = 5, 1, 3
    h, g, B = small_cas(n, 13)
    gam, Gam, e_ci = cas_ci_rdms(h, g, n, n_core, n_act, 4, 0)
    e = orbital.energy(h, B, np.zeros((n, n)), gam, Gam, n_core, n_act)
    assert abs(e - e_ci) < 1e-10
    assert abs(np.trace(gam) - 4.0) < 1e-12
    assert abs(np.einsum("tuut->", Gam) - 4.0 * 3.0) < 1e-10  # N(N-1)


def test_orbital_gradient_closed_form_equals_finite_differences_and_has_zero_redundant_blocks():
    from oracle import orbital
    n, n_core, n_act = 6, 2, 2
    h, g, B = small_cas(n, 3)
    gam, Gam, _ = cas_ci_rdms(h, g, n, n_core, n_act, 2, 0)
    fd = orbital.gradient_fd(h, B, np.zeros((n, n)), gam, Gam, n_core, n_act, step=1e-5)
    cf = orbital.generalized_fock_gradient(h, B, gam, Gam, n_core, n_act)
    assert np.abs(fd - cf).max() < 1e-7 * max(1.0, np.abs(cf).max())
    assert np.abs(cf).max() > 1e-3
    # core-core and virtual-virtual rotations leave E unchanged
    assert np.abs(cf[:n_core, :n_core]).max() < 1e-12
    assert np.abs(cf[n_core + n_act:, n_core + n_act:]).max() < 1e-12
    rng = np.random.default_rng(1)
    k = np.zeros((n, n))
    k[1, 0] = 0.3
    k[5, 4] = -0.2
    e0 = orbital.energy(h, B, np.zeros((n, n)), gam, Gam, n_core, n_act)
    assert abs(orbital.energy(h, B, k, gam, Gam, n_core, n_act) - e0) < 1e-12
    # away from zero the finite differences still see a smooth function
    k = np.tril(rng.normal(scale=1e-2, size=(n, n)), -1)
    f1 = orbital.gradient_fd(h, B, k, gam, Gam, n_core, n_act, step=1e-4)
    f2 = orbital.gradient_fd(h, B, k, gam, Gam, n_core, n_act, step=2e-4)
    assert np.abs(f1 - f2).max() < 1e-6
