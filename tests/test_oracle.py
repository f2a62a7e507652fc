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
