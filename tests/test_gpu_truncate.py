"""GPU truncation (dmrg_truncate) and operator-block growth against the oracle.

* The full multiplet spectrum of the cut, each weight w of spin S expanded to
  2S+1 Schmidt values sqrt(w/(2S+1)), equals the oracle's Schmidt values from
  an SVD of the explicit Fock-space wavefunction (singlet states).
* With truncation to D multiplets, the kept weights are the D largest and
  the reported error is the discarded fraction.
* After truncation the grown operator block feeds H*psi at the next two-site
  position; that H*psi equals the oracle's V^T H V psi for the MPS carrying
  the new site tensor (both sweep directions).
"""
import copy

import numpy as np
import pytest

from oracle import heff
from oracle import truncate as otr
from synth.integrals import small_cas
from synth.mps import left_site_blocks, psi_layout, random_mps, random_psi, right_site_blocks

pytestmark = pytest.mark.gpu


def _ctx(case, keep=False):
    from paper_2503_20700_amd.binding import DMRG
    n, ne, ts, d, k, seed = case
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 10)
    psi, lay = random_psi(mps, seed=seed + 20)
    dm = DMRG(h, g, ne, ts, keep_blocks=keep)
    bs, cnt = mps.bond_table()
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    return h, g, mps, psi, lay, dm


@pytest.mark.parametrize("direction", [1, -1])
def test_full_cut_spectrum_matches_fock_svd(direction):
    h, g, mps, psi, lay, dm = _ctx((8, 8, 0, 64, 3, 0))
    err, kept = dm.truncate(psi, 10 ** 6, 0.0, direction)
    vals, spins = dm.cut_spectrum()
    assert err < 1e-14
    assert abs((vals ** 2).sum() - 1.0) < 1e-12
    sv = otr.schmidt_values(mps, lay, psi)
    expanded = np.sort(np.concatenate([np.full(s + 1, v / np.sqrt(s + 1)) for v, s in zip(vals, spins)]))[::-1]
    m = len(expanded)
    assert np.abs(expanded - sv[:m]).max() < 1e-12
    assert (sv[m:] < 1e-12).all()


def test_truncation_keeps_largest_weights():
    h, g, mps, psi, lay, dm = _ctx((8, 8, 0, 64, 3, 0))
    dm.truncate(psi, 10 ** 6, 0.0, 1)
    full, _ = dm.cut_spectrum()
    h, g, mps, psi, lay, dm = _ctx((8, 8, 0, 64, 3, 0))
    err, kept = dm.truncate(psi, 12, 0.0, 1)
    vals, _ = dm.cut_spectrum()
    assert kept == 12
    w = np.sort(full ** 2)[::-1]
    assert np.abs(np.sort(vals ** 2)[::-1] - w[:12]).max() < 1e-12
    assert abs(err - w[12:].sum()) < 1e-12
    # truncation-error mode: smallest kept set with discarded weight <= eps
    h, g, mps, psi, lay, dm = _ctx((8, 8, 0, 64, 3, 0))
    eps = float(w[20:].sum()) * 1.000001
    err2, kept2 = dm.truncate(psi, 10 ** 6, eps, 1)
    assert kept2 == 20 and err2 <= eps


def _moved_mps(mps, dm, k, direction):
    m2 = copy.deepcopy(mps)
    nb = dm.get_bond(k + 1)
    if direction == 1:
        a = dm.get_site(k)
        blocks, off, lst = left_site_blocks(mps.left_bonds[k], nb), 0, []
        for (il, s, ia) in blocks:
            r, c = mps.left_bonds[k][il][2], nb[ia][2]
            lst.append((il, s, ia, a[off:off + r * c].reshape(r, c)))
            off += r * c
        assert off == a.size
        m2.left_bonds = mps.left_bonds[:k + 1] + [nb]
        m2.A = mps.A + [lst]
        m2.k = k + 1
        m2.right_bonds = {b: v for b, v in mps.right_bonds.items() if b >= k + 3}
        m2.B = {j: v for j, v in mps.B.items() if j >= k + 3}
    else:
        bt = dm.get_site(k + 1)
        blocks, off, lst = right_site_blocks(nb, mps.right_bonds[k + 2]), 0, []
        for (ic, s, ir) in blocks:
            r, c = nb[ic][2], mps.right_bonds[k + 2][ir][2]
            lst.append((ic, s, ir, bt[off:off + r * c].reshape(r, c)))
            off += r * c
        assert off == bt.size
        m2.right_bonds = dict(mps.right_bonds)
        m2.right_bonds[k + 1] = nb
        m2.B = dict(mps.B)
        m2.B[k + 1] = lst
        m2.k = k - 1
        m2.left_bonds = mps.left_bonds[:k]
        m2.A = mps.A[:k - 1]
    return m2


@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("case", [(8, 8, 0, 64, 3, 0), (8, 7, 1, 20, 3, 5)], ids=["s0", "s1/2"])
def test_block_growth_after_truncation_matches_oracle(direction, case):
    n, ne, ts, d, k, seed = case
    h, g, mps, psi, lay, dm = _ctx(case, keep=True)
    err, kept = dm.truncate(psi, 10, 0.0, direction)
    assert dm.k == k + direction
    m2 = _moved_mps(mps, dm, k, direction)
    lay2 = psi_layout(m2.left_bonds[m2.k], m2.right_bonds[m2.k + 2], ne, ts)
    p2 = np.random.default_rng(9).normal(size=sum(b["nrows"] * b["ncols"] for b in lay2))
    he = heff.HeffDefinition(h, g, m2, lay2)
    assert he.isometry_defect() < 1e-11
    y, _ = dm.hpsi(p2)
    ref = he.apply(p2)
    assert np.abs(y - ref).max() < 1e-10 * np.abs(ref).max()


def test_cut_spectrum_at_cas32_d1024_matches_numpy():
    # Full size of the CAS(32,32) D=1024 workload: reduced density matrices of
    # the enlarged left block are up to ~300 wide.  Their spectra from the
    # GPU Jacobi solver equal numpy's eigvalsh of rho_a = sum_c psi_ac psi_ac^T
    # built on the host from the psi layout.
    from paper_2503_20700_amd.binding import DMRG
    from synth.integrals import huckel_chain
    h, g, _ = huckel_chain(32, 1, naux=96)
    mps = random_mps(32, 32, 0, 1024, k=15, seed=1)
    psi, lay = random_psi(mps, seed=2)
    psi /= np.linalg.norm(psi)
    dm = DMRG(h, g, 32, 0)
    bs, cnt = mps.bond_table()
    dm.set_mps(15, bs, cnt, mps.site_blocks_flat())
    err, kept = dm.truncate(psi, 10 ** 6, 0.0, 1)
    vals, spins = dm.cut_spectrum()
    ref = []
    by_a = {}
    for b in lay:
        m = psi[b["offset"]:b["offset"] + b["nrows"] * b["ncols"]].reshape(b["nrows"], b["ncols"])
        by_a.setdefault(b["a"], []).append(m)
    for a, ms in by_a.items():
        rho = sum(m @ m.T for m in ms)
        ref.extend(np.linalg.eigvalsh(rho))
    ref = np.sort(np.clip(ref, 0.0, None))[::-1]
    w = np.sort(vals ** 2)[::-1]
    print(f"[cut spectrum] sectors={len(by_a)} max dim={max(len(ms[0]) for ms in by_a.values())} n={len(w)}", flush=True)
    assert abs(w.sum() - 1.0) < 1e-12
    assert np.abs(w - ref[:len(w)]).max() < 1e-13


@pytest.mark.parametrize("direction", [1, -1])
def test_dbss_selection_matches_oracle(direction):
    # Dynamic block state selection: the kept count and the discarded weight
    # equal the oracle's rule applied to the multiplet weights it derives from
    # the Fock-space Schmidt values of the same (singlet) wavefunction.
    case = (8, 8, 0, 64, 3, 0)
    h, g, mps, psi, lay, dm = _ctx(case)
    w, _ = otr.multiplet_weights(otr.schmidt_values(mps, lay, psi))
    tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]]) / w.sum()
    eps20 = tail[20] * 1.000001  # just admits discarding everything past 20
    eps31 = tail[31] * 0.999999  # just too small to stop at 31
    for eps, d_min, d_max in [(eps20, 0, 10 ** 6), (eps20, 25, 10 ** 6), (eps20, 0, 15), (eps31, 0, 10 ** 6),
                              (0.5, 3, 100), (0.0, 0, 17)]:
        print(f"[dbss] dir={direction} eps={eps:.3e} d_min={d_min} d_max={d_max}", flush=True)
        h, g, mps, psi, lay, dm = _ctx(case)
        err, kept = dm.truncate(psi, d_max, eps, direction, d_min=d_min)
        want = otr.dbss_keep(w, eps, d_min, d_max)
        assert kept == want, (kept, want)
        assert abs(err - tail[want]) < 1e-12
        if eps > 0 and d_min < kept < d_max:  # neither clamp active
            assert err <= eps


@pytest.mark.parametrize("direction", [1, -1], ids=["right", "left"])
@pytest.mark.parametrize("d_max", [10 ** 6, 12], ids=["complete", "truncated"])
@pytest.mark.parametrize("case", [(8, 8, 0, 64, 3, 0), (8, 7, 1, 20, 3, 5)], ids=["s0", "s1/2"])
def test_next_block_guess_is_the_kept_state(case, d_max, direction):
    # The start vector carried from (k, k+1) to (k+1, k+2) (or (k-1, k)):
    # expanded into determinants through the moved MPS it is exactly the old
    # wavefunction when nothing is discarded, and its orthogonal projection
    # onto the kept states of the cut side otherwise (overlap = norm^2 =
    # 1 - trunc_err).
    from oracle.mps_fock import Embedding
    from paper_2503_20700_amd.binding import DMRG
    n, ne, ts, d, k, seed = case
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 10)
    psi, lay = random_psi(mps, seed=seed + 20)
    psi = psi / np.linalg.norm(psi)
    dm = DMRG(h, g, ne, ts, keep_blocks=True, next_guess=True)
    bs, cnt = mps.bond_table()
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    err, kept = dm.truncate(psi, d_max, 0.0, direction)
    assert dm.k == k + direction
    guess = dm.next_guess()
    m2 = _moved_mps(mps, dm, k, direction)
    lay2 = psi_layout(m2.left_bonds[m2.k], m2.right_bonds[m2.k + 2], ne, ts)
    old = Embedding(mps, lay).expand(psi)
    new = Embedding(m2, lay2).expand(guess)
    assert abs(guess @ guess - (1.0 - err)) < 1e-12
    assert abs(old @ new - new @ new) < 1e-12
    if d_max > 1000:
        assert err < 1e-14
        assert np.abs(new - old).max() < 1e-12
    else:
        assert err > 1e-6


def test_keep_blocks_right_side_only():
    # keep_blocks -m keeps the m nearest right blocks only: m moves to the
    # right, none to the left (keep_blocks m keeps both sides)
    from paper_2503_20700_amd.binding import DMRG
    n, ne, ts, d, k, seed = 8, 8, 0, 64, 3, 0
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 10)
    psi, lay = random_psi(mps, seed=seed + 20)
    bs, cnt = mps.bond_table()
    for keep, moves in ((-2, [(1, 4), (1, 5), (1, -1)]), (-2, [(-1, -1)]), (2, [(-1, 2)])):
        dm = DMRG(h, g, ne, ts, keep_blocks=keep)
        dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
        for direction, want in moves:
            _, nel = dm.psi_layout()
            p = np.random.default_rng(3).normal(size=nel)
            dm.truncate(p, 10 ** 6, 0.0, direction)
            assert dm.k == want, (keep, direction, dm.k, want)
            if want < 0:
                break
        dm.close()
