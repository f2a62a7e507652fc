"""Exact identities of H_eff through the C ABI (FP64 path), at the oracle's
small sizes and -- where no oracle reaches -- at the full CAS(32,32) D=1024
and CAS(82,82) D=4096 workloads in the launch configuration bench.py times.

With (h, g) shifted by alpha*1 and beta*delta_pq*delta_rs and the orbital
sign gauge a_p -> -a_p applied to a set F of orbitals (integrals, site
tensors and the two-site coefficients; tests/identities.py),

    P H'_eff P psi = H_eff psi + (alpha*N + beta*N(N-1)/2) psi

exactly.  The gauge changes the sign of every integral with an odd count of
indices in F and of every renormalised operator built from a flipped site, so
an integral taken with a wrong index (one that changes the count parity of F)
or a fermion sign applied at the wrong place breaks the identity; the shifts
check the one-body diagonal and the Coulomb pieces through every block.  The
bar is relative max-norm 1e-10, the FP64 parity bar.
"""
import numpy as np
import pytest

import identities as ident

pytestmark = pytest.mark.gpu

ALPHA, BETA = 0.37, -0.021


def _hpsi(h, g, mps, k, ne, ts, psi):
    from paper_2503_20700_amd.binding import DMRG, FP64
    dm = DMRG(h, g, ne, ts)
    bs, cnt = mps.bond_table()
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    y, _ = dm.hpsi(psi, FP64)
    dm.close()
    return y


def _check(h, g, mps, lay, psi, k, ne, ts, flips):
    y = _hpsi(h, g, mps, k, ne, ts, psi)
    h2, g2, mps2 = ident.transformed(h, g, mps, ALPHA, BETA, flips)
    y2 = _hpsi(h2, g2, mps2, k, ne, ts, ident.gauge_psi(psi, lay, k, flips))
    c = ident.shift_value(ne, ts, ALPHA, BETA)
    err = np.abs(ident.gauge_psi(y2, lay, k, flips) - y - c * psi).max() / np.abs(y).max()
    print(f"[identities] rel err {err:.2e}", flush=True)
    assert err < 1e-10, err


@pytest.mark.parametrize("n,ne,ts,d,k,seed", [(6, 6, 0, 16, 2, 2), (7, 7, 1, 16, 2, 3), (6, 6, 2, 16, 2, 4),
                                              (10, 10, 0, 40, 4, 6), (11, 11, 1, 500, 4, 7)])
def test_shift_and_gauge_identity_small(n, ne, ts, d, k, seed):
    from synth.integrals import small_cas
    from synth.mps import random_mps, random_psi
    print(f"[identities] n={n} N={ne} 2S={ts} D={d} k={k}", flush=True)
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    flips = {0, k, k + 1, n - 1} | ({k - 1} if k > 1 else set())
    _check(h, g, mps, lay, psi, k, ne, ts, flips)


@pytest.mark.parametrize("name", ["cas32_d1024", "cas82_d4096"], ids=["cas32_d1024", "cas82_d4096"])
def test_shift_and_gauge_identity_fullsize(name):
    import bench
    from synth.mps import random_mps, random_psi
    w = bench.workload(name)
    print(f"[identities] {w['name']}", flush=True)
    mps = random_mps(w["n"], w["N"], w["two_s"], w["D"], k=w["k"], seed=w["seed"])
    psi, lay = random_psi(mps, seed=w["seed"] + 1)
    k, n = w["k"], w["n"]
    flips = {1, k // 2, k - 1, k, k + 1, k + 3, (k + n) // 2, n - 1}
    _check(w["h"], w["g"], mps, lay, psi, k, w["N"], w["two_s"], flips)
