"""Error paths of the C ABI that need a device: the device-memory budget
(DMRG_ERR_BUDGET, raised on the host before the allocation that would pass
it) and an unconverged Davidson (DMRG_ERR_NOCONV, with the best iterate still
written)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case():
    from synth.integrals import small_cas
    from synth.mps import random_mps, random_psi
    h, g, _ = small_cas(10, 6)
    mps = random_mps(10, 10, 0, 40, k=4, seed=106)
    psi, lay = random_psi(mps, seed=206)
    return h, g, mps, psi


def test_budget_exceeded_is_reported_before_allocating():
    from paper_2503_20700_amd.binding import DMRG, DMRGError
    print("[errors] budget", flush=True)
    h, g, mps, psi = _case()
    bs, cnt = mps.bond_table()
    dm = DMRG(h, g, 10, 0, hbm_budget_bytes=64 * 1024)
    with pytest.raises(DMRGError) as e:
        dm.set_mps(4, bs, cnt, mps.site_blocks_flat())
    assert e.value.code == -4 and "budget" in str(e.value)
    dm.close()
    # a budget that fits: same result as without one
    ref = DMRG(h, g, 10, 0)
    ref.set_mps(4, bs, cnt, mps.site_blocks_flat())
    y0, _ = ref.hpsi(psi)
    peak = ref.stats()["peak_bytes"]
    ref.close()
    dm = DMRG(h, g, 10, 0, hbm_budget_bytes=int(peak) + 1)
    dm.set_mps(4, bs, cnt, mps.site_blocks_flat())
    y1, _ = dm.hpsi(psi)
    assert np.array_equal(y0, y1)
    # the low-precision copies need more: refused, the FP64 path still works
    with pytest.raises(DMRGError) as e:
        dm.hpsi(psi, 2)
    assert e.value.code == -4
    y2, _ = dm.hpsi(psi)
    assert np.array_equal(y0, y2)
    dm.close()


@pytest.mark.parametrize("prec", [0, 2])
def test_unconverged_davidson_returns_its_best_iterate(prec):
    from paper_2503_20700_amd.binding import DMRG
    print(f"[errors] noconv prec={prec}", flush=True)
    h, g, mps, psi = _case()
    bs, cnt = mps.bond_table()
    dm = DMRG(h, g, 10, 0, hpsi_prec=prec, davidson_max_iter=1, davidson_jd_inner=4 if prec else 0)
    dm.set_mps(4, bs, cnt, mps.site_blocks_flat())
    r = dm.davidson(psi)
    assert not r["converged"] and r["resid"] > 1e-7
    x = r["psi"]
    assert abs(np.linalg.norm(x) - 1.0) < 1e-12
    y, _ = dm.hpsi(x)
    # the energy and residual reported are those of the returned vector
    assert abs(x @ y - r["energy"]) < 1e-10 * abs(r["energy"])
    assert abs(np.linalg.norm(y - r["energy"] * x) - r["resid"]) < 1e-8 * max(1.0, r["resid"])
    # and it is no worse than the start vector's Rayleigh quotient
    p0 = psi / np.linalg.norm(psi)
    y0, _ = dm.hpsi(p0)
    assert r["energy"] <= p0 @ y0 + 1e-12 * abs(r["energy"])
    dm.close()
