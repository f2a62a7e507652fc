"""Checks at the full sizes of the CAS(32,32) D=1024 and CAS(82,82) D=4096
workloads, in the launch configuration bench.py times (centre two-site block,
default work budget).  The oracle cannot build these spaces, so the checks are
properties that hold at any size:

* FP64 H_eff is symmetric: <phi|H psi> = <H phi|psi> for random phi, psi;
* FP64 H*psi is bitwise reproducible (fixed summation order);
* the BF16 path (lean kernel) agrees with FP64 within the bound of BF16
  operands with FP32 accumulation used at small sizes, and its Rayleigh
  quotient is within the same relative bound.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _workload(name):
    import bench
    return bench.workload(name)


@pytest.mark.parametrize("name", ["cas32_d1024", "cas82_d4096"], ids=["cas32_d1024", "cas82_d4096"])
def test_fullsize_properties(name):
    from paper_2503_20700_amd.binding import BF16, DMRG, FP64
    from synth.mps import random_mps, random_psi
    w = _workload(name)
    print(f"[fullsize] {w['name']}", flush=True)
    mps = random_mps(w["n"], w["N"], w["two_s"], w["D"], k=w["k"], seed=w["seed"])
    psi, _ = random_psi(mps, seed=w["seed"] + 1)
    dm = DMRG(w["h"], w["g"], w["N"], w["two_s"])
    bs, cnt = mps.bond_table()
    dm.set_mps(w["k"], bs, cnt, mps.site_blocks_flat())
    print("[fullsize] operator blocks built", flush=True)
    y, flops = dm.hpsi(psi, FP64)
    assert flops > 0 and np.all(np.isfinite(y))
    phi = np.random.default_rng(3).normal(size=psi.size)
    hphi, _ = dm.hpsi(phi, FP64)
    scale = np.linalg.norm(phi) * np.linalg.norm(y)
    assert abs(phi @ y - hphi @ psi) <= 1e-12 * scale
    y2, _ = dm.hpsi(psi, FP64)
    assert np.array_equal(y, y2)
    ylo, _ = dm.hpsi(psi, BF16)
    assert np.abs(ylo - y).max() <= 2.0 ** -8 * 8 * np.abs(y).max()
    e64, elo = psi @ y, psi @ ylo
    assert abs(elo - e64) <= 2.0 ** -8 * 8 * abs(e64)
    dm.close()
