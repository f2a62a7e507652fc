"""Full DMRG sweeps through the C ABI: Davidson (FP64, and BF16 bulk with
Jacobi-Davidson refinement) at every two-site block, truncation to D
multiplets and growth of the operator block, moving right to the chain end,
back to the left end and right to the centre (keep_blocks holds the blocks
the return trip needs), at CAS(8,8), S=0.

* D = 200 keeps every bond complete (the middle bond of CAS(8,8) needs 126
  multiplets): every step's energy is the exact FCI ground state and no
  weight is discarded.
* D = 64 truncates the middle bond: every energy lies above FCI
  (variational), the steps next to the middle bond discard weight, and the
  energies of the second pass over a block repeat those of the first
  (the sweep has converged at this D)."""
import numpy as np
import pytest

from oracle import fock
from synth.integrals import small_cas
from synth.mps import random_mps

pytestmark = pytest.mark.gpu


def _sweep(prec, d):
    from paper_2503_20700_amd.binding import DMRG
    n, ne, ts = 8, 8, 0
    h, g, _ = small_cas(n, 0)
    e_fci = fock.fci_spectrum(h, g, ne, ts)[0]
    mps = random_mps(n, ne, ts, d, k=3, seed=7)
    dm = DMRG(h, g, ne, ts, keep_blocks=True, hpsi_prec=prec, davidson_max_iter=300, davidson_jd_inner=10)
    bs, cnt = mps.bond_table()
    dm.set_mps(3, bs, cnt, mps.site_blocks_flat())
    steps = []
    for direction in [1] * 3 + [-1] * 6 + [1] * 6 + [-1] * 3:  # 3 -> 6 -> 0 -> 6 -> 3
        k = dm.k
        _, nel = dm.psi_layout()
        r = dm.davidson(np.zeros(nel))
        assert r["converged"], r
        err, kept = dm.truncate(r["psi"], d, 0.0, direction)
        steps.append((k, direction, r["energy"], err))
        assert dm.k >= 0
    dm.close()
    return e_fci, steps


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "bf16+jd"])
def test_sweep_complete_bonds_is_exact(prec):
    e_fci, steps = _sweep(prec, 200)
    print(f"[sweep D=200] prec={prec} worst |E-FCI|={max(abs(e - e_fci) for _, _, e, _ in steps):.2e}", flush=True)
    for k, _, e, err in steps:
        assert abs(e - e_fci) < 1e-8, (k, e, e_fci)
        assert err < 1e-12


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "bf16+jd"])
def test_sweep_truncated_is_variational_and_converged(prec):
    e_fci, steps = _sweep(prec, 64)
    print(f"[sweep D=64] prec={prec} E-FCI=" + " ".join(f"{e - e_fci:.2e}" for _, _, e, _ in steps), flush=True)
    assert min(e for _, _, e, _ in steps) >= e_fci - 1e-8
    assert max(err for _, _, _, err in steps) > 1e-4  # the middle bond is truncated
    # blocks visited twice in the same direction give the same energy
    first = {}
    for k, direction, e, _ in steps:
        key = (k, direction)
        if key in first:
            assert abs(e - first[key]) < 1e-6, (key, e, first[key])
        else:
            first[key] = e
