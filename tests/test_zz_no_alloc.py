"""The allocation-free H*psi entry point (dmrg_hpsi_dev_noalloc) against
dmrg_hpsi_dev, through the C ABI: two calls in a row on different contexts,
the second with a smaller input, in FP64 and BF16, then a block that needs
more scratch than the fixed array holds (refused before any launch)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ctx(n, ne, ts, d, k, seed, budget=0):
    from paper_2503_20700_amd.binding import DMRG
    from synth.integrals import small_cas
    from synth.mps import random_mps, random_psi
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    dm = DMRG(h, g, ne, ts, work_budget_elems=budget)
    bs, cnt = mps.bond_table()
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    return dm, psi


@pytest.mark.parametrize("prec,bound", [(0, 1e-10), (2, 2.0 ** -8 * 8)], ids=["fp64", "bf16"])
def test_noalloc_matches_hpsi_dev_on_two_calls(prec, bound):
    import torch
    dev = torch.device("cuda:0")
    # the first block in several chunks of at most 2^22 X elements (so that it
    # fits the fixed array), the second a smaller input
    cases = [(11, 11, 1, 500, 4, 7, 1 << 22), (8, 8, 0, 64, 3, 0, 0)]
    ctxs = []
    for case in cases:
        print(f"[noalloc] prec={prec} case={case}", flush=True)
        dm, psi = _ctx(*case)
        x = torch.from_numpy(psi).to(dev)
        want = torch.empty_like(x)
        dm.hpsi_dev(x.data_ptr(), want.data_ptr(), prec)  # makes the plan and the operator copies
        torch.cuda.synchronize()
        ctxs.append((dm, x, want))
    for dm, x, want in ctxs:
        got = torch.full_like(x, float("nan"))
        dm.hpsi_dev_noalloc(x.data_ptr(), got.data_ptr(), prec)
        torch.cuda.synchronize()
        w, g = want.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(g))
        assert np.abs(g - w).max() <= bound * np.abs(w).max()
        if prec == 0:
            ref = dm.hpsi(x.cpu().numpy(), 0)[0]
            assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()
    for dm, _, _ in ctxs:
        dm.close()


def test_noalloc_refuses_what_does_not_fit_and_unprepared_contexts():
    import torch

    from paper_2503_20700_amd.binding import DMRGError
    dev = torch.device("cuda:0")
    print("[noalloc] refusals", flush=True)
    dm, psi = _ctx(10, 10, 0, 40, 4, 6)
    x = torch.from_numpy(psi).to(dev)
    y = torch.zeros_like(x)
    dm.psi_layout()  # the plan; no BF16 operator copies yet
    with pytest.raises(DMRGError) as e:
        dm.hpsi_dev_noalloc(x.data_ptr(), y.data_ptr(), 2)
    assert e.value.code == -1
    dm.hpsi_dev_noalloc(x.data_ptr(), y.data_ptr(), 0)  # FP64 needs no copies
    torch.cuda.synchronize()
    dm.close()
    # a block whose intermediates exceed the fixed array
    big, psi = _ctx(12, 12, 0, 400, 5, 3)
    x = torch.from_numpy(psi).to(dev)
    y = torch.zeros_like(x)
    big.psi_layout()
    with pytest.raises(DMRGError) as e:
        big.hpsi_dev_noalloc(x.data_ptr(), y.data_ptr(), 0)
    assert e.value.code == -4 and "scratch" in str(e.value)
    big.close()
