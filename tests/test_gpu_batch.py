"""GPU parity of the batched H*psi (dmrg_batch_*): several independent
instances -- different integrals, electron counts, spins, bond dimensions and
two-site positions -- run in one grouped launch per stage and chunk.  Each
instance's result is checked against the FP64 oracle and against the same
instance's own dmrg_hpsi_dev, in every precision."""
import numpy as np
import pytest
import torch  # before the library: torch's HIP runtime must be loaded first

from oracle import heff
from synth.integrals import small_cas
from synth.mps import random_mps, random_psi

pytestmark = pytest.mark.gpu

INSTANCES = [
    # n, N, 2S, D, k, seed, work budget (elements; small values force several chunks)
    (6, 6, 0, 16, 2, 2, 0),
    (7, 7, 1, 16, 2, 3, 0),
    (8, 8, 0, 64, 3, 0, 0),
    (10, 10, 0, 40, 4, 6, 3000),
    (8, 7, 1, 20, 3, 5, 0),
]


def _make(n, ne, ts, d, k, seed, budget):
    from paper_2503_20700_amd.binding import DMRG
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    dm = DMRG(h, g, ne, ts, work_budget_elems=budget)
    bs, cnt = mps.bond_table()
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    return dict(h=h, g=g, mps=mps, psi=psi, lay=lay, dm=dm)


@pytest.fixture(scope="module")
def instances():
    out = [_make(*c) for c in INSTANCES]
    for x in out:
        x["ref"] = heff.hpsi(x["h"], x["g"], x["mps"], x["lay"], x["psi"])
    return out


def _run_batch(insts, prec):
    from paper_2503_20700_amd.binding import HpsiBatch
    dev = torch.device("cuda:0")
    d_in = [torch.from_numpy(x["psi"]).to(dev) for x in insts]
    d_out = [torch.full_like(t, float("nan")) for t in d_in]
    torch.cuda.synchronize()
    b = HpsiBatch([x["dm"] for x in insts], prec)
    b.run([t.data_ptr() for t in d_in], [t.data_ptr() for t in d_out])
    first = [t.cpu().numpy() for t in d_out]
    b.run([t.data_ptr() for t in d_in], [t.data_ptr() for t in d_out])
    second = [t.cpu().numpy() for t in d_out]
    b.close()
    return first, second


@pytest.mark.parametrize("prec,bound", [(0, 1e-10), (1, 2.0 ** -24 * 64), (2, 2.0 ** -8 * 8)],
                         ids=["fp64", "fp32", "bf16"])
def test_batch_matches_oracle_and_single(instances, prec, bound):
    print(f"[batch hpsi] prec={prec} instances={len(instances)}", flush=True)
    first, second = _run_batch(instances, prec)
    for x, y, y2 in zip(instances, first, second):
        ref = x["ref"]
        scale = np.abs(ref).max()
        assert np.all(np.isfinite(y))
        assert np.abs(y - ref).max() < bound * scale
        # fixed plan: repeated batched calls are bitwise identical
        assert np.array_equal(y, y2)
        single, _ = x["dm"].hpsi(x["psi"], prec)
        # same block products; only split-K partition and tile choice may differ
        tol = 1e-12 if prec == 0 else 2 * bound
        assert np.abs(y - single).max() < tol * scale


def test_batch_of_one_equals_single_fp64(instances):
    x = instances[2]
    (y,), _ = _run_batch([x], 0)
    single, _ = x["dm"].hpsi(x["psi"], 0)
    assert np.abs(y - single).max() < 1e-12 * np.abs(single).max()


def test_batch_rejects_changed_context():
    from paper_2503_20700_amd.binding import DMRGError, HpsiBatch
    a = _make(6, 6, 0, 16, 2, 2, 0)
    c = _make(7, 7, 1, 16, 2, 3, 0)
    b = HpsiBatch([a["dm"], c["dm"]], 0)
    dev = torch.device("cuda:0")
    d_in = [torch.from_numpy(x["psi"]).to(dev) for x in (a, c)]
    d_out = [torch.empty_like(t) for t in d_in]
    b.run([t.data_ptr() for t in d_in], [t.data_ptr() for t in d_out])
    bs, cnt = a["mps"].bond_table()
    a["dm"].set_mps(2, bs, cnt, a["mps"].site_blocks_flat())  # new plan for the first context
    with pytest.raises(DMRGError) as e:
        b.run([t.data_ptr() for t in d_in], [t.data_ptr() for t in d_out])
    assert e.value.code == -1
    # closing a context closes its batches first
    a["dm"].close()
    assert not b._h


def test_batch48_full_size_self_consistent():
    # The 48-instance workload in the launch configuration bench.py times:
    # every batched result equals its single-instance run, and the batched
    # FP64 operator is symmetric, <phi|H psi> = <H phi|psi>, per instance.
    import bench
    from paper_2503_20700_amd.binding import DMRG, HpsiBatch
    dev = torch.device("cuda:0")
    insts = bench.batch_instances()
    dms, xs = [], []
    for w in insts:
        print(f"[batch48] n={w['n']} 2S={w['two_s']} D={w['D']} seed={w['seed']}", flush=True)
        mps = random_mps(w["n"], w["N"], w["two_s"], w["D"], k=w["k"], seed=w["seed"])
        psi, _ = random_psi(mps, seed=w["seed"] + 1)
        dm = DMRG(w["h"], w["g"], w["N"], w["two_s"])
        bs, cnt = mps.bond_table()
        dm.set_mps(w["k"], bs, cnt, mps.site_blocks_flat())
        dms.append(dm)
        xs.append(torch.from_numpy(psi).to(dev))
    rng = np.random.default_rng(3)
    phis = [torch.from_numpy(rng.normal(size=x.numel())).to(dev) for x in xs]
    for prec, tol in ((0, 1e-12), (2, 2.0 ** -8 * 16)):
        print(f"[batch48] prec={prec}", flush=True)
        b = HpsiBatch(dms, prec)
        ys = [torch.empty_like(x) for x in xs]
        qs = [torch.empty_like(x) for x in xs]
        b.run([x.data_ptr() for x in xs], [y.data_ptr() for y in ys])
        b.run([p.data_ptr() for p in phis], [q.data_ptr() for q in qs])
        torch.cuda.synchronize()
        b.close()
        for dm, x, y, p, q in zip(dms, xs, ys, phis, qs):
            single = torch.empty_like(x)
            dm.hpsi_dev(x.data_ptr(), single.data_ptr(), prec)
            torch.cuda.synchronize()
            scale = float(single.abs().max())
            assert float((y - single).abs().max()) < tol * scale
            if prec == 0:
                herm = abs(float(p @ y) - float(q @ x)) / float(p.norm() * y.norm())
                assert herm < 1e-12, herm
    for dm in dms:
        dm.close()


@pytest.mark.parametrize("wave", ["0", "1"], ids=["lean", "wave"])
def test_batch_bf16_each_kernel(instances, wave, monkeypatch):
    # the merged BF16 launches on either padded kernel, against the oracle
    monkeypatch.setenv("DMRG_WAVE", wave)
    first, _ = _run_batch(instances, 2)
    for x, y in zip(instances, first):
        assert np.abs(y - x["ref"]).max() < 2.0 ** -8 * 8 * np.abs(x["ref"]).max()


@pytest.mark.parametrize("prec,jd", [(0, 0), (2, 10)], ids=["fp64", "bf16+jd"])
def test_batch_davidson_matches_single_and_dense(prec, jd):
    # dmrg_batch_davidson: every instance's solve, with its matvecs gathered
    # into the merged launches, converges to the same eigenpair as its own
    # dmrg_davidson_step; the smallest instance also against the dense
    # lowest eigenvalue of the oracle's H_eff.
    from paper_2503_20700_amd.binding import DMRG, HpsiBatch
    singles, batched, starts, dense_case = [], [], [], None
    for n, ne, ts, d, k, seed, budget in INSTANCES:
        h, g, _ = small_cas(n, seed)
        mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
        psi, lay = random_psi(mps, seed=seed + 200)
        if dense_case is None:
            dense_case = np.linalg.eigvalsh(heff.HeffDefinition(h, g, mps, lay).dense())[0]
        for lst in (singles, batched):
            dm = DMRG(h, g, ne, ts, work_budget_elems=budget, hpsi_prec=prec, davidson_jd_inner=jd,
                      davidson_max_iter=300)
            bs, cnt = mps.bond_table()
            dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
            lst.append(dm)
        starts.append(psi)
    print(f"[batch davidson] prec={prec} jd={jd}", flush=True)
    ref = [dm.davidson(p) for dm, p in zip(singles, starts)]
    b = HpsiBatch(batched, prec)
    got = b.davidson(starts)
    b.close()
    for r, s in zip(got, ref):
        assert r["converged"] and s["converged"]
        assert r["resid"] <= 1e-7
        assert abs(r["energy"] - s["energy"]) < 1e-9
        assert abs(abs(r["psi"] @ s["psi"]) - 1.0) < 1e-8
    assert abs(got[0]["energy"] - dense_case) < 1e-9


def test_batch_davidson_rejects_changed_context():
    from paper_2503_20700_amd.binding import DMRGError, HpsiBatch
    a = _make(6, 6, 0, 16, 2, 2, 0)
    c = _make(7, 7, 1, 16, 2, 3, 0)
    b = HpsiBatch([a["dm"], c["dm"]], 0)
    bs, cnt = c["mps"].bond_table()
    c["dm"].set_mps(2, bs, cnt, c["mps"].site_blocks_flat())
    with pytest.raises(DMRGError) as e:
        b.davidson([a["psi"], c["psi"]])
    assert e.value.code == -1
    b.close()
