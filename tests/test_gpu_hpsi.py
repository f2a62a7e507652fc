"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

H*psi is compared element by element with the oracle's V^T H V psi on the same
seeded MPS and psi, at sizes where the oracle runs in seconds.  Sizes are
chosen so that operator blocks span several 64-wide MFMA tiles with ragged
tails (sector dimensions up to 75), and cover S = 0, 1/2, 1, complete and
truncated bonds.  The FP64 bar is relative max-norm error 1e-10 (the bar the
target path is held to); FP32 and BF16 operands are checked against bounds
derived from their unit roundoff (2^-24, 2^-8) times the accumulated size.
"""
import numpy as np
import pytest

from oracle import heff
from synth.integrals import small_cas
from synth.mps import random_mps, random_psi

pytestmark = pytest.mark.gpu

CASES = [
    # n, N, 2S, D, k, seed
    (4, 4, 0, 16, 1, 1),
    (6, 6, 0, 16, 2, 2),
    (7, 7, 1, 16, 2, 3),
    (6, 6, 2, 16, 2, 4),
    (8, 8, 0, 64, 3, 0),     # CAS(8,8) centre, complete two-site space
    (8, 7, 1, 20, 3, 5),
    (10, 10, 0, 40, 4, 6),
    (11, 11, 1, 500, 4, 7),  # right block complete: sectors up to 75
]


def _setup(n, ne, ts, d, k, seed):
    from paper_2503_20700_amd.binding import DMRG
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    dm = DMRG(h, g, ne, ts)
    bs, cnt = mps.bond_table()
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    return h, g, mps, psi, lay, dm


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}N{c[1]}S{c[2]}D{c[3]}" for c in CASES])
def test_hpsi_fp64_matches_oracle(case):
    n, ne, ts, d, k, seed = case
    print(f"[hpsi parity] n={n} N={ne} 2S={ts} D={d} k={k}", flush=True)
    h, g, mps, psi, lay, dm = _setup(*case)
    desc, nel = dm.psi_layout()
    assert nel == psi.size
    for i, b in enumerate(lay):
        assert tuple(desc[i]) == (b["a"][0], b["a"][1], b["c"][0], b["c"][1], b["nrows"], b["ncols"], b["offset"])
    y, flops = dm.hpsi(psi)
    ref = heff.hpsi(h, g, mps, lay, psi)
    rel = np.abs(y - ref).max() / np.abs(ref).max()
    assert rel < 1e-10, rel
    assert flops > 0
    # bitwise reproducible (fixed summation order, no atomics)
    y2, _ = dm.hpsi(psi)
    assert np.array_equal(y, y2)


def test_heff_diag_matches_oracle_dense():
    from paper_2503_20700_amd.binding import DMRG
    n, ne, ts, d, k, seed = 6, 6, 0, 16, 2, 2
    h, g, mps, psi, lay, dm = _setup(n, ne, ts, d, k, seed)
    hd = heff.HeffDefinition(h, g, mps, lay).dense()
    diag = dm.heff_diag(psi.size)
    assert np.abs(diag - np.diag(hd)).max() < 1e-10 * np.abs(np.diag(hd)).max()


F64_KERNELS = ["static", "f64pipe64x64", "f64pipe2s64x64", "f64pipe2s128x64", "f64pipe2s64x128"]


@pytest.mark.parametrize("kernel", F64_KERNELS)
@pytest.mark.parametrize("case", [CASES[2], CASES[4], CASES[7]], ids=["n7S1", "n8S0", "n11S1D500"])
def test_hpsi_fp64_kernels_match_oracle(case, kernel, monkeypatch):
    # Every FP64 kernel the tuner chooses from, forced for all H*psi launches.
    if kernel == "static":
        monkeypatch.setenv("DMRG_PIPE", "0")
    else:
        monkeypatch.setenv("DMRG_TILE", kernel)
    print(f"[hpsi fp64 kernel] {kernel} case={case}", flush=True)
    h, g, mps, psi, lay, dm = _setup(*case)
    y, _ = dm.hpsi(psi)
    ref = heff.hpsi(h, g, mps, lay, psi)
    assert np.abs(y - ref).max() < 1e-10 * np.abs(ref).max()
    y2, _ = dm.hpsi(psi)
    assert np.array_equal(y, y2)


@pytest.mark.parametrize("prec,bound,kt", [(1, 2.0 ** -24 * 64, ""), (2, 2.0 ** -8 * 8, "32"),
                                           (2, 2.0 ** -8 * 8, "64"), (2, 2.0 ** -8 * 8, "")])
@pytest.mark.parametrize("kernel", ["lean", "generic", "64x64", "64x128", "128x64", "128x128", "pipe64x64",
                                    "pipe64x128", "pipe128x64", "pipe128x128", "pipe2s64x64", "pipe2s64x128",
                                    "pipe2s128x64", "wave"])
def test_hpsi_low_precision_error_bound(prec, bound, kt, kernel, monkeypatch):
    # BF16 H*psi launches run on the lean padded-operand kernel unless it is
    # switched off; the generic kernel then runs with K slabs of 32 or 64.
    if kt:
        monkeypatch.setenv("DMRG_BF16_KT", kt)  # else chosen per launch
    if kernel == "generic":
        monkeypatch.setenv("DMRG_NO_PADDED_KERNEL", "1")
    elif kernel == "wave":
        monkeypatch.setenv("DMRG_WAVE", "1")  # 32x32 tile per wave, identity products included
    else:
        monkeypatch.setenv("DMRG_WAVE", "0")
        if kernel != "lean":
            monkeypatch.setenv("DMRG_TILE", kernel)
    case = (10, 10, 0, 40, 4, 6)
    h, g, mps, psi, lay, dm = _setup(*case)
    y64, _ = dm.hpsi(psi, 0)
    ylo, _ = dm.hpsi(psi, prec)
    rel = np.abs(ylo - y64).max() / np.abs(y64).max()
    assert rel < bound, rel
    assert rel > 0.0


def test_hermiticity_fp64():
    case = (11, 11, 1, 500, 4, 7)
    h, g, mps, psi, lay, dm = _setup(*case)
    rng = np.random.default_rng(11)
    x = rng.normal(size=psi.size)
    y = rng.normal(size=psi.size)
    hx, _ = dm.hpsi(x)
    hy, _ = dm.hpsi(y)
    lhs, rhs = x @ hy, hx @ y
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(hx) * np.linalg.norm(y)


@pytest.mark.parametrize("steps", ["1", "3"])
@pytest.mark.parametrize("wave", ["0", "1"], ids=["tile64", "wave32"])
def test_hpsi_split_k_matches_oracle(steps, wave, monkeypatch):
    # Force the executor to cut every output tile's product list into pieces
    # of at most `steps` K steps, so that nearly every tile is summed from
    # partial tiles by the reduction launch (block builds included), with
    # 64x64 tiles or with the 32x32 one-wave tiles.
    monkeypatch.setenv("DMRG_SPLIT_STEPS", steps)
    monkeypatch.setenv("DMRG_WAVE", wave)
    case = (10, 10, 0, 40, 4, 6)
    print(f"[hpsi split-K] steps={steps} case={case}", flush=True)
    h, g, mps, psi, lay, dm = _setup(*case)
    y, _ = dm.hpsi(psi)
    ref = heff.hpsi(h, g, mps, lay, psi)
    assert np.abs(y - ref).max() < 1e-10 * np.abs(ref).max()
    y2, _ = dm.hpsi(psi)
    assert np.array_equal(y, y2)
    ylo, _ = dm.hpsi(psi, 2)
    assert np.abs(ylo - ref).max() < 2.0 ** -8 * 8 * np.abs(ref).max()


@pytest.mark.parametrize("wave", ["0", "1"], ids=["tile64", "wave32"])
@pytest.mark.parametrize("case", [CASES[2], CASES[6], CASES[7]], ids=["n7S1", "n10D40", "n11D500"])
def test_hpsi_fp64_each_kernel(case, wave, monkeypatch):
    # every FP64 launch (block builds included) on one kernel or the other
    monkeypatch.setenv("DMRG_WAVE", wave)
    print(f"[hpsi fp64 kernel] wave={wave} case={case}", flush=True)
    h, g, mps, psi, lay, dm = _setup(*case)
    y, _ = dm.hpsi(psi)
    ref = heff.hpsi(h, g, mps, lay, psi)
    assert np.abs(y - ref).max() < 1e-10 * np.abs(ref).max()
    y2, _ = dm.hpsi(psi)
    assert np.array_equal(y, y2)


def test_hpsi_graph_replays_equal_eager():
    # opts.hpsi_graph: the H*psi launch sequence is recorded once per
    # precision and replayed.  Every replay -- with other work and device
    # synchronisations in between, across precisions, and after the shared
    # scratch buffer has moved (re-recorded) -- equals the eager result bit
    # for bit.
    from paper_2503_20700_amd.binding import DMRG
    case = (10, 10, 0, 40, 4, 6)
    n, ne, ts, d, k, seed = case
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    bs, cnt = mps.bond_table()
    eager = DMRG(h, g, ne, ts)
    graph = DMRG(h, g, ne, ts, hpsi_graph=True)
    for dm in (eager, graph):
        dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    rng = np.random.default_rng(5)
    vecs = [psi] + [rng.normal(size=psi.size) for _ in range(3)]
    for rep in range(3):
        for prec in (0, 2, 1):
            for v in vecs:
                print(f"[hpsi graph] rep={rep} prec={prec}", flush=True)
                want, _ = eager.hpsi(v, prec)
                got, _ = graph.hpsi(v, prec)
                assert np.array_equal(got, want)
        # eager work on the graph context's own stream between replays
        graph.heff_diag(psi.size)
    ref = heff.hpsi(h, g, mps, lay, psi)
    got, _ = graph.hpsi(psi, 0)
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("split", ["", "1"], ids=["default", "split1"])
def test_hpsi_graph_rerecords_after_scratch_moves(split, monkeypatch):
    # A later launch plan that needs a larger partial-tile buffer moves the
    # executor's scratch; the recorded graph must then be re-recorded, not
    # replayed against the freed buffer.
    from paper_2503_20700_amd.binding import DMRG
    case = (8, 8, 0, 64, 3, 0)
    n, ne, ts, d, k, seed = case
    h, g, _ = small_cas(n, seed)
    mps = random_mps(n, ne, ts, d, k=k, seed=seed + 100)
    psi, lay = random_psi(mps, seed=seed + 200)
    bs, cnt = mps.bond_table()
    dm = DMRG(h, g, ne, ts, hpsi_graph=True)
    dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
    first, _ = dm.hpsi(psi, 0)             # recorded with the current scratch
    if split:
        monkeypatch.setenv("DMRG_SPLIT_STEPS", split)
    dm.hpsi(psi, 2)                          # BF16 plan, with every tile split: more scratch
    again, _ = dm.hpsi(psi, 0)             # must re-record if the scratch moved
    assert np.array_equal(first, again)
    ref = heff.hpsi(h, g, mps, lay, psi)
    assert np.abs(again - ref).max() < 1e-10 * np.abs(ref).max()


def test_hpsi_dev_stream_orders_with_caller_stream():
    # dmrg_hpsi_dev_stream: the input is written on the caller's stream behind
    # ~30 ms of queued work, and the output is consumed on that stream right
    # after the call; with the stream ordering both see the right data
    # (without it the product would read the zero input, or the consumer NaN).
    import torch
    case = (10, 10, 0, 40, 4, 6)
    h, g, mps, psi, lay, dm = _setup(*case)
    want, _ = dm.hpsi(psi, 0)
    dev = torch.device("cuda:0")
    src = torch.from_numpy(psi).to(dev)
    x = torch.zeros_like(src)
    y = torch.full_like(src, float("nan"))
    a = torch.randn(4096, 4096, device=dev)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(20):
            a = (a @ a) * 1e-2  # keeps the stream busy before the input exists
        x.copy_(src)
        dm.hpsi_dev(x.data_ptr(), y.data_ptr(), 0, stream=s.cuda_stream)
        z = y * 1.0
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), want)
    # the call only queues its work: it returns while the caller's stream is
    # still busy with the work queued before it (~30 ms of products here)
    with torch.cuda.stream(s):
        for _ in range(20):
            a = (a @ a) * 1e-2
        x.copy_(src)
        dm.hpsi_dev(x.data_ptr(), y.data_ptr(), 0, stream=s.cuda_stream)
        busy = not s.query()
        z = y * 1.0
    torch.cuda.synchronize()
    assert busy
    assert np.array_equal(z.cpu().numpy(), want)


EDGE_CASES = [
    # n, N, 2S, D, k, seed: the degenerate shapes of the method
    (6, 6, 0, 16, 0, 11),   # two-site block at the left end: left block is the vacuum
    (6, 6, 0, 16, 4, 12),   # at the right end: right block is the vacuum
    (7, 7, 1, 20, 5, 13),   # right end, doublet
    (6, 2, 0, 16, 2, 14),   # two electrons in six orbitals
    (6, 4, 4, 16, 2, 15),   # high spin, 2S = N
    (5, 5, 5, 8, 1, 16),    # fully polarised half filling: a one-coefficient space
    (6, 10, 0, 16, 2, 17),  # two holes in six orbitals
]


@pytest.mark.parametrize("prec,bound", [(0, 1e-10), (1, 2.0 ** -24 * 64), (2, 2.0 ** -8 * 8), (3, 2.0 ** -4 * 2)],
                         ids=["fp64", "fp32", "bf16", "fp8"])
@pytest.mark.parametrize("case", EDGE_CASES, ids=[f"n{c[0]}N{c[1]}S{c[2]}k{c[4]}" for c in EDGE_CASES])
def test_hpsi_edge_cases_match_oracle(case, prec, bound):
    print(f"[hpsi edge] case={case} prec={prec}", flush=True)
    h, g, mps, psi, lay, dm = _setup(*case)
    y, _ = dm.hpsi(psi, prec)
    ref = heff.hpsi(h, g, mps, lay, psi)
    assert np.all(np.isfinite(y))
    assert np.abs(y - ref).max() <= bound * np.abs(ref).max()


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}N{c[1]}S{c[2]}D{c[3]}" for c in CASES])
def test_hpsi_fp8_error_bound(case):
    """FP8 operands (OCP E4M3, unit roundoff 2^-4) with BF16 intermediates:
    max-norm error against the oracle within 2 * 2^-4 of the largest element."""
    print(f"[hpsi fp8] case={case}", flush=True)
    h, g, mps, psi, lay, dm = _setup(*case)
    y8, _ = dm.hpsi(psi, 3)
    ref = heff.hpsi(h, g, mps, lay, psi)
    rel = np.abs(y8 - ref).max() / np.abs(ref).max()
    assert np.all(np.isfinite(y8))
    assert 0.0 < rel < 2.0 ** -4 * 2, rel
    # the Rayleigh quotient within the same relative bound
    assert abs(psi @ y8 - psi @ ref) <= 2.0 ** -4 * 2 * abs(psi @ ref)
