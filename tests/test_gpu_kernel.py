"""The grouped MFMA GEMM kernel on its own (through dmrg_gemm_selftest) against
numpy's matmul: tile interiors, ragged tails in m, n and k, transposed
operands, identity operands, accumulation, and the three arithmetic paths."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (16, 16, 4), (64, 64, 16), (65, 63, 17), (130, 70, 33), (7, 200, 129), (200, 9, 5)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("wave", ["", "0", "1"], ids=["auto", "tile64", "wave32"])
def test_gemm_fp64(m, n, k, ta, tb, wave, monkeypatch):
    # FP64 on the 64x64-tile kernel and on the one-wave-per-32x32-tile kernel
    if wave:
        monkeypatch.setenv("DMRG_WAVE", wave)
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    c0 = rng.normal(size=(m, n))
    got = gemm_selftest(a.T.copy() if ta else a, b.T.copy() if tb else b, C=c0, trans_a=bool(ta), trans_b=bool(tb),
                        alpha=0.75, beta=1.0)
    ref = c0 + 0.75 * (a @ b)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("m,n", [(1, 1), (65, 63), (130, 7)])
@pytest.mark.parametrize("wave", ["0", "1"], ids=["tile64", "wave32"])
def test_gemm_identity_operands(m, n, wave, monkeypatch):
    monkeypatch.setenv("DMRG_WAVE", wave)
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(3)
    b = rng.normal(size=(m, n))
    got = gemm_selftest(None, b, ident_a=True, alpha=-2.0)
    assert np.abs(got + 2.0 * b).max() < 1e-14
    a = rng.normal(size=(m, n))
    got = gemm_selftest(a.T.copy(), None, trans_a=True, ident_b=True, alpha=0.5)
    assert np.abs(got - 0.5 * a).max() < 1e-14


@pytest.mark.parametrize("prec,eps,kt", [(1, 2.0 ** -24, "32"), (2, 2.0 ** -8, "32"), (2, 2.0 ** -8, "64")])
@pytest.mark.parametrize("m,n,k", [(65, 63, 17), (130, 70, 300)])
def test_gemm_low_precision(prec, eps, kt, m, n, k, monkeypatch):
    monkeypatch.setenv("DMRG_BF16_KT", kt)
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(5)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    got = gemm_selftest(a, b, prec=prec)
    ref = a @ b
    # |error| <= ~2 eps * sum_k |a||b| (operand rounding) + k * 2^-24 * ... (fp32 accumulation)
    bound = (2 * eps + k * 2.0 ** -24) * (np.abs(a) @ np.abs(b))
    assert np.all(np.abs(got - ref) <= 4 * bound + 1e-30)


@pytest.mark.parametrize("prec,kt", [(0, "32"), (1, "32"), (2, "32"), (2, "64")])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 32), (65, 63, 17), (130, 70, 33), (7, 200, 129), (200, 9, 5)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_padded_vector_path(prec, kt, m, n, k, ta, tb, monkeypatch):
    # Rows padded to a multiple of 8 with NaN padding: the 16-byte vector
    # loads must mask everything past the logical extent (a leaked NaN fails).
    # BF16 runs with K slabs of 32 and of 64.
    monkeypatch.setenv("DMRG_BF16_KT", kt)
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    c0 = rng.normal(size=(m, n))
    for pa, pb in [(True, True), (True, False), (False, True)]:
        got = gemm_selftest(a.T.copy() if ta else a, b.T.copy() if tb else b, C=c0, trans_a=bool(ta),
                            trans_b=bool(tb), alpha=0.75, beta=1.0, prec=prec, pad_a=pa, pad_b=pb)
        ref = c0 + 0.75 * (a @ b)
        assert np.all(np.isfinite(got))
        if prec == 0:
            assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
        else:
            eps = 2.0 ** -24 if prec == 1 else 2.0 ** -8
            bound = (2 * eps + k * 2.0 ** -24) * 0.75 * (np.abs(a) @ np.abs(b)) + 2.0 ** -24 * np.abs(ref)
            assert np.all(np.abs(got - ref) <= 4 * bound + 1e-30)


@pytest.mark.parametrize("m,n,k", [(65, 63, 17), (130, 70, 300), (7, 200, 129)])
def test_gemm_bf16_lean_and_generic_kernels_agree(m, n, k, monkeypatch):
    # Fully padded BF16 operands run on the lean kernel; with it switched off
    # the generic kernel computes the same product (both accumulate in FP32).
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(11)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    monkeypatch.setenv("DMRG_WAVE", "0")
    lean = gemm_selftest(a, b, alpha=-1.25, prec=2, pad_a=True, pad_b=True)
    monkeypatch.setenv("DMRG_WAVE", "1")
    wave = gemm_selftest(a, b, alpha=-1.25, prec=2, pad_a=True, pad_b=True)
    monkeypatch.setenv("DMRG_NO_PADDED_KERNEL", "1")
    generic = gemm_selftest(a, b, alpha=-1.25, prec=2, pad_a=True, pad_b=True)
    assert np.abs(lean - generic).max() <= 1e-5 * np.abs(generic).max()
    assert np.abs(wave - generic).max() <= 1e-5 * np.abs(generic).max()


@pytest.mark.parametrize("tile", ["64x64", "64x128", "128x64", "128x128", "pipe64x64", "pipe64x128", "pipe128x64",
                                  "pipe128x128", "pipe2s64x64", "pipe2s64x128", "pipe2s128x64"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (65, 63, 17), (130, 70, 300), (7, 200, 129), (200, 9, 5), (129, 257, 40)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_bf16_lean_tile_shapes(tile, m, n, k, ta, tb, monkeypatch):
    # Every output tile shape of the lean BF16 kernel on NaN-padded operands.
    monkeypatch.setenv("DMRG_TILE", tile)
    monkeypatch.setenv("DMRG_WAVE", "0")
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(m + 3 * n + 7 * k)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    c0 = rng.normal(size=(m, n))
    got = gemm_selftest(a.T.copy() if ta else a, b.T.copy() if tb else b, C=c0, trans_a=bool(ta), trans_b=bool(tb),
                        alpha=0.5, beta=1.0, prec=2, pad_a=True, pad_b=True)
    ref = c0 + 0.5 * (a @ b)
    bound = (2 * 2.0 ** -8 + k * 2.0 ** -24) * 0.5 * (np.abs(a) @ np.abs(b)) + 2.0 ** -24 * np.abs(ref)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= 4 * bound + 1e-30)


@pytest.mark.parametrize("tile", ["f64pipe64x64", "f64pipe2s64x64", "f64pipe2s128x64", "f64pipe2s64x128"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (65, 63, 17), (130, 70, 300), (7, 200, 129), (200, 9, 5), (129, 257, 40)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_f64_pipelined_tile_shapes(tile, m, n, k, ta, tb, monkeypatch):
    # The FP64 LDS-pipelined kernel on NaN-padded operands: both storage
    # orientations of each operand, ragged edges, k tails, accumulation.
    monkeypatch.setenv("DMRG_TILE", tile)
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(m + 5 * n + 11 * k)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    c0 = rng.normal(size=(m, n))
    got = gemm_selftest(a.T.copy() if ta else a, b.T.copy() if tb else b, C=c0, trans_a=bool(ta), trans_b=bool(tb),
                        alpha=0.5, beta=1.0, prec=0, pad_a=True, pad_b=True)
    ref = c0 + 0.5 * (a @ b)
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() <= 1e-13 * (1.0 + np.abs(ref).max()) * k


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (5, 3, 40), (32, 32, 32), (33, 31, 65), (65, 63, 17), (7, 200, 129),
                                   (200, 9, 5)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_gemm_bf16_wave_kernel(m, n, k, ta, tb, beta, monkeypatch):
    # The one-wave-per-32x32-tile BF16 kernel on NaN-padded operands: vector
    # loads along k, element loads along m / n, ragged edges, accumulation.
    monkeypatch.setenv("DMRG_WAVE", "1")
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(m + 5 * n + 11 * k)
    a = rng.normal(size=(m, k))
    b = rng.normal(size=(k, n))
    c0 = rng.normal(size=(m, n))
    got = gemm_selftest(a.T.copy() if ta else a, b.T.copy() if tb else b, C=c0, trans_a=bool(ta), trans_b=bool(tb),
                        alpha=-0.625, beta=beta, prec=2, pad_a=True, pad_b=True)
    ref = beta * c0 - 0.625 * (a @ b)
    bound = (2 * 2.0 ** -8 + k * 2.0 ** -24) * 0.625 * (np.abs(a) @ np.abs(b)) + 2.0 ** -24 * np.abs(ref)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= 4 * bound + 1e-30)


def _e4m3_values():
    """All finite non-negative OCP E4M3 values (bias 7, subnormals m * 2^-9, max 448)."""
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue  # NaN
            vals.append(m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
    return np.array(sorted(set(vals)))


def _quantize_e4m3(x):
    """Round to the nearest E4M3 value, ties to the even code, saturating at 448."""
    grid = _e4m3_values()
    codes = {v: i for i, v in enumerate(grid)}  # in increasing order, code parity = mantissa parity
    out = np.empty_like(x)
    for i, v in enumerate(np.asarray(x, dtype=np.float32).astype(np.float64).ravel()):
        a = min(abs(v), 448.0)
        j = np.searchsorted(grid, a)
        cand = [grid[max(j - 1, 0)], grid[min(j, len(grid) - 1)]]
        d0, d1 = abs(a - cand[0]), abs(a - cand[1])
        q = cand[0] if d0 < d1 else cand[1] if d1 < d0 else (cand[0] if codes[cand[0]] % 2 == 0 else cand[1])
        out.ravel()[i] = np.copysign(q, v)
    return out


@pytest.mark.parametrize("m,n", [(65, 63), (130, 7)])
def test_gemm_fp8_operands_are_ocp_e4m3(m, n):
    """FP8 operands: x / s rounded to OCP E4M3 (nearest, ties to even,
    saturating), s the smallest power of two with max|x| / s <= 448, widened
    exactly for the BF16 MFMA.  A times the identity (stored in FP8 too)
    returns s * E4M3(A / s) exactly."""
    from paper_2503_20700_amd.binding import gemm_selftest
    rng = np.random.default_rng(11)
    a = rng.normal(size=(m, n)) * np.exp(rng.uniform(-6, 6, size=(m, n)))
    a[0, 0] = 0.0
    eye = np.eye(n)
    got = gemm_selftest(a, eye, prec=3, pad_a=True, pad_b=True)
    s = 2.0 ** np.ceil(np.log2(np.abs(a).max() / 448.0))
    assert np.abs(a).max() / s <= 448.0 < 2 * np.abs(a).max() / s
    want = s * _quantize_e4m3(a / s)
    assert np.array_equal(got, want)
    # a product: operand rounding 2^-4 each, FP32 accumulation
    b = rng.normal(size=(n, 40))
    got = gemm_selftest(a, b, prec=3, pad_a=True, pad_b=True)
    ref = a @ b
    bound = (2 * 2.0 ** -4 + n * 2.0 ** -24) * (np.abs(a) @ np.abs(b))
    assert np.all(np.abs(got - ref) <= 2 * bound + 1e-300)
