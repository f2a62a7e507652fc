"""Host-side checks of the C ABI: the library loads, exports every symbol
include/dmrg.h declares, and rejects bad arguments before any GPU work
(no compute call is made here)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmrg.h")
LIB = os.path.join(ROOT, "paper_2503_20700_amd", "_lib", "libdmrg_mi355x.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b((?:dmrg|orb)_[a-z_0-9]+)\s*\(", txt)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="native library not built")
def test_library_exports_every_declared_symbol():
    lib = ct.CDLL(LIB)
    names = declared()
    assert "dmrg_hpsi" in names and "dmrg_set_mps" in names
    for name in names:
        assert hasattr(lib, name), name
    from paper_2503_20700_amd.binding import exported_symbols
    assert sorted(exported_symbols()) == names


@pytest.mark.skipif(not os.path.exists(LIB), reason="native library not built")
def test_create_rejects_bad_symmetry_and_nonfinite():
    from paper_2503_20700_amd.binding import DMRG, DMRGError
    h = np.eye(4)
    g = np.zeros((4, 4, 4, 4))
    with pytest.raises(DMRGError) as e:
        DMRG(h, g, 5, 0)  # odd N with integer spin
    assert e.value.code == -3
    with pytest.raises(DMRGError) as e:
        DMRG(h, g, 4, 6)  # S too large
    assert e.value.code == -3
    g2 = g.copy()
    g2[0, 0, 0, 0] = np.nan
    with pytest.raises(DMRGError) as e:
        DMRG(h, g2, 4, 0)
    assert e.value.code == -7


@pytest.mark.skipif(not os.path.exists(LIB), reason="native library not built")
def test_batch_rejects_bad_arguments():
    lib = ct.CDLL(LIB)
    lib.dmrg_batch_create.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.POINTER(ct.c_void_p)]
    lib.dmrg_batch_hpsi.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.dmrg_batch_destroy.argtypes = [ct.c_void_p]
    out = ct.c_void_p()
    assert lib.dmrg_batch_create(None, 1, 0, ct.byref(out)) == -1
    null_ctx = (ct.c_void_p * 2)(None, None)
    assert lib.dmrg_batch_create(null_ctx, 0, 0, ct.byref(out)) == -1
    assert lib.dmrg_batch_create(null_ctx, 2, 0, ct.byref(out)) == -1
    assert lib.dmrg_batch_create(null_ctx, 2, 7, ct.byref(out)) == -1
    assert not out.value
    assert lib.dmrg_batch_hpsi(None, None, None) == -1
    lib.dmrg_batch_destroy(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="native library not built")
def test_truncate_dbss_rejects_bad_arguments():
    lib = ct.CDLL(LIB)
    f = lib.dmrg_truncate_dbss
    f.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_void_p,
                  ct.c_void_p]
    err, kept = ct.c_double(), ct.c_int()
    assert f(None, 0, None, 1, 0, 10, 0.0, ct.byref(err), ct.byref(kept)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="native library not built")
def test_create_rejects_integrals_without_their_symmetries_and_a_negative_budget():
    from paper_2503_20700_amd.binding import DMRG, DMRGError
    rng = np.random.default_rng(0)
    n = 4
    h = rng.normal(size=(n, n))
    h = h + h.T
    b = rng.normal(size=(3, n, n))
    b = b + b.transpose(0, 2, 1)
    g = np.einsum("lpq,lrs->pqrs", b, b)
    h_bad = h.copy()
    h_bad[0, 1] += 1e-3
    g_bad = g.copy()
    g_bad[0, 1, 2, 3] += 1e-3  # (01|23) no longer equals (10|23)
    for hh, gg in ((h_bad, g), (h, g_bad)):
        with pytest.raises(DMRGError) as e:
            DMRG(hh, gg, 4, 0)
        assert e.value.code == -1
    # the integrals of S^2 pair exchange without pair hopping: not 8-fold symmetric
    gs = np.zeros((n, n, n, n))
    for p in range(n):
        for q in range(n):
            gs[p, q, q, p] -= 1.0
    with pytest.raises(DMRGError) as e:
        DMRG(h, gs, 4, 0)
    assert e.value.code == -1
    with pytest.raises(DMRGError) as e:
        DMRG(h, g, 4, 0, hbm_budget_bytes=-1)
    assert e.value.code == -1
    for bad in (dict(keep_blocks=-1), dict(davidson_mid_fp32=2), dict(davidson_graph=2)):
        with pytest.raises(DMRGError) as e:
            DMRG(h, g, 4, 0, **bad)
        assert e.value.code == -1, bad


@pytest.mark.skipif(not os.path.exists(LIB), reason="native library not built")
def test_library_su2_coefficients_match_sympy():
    """The library's own CG, 6j and 9j (the weights of every H*psi term) against
    sympy.physics.wigner, a library routine independent of both the library
    and the oracle."""
    from sympy import Rational
    from sympy.physics.wigner import clebsch_gordan, wigner_6j, wigner_9j

    from paper_2503_20700_amd.binding import DMRGError, su2_coefficient
    H = lambda x: Rational(x, 2)  # noqa: E731
    rng = np.random.default_rng(7)
    worst = 0.0
    # Clebsch-Gordan, all projections of small spins
    for j1 in range(0, 5):
        for j2 in range(0, 4):
            for J in range(abs(j1 - j2), j1 + j2 + 1, 2):
                for m1 in range(-j1, j1 + 1, 2):
                    for m2 in range(-j2, j2 + 1, 2):
                        if abs(m1 + m2) > J:
                            continue
                        ref = float(clebsch_gordan(H(j1), H(j2), H(J), H(m1), H(m2), H(m1 + m2)))
                        worst = max(worst, abs(ref - su2_coefficient(0, [j1, m1, j2, m2, J, m1 + m2])))
    # 6j: every triangle-allowed set with spins up to 3, plus random larger ones
    cnt6 = 0
    for t in rng.integers(0, 7, size=(4000, 6)):
        a, b, c, d, e, f = (int(x) for x in t)
        try:
            ref = float(wigner_6j(H(a), H(b), H(c), H(d), H(e), H(f)))
        except ValueError:  # a triad with a half-integer sum: the symbol is zero
            ref = 0.0
        worst = max(worst, abs(ref - su2_coefficient(1, [a, b, c, d, e, f])))
        cnt6 += ref != 0.0
    # 9j, including the spin-1/2 and spin-1 rows the operator couplings use
    def tri(a, b, c):
        return abs(a - b) <= c <= a + b and (a + b + c) % 2 == 0

    valid9 = []
    while len(valid9) < 150:  # rows and columns all triangle-allowed (mostly non-zero symbols)
        v = [int(x) for x in rng.integers(0, 5, size=9)]
        if all(tri(*v[3 * r:3 * r + 3]) for r in range(3)) and all(tri(v[c], v[c + 3], v[c + 6]) for c in range(3)):
            valid9.append(v)
    cnt9 = 0
    for v in valid9 + [[int(x) for x in t] for t in rng.integers(0, 5, size=(200, 9))]:
        try:
            ref = float(wigner_9j(*[H(x) for x in v]))
        except ValueError:
            ref = 0.0
        worst = max(worst, abs(ref - su2_coefficient(2, v)))
        cnt9 += ref != 0.0
    assert worst < 1e-12, worst
    assert cnt6 > 50 and cnt9 > 10  # enough non-zero symbols were compared
    with pytest.raises(DMRGError):
        su2_coefficient(3, [0] * 9)
