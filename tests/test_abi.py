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
    return sorted(set(re.findall(r"\b(dmrg_[a-z_0-9]+)\s*\(", txt)))


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
