"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The library's host sources (SU(2) coefficients, site operators, planner,
H*psi plan, Davidson driver, truncation, batching, orbital step, C ABI) are
compiled with -fsanitize=address,undefined into a separate library together
with tests/asan/host_executor.cpp, a plain-loop stand-in for the HIP
executor; a child Python process then drives that library through the
binding over a small workload -- H*psi in every precision, Davidson with and
without the FP32 middle phase, Davidson iterations recorded as graphs against
eager ones, truncation both ways with carried start vectors, checkpoint and
resume, a batch of two instances, the orbital step and the argument checks.  Any sanitizer report fails the test.  The product
library is not involved: this checks the host-side index arithmetic, which
the GPU tests exercise only through results."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_20700_amd", "csrc")
HOST = ["su2.cpp", "spin.cpp", "planner.cpp", "hpsi.cpp", "api.cpp", "driver.cpp", "batch.cpp", "orbital.cpp"]
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined"]

DRIVER = r'''
import sys
sys.modules["torch"] = None  # keep torch's runtime out of the sanitized process
sys.path.insert(0, ROOT)
import numpy as np
from paper_2503_20700_amd.binding import DMRG, DMRGError, HpsiBatch, load_checkpoint, orb_grad
from synth.integrals import small_cas
from synth.mps import random_mps, random_psi

n, ne, ts, d, k = 8, 8, 0, 20, 3
h, g, B = small_cas(n, 0)
mps = random_mps(n, ne, ts, d, k=k, seed=7)
psi, lay = random_psi(mps, seed=8)
bs, cnt = mps.bond_table()
dm = DMRG(h, g, ne, ts, keep_blocks=True, next_guess=True, hpsi_prec=2, davidson_mid_fp32=True,
          davidson_max_iter=80)
dm.set_mps(k, bs, cnt, mps.site_blocks_flat())
for prec in (0, 1, 2, 3):
    dm.hpsi(psi, prec)
dm.heff_diag(psi.size)
r = dm.davidson(psi)
dm.truncate(r["psi"], 12, 0.0, 1)
r2 = dm.davidson(dm.next_guess())
dm.save_checkpoint(TMP + "/ck.npz", r2["psi"])
dm.truncate(r2["psi"], 12, 1e-6, -1, d_min=4)
dm.davidson(dm.next_guess())
dm.stats(); dm.cut_spectrum(); dm.get_bond(4); dm.tuner_report()
other = DMRG(h, g, ne, ts, davidson_max_iter=40)
p0 = other.resume(TMP + "/ck.npz")
other.hpsi(p0)
a = DMRG(h, g, ne, ts, davidson_max_iter=40)
b = DMRG(h, g, ne, ts, davidson_max_iter=40)
for x in (a, b):
    x.set_mps(k, bs, cnt, mps.site_blocks_flat())
bt = HpsiBatch([a, b], 0)
bt.davidson([psi, psi])
bt.close()
# Davidson iterations recorded as graphs (replayed closures on this
# executor) against the eager iteration: the same eigenpair bit for bit and
# the same matvec counts, with restarts (subspace 8) between recorded steps
mps_h = random_mps(7, 7, 1, 12, k=2, seed=9)  # a doublet
psi_h, _ = random_psi(mps_h, seed=10)
h7, g7, _ = small_cas(7, 3)
cases = [(0, {}, None), (2, dict(davidson_mid_fp32=True), None), (2, dict(davidson_jd_inner=4), None),
         (3, {}, None), (2, {}, "doublet")]
for prec, extra, which in cases:
    res = []
    for rec in (False, True):
        if which is None:
            x = DMRG(h, g, ne, ts, hpsi_prec=prec, davidson_max_iter=80, davidson_max_subspace=8,
                     davidson_graph=rec, hpsi_graph=rec, **extra)
            x.set_mps(k, bs, cnt, mps.site_blocks_flat())
            res.append(x.davidson(psi))
        else:
            x = DMRG(h7, g7, 7, 1, hpsi_prec=prec, davidson_max_iter=80, davidson_max_subspace=8,
                     davidson_graph=rec, **extra)
            b7, c7 = mps_h.bond_table()
            x.set_mps(2, b7, c7, mps_h.site_blocks_flat())
            res.append(x.davidson(psi_h))
        x.close()
    e, f = res
    assert e["energy"] == f["energy"] and np.array_equal(e["psi"], f["psi"]), (prec, extra)
    assert (e["n_lo"], e["n_fp64"]) == (f["n_lo"], f["n_fp64"]), (prec, extra, e["n_lo"], f["n_lo"])
    print("recorded iterations", prec, extra, e["n_lo"], e["n_fp64"], flush=True)
for bad in (lambda: DMRG(h, g, ne, ts, keep_blocks=-1), lambda: dm.hpsi(psi[:-1]), lambda: dm.truncate(psi, 0, 0.0, 1)):
    try:
        bad()
    except (DMRGError, ValueError):
        pass
nc, na, nv = 1, 4, 3
rng = np.random.default_rng(1)
hh, BB = h[: nc + na + nv, : nc + na + nv].copy(), B[:, : nc + na + nv, : nc + na + nv].copy()
gam = np.eye(na) * 0.5
Gam = np.zeros((na, na, na, na))
kap = np.tril(rng.normal(scale=1e-3, size=(nc + na + nv, nc + na + nv)), -1)
orb_grad(nc, na, nv, hh, BB, kap, gam, Gam)
print("host flow done", flush=True)
'''


def _asan_runtime():
    out = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = out.stdout.strip()
    return p if out.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_address_and_ub_sanitizers():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("libasan not available")
    with tempfile.TemporaryDirectory() as tmp:
        objs, procs = [], []
        for src in HOST + [os.path.join(ROOT, "tests", "asan", "host_executor.cpp")]:
            path = src if os.path.isabs(src) else os.path.join(CSRC, src)
            obj = os.path.join(tmp, os.path.basename(path) + ".o")
            objs.append(obj)
            procs.append(subprocess.Popen(["g++", *FLAGS, "-c", path, "-o", obj], stderr=subprocess.PIPE, text=True))
        for pr in procs:
            _, err = pr.communicate()
            assert pr.returncode == 0, err[-3000:]
        lib = os.path.join(tmp, "libdmrg_host_asan.so")
        link = subprocess.run(["g++", "-shared", "-fsanitize=address,undefined", *objs, "-o", lib],
                              capture_output=True, text=True)
        assert link.returncode == 0, link.stderr[-3000:]
        env = dict(os.environ, DMRG_MI355X_LIB=lib, LD_PRELOAD=rt,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        script = "ROOT = %r\nTMP = %r\n" % (ROOT, tmp) + DRIVER
        run = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=900)
        report = run.stdout[-2000:] + run.stderr[-6000:]
        assert "AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, report
        assert run.returncode == 0 and "host flow done" in run.stdout, report
