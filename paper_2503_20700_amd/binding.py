"""ctypes binding of the C ABI declared in include/dmrg.h (argument marshalling only).

Every computation happens in the native library; this module converts numpy
arrays to pointers, checks return codes and raises ``DMRGError`` with the
library's message.  The library is loaded from the package's ``_lib``
directory (built by ``__graft_entry__.build()``); if it is missing the import
of this module succeeds but constructing ``DMRG`` raises immediately -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(_HERE, "_lib", "libdmrg_mi355x.so")

FP64, FP32, BF16, FP8 = 0, 1, 2, 3
ERRORS = {-1: "ARG", -2: "SHAPE", -3: "SYMMETRY", -4: "BUDGET", -5: "HIP", -6: "NOCONV", -7: "NONFINITE"}


class DMRGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Opts(ct.Structure):
    _fields_ = [("n_orb", ct.c_int), ("n_elec", ct.c_int), ("two_s", ct.c_int), ("e_core", ct.c_double),
                ("davidson_tol", ct.c_double), ("davidson_max_iter", ct.c_int),
                ("davidson_max_subspace", ct.c_int), ("hpsi_prec", ct.c_int),
                ("work_budget_elems", ct.c_longlong), ("keep_blocks", ct.c_int),
                ("davidson_refine_iter", ct.c_int), ("davidson_jd_inner", ct.c_int),
                ("davidson_lowprec_iter", ct.c_int), ("hpsi_graph", ct.c_int), ("next_guess", ct.c_int),
                ("hbm_budget_bytes", ct.c_longlong), ("davidson_mid_fp32", ct.c_int),
                ("davidson_graph", ct.c_int)]


_LIBS = {}


def load(path=None):
    path = os.path.abspath(path or os.environ.get("DMRG_MI355X_LIB", DEFAULT_LIB))
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        raise FileNotFoundError(f"native library not built: {path} (run __graft_entry__.build())")
    # PyTorch-ROCm ships its own HIP runtime.  If the library's runtime is
    # loaded into the process first, torch's later finds no GPU; loaded in
    # this order both see it, so callers may hand torch device buffers to
    # the *_dev entry points.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(path)
    P, I, D, LL, V = ct.c_void_p, ct.c_int, ct.c_double, ct.c_longlong, None
    dp = ct.POINTER(ct.c_double)
    ip = ct.POINTER(ct.c_int)
    llp = ct.POINTER(ct.c_longlong)
    sig = {
        "dmrg_create": (I, [ct.POINTER(P), ct.POINTER(Opts), dp, dp]),
        "dmrg_set_mps": (I, [P, I, ip, ip, dp, LL]),
        "dmrg_psi_layout": (I, [P, I, llp, llp, llp]),
        "dmrg_hpsi": (I, [P, I, dp, dp, I, dp]),
        "dmrg_hpsi_dev": (I, [P, I, P, P, I]),
        "dmrg_hpsi_dev_stream": (I, [P, I, P, P, I, P]),
        "dmrg_heff_diag": (I, [P, I, dp]),
        "dmrg_davidson_step": (I, [P, I, dp, dp, dp, ip, ip]),
        "dmrg_truncate": (I, [P, I, dp, I, I, D, dp, ip]),
        "dmrg_truncate_dbss": (I, [P, I, dp, I, I, I, D, dp, ip]),
        "dmrg_cut_spectrum": (I, [P, dp, ip, ip, I]),
        "dmrg_stats": (I, [P, dp, I]),
        "dmrg_su2_coefficient": (I, [I, ip, dp]),
        "dmrg_update_opts": (I, [P, ct.POINTER(Opts)]),
        "dmrg_tuner_report": (I, [P, ct.c_char_p, I]),
        "dmrg_hpsi_dev_noalloc": (I, [P, I, P, P, I]),
        "orb_grad": (I, [I, I, I, dp, dp, I, dp, dp, dp, dp, dp]),
        "dmrg_gemm_selftest": (I, [I, I, I, dp, I, I, dp, I, I, D, D, dp, I]),
        "dmrg_kernel_timing": (I, [P, I, dp, llp]),
        "dmrg_current_block": (I, [P, ip]),
        "dmrg_next_guess": (I, [P, I, dp, LL]),
        "dmrg_get_bond": (I, [P, I, ip, ip]),
        "dmrg_get_site": (I, [P, I, dp, llp]),
        "dmrg_batch_create": (I, [ct.POINTER(P), I, I, ct.POINTER(P)]),
        "dmrg_batch_hpsi": (I, [P, ct.POINTER(P), ct.POINTER(P)]),
        "dmrg_batch_destroy": (V, [P]),
        "dmrg_batch_davidson": (I, [P, ct.POINTER(dp), dp, dp, ip, ip, ip]),
        "dmrg_last_error": (ct.c_char_p, []),
        "dmrg_destroy": (V, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIBS[path] = lib
    return lib


def exported_symbols():
    return ["dmrg_create", "dmrg_set_mps", "dmrg_psi_layout", "dmrg_hpsi", "dmrg_hpsi_dev", "dmrg_hpsi_dev_stream",
            "dmrg_heff_diag",
            "dmrg_davidson_step", "dmrg_truncate", "dmrg_truncate_dbss", "dmrg_cut_spectrum", "dmrg_stats", "dmrg_gemm_selftest",
            "dmrg_kernel_timing", "dmrg_current_block", "dmrg_next_guess", "dmrg_get_bond", "dmrg_get_site", "dmrg_batch_create",
            "dmrg_batch_hpsi", "dmrg_batch_destroy", "dmrg_batch_davidson", "dmrg_su2_coefficient", "dmrg_update_opts",
            "dmrg_hpsi_dev_noalloc", "orb_grad", "dmrg_tuner_report",
            "dmrg_last_error",
            "dmrg_destroy"]


def su2_coefficient(kind, two_j, lib=None):
    """The library's CG (kind 0), 6j (kind 1) or 9j (kind 2) coefficient for
    doubled spins two_j (dmrg_su2_coefficient)."""
    L = load(lib)
    a = (ct.c_int * len(two_j))(*[int(x) for x in two_j])
    v = ct.c_double()
    rc = L.dmrg_su2_coefficient(int(kind), a, ct.byref(v))
    if rc != 0:
        raise DMRGError(rc, L.dmrg_last_error().decode())
    return v.value


def orb_grad(n_core, n_act, n_virt, h, B, kappa, gamma, Gamma, lib=None):
    """Energy at fixed active-space RDMs after the orbital rotation kappa, and
    dE/dkappa (orb_grad): returns (energy, grad) with grad antisymmetric,
    grad[p, q] = dE/dkappa_pq for p > q.  h: n x n, B: naux x n x n symmetric
    density-fitting factors, kappa: n x n (strict lower triangle read),
    gamma: n_act^2, Gamma: n_act^4 (Gamma~_tuvw = <a+_ts a+_ut a_vt a_ws>)."""
    L = load(lib)
    n = n_core + n_act + n_virt
    h = np.ascontiguousarray(h, dtype=np.float64).reshape(n, n)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1, n, n)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64).reshape(n, n)
    gamma = np.ascontiguousarray(gamma, dtype=np.float64).reshape(n_act, n_act)
    Gamma = np.ascontiguousarray(Gamma, dtype=np.float64).reshape((n_act,) * 4)
    e = np.zeros(1)
    grad = np.zeros((n, n))
    rc = L.orb_grad(n_core, n_act, n_virt, _dp(h), _dp(B), B.shape[0], _dp(kappa), _dp(gamma), _dp(Gamma), _dp(e),
                    _dp(grad))
    if rc != 0:
        raise DMRGError(rc, L.dmrg_last_error().decode())
    return float(e[0]), grad


def orbital_energy_function():
    """torch.autograd.Function E(kappa) at fixed integrals and RDMs: forward and
    backward both run in the library (orb_grad: the gradient is the
    hand-written backward on the GPU); backward scales it by the incoming
    gradient.  Use: E = F.apply(kappa, n_core, n_act, n_virt, h, B, gamma, Gamma)
    with kappa a float64 tensor (n x n, strict lower triangle read); the
    gradient returned for kappa is dE/dkappa in its strict lower triangle."""
    import torch

    class OrbitalEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, kappa, n_core, n_act, n_virt, h, B, gamma, Gamma):
            k = kappa.detach().to("cpu", torch.float64).numpy()
            e, grad = orb_grad(n_core, n_act, n_virt, h, B, k, gamma, Gamma)
            ctx.save_for_backward(torch.from_numpy(np.tril(grad, -1)).to(kappa.device, kappa.dtype))
            return torch.tensor(e, dtype=kappa.dtype, device=kappa.device)

        @staticmethod
        def backward(ctx, g_out):
            (grad,) = ctx.saved_tensors
            return (g_out * grad, None, None, None, None, None, None, None)

    return OrbitalEnergy


def gemm_selftest(A, B, C=None, trans_a=False, trans_b=False, ident_a=False, ident_b=False, alpha=1.0, beta=0.0,
                  prec=FP64, pad_a=False, pad_b=False, lib=None):
    """C = beta*C + alpha op(A) op(B) through the library's grouped MFMA kernel.
    pad_a / pad_b store that operand with NaN-padded rows (multiple of 8) and
    select the kernel's vector staging path."""
    lib = load(lib)
    if ident_a:
        B = np.ascontiguousarray(B, dtype=np.float64)
        k, n = (B.shape[1], B.shape[0]) if trans_b else B.shape
        m = k
    else:
        A = np.ascontiguousarray(A, dtype=np.float64)
        m, k = (A.shape[1], A.shape[0]) if trans_a else A.shape
        if ident_b:
            n = k
        else:
            B = np.ascontiguousarray(B, dtype=np.float64)
            n = B.shape[0] if trans_b else B.shape[1]
    C = np.zeros((m, n)) if C is None else np.ascontiguousarray(C, dtype=np.float64).copy()
    dummy = np.zeros(1)
    rc = lib.dmrg_gemm_selftest(m, n, k, _dp(dummy if ident_a else A), int(trans_a) | (2 if pad_a else 0),
                                int(ident_a), _dp(dummy if ident_b else B), int(trans_b) | (2 if pad_b else 0),
                                int(ident_b), alpha, beta, _dp(C), prec)
    if rc != 0:
        raise DMRGError(rc, lib.dmrg_last_error().decode())
    return C


def load_checkpoint(path):
    """Contents of a save_checkpoint file as a dict (plain arrays; nothing
    in the file is executed)."""
    with np.load(path, allow_pickle=False) as z:
        out = {key: z[key] for key in z.files}
    for key in ("k", "n_orb", "n_elec", "two_s"):
        out[key] = int(out[key])
    return out


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


class DMRG:
    """One context: integrals, an MPS around a two-site block, and its H*psi."""

    def __init__(self, h, g, n_elec, two_s, e_core=0.0, davidson_tol=1e-7, davidson_max_iter=60,
                 davidson_max_subspace=24, hpsi_prec=FP64, work_budget_elems=0, keep_blocks=False,
                 davidson_refine_iter=0, davidson_jd_inner=0, davidson_lowprec_iter=-1, hpsi_graph=False,
                 next_guess=False, hbm_budget_bytes=0, davidson_mid_fp32=False, davidson_graph=False, lib=None):
        self.lib = load(lib)
        h = np.ascontiguousarray(h, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        n = h.shape[0]
        self.opts = Opts(n, n_elec, two_s, e_core, davidson_tol, davidson_max_iter, davidson_max_subspace,
                         hpsi_prec, work_budget_elems, int(keep_blocks), davidson_refine_iter,
                         davidson_jd_inner, davidson_lowprec_iter, int(hpsi_graph), int(next_guess),
                         int(hbm_budget_bytes), int(davidson_mid_fp32), int(davidson_graph))
        self._h = ct.c_void_p()
        self._batches = weakref.WeakSet()
        self._check(self.lib.dmrg_create(ct.byref(self._h), ct.byref(self.opts), _dp(h), _dp(g)))
        self.k = None

    def _check(self, rc):
        if rc != 0:
            raise DMRGError(rc, self.lib.dmrg_last_error().decode())
        return rc

    def tuner_report(self):
        """The tile autotuner's choices so far (dmrg_tuner_report), as a dict."""
        import json
        buf = ct.create_string_buffer(4096)
        self._check(self.lib.dmrg_tuner_report(self._h, buf, 4096))
        return json.loads(buf.value.decode()) if buf.value else {}

    def update_opts(self, **kw):
        """Change Davidson / precision / graph / next-guess options in place
        (dmrg_update_opts); keyword names are the dmrg_opts fields."""
        o = Opts()
        ct.pointer(o)[0] = self.opts
        for key, val in kw.items():
            if key not in dict(Opts._fields_):
                raise TypeError(f"unknown option {key}")
            setattr(o, key, int(val) if isinstance(val, bool) else val)
        self._check(self.lib.dmrg_update_opts(self._h, ct.byref(o)))
        self.opts = o

    def close(self):
        for b in list(getattr(self, "_batches", ())):
            b.close()
        if self._h:
            self.lib.dmrg_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mps(self, k, bond_sectors, sectors_per_bond, blocks):
        bs = np.ascontiguousarray(bond_sectors, dtype=np.int32).reshape(-1)
        cnt = np.ascontiguousarray(sectors_per_bond, dtype=np.int32)
        blk = np.ascontiguousarray(blocks, dtype=np.float64)
        self._check(self.lib.dmrg_set_mps(self._h, k, bs.ctypes.data_as(ct.POINTER(ct.c_int)),
                                          cnt.ctypes.data_as(ct.POINTER(ct.c_int)), _dp(blk), blk.size))
        self.k = k

    def psi_layout(self):
        nsb, nel = ct.c_longlong(), ct.c_longlong()
        self._check(self.lib.dmrg_psi_layout(self._h, self.k, ct.byref(nsb), None, ct.byref(nel)))
        desc = np.zeros(7 * nsb.value, dtype=np.int64)
        self._check(self.lib.dmrg_psi_layout(self._h, self.k, ct.byref(nsb),
                                             desc.ctypes.data_as(ct.POINTER(ct.c_longlong)), ct.byref(nel)))
        return desc.reshape(-1, 7), nel.value

    def hpsi(self, psi, prec=FP64):
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        out = np.empty_like(psi)
        fl = ct.c_double()
        self._check(self.lib.dmrg_hpsi(self._h, self.k, _dp(psi), _dp(out), prec, ct.byref(fl)))
        return out, fl.value

    def hpsi_dev(self, d_in, d_out, prec=FP64, stream=None):
        """d_out = H d_in on device FP64 buffers.  stream: a HIP stream handle
        (e.g. torch.cuda.current_stream().cuda_stream) to order the product
        with; without it the caller synchronises the device itself."""
        if stream is None:
            self._check(self.lib.dmrg_hpsi_dev(self._h, self.k, ct.c_void_p(d_in), ct.c_void_p(d_out), prec))
        else:
            self._check(self.lib.dmrg_hpsi_dev_stream(self._h, self.k, ct.c_void_p(d_in), ct.c_void_p(d_out), prec,
                                                      ct.c_void_p(stream)))

    def hpsi_dev_noalloc(self, d_in, d_out, prec=FP64):
        """d_out = H d_in on device FP64 buffers through the allocation-free
        entry point (intermediates in the library's fixed device array)."""
        self._check(self.lib.dmrg_hpsi_dev_noalloc(self._h, self.k, ct.c_void_p(d_in), ct.c_void_p(d_out), prec))

    def heff_diag(self, size):
        out = np.empty(size)
        self._check(self.lib.dmrg_heff_diag(self._h, self.k, _dp(out)))
        return out

    def davidson(self, psi0):
        psi = np.ascontiguousarray(psi0, dtype=np.float64).copy()
        e, r = ct.c_double(), ct.c_double()
        nlo, nhi = ct.c_int(), ct.c_int()
        rc = self.lib.dmrg_davidson_step(self._h, self.k, _dp(psi), ct.byref(e), ct.byref(r), ct.byref(nlo),
                                         ct.byref(nhi))
        if rc not in (0, -6):
            self._check(rc)
        return dict(psi=psi, energy=e.value, resid=r.value, n_lo=nlo.value, n_fp64=nhi.value, converged=rc == 0)

    def truncate(self, psi, d_max, eps_tr=0.0, direction=1, d_min=0):
        """Truncate to d_max multiplets, or with eps_tr > 0 to the fewest whose
        discarded weight is <= eps_tr (dynamic block state selection), kept
        within [d_min, d_max]."""
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        err, kept = ct.c_double(), ct.c_int()
        self._check(self.lib.dmrg_truncate_dbss(self._h, self.k, _dp(psi), direction, d_min, d_max, eps_tr,
                                                ct.byref(err), ct.byref(kept)))
        kk = ct.c_int()
        self._check(self.lib.dmrg_current_block(self._h, ct.byref(kk)))
        self.k = kk.value
        return err.value, kept.value

    def next_guess(self):
        """Start vector carried to the current block by the last right-moving
        truncation (opts next_guess)."""
        _, nel = self.psi_layout()
        out = np.zeros(nel)
        self._check(self.lib.dmrg_next_guess(self._h, self.k, _dp(out), nel))
        return out

    def get_bond(self, b):
        n = ct.c_int()
        self._check(self.lib.dmrg_get_bond(self._h, b, None, ct.byref(n)))
        out = np.zeros(3 * max(n.value, 1), dtype=np.int32)
        self._check(self.lib.dmrg_get_bond(self._h, b, out.ctypes.data_as(ct.POINTER(ct.c_int)), ct.byref(n)))
        return [tuple(int(x) for x in out[3 * i:3 * i + 3]) for i in range(n.value)]

    def get_site(self, j):
        n = ct.c_longlong()
        self._check(self.lib.dmrg_get_site(self._h, j, None, ct.byref(n)))
        out = np.zeros(max(n.value, 1))
        self._check(self.lib.dmrg_get_site(self._h, j, _dp(out), ct.byref(n)))
        return out[:n.value]

    def save_checkpoint(self, path, psi):
        """Write the MPS around the current two-site block (k, k+1) to one
        .npz file: the sectors of bonds 0..n (bond k+1, inside the block,
        empty), the site tensors outside the block (dmrg_get_site, in the
        order dmrg_set_mps reads them), the two-site psi and the system's
        orbital / electron / spin numbers.  resume() reloads it."""
        n, k = self.opts.n_orb, self.k
        rows, counts = [], []
        for b in range(n + 1):
            secs = [] if b == k + 1 else self.get_bond(b)
            counts.append(len(secs))
            rows.extend(secs)
        sites = [self.get_site(j) for j in range(n) if j not in (k, k + 1)]
        np.savez(path, k=np.int64(k), n_orb=np.int64(n), n_elec=np.int64(self.opts.n_elec),
                 two_s=np.int64(self.opts.two_s), bond_sectors=np.asarray(rows, dtype=np.int32).reshape(-1, 3),
                 counts=np.asarray(counts, dtype=np.int32),
                 sites=np.concatenate(sites) if sites else np.zeros(0),
                 psi=np.ascontiguousarray(psi, dtype=np.float64))

    def resume(self, path):
        """Load a checkpoint written by save_checkpoint into this context
        (same orbitals, electrons and spin; its integrals are this
        context's): builds the operator blocks around the saved block and
        returns the saved psi."""
        ck = load_checkpoint(path)
        if (ck["n_orb"], ck["n_elec"], ck["two_s"]) != (self.opts.n_orb, self.opts.n_elec, self.opts.two_s):
            raise ValueError("checkpoint is for a different system (orbitals, electrons or spin)")
        self.set_mps(ck["k"], ck["bond_sectors"], ck["counts"], ck["sites"])
        return ck["psi"]

    def cut_spectrum(self, capacity=1 << 20):
        vals = np.zeros(capacity)
        spins = np.zeros(capacity, dtype=np.int32)
        n = ct.c_int()
        self._check(self.lib.dmrg_cut_spectrum(self._h, _dp(vals), spins.ctypes.data_as(ct.POINTER(ct.c_int)),
                                               ct.byref(n), capacity))
        return vals[:n.value].copy(), spins[:n.value].copy()

    def kernel_timing(self, mode):
        ms, n = ct.c_double(), ct.c_longlong()
        self._check(self.lib.dmrg_kernel_timing(self._h, mode, ct.byref(ms), ct.byref(n)))
        return ms.value, n.value

    def stats(self):
        out = np.zeros(7)
        self._check(self.lib.dmrg_stats(self._h, _dp(out), 7))
        return dict(hpsi_flops=out[0], op_bytes=out[1], peak_bytes=out[2], n_terms=int(out[3]),
                    n_tasks=int(out[4]), hpsi_flops_executed=out[5], hpsi_flops_dense_regions=out[6])


class HpsiBatch:
    """H*psi of several contexts in one grouped launch per stage (dmrg_batch_*).

    The batch keeps its contexts alive; closing any of them closes the batch
    first."""

    def __init__(self, contexts, prec=FP64):
        self.contexts = list(contexts)
        if not self.contexts:
            raise ValueError("HpsiBatch needs at least one context")
        self.lib = self.contexts[0].lib
        self.prec = prec
        arr = (ct.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        self._h = ct.c_void_p()
        rc = self.lib.dmrg_batch_create(arr, len(self.contexts), prec, ct.byref(self._h))
        if rc != 0:
            raise DMRGError(rc, self.lib.dmrg_last_error().decode())
        for c in self.contexts:
            c._batches.add(self)

    def run(self, d_in, d_out):
        """d_in[i], d_out[i]: device addresses of FP64 vectors of context i's length."""
        n = len(self.contexts)
        if len(d_in) != n or len(d_out) != n:
            raise ValueError("one input and one output per context")
        if not self._h:
            raise DMRGError(-1, "batch is closed")
        a = (ct.c_void_p * n)(*[int(p) for p in d_in])
        b = (ct.c_void_p * n)(*[int(p) for p in d_out])
        rc = self.lib.dmrg_batch_hpsi(self._h, a, b)
        if rc != 0:
            raise DMRGError(rc, self.lib.dmrg_last_error().decode())

    def davidson(self, psis):
        """dmrg_davidson_step on every context at once, matvecs batched.
        psis: host start vectors (zero: random start).  Returns one dict per
        context, like DMRG.davidson, plus its status code."""
        n = len(self.contexts)
        if len(psis) != n:
            raise ValueError("one start vector per context")
        if not self._h:
            raise DMRGError(-1, "batch is closed")
        vecs = [np.ascontiguousarray(p, dtype=np.float64).copy() for p in psis]
        arr = (ct.POINTER(ct.c_double) * n)(*[_dp(v) for v in vecs])
        e, r = np.zeros(n), np.zeros(n)
        nlo, nhi, st = (np.zeros(n, dtype=np.int32) for _ in range(3))
        ip_ = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_int))
        rc = self.lib.dmrg_batch_davidson(self._h, arr, _dp(e), _dp(r), ip_(nlo), ip_(nhi), ip_(st))
        if rc not in (0, -6):
            raise DMRGError(rc, self.lib.dmrg_last_error().decode())
        return [dict(psi=v, energy=float(e[i]), resid=float(r[i]), n_lo=int(nlo[i]), n_fp64=int(nhi[i]),
                     converged=int(st[i]) == 0, status=int(st[i])) for i, v in enumerate(vecs)]

    def close(self):
        if self._h:
            self.lib.dmrg_batch_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
