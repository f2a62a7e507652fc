"""The CAS-SCF orbital step on the GPU (orb_grad and its torch.autograd.Function)
against the oracle (oracle/orbital.py): the energy after a rotation kappa and
dE/dkappa, at small sizes with CAS-CI density matrices, and at the full
orbital-gradient workload shape (120 orbitals: 48 core, 24 active, 48
virtual, 360 density-fitting vectors, kappa ~ N(0, 1e-3)) against central
finite differences with step 1e-4."""
import numpy as np
import pytest

from casci import cas_ci_rdms

pytestmark = pytest.mark.gpu


def _sym_rdms(na, rng):
    """Random tensors with the permutation symmetries of spin-summed RDMs
    (gamma symmetric; Gamma~_tuvw = Gamma~_utwv = Gamma~_wvut).  E(kappa) and
    its gradient are defined for any such tensors."""
    gam = rng.normal(size=(na, na))
    gam = gam + gam.T
    G = rng.normal(size=(na,) * 4)
    G = G + G.transpose(1, 0, 3, 2)
    G = G + G.transpose(3, 2, 1, 0)
    return gam, G


@pytest.mark.parametrize("n,nc,na,nel,kscale", [(5, 1, 3, 4, 0.0), (6, 2, 2, 2, 1e-2), (6, 1, 4, 4, 0.2)])
def test_orb_grad_matches_oracle_small(n, nc, na, nel, kscale):
    from oracle import orbital
    from paper_2503_20700_amd.binding import orb_grad
    from synth.integrals import small_cas
    print(f"[orbital] n={n} core={nc} active={na} kappa~{kscale}", flush=True)
    h, g, B = small_cas(n, 40 + n)
    gam, Gam, _ = cas_ci_rdms(h, g, n, nc, na, nel, 0)
    rng = np.random.default_rng(n)
    k = np.tril(rng.normal(scale=kscale, size=(n, n)), -1) if kscale else np.zeros((n, n))
    e, grad = orb_grad(nc, na, n - nc - na, h, B, k, gam, Gam)
    e_ref = orbital.energy(h, B, k, gam, Gam, nc, na)
    assert abs(e - e_ref) <= 1e-10 * max(1.0, abs(e_ref))
    fd = orbital.gradient_fd(h, B, k, gam, Gam, nc, na, step=1e-5)
    assert np.abs(grad - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())
    assert np.allclose(grad, -grad.T, atol=0.0)
    if kscale == 0.0:
        cf = orbital.generalized_fock_gradient(h, B, gam, Gam, nc, na)
        assert np.abs(grad - cf).max() <= 1e-10 * max(1.0, np.abs(cf).max())
    # core-core and virtual-virtual rotations are redundant at kappa = 0
    if kscale == 0.0:
        assert np.abs(grad[:nc, :nc]).max() < 1e-12
        assert np.abs(grad[nc + na:, nc + na:]).max() < 1e-12


def test_orb_grad_autograd_function():
    import torch

    from paper_2503_20700_amd.binding import orb_grad, orbital_energy_function
    from synth.integrals import small_cas
    print("[orbital] autograd", flush=True)
    n, nc, na = 7, 2, 3
    h, g, B = small_cas(n, 17)
    gam, Gam = _sym_rdms(na, np.random.default_rng(3))
    F = orbital_energy_function()
    k0 = np.tril(np.random.default_rng(4).normal(scale=1e-2, size=(n, n)), -1)
    kappa = torch.tensor(k0, dtype=torch.float64, device="cuda:0", requires_grad=True)
    e = F.apply(kappa, nc, na, n - nc - na, h, B, gam, Gam)
    (gk,) = torch.autograd.grad(3.0 * e, kappa)
    e_ref, grad = orb_grad(nc, na, n - nc - na, h, B, k0, gam, Gam)
    assert abs(e.item() - e_ref) < 1e-12 * abs(e_ref)
    assert np.allclose(gk.cpu().numpy(), 3.0 * np.tril(grad, -1), rtol=0, atol=1e-12)
    # a directional derivative by central differences through the Function itself
    d = np.tril(np.random.default_rng(5).normal(size=(n, n)), -1)
    s = 1e-5
    ep = F.apply(torch.tensor(k0 + s * d, device="cuda:0"), nc, na, n - nc - na, h, B, gam, Gam).item()
    em = F.apply(torch.tensor(k0 - s * d, device="cuda:0"), nc, na, n - nc - na, h, B, gam, Gam).item()
    assert abs((ep - em) / (2 * s) - float((gk.cpu().numpy() / 3.0 * d).sum())) < 1e-6


def test_orb_grad_full_workload_against_finite_differences():
    """120 orbitals (48 core, 24 active, 48 virtual), 360 density-fitting
    vectors, kappa ~ N(0, 1e-3): the gradient against central differences of
    the GPU energy (step 1e-4) on entries of every block and 16 random
    directions, against the oracle's energy and its finite differences on a
    sample of entries, and with zero core-core and virtual-virtual blocks at
    kappa = 0.  The density matrices are random tensors with RDM symmetries
    (the orbital step is defined for any)."""
    from oracle import orbital
    from paper_2503_20700_amd.binding import orb_grad
    from synth.integrals import embedded_cas
    print("[orbital] 120 orbitals, CAS(24,24) inside", flush=True)
    nc, na, nv = 48, 24, 48
    n = nc + na + nv
    h, B = embedded_cas(nc, na, nv, seed=3)
    rng = np.random.default_rng(3)
    gam, Gam = _sym_rdms(na, rng)
    gam *= 0.1
    Gam *= 0.01
    k = np.tril(rng.normal(scale=1e-3, size=(n, n)), -1)
    e, grad = orb_grad(nc, na, nv, h, B, k, gam, Gam)
    e_ref = orbital.energy(h, B, k, gam, Gam, nc, na)
    assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
    step = 1e-4
    blocks = [(5, 2), (60, 10), (60, 50), (100, 3), (100, 60), (110, 90), (70, 55)]
    for p, q in blocks:
        kp, km = k.copy(), k.copy()
        kp[p, q] += step
        km[p, q] -= step
        fd = (orb_grad(nc, na, nv, h, B, kp, gam, Gam)[0] - orb_grad(nc, na, nv, h, B, km, gam, Gam)[0]) / (2 * step)
        assert abs(fd - grad[p, q]) <= 1e-6 * max(1.0, abs(grad[p, q])), (p, q, fd, grad[p, q])
    for i in range(16):
        d = np.tril(rng.normal(size=(n, n)), -1)
        d /= np.linalg.norm(d)
        fd = (orb_grad(nc, na, nv, h, B, k + step * d, gam, Gam)[0] -
              orb_grad(nc, na, nv, h, B, k - step * d, gam, Gam)[0]) / (2 * step)
        assert abs(fd - (grad * d).sum()) <= 1e-6 * max(1.0, np.abs(grad).max())
    ofd = orbital.gradient_fd(h, B, k, gam, Gam, nc, na, step=step, pairs=[(60, 10), (100, 60)])
    assert abs(ofd[60, 10] - grad[60, 10]) <= 1e-6 * max(1.0, abs(grad[60, 10]))
    assert abs(ofd[100, 60] - grad[100, 60]) <= 1e-6 * max(1.0, abs(grad[100, 60]))
    _, g0 = orb_grad(nc, na, nv, h, B, np.zeros((n, n)), gam, Gam)
    assert np.abs(g0[:nc, :nc]).max() < 1e-10 * np.abs(g0).max()
    assert np.abs(g0[nc + na:, nc + na:]).max() < 1e-10 * np.abs(g0).max()
    assert np.abs(g0[nc:nc + na, :nc]).max() > 1e-6
