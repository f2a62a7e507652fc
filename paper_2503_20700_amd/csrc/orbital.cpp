// CAS-SCF orbital step: the energy at fixed reduced density matrices as a
// function of an orbital rotation, E(kappa), and its gradient dE/dkappa, on
// the GPU (Sec. "Complete active space SCF": the orbital optimisation at
// fixed RDMs between DMRG solves, with h(kappa) and (pq|rs)(kappa) from the
// rotated orbitals).
//
// Reading (the paper gives no formulas for this step):
//   U = exp(-K), K_pq = kappa_pq (p > q), K_qp = -kappa_pq;
//   h(kappa) = U^T h U,  B^L(kappa) = U^T B^L U  ((pq|rs) = sum_L B^L_pq B^L_rs);
//   E = 2 sum_i h_ii + sum_ij [2(ii|jj) - (ij|ji)] + sum_tu F^c_tu gam_tu
//       + 1/2 sum_tuvw (tu|vw) Gam_tvwu,  F^c_pq = h_pq + sum_i [2(pq|ii) - (pi|iq)]
// over core (i, j) and active (t, u, v, w) orbitals, in that order.
//
// Forward: U by a scaled Taylor series with repeated squaring; the batched
// congruence transforms; per auxiliary index the scalars J = tr B_cc,
// t = <gam, B_aa>, q = |B_cc|^2, r = <gam B_ac, B_ac> and the active block
// b_L, so that E = <G_h, h'> + sum_L [2J^2 - q + 2Jt - r + 1/2 b_L.D b_L] with
// D_(tu),(vw) = Gam_tvwu and G_h = 2 (core identity) + gam.
// Backward (by hand, in reverse order): G_L = dE/dB'_L per auxiliary index,
// dE/dU = sum_L B_L U (G_L + G_L^T) + h U (G_h + G_h^T), and through the
// exponential with the adjoint of its Frechet derivative,
//   dE/dA = [exp([[A^T, dE/dU], [0, A^T]])]_12,  A = -K,
// then dE/dkappa_pq = (dE/dK)_pq - (dE/dK)_qp.  All arithmetic is FP64 (the
// central finite differences the gradient is checked against, step 1e-4, need
// the energy to about 1e-12 relative).
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dmrg.h"
#include "exec.hpp"
#include "session.hpp"

using namespace dmrg;

namespace {

struct DBuf {
  Executor* ex = nullptr;
  double* p = nullptr;
  DBuf(Executor* e, size_t n) : ex(e) {
    p = (double*)ex->alloc(std::max<size_t>(n, 1) * 8);
    ex->zero(p, std::max<size_t>(n, 1) * 8);
  }
  ~DBuf() {
    if (p) ex->release(p);
  }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
};

// One grouped launch of FP64 products on the library's GEMM kernels.
struct Gemm {
  std::vector<RawJob> jobs;
  std::vector<RawTerm> terms;
  void job(double* C, int m, int n, int64_t ldc, bool acc) {
    RawJob j{};
    j.C = C;
    j.m = m;
    j.n = n;
    j.ldc = ldc;
    j.accumulate = acc ? 1 : 0;
    j.tbeg = j.tend = (int64_t)terms.size();
    jobs.push_back(j);
  }
  // op(A) (m x k) @ op(B) (k x n) added to the last job; A or B null: identity
  void prod(const double* A, int64_t lda, bool ta, const double* B, int64_t ldb, bool tb, int k, double alpha) {
    RawTerm t{};
    t.A = A;
    t.B = B;
    t.lda = lda;
    t.ldb = ldb;
    t.k = k;
    t.flags = (ta ? TF_TRANS_A : 0) | (tb ? TF_TRANS_B : 0) | (A ? 0 : TF_IDENT_A) | (B ? 0 : TF_IDENT_B);
    t.alpha = alpha;
    terms.push_back(t);
    jobs.back().tend = (int64_t)terms.size();
  }
  void run(Executor* ex) {
    if (jobs.empty()) return;
    void* h = ex->prepare(jobs, terms, DT_F64, DT_F64, DT_F64);
    ex->run(h);
    ex->drop(h);
    jobs.clear();
    terms.clear();
  }
};

// out = exp(A) for an m x m device matrix A with ||A||_1 <= norm1: Taylor
// polynomial of degree 18 in A / 2^s with ||A / 2^s||_1 <= 1/2 (truncation
// below 1e-22 relative), evaluated by Horner's rule, then squared s times.
void expm_device(Executor* ex, const double* A, double* out, int m, double norm1) {
  int s = 0;
  while (norm1 / std::ldexp(1.0, s) > 0.5 && s < 60) ++s;
  const double scale = std::ldexp(1.0, -s);
  DBuf t(ex, (size_t)m * m), eye(ex, (size_t)m * m);
  {
    std::vector<double> I((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
    ex->upload(eye.p, I.data(), I.size() * 8);
    ex->upload(out, I.data(), I.size() * 8);  // P = I
  }
  Gemm g;
  double* P = out;
  double* Q = t.p;
  for (int j = 18; j >= 1; --j) {  // P <- I + (A / 2^s / j) P
    g.job(Q, m, m, m, false);
    g.prod(A, m, false, P, m, false, m, scale / j);
    g.prod(eye.p, m, false, nullptr, 0, false, m, 1.0);
    g.run(ex);
    std::swap(P, Q);
  }
  for (int i = 0; i < s; ++i) {
    g.job(Q, m, m, m, false);
    g.prod(P, m, false, P, m, false, m, 1.0);
    g.run(ex);
    std::swap(P, Q);
  }
  if (P != out) ex->copy_d2d(out, P, (size_t)m * m * 8);
  ex->sync();
}

double norm1(const std::vector<double>& a, int m) {
  double best = 0.0;
  for (int j = 0; j < m; ++j) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += std::fabs(a[(size_t)i * m + j]);
    best = std::max(best, s);
  }
  return best;
}

bool finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

extern "C" int orb_grad(int n_core, int n_act, int n_virt, const double* h_full, const double* B, int naux,
                        const double* kappa, const double* gamma, const double* Gamma, double* energy,
                        double* grad) {
  if (!h_full || !B || !kappa || !energy || !grad || (n_act > 0 && (!gamma || !Gamma)))
    return dmrg_fail(DMRG_ERR_ARG, "orb_grad: null argument");
  if (n_core < 0 || n_act < 0 || n_virt < 0 || naux < 1 || n_core + n_act + n_virt < 1 ||
      n_core + n_act + n_virt > 4096)
    return dmrg_fail(DMRG_ERR_SHAPE, "orb_grad: bad orbital or auxiliary counts");
  const int n = n_core + n_act + n_virt, na = n_act, nc = n_core;
  const size_t nn = (size_t)n * n, na2 = (size_t)na * na;
  if (!finite(h_full, nn) || !finite(B, nn * naux) || !finite(kappa, nn) || (na && !finite(gamma, na2)) ||
      (na && !finite(Gamma, na2 * na2)))
    return dmrg_fail(DMRG_ERR_NONFINITE, "orb_grad: non-finite input");
  {
    double hm = 0.0, bm = 0.0;
    for (size_t i = 0; i < nn; ++i) hm = std::max(hm, std::fabs(h_full[i]));
    for (size_t i = 0; i < nn * naux; ++i) bm = std::max(bm, std::fabs(B[i]));
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < p; ++q) {
        if (std::fabs(h_full[(size_t)p * n + q] - h_full[(size_t)q * n + p]) > 1e-12 * std::max(hm, 1e-300))
          return dmrg_fail(DMRG_ERR_ARG, "orb_grad: h is not symmetric");
        for (int L = 0; L < naux; ++L)
          if (std::fabs(B[L * nn + (size_t)p * n + q] - B[L * nn + (size_t)q * n + p]) > 1e-12 * std::max(bm, 1e-300))
            return dmrg_fail(DMRG_ERR_ARG, "orb_grad: a density-fitting matrix B^L is not symmetric");
      }
  }
  try {
    std::unique_ptr<Executor> exo(make_hip_executor());
    Executor* ex = exo.get();
    // ---- inputs on the device
    std::vector<double> K(nn, 0.0);
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < p; ++q) {
        K[(size_t)p * n + q] = kappa[(size_t)p * n + q];
        K[(size_t)q * n + p] = -kappa[(size_t)p * n + q];
      }
    std::vector<double> mK(nn), Gh(nn, 0.0), Dm(na2 * na2);
    for (size_t i = 0; i < nn; ++i) mK[i] = -K[i];
    for (int i = 0; i < nc; ++i) Gh[(size_t)i * n + i] = 2.0;
    for (int t = 0; t < na; ++t)
      for (int u = 0; u < na; ++u) Gh[(size_t)(nc + t) * n + nc + u] = gamma[(size_t)t * na + u];
    // D_(tu),(vw) = Gam_tvwu
    for (int t = 0; t < na; ++t)
      for (int u = 0; u < na; ++u)
        for (int v = 0; v < na; ++v)
          for (int w = 0; w < na; ++w)
            Dm[((size_t)t * na + u) * na2 + (size_t)v * na + w] = Gamma[(((size_t)t * na + v) * na + w) * na + u];
    DBuf dh(ex, nn), dB(ex, nn * naux), dmK(ex, nn), dGh(ex, nn), dgam(ex, std::max<size_t>(na2, 1)),
        dD(ex, std::max<size_t>(na2 * na2, 1));
    ex->upload(dh.p, h_full, nn * 8);
    ex->upload(dB.p, B, nn * naux * 8);
    ex->upload(dmK.p, mK.data(), nn * 8);
    ex->upload(dGh.p, Gh.data(), nn * 8);
    if (na) {
      ex->upload(dgam.p, gamma, na2 * 8);
      ex->upload(dD.p, Dm.data(), na2 * na2 * 8);
    }
    // ---- forward: U, h', B'
    DBuf dU(ex, nn), dT(ex, nn * naux), dBp(ex, nn * naux), dhp(ex, nn), dth(ex, nn);
    expm_device(ex, dmK.p, dU.p, n, norm1(mK, n));
    Gemm g;
    for (int L = 0; L < naux; ++L) {
      g.job(dT.p + L * nn, n, n, n, false);
      g.prod(dB.p + L * nn, n, false, dU.p, n, false, n, 1.0);
    }
    g.job(dth.p, n, n, n, false);
    g.prod(dh.p, n, false, dU.p, n, false, n, 1.0);
    g.run(ex);
    for (int L = 0; L < naux; ++L) {
      g.job(dBp.p + L * nn, n, n, n, false);
      g.prod(dU.p, n, true, dT.p + L * nn, n, false, n, 1.0);
    }
    g.job(dhp.p, n, n, n, false);
    g.prod(dU.p, n, true, dth.p, n, false, n, 1.0);
    g.run(ex);
    // ---- energy terms and dE/dB'
    DBuf dbact(ex, std::max<size_t>(na2 * naux, 1)), dscal(ex, 4 * (size_t)naux), dY(ex, std::max<size_t>(na2 * naux, 1)),
        dZ(ex, std::max<size_t>(na2 * naux, 1)), dG(ex, nn * naux), de2(ex, naux);
    ex->orb_scalars(dBp.p, naux, n, nc, na, dgam.p, dbact.p, dscal.p);
    if (na) {
      g.job(dY.p, naux, (int)na2, (int64_t)na2, false);  // Y_L = D b_L
      g.prod(dbact.p, (int64_t)na2, false, dD.p, (int64_t)na2, true, (int)na2, 1.0);
      g.job(dZ.p, naux, (int)na2, (int64_t)na2, false);  // Z_L = D^T b_L
      g.prod(dbact.p, (int64_t)na2, false, dD.p, (int64_t)na2, false, (int)na2, 1.0);
      g.run(ex);
    }
    ex->orb_assemble(dBp.p, naux, n, nc, na, dgam.p, dscal.p, dbact.p, dY.p, dZ.p, dG.p, de2.p);
    double e1 = 0.0;
    ex->multidot(dGh.p, (int64_t)nn, 1, dhp.p, (int64_t)nn, &e1);
    std::vector<double> scal(4 * (size_t)naux), e2(naux);
    ex->download(scal.data(), dscal.p, scal.size() * 8);
    ex->download(e2.data(), de2.p, e2.size() * 8);
    double e = e1;
    for (int L = 0; L < naux; ++L) {
      const double J = scal[4 * L], t = scal[4 * L + 1], q = scal[4 * L + 2], r = scal[4 * L + 3];
      e += 2.0 * J * J - q + 2.0 * J * t - r + e2[L];
    }
    // ---- backward: dE/dU = sum_L B_L U (G_L + G_L^T) + h U (G_h + G_h^T)
    DBuf dS(ex, nn * naux), dSh(ex, nn), dW(ex, nn);
    for (int L = 0; L < naux; ++L) {
      g.job(dS.p + L * nn, n, n, n, false);
      g.prod(dU.p, n, false, dG.p + L * nn, n, false, n, 1.0);
      g.prod(dU.p, n, false, dG.p + L * nn, n, true, n, 1.0);
    }
    g.job(dSh.p, n, n, n, false);
    g.prod(dU.p, n, false, dGh.p, n, false, n, 2.0);  // G_h is symmetric
    g.run(ex);
    g.job(dW.p, n, n, n, false);
    for (int L = 0; L < naux; ++L) g.prod(dB.p + L * nn, n, false, dS.p + L * nn, n, false, n, 1.0);
    g.prod(dh.p, n, false, dSh.p, n, false, n, 1.0);
    g.run(ex);
    // ---- through U = exp(A), A = -K: dE/dA = [exp([[A^T, W], [0, A^T]])]_12, A^T = K
    const int m2 = 2 * n;
    std::vector<double> W(nn), M((size_t)m2 * m2, 0.0);
    ex->download(W.data(), dW.p, nn * 8);
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        M[(size_t)p * m2 + q] = K[(size_t)p * n + q];
        M[(size_t)(n + p) * m2 + n + q] = K[(size_t)p * n + q];
        M[(size_t)p * m2 + n + q] = W[(size_t)p * n + q];
      }
    DBuf dM(ex, (size_t)m2 * m2), dE(ex, (size_t)m2 * m2);
    ex->upload(dM.p, M.data(), M.size() * 8);
    expm_device(ex, dM.p, dE.p, m2, norm1(M, m2));
    std::vector<double> X((size_t)m2 * m2);
    ex->download(X.data(), dE.p, X.size() * 8);
    // dE/dK = -dE/dA ; dE/dkappa_pq = (dE/dK)_pq - (dE/dK)_qp
    for (int p = 0; p < n; ++p) {
      grad[(size_t)p * n + p] = 0.0;
      for (int q = 0; q < p; ++q) {
        const double dApq = X[(size_t)p * m2 + n + q], dAqp = X[(size_t)q * m2 + n + p];
        const double v = -(dApq - dAqp);
        grad[(size_t)p * n + q] = v;
        grad[(size_t)q * n + p] = -v;
      }
    }
    *energy = e;
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return dmrg_fail(DMRG_ERR_BUDGET, std::string("orb_grad: ") + e.what());
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("orb_grad: ") + e.what());
  }
}
