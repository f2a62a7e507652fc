// Davidson eigensolver at the two-site block (lowest state of H_eff).
//
// The residual criterion ||H x - theta x||_2 <= tol for ||x|| = 1 is the
// paper's (Sec. "Numerical procedure", residual 1e-7).  With a low-precision
// bulk matvec (FP32 or BF16 operands, FP32 accumulation) the iteration runs
// in two phases: (1) Davidson with low-precision matvecs until the residual
// reaches the precision's noise floor, (2) FP64 refinement: Davidson
// restarted from the phase-1 Ritz vector with FP64 matvecs until tol.  In
// the refinement the basis images, Ritz pairs and residuals are FP64, and
// each new basis vector is, with davidson_jd_inner = k > 0, the Jacobi-
// Davidson correction: k conjugate-gradient steps on
//     (I - x x^T)(H - theta)(I - x x^T) t = -r,   t orthogonal to x,
// whose matvecs use the low precision.  The FP64 matvecs then only measure
// the residual of each refined vector, and their count drops to a few
// (iterative refinement of the eigenpair).  All vectors, projections (dot
// products), orthogonalisation and residuals are FP64 on the GPU; only the
// small projected matrix (<= 48 x 48) is diagonalised on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <random>
#include <tuple>
#include <string>
#include <vector>

#include "su2.hpp"

#include "../../include/dmrg.h"
#include "session.hpp"

using namespace dmrg;

namespace {


// Cyclic Jacobi for a small symmetric matrix (row-major m x m); returns
// eigenvalues ascending and eigenvectors as columns of V.
void jacobi_eig(int m, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
    if (off < 1e-30) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < m; ++k) {
          const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = c * akp - s * akq;
          A[(size_t)k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = c * apk - s * aqk;
          A[(size_t)q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
          V[(size_t)k * m + p] = c * vkp - s * vkq;
          V[(size_t)k * m + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return A[(size_t)a * m + a] < A[(size_t)b * m + b]; });
  w.resize(m);
  std::vector<double> Vs((size_t)m * m);
  for (int j = 0; j < m; ++j) {
    w[j] = A[(size_t)order[j] * m + order[j]];
    for (int i = 0; i < m; ++i) Vs[(size_t)i * m + j] = V[(size_t)i * m + order[j]];
  }
  V.swap(Vs);
}

struct Workspace {
  int bV = -1, bW = -1, bx = -1, bhx = -1, br = -1, bt = -1, bp = -1, bq = -1, bs = -1;
  int bc = -1;  // scalars of the recorded iterations (layout: enum Cf)
  int64_t n = 0;
  int mmax = 0;
};

constexpr int kKeep = 4;  // Ritz vectors kept at a restart

constexpr int kStall = 6;  // low-precision phase: iterations over which the residual must fall

double* P(dmrg_ctx* c, int b) { return (double*)c->C->ptr(b); }

// Device scalars of a recorded Davidson iteration (offsets into ws.bc):
// Ritz coefficients y, theta, <r,r>, <t,t>, 1/||t||, the orthogonalisation
// coefficients, and the new row and column of the projected matrix.
enum Cf : int { CF_Y = 0, CF_THETA = 64, CF_RR = 65, CF_TT = 66, CF_INV = 67, CF_ORTH = 68, CF_ROW = 132,
                CF_COL = 196, CF_SIZE = 260 };

// Davidson iterations recorded as graphs (opts.davidson_graph): while the
// basis holds m < mmax vectors, an iteration is the host's Rayleigh-Ritz
// step and stop tests plus two recorded sequences, each replayed after the
// host has written the scalars it needs:
//   part 1: x = V y, Hx = W y, r = Hx - theta x, <r,r>, t = the
//           preconditioned residual orthogonalised against V twice, <t,t>;
//   part 2: V_m = t / ||t||, W_m = H V_m, <W_j, V_m> and <V_j, W_m>, j <= m.
// They issue the launches of the eager iteration with the same scalars, so
// the results are the same bit for bit.  Not used for Jacobi-Davidson
// corrections (their CG steps branch on the host), by the batched solve,
// or while kernel timing records.
bool dav_graph_on(dmrg_ctx* c, int jd_steps) {
  return c->opts.davidson_graph && jd_steps == 0 && !c->mv_hook && c->ex->graphs() && !c->ex->timing_on();
}

// The recorded sequence `part` for precision prec and basis size m: recorded
// from `body` on first use, and again after the executor's scratch moved.
void* dav_graph(dmrg_ctx* c, int prec, int m, int part, const std::function<void()>& body) {
  Executor* ex = c->ex.get();
  if (c->dav_gen != ex->scratch_generation()) {
    c->drop_dav_graphs();
    c->dav_gen = ex->scratch_generation();
  }
  const int key = (prec * 64 + m) * 2 + part;
  auto it = c->dav_graphs.find(key);
  if (it != c->dav_graphs.end()) return it->second;
  ex->capture_begin();
  try {
    body();
  } catch (...) {
    ex->capture_abort();
    throw;
  }
  void* g = ex->capture_end();
  c->dav_graphs[key] = g;
  return g;
}

// Ritz vectors carried from the low-precision phase into the FP64 phase
// (DMRG_REFINE_KEEP overrides; 1 carries only the Ritz vector).
int refine_keep(dmrg_ctx* c) {
  (void)c;
  if (const char* e = std::getenv("DMRG_REFINE_KEEP")) return std::max(1, std::min(kKeep, std::atoi(e)));
  return kKeep;
}

// Scale of the spectrum for the rounding-level stop of the low-precision
// phase: the largest |diagonal element| of H_eff (host copy of the diagonal).
double diag_scale(dmrg_ctx* c, int64_t n) {
  std::vector<double> d((size_t)n);
  c->ex->download(d.data(), c->C->ptr(c->b_diag), (size_t)n * 8);
  double m = 0.0;
  for (double v : d) m = std::max(m, std::fabs(v));
  return m;
}

// y = H x for device FP64 vectors via the plan buffers.
void matvec(dmrg_ctx* c, const double* x, double* y, int prec, int64_t n) {
  if (c->mv_hook) {
    c->mv_hook(x, y, prec);
    return;
  }
  c->ex->copy_d2d(c->C->ptr(c->b_in), x, (size_t)n * 8);
  c->hpsi_device(prec);
  c->ex->copy_d2d(y, c->C->ptr(c->b_out), (size_t)n * 8);
}

struct PhaseResult {
  double theta = 0.0, resid = 0.0;
  int matvecs = 0;       // matvecs in the phase's own precision
  int inner_matvecs = 0;  // low-precision matvecs of the correction solves
  bool converged = false;
  bool stalled = false;   // stopped because the residual no longer fell
  int ritz_kept = 0;      // Ritz vectors left in the spare rows of V (lowest first)
};

double dot(Executor* ex, const double* a, const double* b, int64_t n) {
  double v = 0.0;
  ex->multidot(a, n, 1, b, n, &v);
  return v;
}

// Jacobi-Davidson correction: approximately solve
//   (I - x x^T)(H_lo - theta)(I - x x^T) t = -r,  t orthogonal to x,
// with at most `steps` conjugate-gradient iterations (H_lo: matvecs in
// precision lo_prec).  Returns the matvecs used; t = 0 if none succeeded.
int jd_correction(dmrg_ctx* c, const Workspace& ws, int lo_prec, double theta, int steps) {
  Executor* ex = c->ex.get();
  const int64_t n = ws.n;
  double* x = P(c, ws.bx);
  double* r = P(c, ws.br);
  double* t = P(c, ws.bt);
  double* p = P(c, ws.bp);
  double* q = P(c, ws.bq);
  double* res = P(c, ws.bs);
  auto project = [&](double* v) {  // v -= x (x.v)
    const double a = dot(ex, x, v, n);
    ex->axpby(v, 1.0, v, -a, x, n);
  };
  ex->axpby(t, 0.0, r, 0.0, r, n);   // t = 0
  ex->axpby(res, -1.0, r, 0.0, r, n);  // res = -r
  project(res);
  ex->copy_d2d(p, res, (size_t)n * 8);
  double rr = dot(ex, res, res, n);
  const double rr0 = rr;
  int used = 0;
  for (int j = 0; j < steps && rr > 1e-30 * std::max(rr0, 1e-300); ++j) {
    matvec(c, p, q, lo_prec, n);
    ++used;
    ex->axpby(q, 1.0, q, -theta, p, n);
    project(q);
    const double pq = dot(ex, p, q, n);
    if (!(pq > 0.0)) break;  // the projected operator is not positive on p
    const double a = rr / pq;
    ex->axpby(t, 1.0, t, a, p, n);
    ex->axpby(res, 1.0, res, -a, q, n);
    const double rr2 = dot(ex, res, res, n);
    ex->axpby(p, 1.0, res, rr2 / rr, p, n);
    rr = rr2;
  }
  return used;
}

// Davidson on the device basis V (rows), W = H V.  Starts from x (normalised),
// or with n_start > 1 from the orthonormal vectors in the spare rows
// mmax..mmax+n_start-1 of V (lowest Ritz vector first).  stall > 0: stop
// (stalled) when, over the last `stall` iterations, the residual has not
// fallen below 0.7 of its earlier value and the Ritz value has moved down by
// less than 1 % of the residual -- a low-precision operator stops improving
// the Ritz pair at its rounding level, while from a poor start the residual
// can stay flat as the Ritz value still falls.  keep_out > 0: on return the
// keep_out lowest Ritz vectors of the final basis are left in the spare rows
// of V.
PhaseResult davidson_phase(dmrg_ctx* c, Workspace& ws, int prec, double tol, int max_iter, int jd_steps = 0,
                           int jd_prec = DMRG_FP64, int n_start = 1, int stall = 0, int keep_out = 0) {
  Executor* ex = c->ex.get();
  const int64_t n = ws.n;
  const int mmax = ws.mmax;
  double* V = P(c, ws.bV);
  double* W = P(c, ws.bW);
  double* x = P(c, ws.bx);
  double* hx = P(c, ws.bhx);
  double* r = P(c, ws.br);
  double* t = P(c, ws.bt);
  const double* diag = (const double*)c->C->ptr(c->b_diag);
  PhaseResult res;
  std::vector<double> G((size_t)mmax * mmax, 0.0), tmp(mmax), w, Y, hist, thist;
  int m = 0;
  if (n_start > 1) {
    // V_0..V_{n_start-1} = the given vectors, W_i = H V_i in this phase's precision
    n_start = std::min(n_start, std::min(kKeep, mmax - 1));
    for (int q = 0; q < n_start; ++q) ex->copy_d2d(V + (int64_t)q * n, V + (int64_t)(mmax + q) * n, (size_t)n * 8);
    for (int q = 0; q < n_start; ++q) {
      matvec(c, V + (int64_t)q * n, W + (int64_t)q * n, prec, n);
      res.matvecs++;
    }
    m = n_start;
    for (int q = 0; q < m; ++q) {
      ex->multidot(W, n, m, V + (int64_t)q * n, n, tmp.data());  // <W_j, V_q>
      for (int j = 0; j < m; ++j) G[(size_t)q * mmax + j] = tmp[j];
    }
  } else {
    // V_0 = x, W_0 = H x
    ex->copy_d2d(V, x, (size_t)n * 8);
    matvec(c, V, W, prec, n);
    res.matvecs++;
    m = 1;
    ex->multidot(W, n, 1, V, n, tmp.data());
    G[0] = tmp[0];
  }
  auto save_ritz = [&](int mm) {
    const int kq = std::min(keep_out, mm);
    for (int q = 0; q < kq; ++q) {
      std::vector<double> yq(mm);
      for (int i = 0; i < mm; ++i) yq[i] = Y[(size_t)i * mm + q];
      ex->combine(V + (int64_t)(mmax + q) * n, V, n, mm, yq.data(), n, 0.0);
    }
    res.ritz_kept = kq;
  };
  const bool graph = dav_graph_on(c, jd_steps);
  double* cf = graph ? P(c, ws.bc) : nullptr;
  for (int it = 0; it < max_iter; ++it) {
    // Rayleigh-Ritz on span(V)
    std::vector<double> Gm((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Gm[(size_t)i * m + j] = 0.5 * (G[(size_t)i * mmax + j] + G[(size_t)j * mmax + i]);
    jacobi_eig(m, Gm, w, Y);
    const double theta = w[0];
    std::vector<double> y0(m);
    for (int i = 0; i < m; ++i) y0[i] = Y[(size_t)i * m + 0];
    double rr = 0.0, tt = 0.0;
    const bool rec = graph && m < mmax;  // this iteration runs the recorded parts
    if (rec) {
      const int mm = m;
      void* g1 = dav_graph(c, prec, mm, 0, [&] {
        ex->combine_dev(x, V, n, mm, cf + CF_Y, 1.0, n, 0.0);
        ex->combine_dev(hx, W, n, mm, cf + CF_Y, 1.0, n, 0.0);
        ex->axpby_dev(r, 1.0, nullptr, hx, -1.0, cf + CF_THETA, x, n);
        ex->multidot_dev(r, n, 1, r, n, cf + CF_RR);
        ex->precond_dev(t, r, diag, cf + CF_THETA, 1e-8, n);
        for (int pass = 0; pass < 2; ++pass) {
          ex->multidot_dev(V, n, mm, t, n, cf + CF_ORTH);
          ex->combine_dev(t, V, n, mm, cf + CF_ORTH, -1.0, n, 1.0);
        }
        ex->multidot_dev(t, n, 1, t, n, cf + CF_TT);
      });
      std::vector<double> up(CF_THETA + 1, 0.0);
      for (int i = 0; i < m; ++i) up[CF_Y + i] = y0[i];
      up[CF_THETA] = theta;
      ex->upload(cf, up.data(), up.size() * 8);
      ex->replay(g1);
      double st[2];
      ex->download(st, cf + CF_RR, sizeof st);
      rr = st[0];
      tt = st[1];
    } else {
      ex->combine(x, V, n, m, y0.data(), n, 0.0);
      ex->combine(hx, W, n, m, y0.data(), n, 0.0);
      ex->axpby(r, 1.0, hx, -theta, x, n);
      ex->multidot(r, n, 1, r, n, &rr);
    }
    res.theta = theta;
    res.resid = std::sqrt(std::max(rr, 0.0));
    if (std::getenv("DMRG_VERBOSE"))
      std::fprintf(stderr, "[davidson] prec %d it %d m %d theta %.12f resid %.3e\n", prec, it, m, theta, res.resid);
    hist.push_back(res.resid);
    thist.push_back(theta);
    if (res.resid <= tol) {
      res.converged = true;
      save_ritz(m);
      break;
    }
    if (stall > 0 && it >= stall && res.resid > 0.7 * hist[(size_t)(it - stall)] &&
        thist[(size_t)(it - stall)] - theta < 1e-2 * res.resid) {
      res.stalled = true;
      save_ritz(m);
      break;
    }
    if (it == max_iter - 1) {
      save_ritz(m);
      break;
    }
    // thick restart: rotate the basis onto the `keep` lowest Ritz vectors,
    // built in the spare rows mmax..mmax+keep-1 and then moved to the front.
    if (m == mmax) {
      const int keep = kKeep;
      for (int q = 0; q < keep; ++q) {
        std::vector<double> yq(m);
        for (int i = 0; i < m; ++i) yq[i] = Y[(size_t)i * m + q];
        ex->combine(V + (int64_t)(mmax + q) * n, V, n, m, yq.data(), n, 0.0);
        ex->combine(W + (int64_t)(mmax + q) * n, W, n, m, yq.data(), n, 0.0);
      }
      for (int q = 0; q < keep; ++q) {
        ex->copy_d2d(V + (int64_t)q * n, V + (int64_t)(mmax + q) * n, (size_t)n * 8);
        ex->copy_d2d(W + (int64_t)q * n, W + (int64_t)(mmax + q) * n, (size_t)n * 8);
      }
      std::fill(G.begin(), G.end(), 0.0);
      for (int q = 0; q < keep; ++q) G[(size_t)q * mmax + q] = w[q];
      m = keep;
      ex->axpby(r, 1.0, hx, -theta, x, n);
    }
    // new direction: Jacobi-Davidson correction (low-precision inner solve)
    // or the diagonally preconditioned residual t = (theta - D)^-1 r;
    // orthogonalised against V twice (done by the recorded part 1 already)
    if (!rec) {
      bool have_t = false;
      if (jd_steps > 0) {
        res.inner_matvecs += jd_correction(c, ws, jd_prec, theta, jd_steps);
        have_t = dot(ex, t, t, n) > 0.0;
      }
      if (!have_t) ex->precond(t, r, diag, theta, 1e-8, n);
      for (int pass = 0; pass < 2; ++pass) {
        ex->multidot(V, n, m, t, n, tmp.data());
        for (int i = 0; i < m; ++i) tmp[i] = -tmp[i];
        ex->combine(t, V, n, m, tmp.data(), n, 1.0);
      }
      ex->multidot(t, n, 1, t, n, &tt);
    }
    bool fell_back = false;
    if (!(tt > 1e-28)) {
      fell_back = true;
      // preconditioned residual lies in the basis: fall back to the residual
      ex->copy_d2d(t, r, (size_t)n * 8);
      for (int pass = 0; pass < 2; ++pass) {
        ex->multidot(V, n, m, t, n, tmp.data());
        for (int i = 0; i < m; ++i) tmp[i] = -tmp[i];
        ex->combine(t, V, n, m, tmp.data(), n, 1.0);
      }
      ex->multidot(t, n, 1, t, n, &tt);
      if (!(tt > 1e-28)) break;
    }
    const double inv = 1.0 / std::sqrt(tt);
    if (rec && !fell_back) {
      const int mm = m;
      double* vm = V + (int64_t)mm * n;
      double* wm = W + (int64_t)mm * n;
      c->prepare(prec);  // task lists exist before the recording
      void* g2 = dav_graph(c, prec, mm, 1, [&] {
        ex->axpby_dev(vm, 1.0, cf + CF_INV, t, 0.0, nullptr, t, n);
        ex->copy_d2d(c->C->ptr(c->b_in), vm, (size_t)n * 8);
        c->enqueue_hpsi(prec);
        ex->copy_d2d(wm, c->C->ptr(c->b_out), (size_t)n * 8);
        ex->multidot_dev(W, n, mm + 1, vm, n, cf + CF_ROW);
        ex->multidot_dev(V, n, mm + 1, wm, n, cf + CF_COL);
      });
      ex->upload(cf + CF_INV, &inv, 8);
      ex->replay(g2);
      std::vector<double> rc(CF_SIZE - CF_ROW);
      ex->download(rc.data(), cf + CF_ROW, rc.size() * 8);
      for (int j = 0; j <= m; ++j) G[(size_t)m * mmax + j] = rc[j];
      for (int j = 0; j <= m; ++j) G[(size_t)j * mmax + m] = rc[CF_COL - CF_ROW + j];
      res.matvecs++;
      ++m;
      continue;
    }
    ex->axpby(V + (int64_t)m * n, inv, t, 0.0, t, n);
    matvec(c, V + (int64_t)m * n, W + (int64_t)m * n, prec, n);
    res.matvecs++;
    // new row / column of the projected matrix
    ex->multidot(W, n, m + 1, V + (int64_t)m * n, n, tmp.data());  // <W_j, V_m>
    for (int j = 0; j <= m; ++j) G[(size_t)m * mmax + j] = tmp[j];
    ex->multidot(V, n, m + 1, W + (int64_t)m * n, n, tmp.data());  // <V_j, W_m>
    for (int j = 0; j <= m; ++j) G[(size_t)j * mmax + m] = tmp[j];
    ++m;
  }
  return res;
}

// Davidson buffers owned by the context (freed with the H*psi plan).
Workspace workspace(dmrg_ctx* c, int64_t n, int mmax) {
  if (c->work_bufs.empty() || c->work_n != n || c->work_mmax != mmax) {
    c->drop_dav_graphs();
    for (int b : c->work_bufs) c->C->free_buf(b);
    c->work_bufs = {c->C->new_buf((int64_t)(mmax + kKeep) * n), c->C->new_buf((int64_t)(mmax + kKeep) * n), c->C->new_buf(n),
                    c->C->new_buf(n), c->C->new_buf(n), c->C->new_buf(n), c->C->new_buf(n), c->C->new_buf(n),
                    c->C->new_buf(n), c->C->new_buf(CF_SIZE)};
    c->work_n = n;
    c->work_mmax = mmax;
  }
  Workspace ws;
  ws.n = n;
  ws.mmax = mmax;
  ws.bV = c->work_bufs[0];
  ws.bW = c->work_bufs[1];
  ws.bx = c->work_bufs[2];
  ws.bhx = c->work_bufs[3];
  ws.br = c->work_bufs[4];
  ws.bt = c->work_bufs[5];
  ws.bp = c->work_bufs[6];
  ws.bq = c->work_bufs[7];
  ws.bs = c->work_bufs[8];
  ws.bc = c->work_bufs[9];
  return ws;
}
}  // namespace

void step_log(const std::string& json) {
  const char* path = std::getenv("DMRG_LOG");
  if (!path || !*path) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s\n", json.c_str());
    std::fclose(f);
  }
}

namespace {
const char* prec_name(int p) {
  return p == DMRG_FP64 ? "fp64" : p == DMRG_FP32 ? "fp32" : p == DMRG_BF16 ? "bf16" : "fp8";
}
// Multiplets D and U(1) states (sum of dim * (2S+1)) of bond b.
std::pair<long long, long long> bond_dims(const Context& C, int b) {
  long long d = 0, du = 0;
  if (b >= 0 && b < (int)C.bonds.size())
    for (const auto& s : C.bonds[b].secs) {
      d += s.dim;
      du += (long long)s.dim * (s.s2 + 1);
    }
  return {d, du};
}
}  // namespace

extern "C" int dmrg_davidson_step(dmrg_ctx* c, int k, double* psi, double* energy, double* resid, int* nlo, int* nhi) {
  if (!c || !psi || !energy || !resid) return dmrg_fail(DMRG_ERR_ARG, "dmrg_davidson_step: null argument");
  if (!c->C->Lblk || k != c->C->k) return dmrg_fail(DMRG_ERR_ARG, "dmrg_davidson_step: no MPS loaded at this k");
  const long long serial = c->plan_serial;
  const auto t0 = std::chrono::steady_clock::now();
  int lo = 0, hi = 0;
  const int rc = davidson_core(c, psi, energy, resid, &lo, &hi);
  if (nlo) *nlo = lo;
  if (nhi) *nhi = hi;
  if (std::getenv("DMRG_LOG") && (rc == DMRG_OK || rc == DMRG_ERR_NOCONV) && c->plan) {
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    char buf[768];
    std::snprintf(buf, sizeof buf,
                  "{\"event\": \"davidson\", \"block\": [%d, %d], \"n_coeff\": %lld, \"precision\": \"%s\", "
                  "\"energy\": %.12f, \"residual\": %.3e, \"converged\": %s, \"matvecs_lowprec\": %d, "
                  "\"matvecs_fp64\": %d, \"hpsi_flops\": %.6e, \"seconds\": %.3f, \"plan_seconds\": %.3f, "
                  "\"prepare_seconds\": %.3f}",
                  k, k + 1, (long long)c->plan->lay.size, prec_name(c->opts.hpsi_prec), *energy, *resid,
                  rc == DMRG_OK ? "true" : "false", lo, hi, c->plan->flops, sec,
                  c->plan_serial != serial ? c->plan_seconds : 0.0,
                  c->prepare_seconds[0] + c->prepare_seconds[1] + c->prepare_seconds[2] + c->prepare_seconds[3]);
    for (double& x : c->prepare_seconds) x = 0.0;  // each preparation is reported once
    step_log(buf);
  }
  return rc;
}

int davidson_core(dmrg_ctx* c, double* psi, double* energy, double* resid, int* nlo, int* nhi) {
  try {
    c->ensure_plan();
    const int64_t n = c->plan->lay.size;
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(psi[i])) return dmrg_fail(DMRG_ERR_NONFINITE, "dmrg_davidson_step: non-finite start vector");
    const int mmax = std::max(8, std::min(48, c->opts.davidson_max_subspace > 0 ? c->opts.davidson_max_subspace : 24));
    const int max_iter = c->opts.davidson_max_iter > 0 ? c->opts.davidson_max_iter : 60;
    const double tol = c->opts.davidson_tol > 0 ? c->opts.davidson_tol : 1e-7;
    Workspace ws = workspace(c, n, mmax);
    // start vector
    std::vector<double> h0(psi, psi + n);
    double nrm = 0.0;
    for (double v : h0) nrm += v * v;
    if (!(nrm > 0.0) || !std::isfinite(nrm)) {
      std::mt19937_64 rng(12345);
      std::normal_distribution<double> nd;
      nrm = 0.0;
      for (auto& v : h0) {
        v = nd(rng);
        nrm += v * v;
      }
    }
    const double s = 1.0 / std::sqrt(nrm);
    for (auto& v : h0) v *= s;
    c->ex->upload(c->C->ptr(ws.bx), h0.data(), (size_t)n * 8);
    const int prec = c->opts.hpsi_prec;
    int lo = 0, hi = 0;
    PhaseResult pr;
    const int lo_iter = c->opts.davidson_lowprec_iter < 0 ? max_iter : c->opts.davidson_lowprec_iter;
    int carried = 1;
    if (prec != DMRG_FP64 && lo_iter > 0) {
      // phase 1: low-precision matvecs until the residual is small enough
      // for the FP64 phase to finish in a few tens of iterations (1e-3 of
      // the spectrum scale for BF16 operands, 1e-2 for FP8, 1e-6 for FP32),
      // or stalls at the precision's rounding level
      const double floor_rel = prec == DMRG_BF16 ? 1e-3 : prec == DMRG_FP8 ? 1e-2 : 1e-6;
      const double floor_tol = floor_rel * std::max(1.0, std::fabs(diag_scale(c, n)));
      pr = davidson_phase(c, ws, prec, std::max(tol, floor_tol), lo_iter, 0, DMRG_FP64, 1, kStall, refine_keep(c));
      lo = pr.matvecs;
      carried = std::max(1, pr.ritz_kept);
      if (c->opts.davidson_mid_fp32 && (prec == DMRG_BF16 || prec == DMRG_FP8) && !(pr.resid <= tol)) {
        // phase 1b: FP32 matvecs (about 1.7x cheaper than FP64 ones at
        // CAS(82,82)) down to the FP32 floor, from phase 1's Ritz vectors
        const double mid_tol = 1e-6 * std::max(1.0, std::fabs(diag_scale(c, n)));
        pr = davidson_phase(c, ws, DMRG_FP32, std::max(tol, mid_tol), lo_iter, 0, DMRG_FP64, carried, kStall,
                            refine_keep(c));
        lo += pr.matvecs;
        carried = std::max(1, pr.ritz_kept);
      }
    }
    // phase 2 (or the whole solve for FP64): FP64 matvecs to tol, starting
    // from phase 1's lowest Ritz vectors, with Jacobi-Davidson corrections
    // from low-precision inner solves if asked
    const int refine_iter =
        (prec != DMRG_FP64 && c->opts.davidson_refine_iter > 0) ? c->opts.davidson_refine_iter : max_iter;
    const int jd = prec != DMRG_FP64 ? c->opts.davidson_jd_inner : 0;
    pr = davidson_phase(c, ws, DMRG_FP64, tol, refine_iter, jd, prec, carried);
    hi = pr.matvecs;
    lo += pr.inner_matvecs;
    c->ex->download(psi, c->C->ptr(ws.bx), (size_t)n * 8);
    *energy = pr.theta + c->opts.e_core;
    *resid = pr.resid;
    if (nlo) *nlo = lo;
    if (nhi) *nhi = hi;
    if (!pr.converged) return dmrg_fail(DMRG_ERR_NOCONV, "dmrg_davidson_step: residual above tolerance");
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return dmrg_fail(DMRG_ERR_BUDGET, std::string("dmrg_davidson_step: ") + e.what());
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_davidson_step: ") + e.what());
  }
}

namespace {
struct CutSector {
  int n = 0, s2 = 0;           // quantum numbers of the enlarged block on the cut side
  int dim = 0;                 // rows (direction +1) or columns (-1) of its super-blocks
  std::vector<int> sbs;        // super-blocks with this sector on the cut side
  int64_t off = 0;             // offset of its rho / eigenvector matrices
};
}  // namespace

// Start vector for the two-site block (k+1, k+2) after a truncation at
// (k, k+1) moving right.  With U_a the kept eigenvectors of cut sector a
// (the new left-canonical tensor at site k), the kept part of psi is
// C = U_a^T psi_(a,c) in the basis |a'> (x) |(sigma2 r) S_c>.  The right
// block state r at bond k+2 is sum B(r; sigma3 r') |(sigma3 r') S_r> with B
// the right-canonical tensor of site k+2, so in the next block's middle-cut
// basis ((a' sigma2) S'', (sigma3 r') S_r) S the coefficients are
//   sum_{S_c} <((a' sigma2) S'', r) S | (a', (sigma2 r) S_c) S> C B,
// one 6j recoupling per block (no fermion sign: the order of the sites is
// unchanged).  Without truncation it is the same state as psi.
static void next_block_guess(dmrg_ctx* c, int k, const PsiLayout& lay, const double* psi,
                      const std::vector<CutSector>& secs, const std::vector<std::vector<int>>& kept,
                      const std::vector<int>& new_of, const std::vector<double>& hV, const Bond& nb) {
  Context& C = *c->C;
  const SiteTensor& B = C.sites[k + 2];
  if (B.left || B.buf < 0) return;
  int64_t nbv = 0;
  for (auto& bk : B.blocks) nbv = std::max<int64_t>(nbv, bk.off + (int64_t)bk.rows * bk.cols);
  std::vector<double> bv((size_t)std::max<int64_t>(nbv, 1));
  if (nbv) c->ex->download(bv.data(), C.ptr(B.buf), (size_t)nbv * 8);
  // C = U^T psi per old super-block whose left sector keeps states
  std::map<std::pair<int, int>, int> sec_index;
  for (size_t si = 0; si < secs.size(); ++si) sec_index[{secs[si].n, secs[si].s2}] = (int)si;
  std::vector<std::vector<double>> Cm(lay.sbs.size());
  for (size_t sbi = 0; sbi < lay.sbs.size(); ++sbi) {
    const auto& sb = lay.sbs[sbi];
    const int si = sec_index.at({sb.an, sb.as2});
    if (new_of[si] < 0) continue;
    const int da = (int)kept[si].size(), dim = secs[si].dim;
    std::vector<double>& m = Cm[sbi];
    m.assign((size_t)da * sb.ncols, 0.0);
    for (int r = 0; r < sb.nrows; ++r) {
      const double* prow = psi + sb.off + (int64_t)r * sb.ncols;
      for (int q = 0; q < da; ++q) {
        const double u = hV[(size_t)secs[si].off + (size_t)r * dim + kept[si][q]];
        if (u == 0.0) continue;
        double* mrow = m.data() + (size_t)q * sb.ncols;
        for (int col = 0; col < sb.ncols; ++col) mrow[col] += u * prow[col];
      }
    }
  }
  const Bond& b2 = C.bonds[k + 2];
  const Bond& b3 = C.bonds[k + 3];
  PsiLayout nl;
  nl.build(nb, b3, c->opts.n_elec, c->opts.two_s);
  std::vector<double> g((size_t)nl.size, 0.0);
  const int S = c->opts.two_s;
  auto loc2s = [](int sig) { return sig == 1 ? 1 : 0; };
  for (const auto& sb2 : nl.sbs) {
    for (const auto& rr : sb2.rows) {
      const Sector& ap = nb.secs[rr.il];  // a' (new bond k+1), site sigma2 = rr.s1
      int si = -1;
      for (size_t q = 0; q < secs.size(); ++q)
        if (new_of[q] == rr.il) si = (int)q;
      if (si < 0) continue;
      for (const auto& cc : sb2.cols) {  // sigma3 = cc.s2, r' = bond k+3 sector cc.ir
        for (size_t ir = 0; ir < b2.secs.size(); ++ir) {
          const Sector& rs = b2.secs[ir];
          if (rs.n != sb2.cn || rs.s2 != sb2.cs2) continue;  // r is (sigma3 r') coupled to S_r = S''_c
          auto bit = B.find.find({(int)ir, cc.s2, cc.ir});
          if (bit == B.find.end()) continue;
          const auto& bk = B.blocks[bit->second];  // D_r x D_r'
          for (size_t sbi = 0; sbi < lay.sbs.size(); ++sbi) {
            const auto& sb = lay.sbs[sbi];
            if (Cm[sbi].empty() || sb.an != ap.n || sb.as2 != ap.s2) continue;
            int c0 = -1, dr = 0;
            for (const auto& col : sb.cols)
              if (col.s2 == rr.s1 && col.ir == (int)ir) {
                c0 = col.c0;
                dr = col.dr;
              }
            if (c0 < 0) continue;
            // <((a' sigma2) S'', r) S | (a', (sigma2 r) S_c) S>
            const int j1 = ap.s2, j2 = loc2s(rr.s1), j3 = rs.s2, J12 = sb2.as2, J23 = sb.cs2;
            const int ph = (j1 + j2 + j3 + S) / 2;
            const double w = ((ph & 1) ? -1.0 : 1.0) * std::sqrt((J12 + 1.0) * (J23 + 1.0)) *
                             sixj2(j1, j2, J12, j3, S, J23);
            if (w == 0.0) continue;
            const int da = rr.dl;
            for (int i = 0; i < da; ++i) {
              const double* crow = Cm[sbi].data() + (size_t)i * sb.ncols + c0;
              double* grow = g.data() + sb2.off + (int64_t)(rr.r0 + i) * sb2.ncols + cc.c0;
              for (int t = 0; t < dr; ++t) {
                const double ct = w * crow[t];
                if (ct == 0.0) continue;
                const double* brow = bv.data() + bk.off + (int64_t)t * bk.cols;
                for (int j = 0; j < cc.dr; ++j) grow[j] += ct * brow[j];
              }
            }
          }
        }
      }
    }
  }
  c->guess.swap(g);
  c->guess_k = k + 1;
}

// Start vector for the two-site block (k-1, k) after a truncation at
// (k, k+1) that moves left: the kept part of psi, psi V (V: the kept
// eigenvectors of the right density matrix, i.e. the new right-canonical
// tensor of site k+1 transposed), contracted with the left-canonical tensor
// of site k-1 and recoupled from ((l s_k) S_a, c') S to (l, (s_k c') S_c) S
// by one 6j per block -- the mirror of next_block_guess; no fermion sign
// enters since the site order is unchanged.
static void prev_block_guess(dmrg_ctx* c, int k, const PsiLayout& lay, const double* psi,
                             const std::vector<CutSector>& secs, const std::vector<std::vector<int>>& kept,
                             const std::vector<int>& new_of, const std::vector<double>& hV, const Bond& nb) {
  Context& C = *c->C;
  const SiteTensor& A = C.sites[k - 1];
  if (!A.left || A.buf < 0) return;
  int64_t nav = 0;
  for (auto& bk : A.blocks) nav = std::max<int64_t>(nav, bk.off + (int64_t)bk.rows * bk.cols);
  std::vector<double> av((size_t)std::max<int64_t>(nav, 1));
  if (nav) c->ex->download(av.data(), C.ptr(A.buf), (size_t)nav * 8);
  // Cm = psi V per old super-block whose right sector keeps states (rows x kept)
  std::map<std::pair<int, int>, int> sec_index;
  for (size_t si = 0; si < secs.size(); ++si) sec_index[{secs[si].n, secs[si].s2}] = (int)si;
  std::vector<std::vector<double>> Cm(lay.sbs.size());
  std::vector<int> cut_of(lay.sbs.size(), -1);
  for (size_t sbi = 0; sbi < lay.sbs.size(); ++sbi) {
    const auto& sb = lay.sbs[sbi];
    const int si = sec_index.at({sb.cn, sb.cs2});
    if (new_of[si] < 0) continue;
    cut_of[sbi] = si;
    const int da = (int)kept[si].size(), dim = secs[si].dim;
    std::vector<double>& m = Cm[sbi];
    m.assign((size_t)sb.nrows * da, 0.0);
    for (int r = 0; r < sb.nrows; ++r) {
      const double* prow = psi + sb.off + (int64_t)r * sb.ncols;
      for (int q = 0; q < da; ++q) {
        double acc = 0.0;
        for (int col = 0; col < sb.ncols; ++col) acc += prow[col] * hV[(size_t)secs[si].off + (size_t)col * dim + kept[si][q]];
        m[(size_t)r * da + q] = acc;
      }
    }
  }
  const Bond& bl = C.bonds[k - 1];
  const Bond& bk = C.bonds[k];
  PsiLayout nl;
  nl.build(bl, nb, c->opts.n_elec, c->opts.two_s);
  std::vector<double> g((size_t)nl.size, 0.0);
  const int S = c->opts.two_s;
  auto loc2s = [](int sig) { return sig == 1 ? 1 : 0; };
  for (const auto& sb2 : nl.sbs) {
    for (const auto& rr : sb2.rows) {  // l'' = bond k-1 sector rr.il, sigma_{k-1} = rr.s1
      for (size_t il = 0; il < bk.secs.size(); ++il) {
        const Sector& ls = bk.secs[il];  // l: (l'' sigma_{k-1}) coupled to the new left sector
        if (ls.n != sb2.an || ls.s2 != sb2.as2) continue;
        auto ait = A.find.find({rr.il, rr.s1, (int)il});
        if (ait == A.find.end()) continue;
        const auto& ab = A.blocks[ait->second];  // D_l'' x D_l
        for (const auto& cc : sb2.cols) {  // sigma_k = cc.s2, c' = new bond k+1 sector cc.ir
          for (size_t sbi = 0; sbi < lay.sbs.size(); ++sbi) {
            const int si = cut_of[sbi];
            if (si < 0 || new_of[si] != cc.ir) continue;
            const auto& sb = lay.sbs[sbi];
            int r0o = -1;
            for (const auto& ro : sb.rows)
              if (ro.il == (int)il && ro.s1 == cc.s2) r0o = ro.r0;
            if (r0o < 0) continue;
            const int da = (int)kept[si].size();
            if (da != cc.dr) throw std::runtime_error("prev_block_guess: kept states do not match the new bond");
            // <(l, (sigma_k c') S_c) S | ((l sigma_k) S_a, c') S>
            const int j1 = ls.s2, j2 = loc2s(cc.s2), j3 = nb.secs[cc.ir].s2, J12 = sb.as2, J23 = sb2.cs2;
            const int ph = (j1 + j2 + j3 + S) / 2;
            const double w = ((ph & 1) ? -1.0 : 1.0) * std::sqrt((J12 + 1.0) * (J23 + 1.0)) *
                             sixj2(j1, j2, J12, j3, S, J23);
            if (w == 0.0) continue;
            for (int i = 0; i < rr.dl; ++i) {
              double* grow = g.data() + sb2.off + (int64_t)(rr.r0 + i) * sb2.ncols + cc.c0;
              for (int t = 0; t < ab.cols; ++t) {
                const double at = w * av[(size_t)ab.off + (size_t)i * ab.cols + t];
                if (at == 0.0) continue;
                const double* crow = Cm[sbi].data() + (size_t)(r0o + t) * da;
                for (int j = 0; j < da; ++j) grow[j] += at * crow[j];
              }
            }
          }
        }
      }
    }
  }
  c->guess.swap(g);
  c->guess_k = k - 1;
}

extern "C" int dmrg_truncate(dmrg_ctx* c, int k, const double* psi, int dir, int d_max, double eps_tr,
                             double* trunc_err, int* d_kept) {
  return dmrg_truncate_dbss(c, k, psi, dir, 0, d_max, eps_tr, trunc_err, d_kept);
}

static int truncate_core(dmrg_ctx* c, int k, const double* psi, int dir, int d_min, int d_max, double eps_tr,
                         double* trunc_err, int* d_kept);

extern "C" int dmrg_truncate_dbss(dmrg_ctx* c, int k, const double* psi, int dir, int d_min, int d_max,
                                  double eps_tr, double* trunc_err, int* d_kept) {
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = truncate_core(c, k, psi, dir, d_min, d_max, eps_tr, trunc_err, d_kept);
  if (rc == DMRG_OK && std::getenv("DMRG_LOG")) {
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    const auto dd = bond_dims(*c->C, k + 1);
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "{\"event\": \"truncate\", \"block\": [%d, %d], \"direction\": %d, \"bond\": %d, "
                  "\"d_kept\": %d, \"d_u1\": %lld, \"trunc_err\": %.6e, \"seconds\": %.3f, \"next_block\": %d}",
                  k, k + 1, dir, k + 1, *d_kept, dd.second, *trunc_err, sec, c->C->k);
    step_log(buf);
  }
  return rc;
}

static int truncate_core(dmrg_ctx* c, int k, const double* psi, int dir, int d_min, int d_max, double eps_tr,
                         double* trunc_err, int* d_kept) {
  if (!c || !psi || !trunc_err || !d_kept) return dmrg_fail(DMRG_ERR_ARG, "dmrg_truncate: null argument");
  if (dir != 1 && dir != -1) return dmrg_fail(DMRG_ERR_ARG, "dmrg_truncate: direction must be +1 or -1");
  if (d_max < 1 || !(eps_tr >= 0.0)) return dmrg_fail(DMRG_ERR_ARG, "dmrg_truncate: bad d_max / eps_tr");
  if (d_min < 0 || d_min > d_max) return dmrg_fail(DMRG_ERR_ARG, "dmrg_truncate: need 0 <= d_min <= d_max");
  if (!c->C->Lblk || k != c->C->k) return dmrg_fail(DMRG_ERR_ARG, "dmrg_truncate: no MPS loaded at this k");
  Context& C = *c->C;
  Executor* ex = c->ex.get();
  try {
    c->ensure_plan();
    const PsiLayout lay = c->plan->lay;  // copy: the plan is reset below
    const int64_t n = lay.size;
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(psi[i])) return dmrg_fail(DMRG_ERR_NONFINITE, "dmrg_truncate: non-finite psi");
    ex->upload(C.ptr(c->b_in), psi, (size_t)n * 8);
    // ---- sectors of the cut side
    std::vector<CutSector> secs;
    std::map<std::pair<int, int>, int> sec_of;
    for (size_t s = 0; s < lay.sbs.size(); ++s) {
      const auto& sb = lay.sbs[s];
      const std::pair<int, int> key = dir > 0 ? std::make_pair(sb.an, sb.as2) : std::make_pair(sb.cn, sb.cs2);
      auto it = sec_of.find(key);
      if (it == sec_of.end()) {
        CutSector cs;
        cs.n = key.first;
        cs.s2 = key.second;
        cs.dim = dir > 0 ? sb.nrows : sb.ncols;
        sec_of[key] = (int)secs.size();
        secs.push_back(cs);
        it = sec_of.find(key);
      }
      secs[it->second].sbs.push_back((int)s);
    }
    std::sort(secs.begin(), secs.end(), [](const CutSector& a, const CutSector& b) {
      return a.n != b.n ? a.n < b.n : a.s2 < b.s2;
    });
    int64_t tot = 0;
    std::vector<int64_t> offs;
    std::vector<int> sizes;
    for (auto& s : secs) {
      s.off = tot;
      offs.push_back(tot);
      sizes.push_back(s.dim);
      tot += (int64_t)s.dim * s.dim;
    }
    // ---- reduced density matrices rho = sum psi psi^T (or psi^T psi) on the GPU
    const int bR = C.new_buf(std::max<int64_t>(tot, 1)), bV = C.new_buf(std::max<int64_t>(tot, 1));
    GemmBatch gb;
    for (auto& s : secs) {
      GemmJob j;
      j.C = BufRef{bR, s.off};
      j.m = s.dim;
      j.n = s.dim;
      j.ldc = s.dim;
      j.tbeg = (int64_t)gb.terms.size();
      for (int sbi : s.sbs) {
        const auto& sb = lay.sbs[sbi];
        GemmTerm t;
        t.A = BufRef{-PH_IN, sb.off};
        t.B = BufRef{-PH_IN, sb.off};
        t.lda = sb.ncols;
        t.ldb = sb.ncols;
        if (dir > 0) {
          t.flags = TF_TRANS_B;
          t.k = sb.ncols;
        } else {
          t.flags = TF_TRANS_A;
          t.k = sb.nrows;
        }
        gb.terms.push_back(t);
      }
      j.tend = (int64_t)gb.terms.size();
      gb.jobs.push_back(j);
    }
    const bool verbose = std::getenv("DMRG_VERBOSE") != nullptr;
    auto tick = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
      if (!verbose) return;
      ex->sync();
      auto now = std::chrono::steady_clock::now();
      std::fprintf(stderr, "[truncate] %s %.3f s\n", what, std::chrono::duration<double>(now - tick).count());
      tick = now;
    };
    c->bind();
    C.run_batch(gb);
    lap("rho");
    double eig_worst = 0.0;
    const int eig_left = ex->sym_eig((double*)C.ptr(bR), (double*)C.ptr(bV), offs, sizes, 40, 1e-15, &eig_worst);
    lap("eigensolve");
    std::vector<double> hR((size_t)tot), hV((size_t)tot);
    ex->download(hR.data(), C.ptr(bR), (size_t)tot * 8);
    ex->download(hV.data(), C.ptr(bV), (size_t)tot * 8);
    C.free_buf(bR);
    C.free_buf(bV);
    // ---- select kept multiplets
    struct W {
      double w;
      int s2, n, sec, idx;
    };
    std::vector<W> all;
    double wsum = 0.0;
    for (size_t si = 0; si < secs.size(); ++si)
      for (int i = 0; i < secs[si].dim; ++i) {
        double w = std::max(0.0, hR[(size_t)secs[si].off + (size_t)i * secs[si].dim + i]);
        all.push_back(W{w, secs[si].s2, secs[si].n, (int)si, i});
        wsum += w;
      }
    if (!(wsum > 0.0)) return dmrg_fail(DMRG_ERR_ARG, "dmrg_truncate: zero wavefunction");
    std::sort(all.begin(), all.end(), [](const W& a, const W& b) {
      if (a.w != b.w) return a.w > b.w;
      if (a.s2 != b.s2) return a.s2 < b.s2;
      if (a.n != b.n) return a.n < b.n;
      return a.sec != b.sec ? a.sec < b.sec : a.idx < b.idx;
    });
    size_t keepn = std::min<size_t>((size_t)d_max, all.size());
    if (eps_tr > 0.0) {
      // dynamic block state selection: the fewest multiplets whose discarded
      // weight stays <= eps_tr, but at least d_min and at most d_max
      double disc = 0.0;
      size_t m = all.size();
      while (m > 1 && disc + all[m - 1].w <= eps_tr * wsum) {
        disc += all[m - 1].w;
        --m;
      }
      keepn = std::min(keepn, std::max(m, std::min<size_t>((size_t)d_min, all.size())));
    }
    double kept_w = 0.0;
    std::vector<std::vector<int>> kept(secs.size());
    c->cut_values.clear();
    c->cut_spins.clear();
    for (size_t i = 0; i < keepn; ++i) {
      kept[all[i].sec].push_back(all[i].idx);
      kept_w += all[i].w;
      c->cut_values.push_back(std::sqrt(all[i].w / wsum));
      c->cut_spins.push_back(all[i].s2);
    }
    *trunc_err = std::max(0.0, 1.0 - kept_w / wsum);
    *d_kept = (int)keepn;
    // ---- new bond and site tensor (kept eigenvectors, descending weight per sector)
    Bond nb;
    std::vector<int> new_of(secs.size(), -1);
    for (size_t si = 0; si < secs.size(); ++si) {
      if (kept[si].empty()) continue;
      new_of[si] = (int)nb.secs.size();
      nb.secs.push_back(Sector{secs[si].n, secs[si].s2, (int)kept[si].size()});
    }
    SiteTensor T;
    T.left = dir > 0;
    T.j = dir > 0 ? k : k + 1;
    const Bond& lb = C.Lblk->bond;
    const Bond& rb = C.Rblk->bond;
    std::vector<double> vals;
    // Left: blocks (l, sigma1, a) in (l, sigma, a) order; rows of a are the (l, sigma1) sub-blocks.
    // Right: blocks (c, sigma2, r) in (c, sigma, r) order; columns of c are the (sigma2, r) sub-blocks.
    auto sub_of = [&](const CutSector& s, int first, int sig, int& off, int& dim) {
      const auto& sb = lay.sbs[s.sbs[0]];
      if (dir > 0) {
        for (auto& r : sb.rows)
          if (r.il == first && r.s1 == sig) {
            off = r.r0;
            dim = r.dl;
            return true;
          }
      } else {
        for (auto& cl : sb.cols)
          if (cl.ir == first && cl.s2 == sig) {
            off = cl.c0;
            dim = cl.dr;
            return true;
          }
      }
      return false;
    };
    const Bond& outer = dir > 0 ? lb : rb;  // the bond on the far side of the site
    int64_t voff = 0;
    if (dir > 0) {
      for (size_t il = 0; il < outer.secs.size(); ++il)
        for (int sig = 0; sig < 3; ++sig)
          for (size_t si = 0; si < secs.size(); ++si) {
            if (new_of[si] < 0) continue;
            int off, dim;
            if (!sub_of(secs[si], (int)il, sig, off, dim)) continue;
            const int da = (int)kept[si].size();
            T.find[{(int)il, sig, new_of[si]}] = (int)T.blocks.size();
            T.blocks.push_back(SiteTensor::Blk{(int)il, sig, new_of[si], voff, dim, da});
            for (int r = 0; r < dim; ++r)
              for (int q = 0; q < da; ++q)
                vals.push_back(hV[(size_t)secs[si].off + (size_t)(off + r) * secs[si].dim + kept[si][q]]);
            voff += (int64_t)dim * da;
          }
    } else {
      for (size_t si = 0; si < secs.size(); ++si) {
        if (new_of[si] < 0) continue;
        for (int sig = 0; sig < 3; ++sig)
          for (size_t ir = 0; ir < outer.secs.size(); ++ir) {
            int off, dim;
            if (!sub_of(secs[si], (int)ir, sig, off, dim)) continue;
            const int dc = (int)kept[si].size();
            T.find[{new_of[si], sig, (int)ir}] = (int)T.blocks.size();
            T.blocks.push_back(SiteTensor::Blk{new_of[si], sig, (int)ir, voff, dc, dim});
            for (int q = 0; q < dc; ++q)
              for (int r = 0; r < dim; ++r)
                vals.push_back(hV[(size_t)secs[si].off + (size_t)(off + r) * secs[si].dim + kept[si][q]]);
            voff += (int64_t)dc * dim;
          }
      }
      // canonical (c, sigma, r) order
      std::vector<size_t> ord(T.blocks.size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
      std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
        const auto &x = T.blocks[a], &y = T.blocks[b];
        return std::tie(x.s0, x.sig, x.s1) < std::tie(y.s0, y.sig, y.s1);
      });
      std::vector<SiteTensor::Blk> nbk;
      std::vector<double> nv;
      T.find.clear();
      for (size_t i : ord) {
        auto bk = T.blocks[i];
        const size_t cnt = (size_t)bk.rows * bk.cols;
        std::vector<double> tmp(vals.begin() + bk.off, vals.begin() + bk.off + cnt);
        bk.off = (int64_t)nv.size();
        nv.insert(nv.end(), tmp.begin(), tmp.end());
        T.find[{bk.s0, bk.sig, bk.s1}] = (int)nbk.size();
        nbk.push_back(bk);
      }
      T.blocks.swap(nbk);
      vals.swap(nv);
    }
    T.buf = C.new_buf(std::max<int64_t>((int64_t)vals.size(), 1));
    if (!vals.empty()) ex->upload(C.ptr(T.buf), vals.data(), vals.size() * 8);
    lap("select + site tensor");
    // ---- start vector for the block (k+1, k+2) the sweep moves to
    c->guess.clear();
    c->guess_k = -1;
    if (dir > 0 && c->opts.next_guess && k + 3 <= C.n) {
      next_block_guess(c, k, lay, psi, secs, kept, new_of, hV, nb);
      lap("next-block start vector");
    } else if (dir < 0 && c->opts.next_guess && k >= 1) {
      prev_block_guess(c, k, lay, psi, secs, kept, new_of, hV, nb);
      lap("previous-block start vector");
    }
    // ---- grow the operator block across the cut, move the two-site block if possible
    c->reset_plan();
    // blocks left behind are kept for a sweep back only with keep_blocks = 1
    const bool keep = c->opts.keep_blocks == 1;
    if (dir > 0) {
      auto N = C.grow_left(*C.Lblk, T, nb);
      if (keep) C.Lhist[k] = std::move(C.Lblk);
      else C.free_block(*C.Lblk);
      C.Lblk = std::move(N);
      C.free_buf(C.sites[k].buf);
      C.sites[k] = T;
      C.bonds[k + 1] = nb;
      if (k + 3 <= C.n && C.Rhist.size() > (size_t)(k + 3) && C.Rhist[k + 3]) {
        if (keep) C.Rhist[k + 2] = std::move(C.Rblk);
        else C.free_block(*C.Rblk);
        C.Rblk = std::move(C.Rhist[k + 3]);
        C.k = k + 1;
      } else {
        C.k = -1;
      }
    } else {
      auto N = C.grow_right(*C.Rblk, T, nb);
      if (keep) C.Rhist[k + 2] = std::move(C.Rblk);
      else C.free_block(*C.Rblk);
      C.Rblk = std::move(N);
      C.free_buf(C.sites[k + 1].buf);
      C.sites[k + 1] = T;
      C.bonds[k + 1] = nb;
      if (k - 1 >= 0 && C.Lhist.size() > (size_t)(k - 1) && C.Lhist[k - 1]) {
        if (keep) C.Lhist[k] = std::move(C.Lblk);
        else C.free_block(*C.Lblk);
        C.Lblk = std::move(C.Lhist[k - 1]);
        C.k = k - 1;
      } else {
        C.k = -1;
      }
    }
    lap("block growth");
    if (eig_left > 0)
      return dmrg_fail(DMRG_ERR_NOCONV, "dmrg_truncate: density-matrix eigensolver left " + std::to_string(eig_left) +
                                            " sector(s) unconverged after 40 sweeps (worst off-diagonal/norm " +
                                            std::to_string(eig_worst) + "); outputs written");
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return dmrg_fail(DMRG_ERR_BUDGET, std::string("dmrg_truncate: ") + e.what());
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_truncate: ") + e.what());
  }
}

extern "C" int dmrg_cut_spectrum(dmrg_ctx* c, double* values, int* two_s, int* n, int capacity) {
  if (!c || !n) return dmrg_fail(DMRG_ERR_ARG, "dmrg_cut_spectrum: null argument");
  const int cnt = (int)c->cut_values.size();
  *n = cnt;
  for (int i = 0; i < cnt && i < capacity; ++i) {
    if (values) values[i] = c->cut_values[i];
    if (two_s) two_s[i] = c->cut_spins[i];
  }
  return DMRG_OK;
}

extern "C" int dmrg_get_bond(dmrg_ctx* c, int b, int* sectors, int* n) {
  if (!c || !n) return dmrg_fail(DMRG_ERR_ARG, "dmrg_get_bond: null argument");
  if (b < 0 || b >= (int)c->C->bonds.size()) return dmrg_fail(DMRG_ERR_ARG, "dmrg_get_bond: bond out of range");
  const Bond& bd = c->C->bonds[b];
  *n = (int)bd.secs.size();
  if (sectors)
    for (size_t i = 0; i < bd.secs.size(); ++i) {
      sectors[3 * i] = bd.secs[i].n;
      sectors[3 * i + 1] = bd.secs[i].s2;
      sectors[3 * i + 2] = bd.secs[i].dim;
    }
  return DMRG_OK;
}

extern "C" int dmrg_get_site(dmrg_ctx* c, int j, double* values, long long* n) {
  if (!c || !n) return dmrg_fail(DMRG_ERR_ARG, "dmrg_get_site: null argument");
  if (j < 0 || j >= (int)c->C->sites.size() || c->C->sites[j].buf < 0)
    return dmrg_fail(DMRG_ERR_ARG, "dmrg_get_site: no tensor held for this site");
  const SiteTensor& T = c->C->sites[j];
  int64_t cnt = 0;
  for (auto& b : T.blocks) cnt += (int64_t)b.rows * b.cols;
  *n = cnt;
  try {
    if (values && cnt) c->ex->download(values, c->C->ptr(T.buf), (size_t)cnt * 8);
  } catch (const std::bad_alloc& e) {
    return dmrg_fail(DMRG_ERR_BUDGET, std::string("dmrg_get_site: ") + e.what());
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_get_site: ") + e.what());
  }
  return DMRG_OK;
}

extern "C" int dmrg_current_block(dmrg_ctx* c, int* k) {
  if (!c || !k) return dmrg_fail(DMRG_ERR_ARG, "dmrg_current_block: null argument");
  *k = c->C->k;
  return DMRG_OK;
}

extern "C" int dmrg_next_guess(dmrg_ctx* c, int k, double* psi, long long n) {
  if (!c || !psi) return dmrg_fail(DMRG_ERR_ARG, "dmrg_next_guess: null argument");
  if (c->guess_k < 0 || c->guess_k != k || c->C->k != k)
    return dmrg_fail(DMRG_ERR_ARG, "dmrg_next_guess: no start vector carried to this block");
  if (n != (long long)c->guess.size()) return dmrg_fail(DMRG_ERR_SHAPE, "dmrg_next_guess: wrong length");
  std::copy(c->guess.begin(), c->guess.end(), psi);
  return DMRG_OK;
}
