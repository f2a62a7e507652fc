// C ABI: argument validation, MPS ingestion, operator-block build and the
// H*psi driver.  See include/dmrg.h for the contract.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <stdexcept>
#include <string>

#include "../../include/dmrg.h"
#include "planner.hpp"
#include "session.hpp"
#include "su2.hpp"

using namespace dmrg;

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}
}  // namespace

extern "C" const char* dmrg_last_error(void) { return g_err.c_str(); }

int dmrg_fail(int code, const std::string& msg) { return fail(code, msg); }

extern "C" int dmrg_create(dmrg_ctx** out, const dmrg_opts* o, const double* h, const double* g) {
  if (!out || !o || !h || !g) return fail(DMRG_ERR_ARG, "dmrg_create: null argument");
  *out = nullptr;
  const int n = o->n_orb;
  if (n < 2 || n > 256) return fail(DMRG_ERR_ARG, "dmrg_create: n_orb must be in [2, 256]");
  if (o->n_elec < 0 || o->n_elec > 2 * n) return fail(DMRG_ERR_SYMMETRY, "dmrg_create: N out of range");
  if (o->two_s < 0 || ((o->n_elec + o->two_s) & 1) || o->two_s > std::min(o->n_elec, 2 * n - o->n_elec))
    return fail(DMRG_ERR_SYMMETRY, "dmrg_create: 2S incompatible with N");
  if (o->hpsi_prec < 0 || o->hpsi_prec > 3) return fail(DMRG_ERR_ARG, "dmrg_create: bad hpsi_prec");
  if (o->davidson_max_iter < 0 || o->davidson_refine_iter < 0 || o->davidson_max_subspace < 0 ||
      o->davidson_jd_inner < 0 || o->davidson_lowprec_iter < -1)
    return fail(DMRG_ERR_ARG, "dmrg_create: negative Davidson budget");
  if (o->hpsi_graph < 0 || o->hpsi_graph > 1) return fail(DMRG_ERR_ARG, "dmrg_create: hpsi_graph must be 0 or 1");
  if (o->next_guess < 0 || o->next_guess > 1) return fail(DMRG_ERR_ARG, "dmrg_create: next_guess must be 0 or 1");
  if (o->hbm_budget_bytes < 0) return fail(DMRG_ERR_ARG, "dmrg_create: negative hbm_budget_bytes");
  if (o->keep_blocks == -1) return fail(DMRG_ERR_ARG, "dmrg_create: keep_blocks -1 (right side only needs -m <= -2)");
  if (o->davidson_mid_fp32 < 0 || o->davidson_mid_fp32 > 1)
    return fail(DMRG_ERR_ARG, "dmrg_create: davidson_mid_fp32 must be 0 or 1");
  if (o->davidson_graph < 0 || o->davidson_graph > 1)
    return fail(DMRG_ERR_ARG, "dmrg_create: davidson_graph must be 0 or 1");
  const size_t n2 = (size_t)n * n, n4 = n2 * n2;
  if (!finite_all(h, n2) || !finite_all(g, n4)) return fail(DMRG_ERR_NONFINITE, "dmrg_create: non-finite integral");
  {
    // the operator scheme pairs (pq|rs) with its index permutations: real
    // orbitals, h symmetric and g 8-fold symmetric
    double hm = 0.0, gm = 0.0;
    for (size_t i = 0; i < n2; ++i) hm = std::max(hm, std::fabs(h[i]));
    for (size_t i = 0; i < n4; ++i) gm = std::max(gm, std::fabs(g[i]));
    const double th = 1e-12 * std::max(hm, 1e-300), tg = 1e-12 * std::max(gm, 1e-300);
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < p; ++q)
        if (std::fabs(h[(size_t)p * n + q] - h[(size_t)q * n + p]) > th)
          return fail(DMRG_ERR_ARG, "dmrg_create: h is not symmetric");
    auto G = [&](int p, int q, int r, int t) { return g[(((size_t)p * n + q) * n + r) * n + t]; };
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q)
        for (int r = 0; r < n; ++r)
          for (int t = 0; t < n; ++t) {
            const double v = G(p, q, r, t);
            if (std::fabs(v - G(q, p, r, t)) > tg || std::fabs(v - G(p, q, t, r)) > tg ||
                std::fabs(v - G(r, t, p, q)) > tg)
              return fail(DMRG_ERR_ARG, "dmrg_create: g is not 8-fold symmetric ((pq|rs) = (qp|rs) = (pq|sr) = (rs|pq))");
          }
  }
  try {
    auto s = std::make_unique<dmrg_ctx>();
    s->opts = *o;
    Integrals I;
    I.n = n;
    I.h.assign(h, h + n2);
    I.g.assign(g, g + n4);
    I.e_core = o->e_core;
    s->ex.reset(make_hip_executor());
    s->C = std::make_unique<Context>(s->ex.get(), I, o->n_elec, o->two_s);
    s->C->budget_bytes = o->hbm_budget_bytes;
    *out = s.release();
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_create: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_create: ") + e.what());
  }
}

extern "C" int dmrg_update_opts(dmrg_ctx* c, const dmrg_opts* o) {
  if (!c || !o) return fail(DMRG_ERR_ARG, "dmrg_update_opts: null argument");
  const dmrg_opts& p = c->opts;
  if (o->n_orb != p.n_orb || o->n_elec != p.n_elec || o->two_s != p.two_s ||
      o->work_budget_elems != p.work_budget_elems || o->keep_blocks != p.keep_blocks ||
      o->hbm_budget_bytes != p.hbm_budget_bytes || o->e_core != p.e_core)
    return fail(DMRG_ERR_ARG, "dmrg_update_opts: only the Davidson, precision, graph and next-guess fields may change");
  if (o->hpsi_prec < 0 || o->hpsi_prec > 3) return fail(DMRG_ERR_ARG, "dmrg_update_opts: bad hpsi_prec");
  if (o->davidson_max_iter < 0 || o->davidson_refine_iter < 0 || o->davidson_max_subspace < 0 ||
      o->davidson_jd_inner < 0 || o->davidson_lowprec_iter < -1 || !(o->davidson_tol >= 0.0))
    return fail(DMRG_ERR_ARG, "dmrg_update_opts: negative Davidson budget or tolerance");
  if (o->hpsi_graph < 0 || o->hpsi_graph > 1 || o->next_guess < 0 || o->next_guess > 1 || o->davidson_mid_fp32 < 0 ||
      o->davidson_mid_fp32 > 1 || o->davidson_graph < 0 || o->davidson_graph > 1)
    return fail(DMRG_ERR_ARG,
                "dmrg_update_opts: hpsi_graph, next_guess, davidson_mid_fp32 and davidson_graph must be 0 or 1");
  c->opts = *o;
  return DMRG_OK;
}

extern "C" void dmrg_destroy(dmrg_ctx* c) { delete c; }

extern "C" int dmrg_set_mps(dmrg_ctx* c, int k, const int* bs, const int* counts, const double* blocks,
                            long long n_values) {
  if (!c || !bs || !counts || (!blocks && n_values > 0)) return fail(DMRG_ERR_ARG, "dmrg_set_mps: null argument");
  Context& C = *c->C;
  const int n = C.n;
  if (k < 0 || k > n - 2) return fail(DMRG_ERR_ARG, "dmrg_set_mps: k out of range");
  // ---- bonds
  std::vector<Bond> bonds(n + 1);
  size_t pos = 0;
  for (int b = 0; b <= n; ++b) {
    if (counts[b] < 0) return fail(DMRG_ERR_SHAPE, "dmrg_set_mps: negative sector count");
    for (int i = 0; i < counts[b]; ++i, ++pos) {
      Sector s{bs[3 * pos], bs[3 * pos + 1], bs[3 * pos + 2]};
      if (s.dim <= 0) return fail(DMRG_ERR_SHAPE, "dmrg_set_mps: non-positive sector dimension");
      if (s.n < 0 || s.s2 < 0 || ((s.n + s.s2) & 1)) return fail(DMRG_ERR_SYMMETRY, "dmrg_set_mps: sector parity");
      const int m = (b <= k) ? b : n - b;  // orbitals in the block this bond describes
      if (s.n > 2 * m || s.s2 > std::min(s.n, 2 * m - s.n))
        return fail(DMRG_ERR_SYMMETRY, "dmrg_set_mps: sector impossible for its block");
      if (bonds[b].find(s.n, s.s2) >= 0) return fail(DMRG_ERR_SHAPE, "dmrg_set_mps: duplicate sector");
      bonds[b].secs.push_back(s);
    }
    if (b == k + 1 && counts[b] != 0) return fail(DMRG_ERR_SHAPE, "dmrg_set_mps: bond k+1 must be empty");
  }
  auto is_vac = [](const Bond& bd) {
    return bd.secs.size() == 1 && bd.secs[0].n == 0 && bd.secs[0].s2 == 0 && bd.secs[0].dim == 1;
  };
  if (!is_vac(bonds[0]) || !is_vac(bonds[n])) return fail(DMRG_ERR_SHAPE, "dmrg_set_mps: bonds 0 and n must be (0,0,1)");
  // ---- site tensors
  std::vector<SiteTensor> sites(n);
  long long need = 0;
  for (int j = 0; j < n; ++j) {
    if (j == k || j == k + 1) continue;
    SiteTensor& T = sites[j];
    T.left = j < k;
    T.j = j;
    const Bond& b0 = bonds[j];
    const Bond& b1 = bonds[j + 1];
    int64_t off = 0;
    for (size_t i0 = 0; i0 < b0.secs.size(); ++i0)
      for (int sig = 0; sig < 3; ++sig)
        for (size_t i1 = 0; i1 < b1.secs.size(); ++i1) {
          const Sector &s0 = b0.secs[i0], &s1 = b1.secs[i1];
          bool ok = T.left ? (s1.n == s0.n + kLocN[sig] && tri2(s0.s2, kLocS2[sig], s1.s2))
                           : (s0.n == kLocN[sig] + s1.n && tri2(kLocS2[sig], s1.s2, s0.s2));
          if (!ok) continue;
          T.find[{(int)i0, sig, (int)i1}] = (int)T.blocks.size();
          T.blocks.push_back(SiteTensor::Blk{(int)i0, sig, (int)i1, off, s0.dim, s1.dim});
          off += (int64_t)s0.dim * s1.dim;
        }
    need += off;
  }
  if (need != n_values) return fail(DMRG_ERR_SHAPE, "dmrg_set_mps: number of tensor values does not match the sectors");
  if (!finite_all(blocks, (size_t)n_values)) return fail(DMRG_ERR_NONFINITE, "dmrg_set_mps: non-finite tensor value");
  try {
    c->reset_plan();
    C.Lblk.reset();
    C.Rblk.reset();
    for (auto& T : C.sites) C.free_buf(T.buf);
    C.k = k;
    C.bonds = bonds;
    const double* src = blocks;
    for (int j = 0; j < n; ++j) {
      if (j == k || j == k + 1) continue;
      int64_t sz = 0;
      for (auto& bl : sites[j].blocks) sz += (int64_t)bl.rows * bl.cols;
      sites[j].buf = C.new_buf(std::max<int64_t>(sz, 1));
      if (sz) C.ex->upload(C.ptr(sites[j].buf), src, (size_t)sz * 8);
      src += sz;
    }
    C.sites = std::move(sites);
    // ---- operator blocks
    const bool verbose = std::getenv("DMRG_VERBOSE") != nullptr;
    auto t_start = std::chrono::steady_clock::now();
    auto progress = [&](const char* side, int b, const Block& blk) {
      if (!verbose) return;
      double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      std::fprintf(stderr, "[dmrg] %s block at bond %d: %.2f GB, %.1f s | %s\n", side, b, blk.bytes_f64() / 1e9, s,
                   c->ex->host_profile().c_str());
      std::fflush(stderr);
    };
    // keep_blocks 1: every bond; m >= 2: the m bonds nearest the block on each
    // side; -m <= -2: the m nearest on the right side only
    const int kb = c->opts.keep_blocks;
    auto keep_left = [&](int bond) { return kb == 1 || (kb >= 2 && bond >= k - kb); };
    auto keep_right = [&](int bond) { return kb == 1 || (kb >= 2 && bond <= k + 2 + kb) || (kb <= -2 && bond <= k + 2 - kb); };
    for (auto& h : C.Lhist)
      if (h) C.free_block(*h);
    for (auto& h : C.Rhist)
      if (h) C.free_block(*h);
    C.Lhist.clear();
    C.Rhist.clear();
    C.Lhist.resize(n + 1);
    C.Rhist.resize(n + 1);
    auto L = C.vacuum_left();
    for (int j = 0; j < k; ++j) {
      auto N = C.grow_left(*L, C.sites[j], C.bonds[j + 1]);
      if (keep_left(j)) C.Lhist[j] = std::move(L);
      else C.free_block(*L);
      L = std::move(N);
      progress("left", j + 1, *L);
    }
    auto R = C.vacuum_right();
    for (int j = n - 1; j >= k + 2; --j) {
      auto N = C.grow_right(*R, C.sites[j], C.bonds[j]);
      if (keep_right(j + 1)) C.Rhist[j + 1] = std::move(R);
      else C.free_block(*R);
      R = std::move(N);
      progress("right", j, *R);
    }
    C.Lblk = std::move(L);
    C.Rblk = std::move(R);
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_set_mps: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_set_mps: ") + e.what());
  }
}

extern "C" int dmrg_psi_layout(dmrg_ctx* c, int k, long long* nsb, long long* desc, long long* nel) {
  if (!c || !nsb || !nel) return fail(DMRG_ERR_ARG, "dmrg_psi_layout: null argument");
  if (!c->C->Lblk || k != c->C->k) return fail(DMRG_ERR_ARG, "dmrg_psi_layout: no MPS loaded at this k");
  try {
    c->ensure_plan();
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_psi_layout: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_psi_layout: ") + e.what());
  }
  const PsiLayout& lay = c->plan->lay;
  *nsb = (long long)lay.sbs.size();
  *nel = lay.size;
  if (desc)
    for (size_t i = 0; i < lay.sbs.size(); ++i) {
      const auto& s = lay.sbs[i];
      long long* d = desc + 7 * i;
      d[0] = s.an; d[1] = s.as2; d[2] = s.cn; d[3] = s.cs2; d[4] = s.nrows; d[5] = s.ncols; d[6] = s.off;
    }
  return DMRG_OK;
}

extern "C" int dmrg_hpsi(dmrg_ctx* c, int k, const double* in, double* out, int prec, double* flops) {
  if (!c || !in || !out) return fail(DMRG_ERR_ARG, "dmrg_hpsi: null argument");
  if (!c->C->Lblk || k != c->C->k) return fail(DMRG_ERR_ARG, "dmrg_hpsi: no MPS loaded at this k");
  if (prec < 0 || prec > 3) return fail(DMRG_ERR_ARG, "dmrg_hpsi: bad precision");
  try {
    c->ensure_plan();
    const int64_t n = c->plan->lay.size;
    if (!finite_all(in, (size_t)n)) return fail(DMRG_ERR_NONFINITE, "dmrg_hpsi: non-finite input");
    c->C->ex->upload(c->C->ptr(c->b_in), in, (size_t)n * 8);
    c->hpsi_device(prec);
    c->C->ex->download(out, c->C->ptr(c->b_out), (size_t)n * 8);
    if (flops) *flops = c->plan->flops;
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_hpsi: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_hpsi: ") + e.what());
  }
}

extern "C" int dmrg_hpsi_dev(dmrg_ctx* c, int k, const void* din, void* dout, int prec) {
  if (!c || !din || !dout) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev: null argument");
  if (!c->C->Lblk || k != c->C->k) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev: no MPS loaded at this k");
  if (prec < 0 || prec > 3) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev: bad precision");
  try {
    c->ensure_plan();
    const int64_t n = c->plan->lay.size;
    c->C->ex->copy_d2d(c->C->ptr(c->b_in), din, (size_t)n * 8);
    c->hpsi_device(prec);
    c->C->ex->copy_d2d(dout, c->C->ptr(c->b_out), (size_t)n * 8);
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_hpsi_dev: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_hpsi_dev: ") + e.what());
  }
}

extern "C" int dmrg_hpsi_dev_stream(dmrg_ctx* c, int k, const void* din, void* dout, int prec, void* hip_stream) {
  if (!c || !din || !dout) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_stream: null argument");
  if (!c->C->Lblk || k != c->C->k) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_stream: no MPS loaded at this k");
  if (prec < 0 || prec > 3) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_stream: bad precision");
  try {
    c->ensure_plan();
    const int64_t n = c->plan->lay.size;
    c->ex->wait_for(hip_stream);  // d_in may still be written by the caller's queued work
    c->ex->copy_d2d(c->C->ptr(c->b_in), din, (size_t)n * 8);
    c->hpsi_device(prec, false);  // queued only: no host wait
    c->ex->copy_d2d(dout, c->C->ptr(c->b_out), (size_t)n * 8);
    c->ex->signal(hip_stream);  // the caller's later work on the stream sees d_out
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_hpsi_dev_stream: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_hpsi_dev_stream: ") + e.what());
  }
}

extern "C" int dmrg_hpsi_dev_noalloc(dmrg_ctx* c, int k, const void* din, void* dout, int prec) {
  if (!c || !din || !dout) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_noalloc: null argument");
  if (!c->C->Lblk || k != c->C->k) return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_noalloc: no MPS loaded at this k");
  if (prec < 0 || prec > 2)
    return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_noalloc: bad precision (FP64, FP32 or BF16; FP8 needs dmrg_hpsi_dev)");
  if (!c->plan)
    return fail(DMRG_ERR_ARG,
                "dmrg_hpsi_dev_noalloc: no H*psi plan at this block yet (dmrg_psi_layout or an H*psi call makes it)");
  if (!c->operators_ready(prec))
    return fail(DMRG_ERR_ARG, "dmrg_hpsi_dev_noalloc: the operator blocks have no copies in this precision yet "
                              "(an H*psi or Davidson call with it makes them)");
  try {
    c->hpsi_fixed(din, dout, prec);
    return DMRG_OK;
  } catch (const dmrg_ctx::FixedTooSmall& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_hpsi_dev_noalloc: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_hpsi_dev_noalloc: ") + e.what());
  }
}

extern "C" int dmrg_heff_diag(dmrg_ctx* c, int k, double* diag) {
  if (!c || !diag) return fail(DMRG_ERR_ARG, "dmrg_heff_diag: null argument");
  if (!c->C->Lblk || k != c->C->k) return fail(DMRG_ERR_ARG, "dmrg_heff_diag: no MPS loaded at this k");
  try {
    c->ensure_plan();
    c->ex->download(diag, c->C->ptr(c->b_diag), (size_t)c->plan->lay.size * 8);
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_heff_diag: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_heff_diag: ") + e.what());
  }
}

extern "C" int dmrg_kernel_timing(dmrg_ctx* c, int mode, double* ms, long long* launches) {
  if (!c) return fail(DMRG_ERR_ARG, "dmrg_kernel_timing: null context");
  try {
    if (mode == 1) {
      c->ex->timing(true);
    } else {
      auto kt = c->ex->kernel_time();
      if (ms) *ms = kt.first;
      if (launches) *launches = kt.second;
      if (mode == 0) c->ex->timing(false);
    }
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("dmrg_kernel_timing: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("dmrg_kernel_timing: ") + e.what());
  }
}

extern "C" int dmrg_gemm_selftest(int m, int n, int k, const double* A, int ta, int ia, const double* B, int tb,
                                  int ib, double alpha, double beta, double* C, int prec) {
  if (m <= 0 || n <= 0 || k <= 0 || !C || (!ia && !A) || (!ib && !B)) return fail(DMRG_ERR_ARG, "gemm_selftest: bad args");
  if ((ia && k != m) || (ib && k != n)) return fail(DMRG_ERR_SHAPE, "gemm_selftest: identity needs k == m / n");
  if (prec < 0 || prec > 3) return fail(DMRG_ERR_ARG, "gemm_selftest: bad precision");
  if (prec == DMRG_FP8 && ((!ia && !(ta & 2)) || (!ib && !(tb & 2))))
    return fail(DMRG_ERR_ARG, "gemm_selftest: FP8 operands must be stored padded (bit 1 of trans)");
  try {
    std::unique_ptr<Executor> ex(make_hip_executor());
    const int dt = prec == DMRG_FP64 ? DT_F64 : prec == DMRG_FP32 ? DT_F32 : prec == DMRG_FP8 ? DT_FP8 : DT_BF16;
    const int dc = prec == DMRG_FP64 ? DT_F64 : DT_F32;
    double fp8_scale = 1.0;  // product of the operands' FP8 scales
    auto put = [&](const double* h, size_t cnt, int d) -> void* {
      void* p64 = ex->alloc(cnt * 8);
      ex->upload(p64, h, cnt * 8);
      if (d == DT_F64) return p64;
      if (d == DT_FP8) {  // one power-of-two scale for the whole operand
        double* sc = (double*)ex->alloc(2 * sizeof(double));
        ex->fp8_scales((const double*)p64, 1, (int64_t)cnt, sc);
        void* p = ex->alloc(cnt);
        ex->to_fp8(p, (const double*)p64, (int64_t)cnt, (int64_t)cnt, sc);
        double hs[2];
        ex->download(hs, sc, sizeof hs);
        fp8_scale *= hs[0];
        ex->release(sc);
        ex->release(p64);
        return p;
      }
      void* p = ex->alloc(cnt * dtype_size(d));
      ex->convert(p, d, p64, DT_F64, cnt);
      ex->sync();
      ex->release(p64);
      return p;
    };
    // bit 1 of ta / tb: store the operand with rows padded to a multiple of 8
    // elements, padding filled with NaN, and flag it as padded
    const bool pa = (ta & 2) != 0, pb = (tb & 2) != 0;
    ta &= 1;
    tb &= 1;
    auto padded = [](const double* h, int rows, int cols, int ld) {
      std::vector<double> v((size_t)rows * ld, std::numeric_limits<double>::quiet_NaN());
      for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) v[(size_t)r * ld + c] = h[(size_t)r * cols + c];
      return v;
    };
    const int rA = ta ? k : m, cA = ta ? m : k, rB = tb ? n : k, cB = tb ? k : n;
    const int ldA = pa ? (cA + 7) / 8 * 8 : cA, ldB = pb ? (cB + 7) / 8 * 8 : cB;
    std::vector<double> hA, hB;
    if (!ia) hA = pa ? padded(A, rA, cA, ldA) : std::vector<double>(A, A + (size_t)m * k);
    if (!ib) hB = pb ? padded(B, rB, cB, ldB) : std::vector<double>(B, B + (size_t)k * n);
    void* dA = ia ? nullptr : put(hA.data(), hA.size(), dt);
    void* dB = ib ? nullptr : put(hB.data(), hB.size(), dt);
    std::vector<double> cb((size_t)m * n);
    for (size_t i = 0; i < cb.size(); ++i) cb[i] = beta * C[i];
    void* dC = put(cb.data(), cb.size(), dc);
    alpha *= fp8_scale;
    RawJob j{dC, m, n, n, 1, 0, 0, 1};
    RawTerm t{dA, dB, ldA, ldB, k,
              (ta ? TF_TRANS_A : 0) | (tb ? TF_TRANS_B : 0) | (ia ? TF_IDENT_A : 0) | (ib ? TF_IDENT_B : 0) |
                  (pa ? TF_PAD_A : 0) | (pb ? TF_PAD_B : 0),
              alpha};
    void* h = ex->prepare({j}, {t}, dt, dt, dc);
    ex->run(h);
    ex->sync();
    ex->drop(h);
    void* c64 = dC;
    if (dc != DT_F64) {
      c64 = ex->alloc(cb.size() * 8);
      ex->convert(c64, DT_F64, dC, dc, cb.size());
      ex->sync();
    }
    ex->download(C, c64, cb.size() * 8);
    for (void* p : {dA, dB, dC}) if (p) ex->release(p);
    if (c64 != dC) ex->release(c64);
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return fail(DMRG_ERR_BUDGET, std::string("gemm_selftest: ") + e.what());
  } catch (const std::exception& e) {
    return fail(DMRG_ERR_HIP, std::string("gemm_selftest: ") + e.what());
  }
}

extern "C" int dmrg_su2_coefficient(int kind, const int* two_j, double* value) {
  if (!two_j || !value) return fail(DMRG_ERR_ARG, "dmrg_su2_coefficient: null argument");
  for (int i = 0; i < (kind == 2 ? 9 : 6); ++i)
    if (two_j[i] < 0 && !(kind == 0 && (i == 1 || i == 3 || i == 5)))
      return fail(DMRG_ERR_ARG, "dmrg_su2_coefficient: negative spin");
  if (kind == 0) *value = cg2(two_j[0], two_j[1], two_j[2], two_j[3], two_j[4], two_j[5]);
  else if (kind == 1) *value = sixj2(two_j[0], two_j[1], two_j[2], two_j[3], two_j[4], two_j[5]);
  else if (kind == 2)
    *value = ninej2(two_j[0], two_j[1], two_j[2], two_j[3], two_j[4], two_j[5], two_j[6], two_j[7], two_j[8]);
  else return fail(DMRG_ERR_ARG, "dmrg_su2_coefficient: kind must be 0 (CG), 1 (6j) or 2 (9j)");
  return DMRG_OK;
}

extern "C" int dmrg_tuner_report(dmrg_ctx* c, char* buf, int capacity) {
  if (!c || !buf || capacity < 1) return fail(DMRG_ERR_ARG, "dmrg_tuner_report: null argument or no capacity");
  const std::string r = c->ex->tuner_report();
  std::snprintf(buf, (size_t)capacity, "%s", r.c_str());
  return (int)r.size() < capacity ? DMRG_OK : fail(DMRG_ERR_ARG, "dmrg_tuner_report: buffer too small");
}

extern "C" int dmrg_stats(dmrg_ctx* c, double* out, int n) {
  if (!c || !out) return fail(DMRG_ERR_ARG, "dmrg_stats: null argument");
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  if (c->plan) {
    v[0] = c->plan->flops;
    v[3] = (double)c->plan->terms.size();
    v[4] = (double)c->plan->n_stage_terms;
    v[5] = c->plan->flops_exec;
    v[6] = c->plan->flops_dense;
  }
  if (c->C->Lblk) v[1] = (double)(c->C->Lblk->bytes_f64() + c->C->Rblk->bytes_f64());
  v[2] = (double)c->C->peak_bytes;
  for (int i = 0; i < n && i < 7; ++i) out[i] = v[i];
  return DMRG_OK;
}
