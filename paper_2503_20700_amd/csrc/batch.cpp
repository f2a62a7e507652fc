// Batched H*psi over independent DMRG contexts: the stage-L task lists of all
// contexts (chunk by chunk) become one grouped launch, and likewise stage R,
// so many small instances share the GPU in a single launch per stage instead
// of one small launch each.  The batched Davidson runs every context's own
// solver on a host thread of its own and gathers their matvecs into those
// launches.
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dmrg.h"
#include "session.hpp"

using namespace dmrg;

namespace {
struct Merged {
  std::vector<void*> stageL, stageR;  // merged launches per chunk index
};
}  // namespace

struct dmrg_batch {
  std::vector<dmrg_ctx*> ctx;
  std::vector<long long> serial;  // plan of each context the launches were built for
  int prec = DMRG_FP64;           // precision of dmrg_batch_hpsi
  Executor* ex = nullptr;         // the first context's executor runs the batch
  std::map<int, Merged> merged;   // by precision, built on first use
};

namespace {
void drop_all(dmrg_batch* b) {
  for (auto& kv : b->merged) {
    for (void* h : kv.second.stageL) b->ex->drop(h);
    for (void* h : kv.second.stageR) b->ex->drop(h);
  }
  b->merged.clear();
}

// Concatenate the resolved task lists of chunk c of every context.
void merge(dmrg_batch* b, Merged& M, size_t c, bool left, int dta, int dtb, int dtc) {
  std::vector<RawJob> jobs, j;
  std::vector<RawTerm> terms, t;
  for (dmrg_ctx* x : b->ctx) {
    if (c >= x->plan->chunks.size()) continue;
    x->bind();
    const auto& ch = x->plan->chunks[c];
    x->C->resolve(left ? ch.stageL : ch.stageR, j, t, dta, dtb, dtc);
    const int64_t base = (int64_t)terms.size();
    for (RawJob& r : j) {
      r.tbeg += base;
      r.tend += base;
    }
    jobs.insert(jobs.end(), j.begin(), j.end());
    terms.insert(terms.end(), t.begin(), t.end());
  }
  void* h = b->ex->prepare_tuned(jobs, terms, dta, dtb, dtc);
  (left ? M.stageL : M.stageR).push_back(h);
}

// The merged launches of precision prec (plans and storage types made ready
// for every context).
Merged& merged_for(dmrg_batch* b, int prec) {
  auto it = b->merged.find(prec);
  if (it != b->merged.end()) return it->second;
  size_t nchunks = 0;
  for (dmrg_ctx* x : b->ctx) {
    x->ready_dtypes(prec);
    x->ex->sync();
    nchunks = std::max(nchunks, x->plan->chunks.size());
  }
  Merged& M = b->merged[prec];
  const int od = dmrg_ctx::op_dt(prec), xd = dmrg_ctx::x_dt(prec), outd = dmrg_ctx::out_dt(prec);
  for (size_t c = 0; c < nchunks; ++c) {
    merge(b, M, c, true, od, od, xd);
    merge(b, M, c, false, xd, od, outd);
  }
  return M;
}

bool stale(const dmrg_batch* b) {
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (!b->ctx[i]->plan || b->ctx[i]->plan_serial != b->serial[i]) return true;
  return false;
}

// y_i = H_i x_i for every i with in[i] != nullptr (device FP64 vectors); the
// merged launches compute every context, the others on stale inputs.
void run_merged(dmrg_batch* b, int prec, const std::vector<const void*>& in, const std::vector<void*>& out) {
  Merged& M = merged_for(b, prec);
  Executor* ex = b->ex;
  const int od = dmrg_ctx::op_dt(prec), outd = dmrg_ctx::out_dt(prec);
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    if (!in[i]) continue;
    dmrg_ctx* x = b->ctx[i];
    x->ex->sync();  // x_i was written on the context's own stream
    const int64_t n = x->plan->lay.size;
    Context& C = *x->C;
    ex->copy_d2d(C.ptr(x->b_in), in[i], (size_t)n * 8);
    x->begin_hpsi(ex, prec);
  }
  for (size_t c = 0; c < M.stageL.size(); ++c) {
    ex->run(M.stageL[c]);
    ex->run(M.stageR[c]);
  }
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    if (!in[i]) continue;
    dmrg_ctx* x = b->ctx[i];
    const int64_t n = x->plan->lay.size;
    Context& C = *x->C;
    x->end_hpsi(ex, prec);
    ex->copy_d2d(out[i], C.ptr(x->b_out), (size_t)n * 8);
  }
  ex->sync();
}

// Rendezvous of the batched Davidson: each worker posts its matvec and
// waits; the worker whose post (or exit) completes the set of active workers
// runs the merged launches for all posted matvecs and wakes the others.
struct Rendezvous {
  static constexpr double kMergedShare = 0.5;
  std::mutex mu;
  std::condition_variable cv;
  dmrg_batch* b = nullptr;
  int active = 0;
  long long generation = 0;
  struct Req {
    const double* x;
    double* y;
    int prec;
  };
  std::vector<Req> req;       // by context index
  std::vector<char> posted;
  int nposted = 0;
  std::string error;          // first failure of a merged launch

  // with mu held: run every posted matvec, clear the posts, wake the waiters.
  // Per precision, the merged launch computes every context, so it runs
  // only when the posting contexts carry most of its flops; a few posts
  // (solvers in another phase, or nearly all finished) run as their own
  // H*psi instead.
  void flush() {
    std::map<int, std::pair<std::vector<const void*>, std::vector<void*>>> by_prec;
    std::map<int, double> posted_flops;
    const size_t n = b->ctx.size();
    double all_flops = 0.0;
    for (size_t i = 0; i < n; ++i) {
      all_flops += b->ctx[i]->plan->flops;
      if (!posted[i]) continue;
      auto& v = by_prec[req[i].prec];
      if (v.first.empty()) {
        v.first.assign(n, nullptr);
        v.second.assign(n, nullptr);
      }
      v.first[i] = req[i].x;
      v.second[i] = req[i].y;
      posted_flops[req[i].prec] += b->ctx[i]->plan->flops;
    }
    try {
      for (auto& kv : by_prec) {
        if (posted_flops[kv.first] >= kMergedShare * all_flops) {
          run_merged(b, kv.first, kv.second.first, kv.second.second);
          continue;
        }
        for (size_t i = 0; i < n; ++i) {
          if (!kv.second.first[i]) continue;
          dmrg_ctx* x = b->ctx[i];
          const int64_t len = x->plan->lay.size;
          x->ex->copy_d2d(x->C->ptr(x->b_in), kv.second.first[i], (size_t)len * 8);
          x->hpsi_device(kv.first);
          x->ex->copy_d2d(kv.second.second[i], x->C->ptr(x->b_out), (size_t)len * 8);
          x->ex->sync();
        }
      }
    } catch (const std::exception& e) {
      if (error.empty()) error = e.what();
    }
    std::fill(posted.begin(), posted.end(), 0);
    nposted = 0;
    ++generation;
    cv.notify_all();
  }

  void matvec(size_t i, const double* x, double* y, int prec) {
    std::unique_lock<std::mutex> lk(mu);
    req[i] = Req{x, y, prec};
    posted[i] = 1;
    ++nposted;
    const long long g = generation;
    if (nposted == active) flush();
    else cv.wait(lk, [&] { return generation != g; });
    if (!error.empty()) throw std::runtime_error("batched matvec: " + error);
  }

  void leave() {
    std::lock_guard<std::mutex> lk(mu);
    --active;
    if (active > 0 && nposted == active) flush();
  }
};
}  // namespace

extern "C" int dmrg_batch_create(dmrg_ctx* const* ctxs, int count, int prec, dmrg_batch** out) {
  if (!ctxs || !out || count < 1) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: bad arguments");
  if (prec < 0 || prec > 3) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: bad precision");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: null context");
    if (!ctxs[i]->C->Lblk) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: context without an MPS");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: context listed twice");
  }
  auto b = std::make_unique<dmrg_batch>();
  b->ctx.assign(ctxs, ctxs + count);
  b->prec = prec;
  b->ex = ctxs[0]->ex.get();
  try {
    for (dmrg_ctx* x : b->ctx) {
      x->ensure_plan();
      b->serial.push_back(x->plan_serial);
    }
    merged_for(b.get(), prec);
    *out = b.release();
    return DMRG_OK;
  } catch (const std::bad_alloc&) {
    drop_all(b.get());
    return dmrg_fail(DMRG_ERR_BUDGET, "dmrg_batch_create: out of memory");
  } catch (const std::exception& e) {
    drop_all(b.get());
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_batch_create: ") + e.what());
  }
}

extern "C" int dmrg_batch_hpsi(dmrg_batch* b, const void* const* d_in, void* const* d_out) {
  if (!b || !d_in || !d_out) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_hpsi: null argument");
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (!d_in[i] || !d_out[i]) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_hpsi: null vector");
  if (stale(b)) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_hpsi: a context changed since the batch was made");
  try {
    run_merged(b, b->prec, std::vector<const void*>(d_in, d_in + b->ctx.size()),
               std::vector<void*>(d_out, d_out + b->ctx.size()));
    return DMRG_OK;
  } catch (const std::bad_alloc& e) {
    return dmrg_fail(DMRG_ERR_BUDGET, std::string("dmrg_batch_hpsi: ") + e.what());
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_batch_hpsi: ") + e.what());
  }
}

extern "C" int dmrg_batch_davidson(dmrg_batch* b, double* const* psi, double* energy, double* resid,
                                   int* n_matvec_lowprec, int* n_matvec_fp64, int* status) {
  if (!b || !psi || !energy || !resid || !status) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_davidson: null argument");
  const size_t n = b->ctx.size();
  for (size_t i = 0; i < n; ++i)
    if (!psi[i]) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_davidson: null vector");
  if (stale(b)) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_davidson: a context changed since the batch was made");
  try {
    // the merged launches every phase can ask for, built before the threads start
    for (dmrg_ctx* x : b->ctx) {
      merged_for(b, x->opts.hpsi_prec);
      if (x->opts.davidson_mid_fp32 && (x->opts.hpsi_prec == DMRG_BF16 || x->opts.hpsi_prec == DMRG_FP8))
        merged_for(b, DMRG_FP32);
      merged_for(b, DMRG_FP64);
    }
  } catch (const std::bad_alloc& e) {
    return dmrg_fail(DMRG_ERR_BUDGET, std::string("dmrg_batch_davidson: ") + e.what());
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_batch_davidson: ") + e.what());
  }
  Rendezvous rv;
  rv.b = b;
  rv.active = (int)n;
  rv.req.resize(n);
  rv.posted.assign(n, 0);
  std::vector<std::string> msg(n);
  std::vector<std::thread> th;
  for (size_t i = 0; i < n; ++i) {
    th.emplace_back([&, i] {
      dmrg_ctx* x = b->ctx[i];
      x->mv_hook = [&rv, i](const double* xv, double* yv, int prec) { rv.matvec(i, xv, yv, prec); };
      int lo = 0, hi = 0;
      status[i] = davidson_core(x, psi[i], &energy[i], &resid[i], &lo, &hi);
      if (status[i] != DMRG_OK) msg[i] = dmrg_last_error();
      x->mv_hook = nullptr;
      if (n_matvec_lowprec) n_matvec_lowprec[i] = lo;
      if (n_matvec_fp64) n_matvec_fp64[i] = hi;
      rv.leave();
    });
  }
  for (auto& t : th) t.join();
  int rc = DMRG_OK;
  std::string first;
  for (size_t i = 0; i < n; ++i) {
    if (status[i] == DMRG_OK) continue;
    if (rc == DMRG_OK || (rc == DMRG_ERR_NOCONV && status[i] != DMRG_ERR_NOCONV)) {
      rc = status[i];
      first = "instance " + std::to_string(i) + ": " + msg[i];
    }
  }
  if (rc != DMRG_OK) return dmrg_fail(rc, "dmrg_batch_davidson: " + first);
  return DMRG_OK;
}

extern "C" void dmrg_batch_destroy(dmrg_batch* b) {
  if (!b) return;
  try {
    drop_all(b);
  } catch (...) {
  }
  delete b;
}
