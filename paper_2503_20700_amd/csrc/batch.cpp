// Batched H*psi over independent DMRG contexts: the stage-L task lists of all
// contexts (chunk by chunk) become one grouped launch, and likewise stage R,
// so many small instances share the GPU in a single launch per stage instead
// of one small launch each.
#include <memory>
#include <string>
#include <vector>

#include "../../include/dmrg.h"
#include "session.hpp"

using namespace dmrg;

struct dmrg_batch {
  std::vector<dmrg_ctx*> ctx;
  std::vector<long long> serial;      // plan of each context the launches were built for
  int prec = DMRG_FP64;
  Executor* ex = nullptr;             // the first context's executor runs the batch
  std::vector<void*> stageL, stageR;  // merged launches per chunk index
};

namespace {
void drop_all(dmrg_batch* b) {
  for (void* h : b->stageL) b->ex->drop(h);
  for (void* h : b->stageR) b->ex->drop(h);
  b->stageL.clear();
  b->stageR.clear();
}

// Concatenate the resolved task lists of chunk c of every context.
void merge(dmrg_batch* b, size_t c, bool left, int dta, int dtb, int dtc) {
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
  void* h = b->ex->prepare(jobs, terms, dta, dtb, dtc);
  (left ? b->stageL : b->stageR).push_back(h);
}
}  // namespace

extern "C" int dmrg_batch_create(dmrg_ctx* const* ctxs, int count, int prec, dmrg_batch** out) {
  if (!ctxs || !out || count < 1) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: bad arguments");
  if (prec < 0 || prec > 2) return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_create: bad precision");
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
    size_t nchunks = 0;
    for (dmrg_ctx* x : b->ctx) {
      x->ensure_plan();
      x->ready_dtypes(prec);
      x->ex->sync();
      nchunks = std::max(nchunks, x->plan->chunks.size());
      b->serial.push_back(x->plan_serial);
    }
    const int od = dmrg_ctx::op_dt(prec), outd = dmrg_ctx::out_dt(prec);
    for (size_t c = 0; c < nchunks; ++c) {
      merge(b.get(), c, true, od, od, od);
      merge(b.get(), c, false, od, od, outd);
    }
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
  try {
    Executor* ex = b->ex;
    const int od = dmrg_ctx::op_dt(b->prec), outd = dmrg_ctx::out_dt(b->prec);
    for (size_t i = 0; i < b->ctx.size(); ++i) {
      dmrg_ctx* x = b->ctx[i];
      if (!x->plan || x->plan_serial != b->serial[i])
        return dmrg_fail(DMRG_ERR_ARG, "dmrg_batch_hpsi: a context changed since the batch was made");
      x->ex->sync();
      const int64_t n = x->plan->lay.size;
      Context& C = *x->C;
      ex->copy_d2d(C.ptr(x->b_in), d_in[i], (size_t)n * 8);
      ex->pack(C.ptr(x->b_inp, od), od, (const double*)C.ptr(x->b_in), (const int*)x->d_pidx,
               (size_t)x->plan->lay.psize);
      ex->zero(C.ptr(x->b_out, outd), (size_t)n * dtype_size(outd));
    }
    for (size_t c = 0; c < b->stageL.size(); ++c) {
      ex->run(b->stageL[c]);
      ex->run(b->stageR[c]);
    }
    for (size_t i = 0; i < b->ctx.size(); ++i) {
      dmrg_ctx* x = b->ctx[i];
      const int64_t n = x->plan->lay.size;
      Context& C = *x->C;
      if (outd != DT_F64) ex->convert(C.ptr(x->b_out), DT_F64, C.ptr(x->b_out, outd), outd, (size_t)n);
      ex->copy_d2d(d_out[i], C.ptr(x->b_out), (size_t)n * 8);
    }
    ex->sync();
    return DMRG_OK;
  } catch (const std::exception& e) {
    return dmrg_fail(DMRG_ERR_HIP, std::string("dmrg_batch_hpsi: ") + e.what());
  }
}

extern "C" void dmrg_batch_destroy(dmrg_batch* b) {
  if (!b) return;
  try {
    drop_all(b);
  } catch (...) {
  }
  delete b;
}
