// Per-context state behind the C ABI: executor, planner context, the H*psi
// plan of the current two-site block and its device buffers.
#pragma once
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <stdexcept>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dmrg.h"
#include "planner.hpp"

// Record the thread-local error message returned by dmrg_last_error().
int dmrg_fail(int code, const std::string& msg);

struct dmrg_ctx;
// The Davidson solve of dmrg_davidson_step at the context's current block
// (argument checks done by the caller); returns a dmrg error code.
int davidson_core(dmrg_ctx* c, double* psi, double* energy, double* resid, int* nlo, int* nhi);
// Appends one JSON object (without newline) as a line to the file that the
// environment variable DMRG_LOG names; nothing if it is unset.
void step_log(const std::string& json);

// psi_in, psi_out, X, ones, diag and padded-psi_in placeholders used by the
// H*psi task lists
// (PH_OUTP: psi' accumulated with rows in the internal order, gathered into
// PH_OUT at the end)
enum { PH_IN = 1, PH_OUT = 2, PH_X = 3, PH_ONES = 4, PH_DIAG = 5, PH_INP = 6, PH_OUTP = 7 };

struct dmrg_ctx {
  dmrg_opts opts{};
  std::unique_ptr<dmrg::Executor> ex;
  std::unique_ptr<dmrg::Context> C;
  std::unique_ptr<dmrg::HpsiPlan> plan;
  int b_in = -1, b_out = -1, b_x = -1, b_ones = -1, b_diag = -1, b_inp = -1, b_outp = -1;
  void* d_pidx = nullptr;  // padded psi index -> caller index (int32, -1 = padding)
  void* d_uidx = nullptr;  // caller index -> index in b_outp (int32)
  double* d_pscale = nullptr;  // (s, 1/s) of the FP8 copy of psi_in
  long long plan_serial = 0;  // bumped whenever a new H*psi plan is made
  // host seconds of the last H*psi plan, and of the task-list preparations
  // (incl. tile tuning) per precision since the step log last reported them
  double plan_seconds = 0.0, prepare_seconds[4] = {0.0, 0.0, 0.0, 0.0};
  // start vector carried by the last truncation to the block it moved to
  std::vector<double> guess;
  int guess_k = -1;
  // When set, the Davidson's matvecs y = H x (device FP64 vectors of the
  // plan's length) go through this instead of hpsi_device: the batched
  // Davidson gathers them into one grouped launch for several contexts.
  std::function<void(const double* x, double* y, int prec)> mv_hook;
  struct Prepared {
    std::vector<void*> L, R;
    bool ready = false;
    void* graph = nullptr;     // recorded H*psi sequence (opts.hpsi_graph)
    long long graph_gen = -1;  // executor scratch generation it was recorded at
  };
  Prepared prep[4];
  // cut spectrum of the last truncation
  std::vector<double> cut_values;
  std::vector<int> cut_spins;
  // Davidson workspace: basis V, images W (mmax x n each), x, Hx, r, t
  std::vector<int> work_bufs;
  int64_t work_n = 0;
  int work_mmax = 0;
  // Davidson iteration sequences recorded as graphs (opts.davidson_graph),
  // keyed by (precision, basis size, part); they hold the addresses of the
  // workspace and of the H*psi buffers, and are valid while both stay and
  // the executor's scratch generation is dav_gen.
  std::map<int, void*> dav_graphs;
  long long dav_gen = -1;
  void drop_dav_graphs() {
    for (auto& g : dav_graphs) ex->drop_graph(g.second);
    dav_graphs.clear();
    dav_gen = -1;
  }

  ~dmrg_ctx() {
    reset_plan();
    C.reset();
    ex.reset();
  }

  int64_t budget() const {
    // default 2^32 elements of X per chunk: 46 chunks at CAS(82,82) D=4096
    // (8.6 GB in BF16, 34 GB in FP64); 2^30 gave 182 launches and 3 % more
    // time, 2^33 and 2^34 longer launch tails
    return opts.work_budget_elems > 0 ? (int64_t)opts.work_budget_elems : ((int64_t)1 << 32);
  }

  void reset_plan() {
    drop_dav_graphs();
    for (auto& p : prep) {
      ex->drop_graph(p.graph);
      p.graph = nullptr;
      p.graph_gen = -1;
      for (void* h : p.L) ex->drop(h);
      for (void* h : p.R) ex->drop(h);
      p.L.clear();
      p.R.clear();
      p.ready = false;
    }
    if (C) {
      for (int b : work_bufs) C->free_buf(b);
      work_bufs.clear();
      work_n = 0;
      work_mmax = 0;
      for (int b : {b_in, b_out, b_x, b_ones, b_diag, b_inp, b_outp}) C->free_buf(b);
      if (d_pidx) ex->release(d_pidx);
      d_pidx = nullptr;
      if (d_uidx) ex->release(d_uidx);
      d_uidx = nullptr;
      if (d_pscale) ex->release(d_pscale);
      d_pscale = nullptr;
      if (C->Lblk) {
        for (auto& t : C->Lblk->tmp) C->free_buf(t.buf);
        C->Lblk->tmp.clear();
      }
      if (C->Rblk) {
        for (auto& t : C->Rblk->tmp) C->free_buf(t.buf);
        C->Rblk->tmp.clear();
      }
    }
    b_in = b_out = b_x = b_ones = b_diag = b_inp = b_outp = -1;
    plan.reset();
  }

  void bind() {
    C->ph[PH_IN] = b_in;
    C->ph[PH_OUT] = b_out;
    C->ph[PH_X] = b_x;
    C->ph[PH_ONES] = b_ones;
    C->ph[PH_DIAG] = b_diag;
    C->ph[PH_INP] = b_inp;
    C->ph[PH_OUTP] = b_outp;
  }

  void ensure_plan() {
    if (plan) return;
    const auto t0 = std::chrono::steady_clock::now();
    plan = C->plan_hpsi(budget());
    plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ++plan_serial;
    const int64_t n = plan->lay.size;
    b_in = C->new_buf(std::max<int64_t>(n, 1));
    b_out = C->new_buf(std::max<int64_t>(n, 1));
    b_x = C->new_buf(std::max<int64_t>(plan->xmax, 1));
    b_diag = C->new_buf(std::max<int64_t>(n, 1));
    b_inp = C->new_buf(std::max<int64_t>(plan->lay.psize, 1));
    b_outp = C->new_buf(std::max<int64_t>(n, 1));
    {
      const std::vector<int> m = plan->lay.pack_map();
      d_pidx = ex->alloc(std::max<size_t>(m.size(), 1) * sizeof(int));
      if (!m.empty()) ex->upload(d_pidx, m.data(), m.size() * sizeof(int));
      d_pscale = (double*)ex->alloc(2 * sizeof(double));
      const std::vector<int> u = plan->lay.unpack_map();
      d_uidx = ex->alloc(std::max<size_t>(u.size(), 1) * sizeof(int));
      if (!u.empty()) ex->upload(d_uidx, u.data(), u.size() * sizeof(int));
    }
    int maxd = 1;
    for (auto& bd : C->bonds)
      for (auto& s : bd.secs) maxd = std::max(maxd, s.dim);
    std::vector<double> ones((size_t)maxd, 1.0);
    b_ones = C->new_buf(maxd);
    ex->upload(C->ptr(b_ones), ones.data(), ones.size() * 8);
    bind();
    C->run_batch(plan->diag);
  }

  // storage of the operator blocks and of psi, of the X intermediates, and of
  // the psi' accumulator for each precision (FP8 operands give BF16 X)
  static int op_dt(int prec) {
    return prec == DMRG_FP64 ? dmrg::DT_F64 : prec == DMRG_FP32 ? dmrg::DT_F32 : prec == DMRG_FP8 ? dmrg::DT_FP8 : dmrg::DT_BF16;
  }
  static int x_dt(int prec) { return prec == DMRG_FP8 ? dmrg::DT_BF16 : op_dt(prec); }
  static int out_dt(int prec) { return prec == DMRG_FP64 ? dmrg::DT_F64 : dmrg::DT_F32; }
  // copy of an operator family buffer in storage type od (FP8: one scale per operator)
  void family_copy(const dmrg::Family& F, int od, const double* src = nullptr) {
    if (F.buf < 0) return;
    if (od == dmrg::DT_FP8) C->ensure_fp8(F.buf, std::max<int64_t>(F.lay->size, 1), src);
    else C->ensure_dtype(F.buf, od);
  }

  // The low-precision copy of a block's Hamiltonian: H - sigma * 1 with sigma
  // the mean of its FP64 diagonal (Block::h_shift, set when the first copy
  // is made; every copy of the block uses it).
  void shifted_h_copy(dmrg::Block* blk, int od) {
    dmrg::Family& F = blk->fam[dmrg::F_H];
    if (F.buf < 0 || C->ptr(F.buf, od) || F.nops < 1 || C->bufs[F.buf].n == 0) {
      family_copy(F, od);
      return;
    }
    std::vector<int> diag;
    for (const auto& b : F.lay->blocks)
      if (b.bra == b.ket)
        for (int i = 0; i < blk->bond.secs[b.bra].dim; ++i) diag.push_back((int)(b.off + (int64_t)i * b.ld + i));
    if (diag.empty()) {
      family_copy(F, od);
      return;
    }
    void* di = ex->alloc(diag.size() * sizeof(int));
    ex->upload(di, diag.data(), diag.size() * sizeof(int));
    const double* h64 = (const double*)C->ptr(F.buf);
    if (!blk->h_shift_set) {
      double* dv = (double*)ex->alloc(diag.size() * 8);
      ex->gather(dv, h64, dmrg::DT_F64, (const int*)di, diag.size());
      std::vector<double> v(diag.size());
      ex->download(v.data(), dv, v.size() * 8);
      ex->release(dv);
      double sum = 0.0;
      for (double x : v) sum += x;
      blk->h_shift = sum / (double)v.size();
      blk->h_shift_set = true;
    }
    if (od == dmrg::DT_FP8) {
      // FP8: convert a shifted FP64 copy, so that the scale fits H - sigma
      const int64_t n = C->bufs[F.buf].n;
      double* tmp = (double*)ex->alloc((size_t)n * 8);
      ex->copy_d2d(tmp, h64, (size_t)n * 8);
      ex->shifted_copy_at(tmp, dmrg::DT_F64, h64, (const int*)di, diag.size(), -blk->h_shift);
      family_copy(F, od, tmp);
      ex->sync();
      ex->release(tmp);
    } else {
      C->ensure_dtype(F.buf, od);
      ex->shifted_copy_at(C->ptr(F.buf, od), od, h64, (const int*)di, diag.size(), -blk->h_shift);
      ex->sync();
    }
    ex->release(di);
  }

  // What the low-precision H*psi leaves out and end_hpsi adds back in FP64:
  // the shifts of the block Hamiltonian terms H_L (x) 1 and 1 (x) H_R.
  double lo_shift() const {
    double s = 0.0;
    for (const auto& t : plan->terms) {
      if (t.hc || t.s1 != dmrg::S_I || t.s2 != dmrg::S_I) continue;
      if (t.L.fam == dmrg::F_H && t.R.is_id() && C->Lblk->h_shift_set) s += t.c * C->Lblk->h_shift;
      if (t.R.fam == dmrg::F_H && t.L.is_id() && C->Rblk->h_shift_set) s += t.c * C->Rblk->h_shift;
    }
    return s;
  }

  // Operator families and plan buffers in the storage type of precision prec.
  void ready_dtypes(int prec) {
    const int od = op_dt(prec), xd = x_dt(prec), outd = out_dt(prec);
    if (od != dmrg::DT_F64) {
      for (dmrg::Block* blk : {C->Lblk.get(), C->Rblk.get()}) {
        shifted_h_copy(blk, od);
        if (std::getenv("DMRG_VERBOSE"))
          std::fprintf(stderr, "[dmrg] %s block Hamiltonian shift %.6f (%s)\n", blk->left ? "left" : "right",
                       blk->h_shift, blk->h_shift_set ? "set" : "unset");
        for (int f = 0; f < dmrg::kNumFam; ++f) family_copy(blk->fam[f], od);
        for (auto& t : blk->tmp) family_copy(t, od);
      }
      C->alloc_dtype(b_inp, od);
      C->alloc_dtype(b_x, xd);
      C->alloc_dtype(b_outp, outd);
    }
  }

  void prepare(int prec) {
    Prepared& P = prep[prec];
    if (P.ready) return;
    const auto t0 = std::chrono::steady_clock::now();
    const int od = op_dt(prec), xd = x_dt(prec), outd = out_dt(prec);
    ready_dtypes(prec);
    bind();
    for (auto& ch : plan->chunks) {
      std::vector<dmrg::RawJob> j;
      std::vector<dmrg::RawTerm> t;
      C->resolve(ch.stageL, j, t, od, od, xd);
      P.L.push_back(ex->prepare_tuned(j, t, od, od, xd));
      C->resolve(ch.stageR, j, t, xd, od, outd);
      P.R.push_back(ex->prepare_tuned(j, t, xd, od, outd));
    }
    P.ready = true;
    prepare_seconds[prec] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Before the stage launches (on executor e): the padded operand copy of
  // b_in and a cleared accumulator b_outp.
  void begin_hpsi(dmrg::Executor* e, int prec) {
    const int od = op_dt(prec), outd = out_dt(prec);
    if (od == dmrg::DT_FP8)  // psi / s with s a power of two from max|psi| (d_pscale)
      e->pack_fp8(C->ptr(b_inp, od), (const double*)C->ptr(b_in), (const int*)d_pidx, (size_t)plan->lay.psize, d_pscale,
                  (const double*)C->ptr(b_in), (size_t)plan->lay.size);
    else
      e->pack(C->ptr(b_inp, od), od, (const double*)C->ptr(b_in), (const int*)d_pidx, (size_t)plan->lay.psize);
    e->zero(C->ptr(b_outp, outd), (size_t)plan->lay.size * dmrg::dtype_size(outd));
  }
  // After them: b_out (FP64, caller layout) from b_outp.
  void end_hpsi(dmrg::Executor* e, int prec) {
    const int outd = out_dt(prec);
    const double sh = prec == DMRG_FP64 ? 0.0 : lo_shift();
    e->gather((double*)C->ptr(b_out), C->ptr(b_outp, outd), outd, (const int*)d_uidx, (size_t)plan->lay.size, sh,
              sh != 0.0 ? (const double*)C->ptr(b_in) : nullptr, prec == DMRG_FP8 ? d_pscale : nullptr);
  }

  // The launches of psi_out = H psi_in on b_in / b_out (prepared already).
  void enqueue_hpsi(int prec) {
    begin_hpsi(ex.get(), prec);
    Prepared& P = prep[prec];
    for (size_t i = 0; i < P.L.size(); ++i) {
      ex->run(P.L[i]);
      ex->run(P.R[i]);
    }
    end_hpsi(ex.get(), prec);
  }

  // True if the operator blocks have their copies in the storage type of prec.
  bool operators_ready(int prec) const {
    const int od = op_dt(prec);
    for (const dmrg::Block* blk : {C->Lblk.get(), C->Rblk.get()}) {
      if (!blk) return false;
      for (int f = 0; f < dmrg::kNumFam; ++f)
        if (blk->fam[f].buf >= 0 && C->bufs[blk->fam[f].buf].n > 0 && !C->ptr(blk->fam[f].buf, od)) return false;
      for (const auto& t : blk->tmp)
        if (t.buf >= 0 && C->bufs[t.buf].n > 0 && !C->ptr(t.buf, od)) return false;
    }
    return true;
  }

  // d_out = H d_in (device FP64, caller layout) with every intermediate --
  // task lists, padded copy of psi, psi' accumulator, X and partial tiles --
  // in the executor's fixed scratch instead of library allocations.  The
  // plan and the operator copies in prec must exist.  Throws FixedTooSmall
  // (before any launch) if one call needs more than the scratch holds.
  struct FixedTooSmall : std::runtime_error {
    using std::runtime_error::runtime_error;
  };
  int v_inp = -1, v_outp = -1, v_x = -1;  // view entries over the fixed scratch
  void hpsi_fixed(const void* din, void* dout, int prec) {
    const int od = op_dt(prec), outd = out_dt(prec);
    size_t cap = 0;
    char* base = (char*)ex->fixed_scratch(&cap);
    if (!base) throw std::runtime_error("the executor has no fixed scratch");
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const dmrg::PsiLayout& lay = plan->lay;
    const size_t o_inp = 0;
    const size_t o_outp = al(o_inp + (size_t)lay.psize * dmrg::dtype_size(od));
    const size_t o_x = al(o_outp + (size_t)lay.size * dmrg::dtype_size(outd));
    const size_t o_part = al(o_x + (size_t)plan->xmax * dmrg::dtype_size(od));
    auto too_small = [&](size_t need) {
      return FixedTooSmall("needs " + std::to_string(need) + " bytes of scratch, the fixed array holds " +
                           std::to_string(cap) + " (a smaller block, or work_budget_elems, fits it)");
    };
    if (o_part > cap) throw too_small(o_part);
    if (v_inp < 0) {
      v_inp = C->view_buf();
      v_outp = C->view_buf();
      v_x = C->view_buf();
    }
    C->set_view(v_inp, od, base + o_inp, lay.psize);
    C->set_view(v_outp, outd, base + o_outp, lay.size);
    C->set_view(v_x, od, base + o_x, plan->xmax);
    C->ph[PH_INP] = v_inp;
    C->ph[PH_OUTP] = v_outp;
    C->ph[PH_X] = v_x;
    std::vector<void*> hs;
    try {
      std::vector<size_t> lb;
      size_t part = 0, lists = 0;
      for (auto& ch : plan->chunks) {
        std::vector<dmrg::RawJob> j;
        std::vector<dmrg::RawTerm> t;
        size_t l = 0, pb = 0;
        C->resolve(ch.stageL, j, t, od, od, od);
        hs.push_back(ex->plan_fixed(j, t, od, od, od, &l, &pb));
        lb.push_back(l);
        lists += al(l);
        part = std::max(part, pb);
        C->resolve(ch.stageR, j, t, od, od, outd);
        hs.push_back(ex->plan_fixed(j, t, od, od, outd, &l, &pb));
        lb.push_back(l);
        lists += al(l);
        part = std::max(part, pb);
      }
      const size_t o_lists = al(o_part + part);
      if (o_lists + lists > cap) throw too_small(o_lists + lists);
      size_t cur = o_lists;
      for (size_t i = 0; i < hs.size(); ++i) {
        ex->place_fixed(hs[i], base + cur, base + o_part);
        cur += al(lb[i]);
      }
      ex->pack(base + o_inp, od, (const double*)din, (const int*)d_pidx, (size_t)lay.psize);
      ex->zero(base + o_outp, (size_t)lay.size * dmrg::dtype_size(outd));
      for (void* h : hs) ex->run(h);
      const double sh = prec == DMRG_FP64 ? 0.0 : lo_shift();
      ex->gather((double*)dout, base + o_outp, outd, (const int*)d_uidx, (size_t)lay.size, sh,
                 sh != 0.0 ? (const double*)din : nullptr);
      ex->sync();
    } catch (...) {
      for (void* h : hs) ex->drop_fixed(h);
      bind();
      throw;
    }
    for (void* h : hs) ex->drop_fixed(h);
    bind();
  }

  // psi_out = H psi_in on the device buffers b_in / b_out (FP64 masters).
  // With opts.hpsi_graph the launch sequence is recorded once per precision
  // and replayed (re-recorded when the executor's scratch moved), except
  // while kernel timing is on.  wait = false only queues the work on the
  // executor's stream (the first call of a precision still prepares its task
  // lists, which blocks the host).
  void hpsi_device(int prec, bool wait = true) {
    prepare(prec);
    Prepared& P = prep[prec];
    if (opts.hpsi_graph && ex->graphs() && !ex->timing_on()) {
      if (!P.graph || P.graph_gen != ex->scratch_generation()) {
        ex->drop_graph(P.graph);
        P.graph = nullptr;
        const long long gen = ex->scratch_generation();
        ex->capture_begin();
        try {
          enqueue_hpsi(prec);
        } catch (...) {
          ex->capture_abort();
          throw;
        }
        P.graph = ex->capture_end();
        P.graph_gen = gen;
      }
      ex->replay(P.graph);
    } else {
      enqueue_hpsi(prec);
    }
    if (wait) ex->sync();
  }
};
