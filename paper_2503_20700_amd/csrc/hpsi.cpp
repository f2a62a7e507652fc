// Task lists of the two-site Davidson matrix-vector product H_eff * psi.
//
// psi is coupled at the middle cut, ((l s1) S_a, (s2 r) S_c) S, and stored as
// super-blocks (a, c).  Every term of H is [[L (x) s1]^kX (x) [s2 (x) R]^kX]^0
// with L a left-block operator (or a linear combination of them), R a
// right-block operator, s1/s2 site operators; its action on a sub-block is
//     psi'[(l' s1') , (s2' r')] += w * L[l'<-l] psi[(l s1), (s2 r)] R[r'<-r]^T
// with w = (term coefficient) x (three Wigner 9j recoupling factors) x
// (site reduced elements) x (fermion signs).  Stage L forms X = L psi for all
// sub-blocks a term touches; stage R accumulates X R^T into psi', summing over
// terms inside each output tile (no atomics).
#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <tuple>
#include <unordered_map>

#include "planner.hpp"
#include "cross.hpp"
#include "su2.hpp"

namespace dmrg {

namespace {
inline double fsign(int parity, int nket) { return (parity & nket & 1) ? -1.0 : 1.0; }
inline int parity_of_ref(const Block& b, const Ref& r) { return r.is_id() ? 0 : (std::abs(b.family(r.fam).dn) & 1); }
inline int dn_of_ref(const Block& b, const Ref& r) { return r.is_id() ? 0 : b.family(r.fam).dn; }

template <class P>
using Expr = std::vector<std::pair<double, P>>;
}  // namespace

std::vector<Term4> Context::hpsi_terms(Block& L, Block& R) {
  const int o1 = L.b, o2 = R.b - 1;
  if (o2 != o1 + 1) throw std::runtime_error("hpsi_terms: blocks are not adjacent to a two-site block");
  std::vector<Term4> out;
  // H of the enlarged left block (x) identity, identity (x) H of the enlarged right block
  for (const LAtom& a : lgrow_h(L)) out.push_back(Term4{a.c, a.L, a.sop, a.kL2, a.ks2, 0, S_I, 0, 0, Ref{}, a.hc});
  for (const RAtom& a : rgrow_h(R)) out.push_back(Term4{a.c, Ref{}, S_I, 0, 0, 0, a.sop, a.ks2, a.kR2, a.R, a.hc});
  // cross terms between L' = L (x) o1 and R' = o2 (x) R
  xterms::CompLeftProv X{*this, L};
  xterms::CompRightProv Y{*this, R};
  xterms::cross_terms(X, Y, [&](double c, const LAtom& x, const RAtom& y, int k2, bool hc) {
    if (c == 0.0) return;
    if (x.hc || y.hc) throw std::runtime_error("hpsi_terms: transposed atom inside a cross term");
    out.push_back(Term4{c, x.L, x.sop, x.kL2, x.ks2, k2, y.sop, y.ks2, y.kR2, y.R, hc});
  });
  return out;
}

namespace {
struct MKey {
  int a[12];
  bool operator<(const MKey& o) const {
    for (int i = 0; i < 12; ++i)
      if (a[i] != o.a[i]) return a[i] < o.a[i];
    return false;
  }
};
}  // namespace

std::unique_ptr<HpsiPlan> Context::plan_hpsi(int64_t x_budget) {
  Block& L = *Lblk;
  Block& R = *Rblk;
  to_complementary(R);  // the middle cut pairs normal operators on the left with complementary ones on the right
  auto plan = std::make_unique<HpsiPlan>();
  plan->k = k;
  plan->lay.build(L.bond, R.bond, n_elec, two_s);
  const PsiLayout& lay = plan->lay;

  // ---- terms, merged: first over left operators, then over right operators
  std::vector<Term4> raw = hpsi_terms(L, R);
  std::vector<std::vector<std::pair<Ref, double>>> pendL, pendR;
  std::vector<int> pfL, pfR;
  std::vector<Term4> t1;
  {
    std::map<MKey, std::vector<size_t>> g;
    for (size_t i = 0; i < raw.size(); ++i) {
      const Term4& t = raw[i];
      g[MKey{{t.s1, t.kL2, t.k12, t.kX2, t.s2, t.k22, t.kR2, t.R.fam, t.R.idx, (int)t.hc, t.L.is_id() ? 1 : 0, 0}}]
          .push_back(i);
    }
    for (auto& [key, idx] : g) {
      if (idx.size() == 1 || key.a[10]) {
        for (size_t i : idx) t1.push_back(raw[i]);
        continue;
      }
      std::vector<std::pair<Ref, double>> parts;
      for (size_t i : idx) parts.push_back({raw[i].L, raw[i].c});
      Term4 t = raw[idx[0]];
      const int dn = dn_of_ref(L, raw[idx[0]].L);
      t.L = make_lincomb(L, t.kL2, dn, parts, &pendL, &pfL);
      t.c = 1.0;
      t1.push_back(t);
    }
  }
  std::vector<Term4>& terms = plan->terms;
  {
    std::map<MKey, std::vector<size_t>> g;
    for (size_t i = 0; i < t1.size(); ++i) {
      const Term4& t = t1[i];
      g[MKey{{t.L.fam, t.L.idx, t.s1, t.kL2, t.k12, t.kX2, t.s2, t.k22, t.kR2, (int)t.hc, t.R.is_id() ? 1 : 0, 0}}]
          .push_back(i);
    }
    for (auto& [key, idx] : g) {
      if (idx.size() == 1 || key.a[10]) {
        for (size_t i : idx) terms.push_back(t1[i]);
        continue;
      }
      std::vector<std::pair<Ref, double>> parts;
      for (size_t i : idx) parts.push_back({t1[i].R, t1[i].c});
      Term4 t = t1[idx[0]];
      const int dn = dn_of_ref(R, t1[idx[0]].R);
      t.R = make_lincomb(R, t.kR2, dn, parts, &pendR, &pfR);
      t.c = 1.0;
      terms.push_back(t);
    }
  }
  materialise_lincombs(L, pendL, pfL);
  materialise_lincombs(R, pendR, pfR);

  // ---- layout lookups
  std::map<std::tuple<int, int, int, int>, int> sb_of;
  for (size_t s = 0; s < lay.sbs.size(); ++s) {
    const auto& sb = lay.sbs[s];
    sb_of[{sb.an, sb.as2, sb.cn, sb.cs2}] = (int)s;
  }
  const int S2 = two_s;

  // ---- per chunk task generation
  //
  // An X region is X_t = (L (x) s1) psi for one (term, direction, output
  // super-block, input super-block); its rows are the row bands (l', s1') of
  // the output super-block in internal order, its columns the padded columns
  // of the input super-block.  A band no stage-L product writes is zero, and
  // a column sub-block no stage-R product reads is not needed; both are left
  // out of the launches and of the flop count.  Stage-R jobs (one per output
  // super-block and column sub-block) are cut into row segments so that each
  // product covers only the bands where its X is non-zero; adjacent segments
  // are merged where fewer, fuller tiles cost less, and a zero band a merged
  // segment reads is then written as zeros by stage L.
  struct XBand {
    std::vector<GemmTerm> prods;  // stage-L products; B offsets at column 0 of the input
    bool zero_read = false;       // no product, but read inside a merged stage-R segment
  };
  struct XRegion {
    int xo = 0, xi = 0;
    int64_t base = 0;
    std::vector<XBand> bands;   // per row sub-block of lay.sbs[xo]
    std::vector<char> colread;  // per column sub-block of lay.sbs[xi]
  };
  struct RProd {
    GemmTerm gt;  // A offset at row 0 of the region
    int reg = 0;
    bool dense = false;  // not an identity product (counts flops)
  };
  std::vector<XRegion> regs;
  std::map<std::tuple<int, int, int, int>, int> xreg;  // (term, dir, out-left sb, in sb) -> region, -1 if zero
  std::map<std::pair<int, int>, std::vector<RProd>> rjobs;  // (out sb, col idx) -> products
  int64_t xoff = 0;
  constexpr int kSegRows = 64;    // row tile of the stage-R launches (cost model of the segment merge)
  constexpr double kSegK = 32.0;  // per-tile overhead, in K elements

  auto new_chunk = [&]() { plan->chunks.emplace_back(); };
  new_chunk();

  auto flush_chunk = [&]() {
    HpsiPlan::Chunk& ch = plan->chunks.back();
    // stage R: row segments per output (super-block, column sub-block)
    for (auto& [key, vec] : rjobs) {
      const auto& sb = lay.sbs[key.first];
      const auto& col = sb.cols[key.second];
      const int nb = (int)sb.rows.size();
      std::vector<int> ord(nb);
      for (int i = 0; i < nb; ++i) ord[i] = i;
      std::sort(ord.begin(), ord.end(), [&](int x, int y) { return sb.rows[x].ir0 < sb.rows[y].ir0; });
      // membership is per X region: every product of a region has its zero bands
      std::vector<int> rlist;
      std::map<int, int> rpos;
      std::vector<double> rk;
      for (const RProd& rp : vec) {
        auto ins = rpos.emplace(rp.reg, (int)rlist.size());
        if (ins.second) {
          rlist.push_back(rp.reg);
          rk.push_back(0.0);
        }
        rk[ins.first->second] += rp.gt.k;
      }
      const size_t nr = rlist.size(), nw = (nr + 63) / 64;
      struct Seg {
        int p0, p1;  // positions in ord
        int rows;
        std::vector<uint64_t> mem;  // member regions
        double kmem;                // summed K of the members' products
      };
      std::vector<Seg> segs;
      std::vector<uint64_t> mem(nw);
      for (int q = 0; q < nb; ++q) {
        const int bi = ord[q];
        std::fill(mem.begin(), mem.end(), 0);
        double km = 0.0;
        bool anyp = false;
        for (size_t r = 0; r < nr; ++r)
          if (!regs[rlist[r]].bands[bi].prods.empty()) {
            mem[r >> 6] |= (uint64_t)1 << (r & 63);
            km += rk[r];
            anyp = true;
          }
        if (!anyp) continue;  // every product is zero here: psi' stays zero
        if (!segs.empty() && segs.back().p1 == q && segs.back().mem == mem) {
          segs.back().p1 = q + 1;
          segs.back().rows += sb.rows[bi].dl;
        } else {
          segs.push_back(Seg{q, q + 1, sb.rows[bi].dl, mem, km});
        }
      }
      auto cost = [&](int rows, double km) { return (double)((rows + kSegRows - 1) / kSegRows) * (km + kSegK); };
      for (size_t i = 0; i + 1 < segs.size();) {
        Seg& A = segs[i];
        Seg& B = segs[i + 1];
        if (A.p1 != B.p0) {
          ++i;
          continue;
        }
        std::vector<uint64_t> u(nw);
        double ku = 0.0;
        for (size_t w = 0; w < nw; ++w) u[w] = A.mem[w] | B.mem[w];
        for (size_t r = 0; r < nr; ++r)
          if (u[r >> 6] >> (r & 63) & 1) ku += rk[r];
        if (cost(A.rows + B.rows, ku) <= cost(A.rows, A.kmem) + cost(B.rows, B.kmem)) {
          A.p1 = B.p1;
          A.rows += B.rows;
          A.mem.swap(u);
          A.kmem = ku;
          segs.erase(segs.begin() + i + 1);
        } else {
          ++i;
        }
      }
      for (const Seg& S : segs) {
        const int row0 = sb.rows[ord[S.p0]].ir0;
        GemmJob j;
        j.C = BufRef{-7, sb.off + (int64_t)row0 * sb.ncols + col.c0};  // -7: psi_out in internal row order
        j.m = S.rows;
        j.n = col.dr;
        j.ldc = sb.ncols;
        j.accumulate = 1;
        j.tbeg = (int64_t)ch.stageR.terms.size();
        std::vector<int> nzrows(nr, 0);
        for (size_t r = 0; r < nr; ++r) {
          if (!(S.mem[r >> 6] >> (r & 63) & 1)) continue;
          XRegion& R = regs[rlist[r]];
          for (int q = S.p0; q < S.p1; ++q) {
            XBand& bd = R.bands[ord[q]];
            if (!bd.prods.empty()) nzrows[r] += sb.rows[ord[q]].dl;
            else bd.zero_read = true;
          }
        }
        for (const RProd& rp : vec) {
          const int r = rpos[rp.reg];
          if (!(S.mem[r >> 6] >> (r & 63) & 1)) continue;
          GemmTerm gt = rp.gt;
          gt.A.off += (int64_t)row0 * gt.lda;
          ch.stageR.terms.push_back(gt);
          if (rp.dense) {
            ch.stageR.flops += 2.0 * nzrows[r] * col.dr * gt.k;
            plan->flops_exec += 2.0 * S.rows * col.dr * gt.k;
          }
        }
        j.tend = (int64_t)ch.stageR.terms.size();
        ch.stageR.jobs.push_back(j);
      }
    }
    // stage L: the bands stage R reads, over runs of the column sub-blocks it reads
    for (const XRegion& R : regs) {
      const auto& O = lay.sbs[R.xo];
      const auto& In = lay.sbs[R.xi];
      const int nc = (int)In.cols.size();
      for (size_t bi = 0; bi < O.rows.size(); ++bi) {
        const XBand& bd = R.bands[bi];
        if (bd.prods.empty() && !bd.zero_read) continue;
        const auto& ro = O.rows[bi];
        for (int c0 = 0; c0 < nc;) {
          if (!R.colread[c0]) {
            ++c0;
            continue;
          }
          int c1 = c0;
          int width = 0;
          while (c1 < nc && R.colread[c1]) width += In.cols[c1++].dr;
          const int pc0 = In.cols[c0].pc0;
          GemmJob j;
          j.C = BufRef{-3, R.base + (int64_t)ro.ir0 * In.pncols + pc0};  // -3: X placeholder
          j.m = ro.dl;
          j.n = In.cols[c1 - 1].pc0 + In.cols[c1 - 1].dr - pc0;
          j.ldc = In.pncols;
          j.accumulate = 0;
          j.tbeg = (int64_t)ch.stageL.terms.size();
          for (const GemmTerm& g0 : bd.prods) {
            GemmTerm gt = g0;
            gt.B.off += pc0;
            ch.stageL.terms.push_back(gt);
            if (!(gt.flags & TF_IDENT_A)) {
              ch.stageL.flops += 2.0 * ro.dl * width * gt.k;
              plan->flops_exec += 2.0 * ro.dl * width * gt.k;
            }
          }
          j.tend = (int64_t)ch.stageL.terms.size();
          ch.stageL.jobs.push_back(j);
          c0 = c1;
        }
      }
    }
    ch.xsize = xoff;
    plan->xmax = std::max(plan->xmax, xoff);
    plan->flops += ch.stageL.flops + ch.stageR.flops;
    plan->n_stage_terms += ch.stageL.terms.size() + ch.stageR.terms.size();
    rjobs.clear();
    xreg.clear();
    regs.clear();
    xoff = 0;
  };

  // Stage-L region: X(rows of left sector of `osb`) x (cols of input sb `isb`)
  // for term t in direction dir (0 forward: L[l'<-l] psi, 1 transposed).
  auto get_x = [&](int ti, int dir, int osb, int isb) -> int {
    auto key = std::make_tuple(ti, dir, osb, isb);
    auto it = xreg.find(key);
    if (it != xreg.end()) return it->second;
    const Term4& t = terms[ti];
    const auto& O = lay.sbs[osb];  // provides output rows
    const auto& In = lay.sbs[isb];
    const Family* LF = t.L.is_id() ? nullptr : &L.family(t.L.fam);
    const SiteOp& so = sops[t.s1];
    XRegion R;
    R.xo = osb;
    R.xi = isb;
    R.bands.resize(O.rows.size());
    R.colread.assign(In.cols.size(), 0);
    bool any = false;
    double dense_flops = 0.0;
    for (size_t bi = 0; bi < O.rows.size(); ++bi) {  // output row sub (l', s1') [dir 0]  /  (l, s1) [dir 1]
      const auto& ro = O.rows[bi];
      for (const auto& ri : In.rows) {
        // forward element is always <bra = (l' s1') of the term's output | ket = (l s1) of its input>
        int bl, kl, bs, ks, bsa, ksa;  // bra / ket sector idx, site idx, enlarged spins
        if (dir == 0) {
          bl = ro.il; bs = ro.s1; bsa = O.as2;
          kl = ri.il; ks = ri.s1; ksa = In.as2;
        } else {
          bl = ri.il; bs = ri.s1; bsa = In.as2;
          kl = ro.il; ks = ro.s1; ksa = O.as2;
        }
        const double r1 = so.r[bs][ks];
        if (r1 == 0.0) continue;
        int blk = -1;
        if (LF) {
          blk = LF->lay->find(bl, kl);
          if (blk < 0) continue;
        } else if (bl != kl) {
          continue;
        }
        const Sector& sb_ = L.bond.secs[bl];
        const Sector& sk_ = L.bond.secs[kl];
        double w = coupled_factor(sb_.s2, sk_.s2, t.kL2, kLocS2[bs], kLocS2[ks], t.k12, bsa, ksa, t.kX2) *
                   fsign(so.parity, sk_.n);
        if (w == 0.0) continue;
        GemmTerm gt;
        gt.flags = 0;
        if (LF) {
          gt.A = BufRef{LF->buf, (int64_t)t.L.idx * LF->lay->size + LF->lay->blocks[blk].off};
          gt.lda = LF->lay->blocks[blk].ld;  // stored block is D_bra x D_ket (padded rows)
          if (dir == 1) gt.flags |= TF_TRANS_A;
        } else {
          gt.flags |= TF_IDENT_A;
        }
        gt.B = BufRef{-6, In.poff + (int64_t)ri.ir0 * In.pncols};  // -6: padded psi_in placeholder
        gt.ldb = In.pncols;
        // operator blocks, padded psi and X all have 8-element padded rows
        gt.flags |= TF_PAD_B | (LF ? TF_PAD_A : 0);
        gt.k = ri.dl;
        gt.alpha = w * r1;
        R.bands[bi].prods.push_back(gt);
        if (LF) dense_flops += 2.0 * ro.dl * In.ncols * ri.dl;
        any = true;
      }
    }
    if (!any) {
      xreg[key] = -1;
      return -1;
    }
    plan->flops_dense += dense_flops;
    R.base = xoff;
    xoff += (int64_t)O.nrows * In.pncols;
    regs.push_back(std::move(R));
    xreg[key] = (int)regs.size() - 1;
    return (int)regs.size() - 1;
  };

  for (size_t ti = 0; ti < terms.size(); ++ti) {
    const Term4& t = terms[ti];
    const int dnL = dn_of_ref(L, t.L);
    const int dnX = dnL + sops[t.s1].dn;
    const int pY = (sops[t.s2].parity + parity_of_ref(R, t.R)) & 1;
    const Family* RF = t.R.is_id() ? nullptr : &R.family(t.R.fam);
    const SiteOp& so2 = sops[t.s2];
    for (size_t isb = 0; isb < lay.sbs.size(); ++isb) {
      const auto& In = lay.sbs[isb];
      for (int as2 = std::abs(In.as2 - t.kX2); as2 <= In.as2 + t.kX2; as2 += 2)
        for (int cs2 = std::abs(In.cs2 - t.kX2); cs2 <= In.cs2 + t.kX2; cs2 += 2) {
          auto it = sb_of.find({In.an + dnX, as2, In.cn - dnX, cs2});
          if (it == sb_of.end()) continue;
          const int osb = it->second;
          const auto& O = lay.sbs[osb];
          const double wout = coupled_factor(O.as2, In.as2, t.kX2, O.cs2, In.cs2, t.kX2, S2, S2, 0) *
                              fsign(pY, In.an);
          if (wout == 0.0) continue;
          for (int dir = 0; dir < (t.hc ? 2 : 1); ++dir) {
            if (t.hc && dir == 0) continue;  // hc terms only act transposed
            const int d = t.hc ? 1 : 0;
            // forward: X over rows of O's left part, cols of In; output O
            // transposed: X over rows of In's left part, cols of O; output In
            const int xo = d ? (int)isb : osb;
            const int xi = d ? osb : (int)isb;
            const int rid = get_x((int)ti, d, xo, xi);
            if (rid < 0) continue;
            const int64_t xbase = regs[rid].base;
            const auto& Xrows = lay.sbs[xo];
            const auto& Xin = lay.sbs[xi];
            const auto& Out = d ? In : O;
            const int outsb = d ? (int)isb : osb;
            for (size_t oc = 0; oc < Out.cols.size(); ++oc) {
              const auto& co = Out.cols[oc];
              for (size_t cidx = 0; cidx < Xin.cols.size(); ++cidx) {
                const auto& ci = Xin.cols[cidx];
                // forward element bra = (s2', r') of O, ket = (s2, r) of In
                int bs, ks, br, kr;
                if (d == 0) {
                  bs = co.s2; br = co.ir; ks = ci.s2; kr = ci.ir;
                } else {
                  bs = ci.s2; br = ci.ir; ks = co.s2; kr = co.ir;
                }
                const double r2 = so2.r[bs][ks];
                if (r2 == 0.0) continue;
                int blk = -1;
                if (RF) {
                  blk = RF->lay->find(br, kr);
                  if (blk < 0) continue;
                } else if (br != kr) {
                  continue;
                }
                const Sector& srb = R.bond.secs[br];
                const Sector& srk = R.bond.secs[kr];
                const double wR = coupled_factor(kLocS2[bs], kLocS2[ks], t.k22, srb.s2, srk.s2, t.kR2, O.cs2, In.cs2,
                                                 t.kX2) *
                                  fsign(RF ? (std::abs(RF->dn) & 1) : 0, kLocN[ks]);
                if (wR == 0.0) continue;
                RProd rp;
                rp.reg = rid;
                rp.dense = RF != nullptr;
                GemmTerm& gt = rp.gt;
                gt.A = BufRef{-3, xbase + ci.pc0};
                gt.lda = Xin.pncols;
                gt.flags = TF_PAD_A;
                if (RF) {
                  gt.B = BufRef{RF->buf, (int64_t)t.R.idx * RF->lay->size + RF->lay->blocks[blk].off};
                  gt.ldb = RF->lay->blocks[blk].ld;
                  if (d == 0) gt.flags |= TF_TRANS_B;  // X @ R^T ; transposed term: X @ R
                  gt.flags |= TF_PAD_B;
                } else {
                  gt.flags |= TF_IDENT_B;
                }
                gt.k = ci.dr;
                gt.alpha = t.c * wout * wR * r2;
                regs[rid].colread[cidx] = 1;
                rjobs[{outsb, (int)oc}].push_back(rp);
                if (RF) plan->flops_dense += 2.0 * Xrows.nrows * co.dr * ci.dr;
              }
            }
          }
        }
    }
    if (xoff >= x_budget && ti + 1 < terms.size()) {
      flush_chunk();
      new_chunk();
    }
  }
  flush_chunk();

  // ---- diagonal of H_eff (Davidson preconditioner)
  {
    GemmBatch& D = plan->diag;
    std::map<std::tuple<int, int, int>, std::vector<GemmTerm>> dj;  // (sb, row, col)
    for (size_t ti = 0; ti < terms.size(); ++ti) {
      const Term4& t = terms[ti];
      const int dnX = dn_of_ref(L, t.L) + sops[t.s1].dn;
      if (dnX != 0) continue;
      const Family* LF = t.L.is_id() ? nullptr : &L.family(t.L.fam);
      const Family* RF = t.R.is_id() ? nullptr : &R.family(t.R.fam);
      const SiteOp& so1 = sops[t.s1];
      const SiteOp& so2 = sops[t.s2];
      const int pY = (so2.parity + parity_of_ref(R, t.R)) & 1;
      const double mult = 1.0;  // the transpose of a term has the same diagonal
      for (size_t isb = 0; isb < lay.sbs.size(); ++isb) {
        const auto& In = lay.sbs[isb];
        const double wout = coupled_factor(In.as2, In.as2, t.kX2, In.cs2, In.cs2, t.kX2, S2, S2, 0) *
                            fsign(pY, In.an);
        if (wout == 0.0) continue;
        for (size_t ir = 0; ir < In.rows.size(); ++ir) {
          const auto& ro = In.rows[ir];
          const double r1 = so1.r[ro.s1][ro.s1];
          if (r1 == 0.0) continue;
          const Sector& sl = L.bond.secs[ro.il];
          int lb = -1;
          if (LF) {
            lb = LF->lay->find(ro.il, ro.il);
            if (lb < 0) continue;
          }
          const double wL = coupled_factor(sl.s2, sl.s2, t.kL2, kLocS2[ro.s1], kLocS2[ro.s1], t.k12, In.as2, In.as2,
                                           t.kX2) *
                            fsign(so1.parity, sl.n);
          if (wL == 0.0) continue;
          for (size_t ic = 0; ic < In.cols.size(); ++ic) {
            const auto& co = In.cols[ic];
            const double r2 = so2.r[co.s2][co.s2];
            if (r2 == 0.0) continue;
            const Sector& sr = R.bond.secs[co.ir];
            int rb = -1;
            if (RF) {
              rb = RF->lay->find(co.ir, co.ir);
              if (rb < 0) continue;
            }
            const double wR = coupled_factor(kLocS2[co.s2], kLocS2[co.s2], t.k22, sr.s2, sr.s2, t.kR2, In.cs2, In.cs2,
                                             t.kX2) *
                              fsign(RF ? (std::abs(RF->dn) & 1) : 0, kLocN[co.s2]);
            if (wR == 0.0) continue;
            GemmTerm gt;
            if (LF) {
              gt.A = BufRef{LF->buf, (int64_t)t.L.idx * LF->lay->size + LF->lay->blocks[lb].off};
              gt.lda = LF->lay->blocks[lb].ld + 1;  // diagonal stride
            } else {
              gt.A = BufRef{-4, 0};  // ones
              gt.lda = 1;
            }
            if (RF) {
              gt.B = BufRef{RF->buf, (int64_t)t.R.idx * RF->lay->size + RF->lay->blocks[rb].off};
              gt.ldb = RF->lay->blocks[rb].ld + 1;
            } else {
              gt.B = BufRef{-4, 0};
              gt.ldb = 1;
            }
            gt.flags = TF_TRANS_B;
            gt.k = 1;
            gt.alpha = mult * t.c * wout * wL * r1 * wR * r2;
            dj[{(int)isb, (int)ir, (int)ic}].push_back(gt);
          }
        }
      }
    }
    for (auto& [key, vec] : dj) {
      const auto& sb = lay.sbs[std::get<0>(key)];
      const auto& ro = sb.rows[std::get<1>(key)];
      const auto& co = sb.cols[std::get<2>(key)];
      GemmJob j;
      j.C = BufRef{-5, sb.off + (int64_t)ro.r0 * sb.ncols + co.c0};
      j.m = ro.dl;
      j.n = co.dr;
      j.ldc = sb.ncols;
      j.accumulate = 0;
      j.tbeg = (int64_t)D.terms.size();
      D.terms.insert(D.terms.end(), vec.begin(), vec.end());
      j.tend = (int64_t)D.terms.size();
      D.jobs.push_back(j);
    }
  }
  return plan;
}

}  // namespace dmrg
