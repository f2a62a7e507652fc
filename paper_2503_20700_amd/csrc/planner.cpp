#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <tuple>
#include <unordered_map>

#include "su2.hpp"
#include "cross.hpp"

namespace dmrg {

// ================================================================ sectors, layouts
int Bond::find(int n_, int s2_) const {
  for (size_t i = 0; i < secs.size(); ++i)
    if (secs[i].n == n_ && secs[i].s2 == s2_) return (int)i;
  return -1;
}

const OpLayout& Block::layout(int k2, int dn) {
  auto key = std::make_pair(k2, dn);
  auto it = layouts.find(key);
  if (it != layouts.end()) return *it->second;
  auto lay = std::make_unique<OpLayout>();
  lay->k2 = k2;
  lay->dn = dn;
  lay->nsec = (int)bond.secs.size();
  lay->lookup.assign((size_t)lay->nsec * lay->nsec, -1);
  for (int br = 0; br < lay->nsec; ++br)
    for (int kt = 0; kt < lay->nsec; ++kt) {
      const Sector &sb = bond.secs[br], &sk = bond.secs[kt];
      if (sb.n != sk.n + dn || !tri2(sk.s2, k2, sb.s2)) continue;
      lay->lookup[(size_t)br * lay->nsec + kt] = (int)lay->blocks.size();
      const int ld = pad_up(sk.dim);
      lay->blocks.push_back(OpBlock{br, kt, lay->size, ld});
      lay->size += (int64_t)sb.dim * ld;
    }
  const OpLayout& ref = *lay;
  layouts[key] = std::move(lay);
  return ref;
}

int Block::op(int f, int i, int j) const {
  const Family& F = family(f);
  if (F.index.empty()) return -1;
  size_t key = (j < 0) ? (size_t)i : (size_t)i * n + j;
  if (key >= F.index.size()) return -1;
  return F.index[key];
}

int64_t Block::bytes_f64() const {
  int64_t s = 0;
  for (int f = 0; f < kNumFam; ++f)
    if (fam[f].lay) s += (int64_t)fam[f].nops * fam[f].lay->size * 8;
  return s;
}

int fam_k2(int f) {
  switch (f) {
    case F_C: case F_D: case F_SL: case F_SR: return 1;
    case F_A1: case F_AB1: case F_B1: case F_P1: case F_K1: return 2;
    default: return 0;
  }
}
int fam_dn(int f) {
  switch (f) {
    case F_C: return 1;
    case F_D: case F_SL: case F_SR: return -1;
    case F_A0: case F_A1: return 2;
    case F_AB0: case F_AB1: case F_P0: case F_P1: return -2;
    default: return 0;
  }
}
const char* fam_name(int f) {
  static const char* names[] = {"H", "C", "D", "A0", "A1", "AB0", "AB1", "B0", "B1", "SL",
                                "P0", "P1", "J", "K0", "K1", "SR"};
  if (f >= 0 && f < kNumFam) return names[f];
  return f == F_ID ? "I" : "TMP";
}
static inline int fam_parity(int f) { return std::abs(fam_dn(f)) & 1; }

// ================================================================ context, buffers
Context::Context(Executor* e, const Integrals& ints, int ne, int ts) : ex(e), I(ints), n_elec(ne), two_s(ts) {
  n = I.n;
  for (int i = 0; i < kNumFixedSite; ++i) sops.push_back(site_op(i));
  for (int o = 0; o < n; ++o) sops.push_back(site_hamiltonian(I.H(o, o), I.G(o, o, o, o)));
}

Context::~Context() {
  Lblk.reset();
  Rblk.reset();
  for (size_t i = 0; i < bufs.size(); ++i) free_buf((int)i);
}

void Context::charge(int64_t bytes) {
  if (budget_bytes > 0 && bytes_in_use + bytes > budget_bytes)
    throw BudgetExceeded("device memory budget of " + std::to_string(budget_bytes) + " bytes exceeded (" +
                         std::to_string(bytes_in_use) + " held, " + std::to_string(bytes) + " more requested)");
}

int Context::new_buf(int64_t nel) {
  DevBuf b;
  b.n = nel;
  if (nel > 0) {
    charge(nel * 8);
    b.p[DT_F64] = ex->alloc((size_t)nel * 8);
    ex->zero(b.p[DT_F64], (size_t)nel * 8);
    bytes_in_use += nel * 8;
    peak_bytes = std::max(peak_bytes, bytes_in_use);
  }
  bufs.push_back(b);
  return (int)bufs.size() - 1;
}

int Context::view_buf() {
  DevBuf b;
  b.view = true;
  bufs.push_back(b);
  return (int)bufs.size() - 1;
}

void Context::set_view(int id, int dt, void* p, int64_t n) {
  DevBuf& b = bufs[id];
  if (!b.view) throw std::runtime_error("set_view: not a view buffer");
  for (auto& q : b.p) q = nullptr;
  b.p[dt] = p;
  b.n = n;
}

void Context::free_buf(int id) {
  if (id < 0 || id >= (int)bufs.size()) return;
  DevBuf& b = bufs[id];
  if (b.view) {
    for (auto& q : b.p) q = nullptr;
    b.n = 0;
    return;
  }
  for (int d = 0; d < 4; ++d)
    if (b.p[d]) {
      ex->release(b.p[d]);
      bytes_in_use -= b.n * (int64_t)dtype_size(d);
      b.p[d] = nullptr;
    }
  b.n = 0;
  b.fp8_seg = 0;
  b.fp8_scale.clear();
}

void Context::ensure_dtype(int id, int dt) {
  DevBuf& b = bufs[id];
  if (dt == DT_F64 || b.p[dt] || b.n == 0) return;
  charge(b.n * (int64_t)dtype_size(dt));
  b.p[dt] = ex->alloc((size_t)b.n * dtype_size(dt));
  bytes_in_use += b.n * (int64_t)dtype_size(dt);
  peak_bytes = std::max(peak_bytes, bytes_in_use);
  ex->convert(b.p[dt], dt, b.p[DT_F64], DT_F64, (size_t)b.n);
}

void Context::ensure_fp8(int id, int64_t seg, const double* src) {
  DevBuf& b = bufs[id];
  if (b.p[DT_FP8] || b.n == 0) return;
  if (seg <= 0 || b.n % seg) throw std::runtime_error("ensure_fp8: segment does not divide the buffer");
  const int64_t nseg = b.n / seg;
  charge(b.n);
  double* d_scale = (double*)ex->alloc((size_t)nseg * 2 * sizeof(double));
  if (!src) src = (const double*)b.p[DT_F64];
  ex->fp8_scales(src, nseg, seg, d_scale);
  b.p[DT_FP8] = ex->alloc((size_t)b.n);
  bytes_in_use += b.n;
  peak_bytes = std::max(peak_bytes, bytes_in_use);
  ex->to_fp8(b.p[DT_FP8], src, b.n, seg, d_scale);
  std::vector<double> sc((size_t)nseg * 2);
  ex->download(sc.data(), d_scale, sc.size() * sizeof(double));
  ex->release(d_scale);
  b.fp8_seg = seg;
  b.fp8_scale.resize((size_t)nseg);
  for (int64_t i = 0; i < nseg; ++i) b.fp8_scale[(size_t)i] = sc[(size_t)(2 * i)];
}

void Context::alloc_dtype(int id, int dt) {
  DevBuf& b = bufs[id];
  if (b.p[dt] || b.n == 0) return;
  charge(b.n * (int64_t)dtype_size(dt));
  b.p[dt] = ex->alloc((size_t)b.n * dtype_size(dt));
  bytes_in_use += b.n * (int64_t)dtype_size(dt);
  peak_bytes = std::max(peak_bytes, bytes_in_use);
}

void Context::free_block(Block& blk) {
  for (int f = 0; f < kNumFam; ++f) {
    free_buf(blk.fam[f].buf);
    blk.fam[f].buf = -1;
  }
  for (auto& t : blk.tmp) free_buf(t.buf);
  blk.tmp.clear();
}

// ================================================================ families
static void add_family(Context& C, Block& blk, int f, const std::vector<std::pair<int, int>>& keys) {
  Family& F = blk.fam[f];
  F.k2 = fam_k2(f);
  F.dn = fam_dn(f);
  F.lay = &blk.layout(F.k2, F.dn);
  const bool pair = !(f == F_H || f == F_C || f == F_D || f == F_SL || f == F_SR);
  F.index.assign(pair ? (size_t)blk.n * blk.n : (f == F_H ? 1 : (size_t)blk.n), -1);
  F.nops = 0;
  for (auto& [i, j] : keys) {
    size_t key = pair ? (size_t)i * blk.n + j : (size_t)i;
    F.index[key] = F.nops++;
  }
  int64_t tot = (int64_t)F.nops * F.lay->size;
  F.buf = tot > 0 ? C.new_buf(tot) : -1;
}

static void init_families(Context& C, Block& blk) {
  const int b = blk.b, n = blk.n;
  std::vector<std::pair<int, int>> k1, ksym, kasym, kall, kout;
  if (blk.left) {
    for (int i = 0; i < b; ++i) k1.push_back({i, -1});
    for (int r = b; r < n; ++r) kout.push_back({r, -1});
  } else {
    for (int q = b; q < n; ++q) k1.push_back({q, -1});
    for (int p = 0; p < b; ++p) kout.push_back({p, -1});
  }
  // pair indices: inside the block (normal pair operators) or, for right
  // blocks in complementary mode, the orbitals to the left of the block
  const bool inside = blk.left || blk.normal;
  const int lo = inside ? (blk.left ? 0 : b) : 0, hi = inside ? (blk.left ? b : n) : b;
  for (int i = lo; i < hi; ++i)
    for (int j = lo; j < hi; ++j) {
      kall.push_back({i, j});
      if (i <= j) ksym.push_back({i, j});
      if (i < j) kasym.push_back({i, j});
    }
  add_family(C, blk, F_H, {{0, -1}});
  add_family(C, blk, F_C, k1);
  add_family(C, blk, F_D, k1);
  if (!blk.left && blk.normal) {
    add_family(C, blk, F_A0, ksym);
    add_family(C, blk, F_A1, kasym);
    add_family(C, blk, F_AB0, ksym);
    add_family(C, blk, F_AB1, kasym);
    add_family(C, blk, F_B0, kall);
    add_family(C, blk, F_B1, kall);
    add_family(C, blk, F_SR, kout);
  } else if (blk.left) {
    add_family(C, blk, F_A0, ksym);
    add_family(C, blk, F_A1, kasym);
    add_family(C, blk, F_AB0, ksym);
    add_family(C, blk, F_AB1, kasym);
    add_family(C, blk, F_B0, kall);
    add_family(C, blk, F_B1, kall);
    add_family(C, blk, F_SL, kout);
  } else {
    add_family(C, blk, F_P0, ksym);
    add_family(C, blk, F_P1, kasym);
    add_family(C, blk, F_J, ksym);
    add_family(C, blk, F_K0, kall);
    add_family(C, blk, F_K1, kall);
    add_family(C, blk, F_SR, kout);
  }
}

std::unique_ptr<Block> Context::vacuum_left() {
  auto blk = std::make_unique<Block>();
  blk->left = true;
  blk->b = 0;
  blk->n = n;
  blk->bond.secs = {Sector{0, 0, 1}};
  init_families(*this, *blk);
  return blk;
}

std::unique_ptr<Block> Context::vacuum_right() {
  auto blk = std::make_unique<Block>();
  blk->left = false;
  blk->normal = true;
  blk->b = n;
  blk->n = n;
  blk->bond.secs = {Sector{0, 0, 1}};
  init_families(*this, *blk);
  return blk;
}

// ================================================================ growth expressions
static Ref R_(int f, int idx) { return Ref{f, idx}; }

std::vector<LAtom> Context::lgrow(const Block& L, int f, int i, int j) const {
  const int o = L.b;  // the site being appended
  const SpinConstants& sc = spin_constants();
  std::vector<LAtom> out;
  auto add = [&](double c, Ref r, int sop, int kL2, int ks2, bool hc = false) {
    if (c == 0.0) return;
    if (!r.is_id() && r.idx < 0) return;
    out.push_back(LAtom{c, r, sop, kL2, ks2, hc});
  };
  auto op = [&](int fam, int a, int b = -1) { return R_(fam, L.op(fam, a, b)); };
  switch (f) {
    case F_C:
    case F_D: {
      const int sop = f == F_C ? S_C : S_D;
      if (i < o) add(1.0, op(f, i), S_I, 1, 0);
      else add(1.0, Ref{}, sop, 0, 1);
      break;
    }
    case F_A0: case F_A1: case F_AB0: case F_AB1: {
      const int S = (f == F_A1 || f == F_AB1) ? 1 : 0;
      const bool cre = (f == F_A0 || f == F_A1);
      if (j < o) add(1.0, op(f, i, j), S_I, 2 * S, 0);
      else if (i < o) add(1.0, op(cre ? F_C : F_D, i), cre ? S_C : S_D, 1, 1);
      else if (S == 0) add(1.0, Ref{}, cre ? S_CC0 : S_DD0, 0, 0);
      break;
    }
    case F_B0: case F_B1: {
      const int k = f == F_B1 ? 1 : 0;
      if (i < o && j < o) add(1.0, op(f, i, j), S_I, 2 * k, 0);
      else if (i < o) add(1.0, op(F_C, i), S_D, 1, 1);
      else if (j < o) add(sc.b_swap[k], op(F_D, j), S_C, 1, 1);
      else add(1.0, Ref{}, k ? S_CD1 : S_CD0, 0, 2 * k);
      break;
    }
    case F_SL: {
      const int r = i;
      add(1.0, op(F_SL, r), S_I, 1, 0);
      add(I.G(o, o, r, o), Ref{}, S_T3, 0, 1);
      for (int k = 0; k < 2; ++k) {
        const int fb = k ? F_B1 : F_B0, scd = k ? S_CD1 : S_CD0;
        for (int p = 0; p < o; ++p)
          for (int s = 0; s < o; ++s) {
            add(sc.t_p1[k] * I.G(p, o, r, s), op(fb, p, s), S_D, 2 * k, 1);  // q = o
            add(sc.t_p2[k] * I.G(p, s, r, o), op(fb, p, s), S_D, 2 * k, 1);  // s = o (here s plays q)
          }
        for (int q = 0; q < o; ++q)
          for (int s = 0; s < o; ++s) {  // p = o: X op [d_s d_q]^S
            const int S = k;
            if (S == 1 && q == s) continue;
            const int fa = S ? F_AB1 : F_AB0;
            double sg = 1.0;
            int a = s, b = q;
            if (s > q) {
              std::swap(a, b);
              sg = (S == 1) ? -1.0 : 1.0;
            }
            add(sc.t_p3[S] * sg * I.G(o, q, r, s), op(fa, a, b), S_C, 2 * S, 1);
          }
        for (int s = 0; s < o; ++s) add(sc.t_p5[k] * I.G(o, o, r, s), op(F_D, s), scd, 1, 2 * k);
        for (int q = 0; q < o; ++q) add(sc.t_p6[k] * I.G(o, q, r, o), op(F_D, q), scd, 1, 2 * k);
      }
      for (int p = 0; p < o; ++p) add(sc.t_p4[0] * I.G(p, o, r, o), op(F_C, p), S_DD0, 1, 0);
      break;
    }
    default:
      throw std::runtime_error("lgrow: unsupported family");
  }
  return out;
}

std::vector<RAtom> Context::rgrow(const Block& R, int f, int i, int j) const {
  const int o = R.b - 1;  // the site being prepended
  const SpinConstants& sc = spin_constants();
  std::vector<RAtom> out;
  auto add = [&](double c, int sop, Ref r, int ks2, int kR2, bool hc = false) {
    if (c == 0.0) return;
    if (!r.is_id() && r.idx < 0) return;
    out.push_back(RAtom{c, sop, r, ks2, kR2, hc});
  };
  auto op = [&](int fam, int a, int b = -1) { return R_(fam, R.op(fam, a, b)); };
  switch (f) {
    case F_C:
    case F_D: {
      const int sop = f == F_C ? S_C : S_D;
      if (i == o) add(1.0, sop, Ref{}, 1, 0);
      else add(1.0, S_I, op(f, i), 0, 1);
      break;
    }
    case F_P0: case F_P1: {
      const int S = f == F_P1 ? 1 : 0;
      add(1.0, S_I, op(f, i, j), 0, 2 * S);
      if (S == 0) add(0.5 * I.G(i, o, j, o), S_DD0, Ref{}, 0, 0);
      for (int q = o + 1; q < n; ++q) add(0.5 * I.G(i, q, j, o), S_D, op(F_D, q), 1, 1);
      for (int s = o + 1; s < n; ++s) add(0.5 * I.G(i, o, j, s) * sc.dd_swap[S], S_D, op(F_D, s), 1, 1);
      break;
    }
    case F_J: {
      add(1.0, S_I, op(F_J, i, j), 0, 0);
      add(I.G(i, j, o, o), S_CD0, Ref{}, 0, 0);
      for (int s = o + 1; s < n; ++s) add(I.G(i, j, o, s), S_C, op(F_D, s), 1, 1);
      for (int r = o + 1; r < n; ++r) add(I.G(i, j, r, o) * sc.cd_swap[0], S_D, op(F_C, r), 1, 1);
      break;
    }
    case F_K0: case F_K1: {
      const int k = f == F_K1 ? 1 : 0;
      add(1.0, S_I, op(f, i, j), 0, 2 * k);
      add(I.G(i, o, o, j), k ? S_CD1 : S_CD0, Ref{}, 2 * k, 0);
      for (int q = o + 1; q < n; ++q) add(I.G(i, q, o, j), S_C, op(F_D, q), 1, 1);
      for (int r = o + 1; r < n; ++r) add(I.G(i, o, r, j) * sc.cd_swap[k], S_D, op(F_C, r), 1, 1);
      break;
    }
    case F_SR: {
      const int p = i;
      add(1.0, S_I, op(F_SR, p), 0, 1);
      add(I.H(p, o), S_D, Ref{}, 1, 0);
      add(I.G(p, o, o, o), S_U3, Ref{}, 1, 0);
      if (std::fabs(sc.u_q3[1]) > 1e-14) throw std::runtime_error("rgrow: unexpected spin-1 Coulomb part");
      if (!R.normal) {
        for (int S = 0; S < 2; ++S) add(2.0 * sc.u_q1[S], S_C, op(S ? F_P1 : F_P0, p, o), 1, 2 * S);
        for (int k = 0; k < 2; ++k) add(sc.u_q2[k], S_D, op(k ? F_K1 : F_K0, p, o), 1, 2 * k);
        add(sc.u_q3[0], S_D, op(F_J, p, o), 1, 0);
      } else {
        // the same three parts with the integral sums over R done on normal pairs
        for (int s = o + 1; s < n; ++s)
          for (int q = o + 1; q < n; ++q) {
            for (int S = 0; S < 2; ++S) {  // sum g_pqos [d_s d_q]^S
              if (S == 1 && s == q) continue;
              const double sg = (s > q && S == 1) ? -1.0 : 1.0;
              add(sc.u_q1[S] * sg * I.G(p, q, o, s), S_C, op(S ? F_AB1 : F_AB0, std::min(s, q), std::max(s, q)), 1,
                  2 * S);
            }
            for (int k = 0; k < 2; ++k)  // sum g_pqro [c_r d_q]^k, here r = s
              add(sc.u_q2[k] * I.G(p, q, s, o), S_D, op(k ? F_B1 : F_B0, s, q), 1, 2 * k);
            add(sc.u_q3[0] * I.G(p, o, s, q), S_D, op(F_B0, s, q), 1, 0);  // sum g_pors [c_r d_s]^0, r = s, s = q
          }
      }
      for (int k = 0; k < 2; ++k) {
        const int scd = k ? S_CD1 : S_CD0;
        for (int q = o + 1; q < n; ++q) add(sc.u_q4[k] * I.G(p, q, o, o), scd, op(F_D, q), 2 * k, 1);
        for (int s = o + 1; s < n; ++s) add(sc.u_q5[k] * I.G(p, o, o, s), scd, op(F_D, s), 2 * k, 1);
      }
      for (int r = o + 1; r < n; ++r) add(sc.u_q6[0] * I.G(p, o, r, o), S_DD0, op(F_C, r), 0, 1);
      break;
    }
    case F_A0: case F_A1: case F_AB0: case F_AB1: {  // normal pairs inside (o (x) R), i <= j
      const int S = (f == F_A1 || f == F_AB1) ? 1 : 0;
      const bool cre = (f == F_A0 || f == F_A1);
      if (i > o) add(1.0, S_I, op(f, i, j), 0, 2 * S);
      else if (j > o) add(1.0, cre ? S_C : S_D, op(cre ? F_C : F_D, j), 1, 1);
      else if (S == 0) add(1.0, cre ? S_CC0 : S_DD0, Ref{}, 0, 0);
      break;
    }
    case F_B0: case F_B1: {
      const int k = f == F_B1 ? 1 : 0;
      if (i > o && j > o) add(1.0, S_I, op(f, i, j), 0, 2 * k);
      else if (j > o) add(1.0, S_C, op(F_D, j), 1, 1);          // [c_o d_j]^k
      else if (i > o) add(sc.cd_swap[k], S_D, op(F_C, i), 1, 1);  // [c_i d_o]^k
      else add(1.0, k ? S_CD1 : S_CD0, Ref{}, 2 * k, 0);
      break;
    }
    default:
      throw std::runtime_error("rgrow: unsupported family");
  }
  return out;
}

// ================================================================ block Hamiltonians
// H of (block (x) site): H_L (x) 1 + 1 (x) h_site + cross terms (L normal, site complementary)
std::vector<LAtom> Context::lgrow_h(const Block& L) const {
  const int o = L.b;
  std::vector<LAtom> raw;
  raw.push_back(LAtom{1.0, Ref{F_H, 0}, S_I, 0, 0, false});
  raw.push_back(LAtom{1.0, Ref{}, site_h(o), 0, 0, false});
  xterms::StoredLeftProv X{L};
  xterms::SiteRightProv Y{I, o};
  xterms::cross_terms(X, Y, [&](double c, const Ref& px, int py, int k2, bool hc) {
    if (c != 0.0 && px.idx >= 0) raw.push_back(LAtom{c, px, py, k2, k2, hc});
  });
  return raw;
}

// H of (site (x) block): h_site (x) 1 + 1 (x) H_R + cross terms (site normal, R complementary)
std::vector<RAtom> Context::rgrow_h(const Block& R) const {
  const int o = R.b - 1;
  std::vector<RAtom> raw;
  raw.push_back(RAtom{1.0, S_I, Ref{F_H, 0}, 0, 0, false});
  raw.push_back(RAtom{1.0, site_h(o), Ref{}, 0, 0, false});
  xterms::SiteLeftProv X{I, o};
  xterms::StoredRightProv Y{R, &I};
  xterms::cross_terms(X, Y, [&](double c, int px, const Ref& py, int k2, bool hc) {
    if (c != 0.0 && py.idx >= 0) raw.push_back(RAtom{c, px, py, k2, k2, hc});
  });
  return raw;
}

// ================================================================ linear combinations
Ref Context::make_lincomb(Block& blk, int k2, int dn, const std::vector<std::pair<Ref, double>>& parts,
                          std::vector<std::vector<std::pair<Ref, double>>>* pending,
                          std::vector<int>* pending_fam) {
  int t = -1;
  for (size_t i = 0; i < blk.tmp.size(); ++i)
    if (blk.tmp[i].k2 == k2 && blk.tmp[i].dn == dn && blk.tmp[i].buf < 0) t = (int)i;
  if (t < 0) {
    Family F;
    F.k2 = k2;
    F.dn = dn;
    F.lay = &blk.layout(k2, dn);
    blk.tmp.push_back(F);
    t = (int)blk.tmp.size() - 1;
  }
  int idx = blk.tmp[t].nops++;
  pending->push_back(parts);
  pending_fam->push_back(t);
  (void)idx;
  return Ref{F_TMP0 + t, idx};
}

void Context::materialise_lincombs(Block& blk, const std::vector<std::vector<std::pair<Ref, double>>>& pending,
                                   const std::vector<int>& pending_fam) {
  // per temp family t and source family f: coefficient matrix (nops_t x nops_f)
  std::map<int, std::vector<size_t>> by_t;
  for (size_t i = 0; i < pending.size(); ++i) by_t[pending_fam[i]].push_back(i);
  GemmBatch batch;
  std::vector<int> coef_bufs;
  for (auto& [t, items] : by_t) {
    Family& T = blk.tmp[t];
    if (T.buf >= 0) continue;
    const int64_t size = T.lay->size;
    T.buf = new_buf((int64_t)T.nops * size);
    if (size == 0 || T.nops == 0) continue;
    std::map<int, std::vector<double>> coef;  // source fam -> dense T.nops x nops_f
    int row = 0;
    for (size_t ii = 0; ii < items.size(); ++ii, ++row) {
      for (auto& [ref, c] : pending[items[ii]]) {
        const Family& S = blk.family(ref.fam);
        if (S.lay != T.lay) throw std::runtime_error("lincomb: layout mismatch");
        auto& m = coef[ref.fam];
        if (m.empty()) m.assign((size_t)T.nops * S.nops, 0.0);
        m[(size_t)row * S.nops + ref.idx] += c;
      }
    }
    GemmJob job;
    job.C = BufRef{T.buf, 0};
    job.m = T.nops;
    job.n = (int)size;
    job.ldc = size;
    job.accumulate = 0;
    job.tbeg = (int64_t)batch.terms.size();
    for (auto& [f, m] : coef) {
      const Family& S = blk.family(f);
      int cb = new_buf((int64_t)m.size());
      ex->upload(ptr(cb), m.data(), m.size() * 8);
      coef_bufs.push_back(cb);
      GemmTerm gt;
      gt.A = BufRef{cb, 0};
      gt.lda = S.nops;
      gt.B = BufRef{S.buf, 0};
      gt.ldb = size;
      gt.k = S.nops;
      gt.alpha = 1.0;
      batch.terms.push_back(gt);
    }
    job.tend = (int64_t)batch.terms.size();
    batch.jobs.push_back(job);
  }
  if (!batch.jobs.empty()) run_batch(batch);
  for (int cb : coef_bufs) free_buf(cb);
}

// Fill family `tf` of blk: op t = sum over rows[t] of coefficient * source op,
// as one GEMM (coefficient matrix) x (source family buffer) per source family.
static void lincomb_into_family(Context& C, Block& blk, int tf,
                                const std::vector<std::vector<std::pair<Ref, double>>>& rows) {
  Family& T = blk.fam[tf];
  const int64_t size = T.lay->size;
  if (size == 0 || T.nops == 0) return;
  std::map<int, std::vector<double>> coef;
  for (size_t r = 0; r < rows.size(); ++r)
    for (auto& [ref, c] : rows[r]) {
      const Family& S = blk.family(ref.fam);
      if (S.lay != T.lay) throw std::runtime_error("lincomb_into_family: layout mismatch");
      auto& m = coef[ref.fam];
      if (m.empty()) m.assign((size_t)T.nops * S.nops, 0.0);
      m[r * (size_t)S.nops + ref.idx] += c;
    }
  GemmBatch batch;
  std::vector<int> cbufs;
  GemmJob job;
  job.C = BufRef{T.buf, 0};
  job.m = T.nops;
  job.n = (int)size;
  job.ldc = size;
  job.accumulate = 0;
  job.tbeg = 0;
  for (auto& [f, m] : coef) {
    const Family& S = blk.family(f);
    int cb = C.new_buf((int64_t)m.size());
    C.ex->upload(C.ptr(cb), m.data(), m.size() * 8);
    cbufs.push_back(cb);
    GemmTerm gt;
    gt.A = BufRef{cb, 0};
    gt.lda = S.nops;
    gt.B = BufRef{S.buf, 0};
    gt.ldb = size;
    gt.k = S.nops;
    batch.terms.push_back(gt);
  }
  job.tend = (int64_t)batch.terms.size();
  batch.jobs.push_back(job);
  C.run_batch(batch);
  for (int cb : cbufs) C.free_buf(cb);
}

void Context::to_complementary(Block& R) {
  if (R.left || !R.normal) return;
  const int b = R.b;
  std::vector<std::pair<int, int>> ksym, kasym, kall;
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < b; ++j) {
      kall.push_back({i, j});
      if (i <= j) ksym.push_back({i, j});
      if (i < j) kasym.push_back({i, j});
    }
  xterms::StoredRightProv Y{R, &I};
  auto build = [&](int f, const std::vector<std::pair<int, int>>& keys, auto expr) {
    add_family(*this, R, f, keys);
    std::vector<std::vector<std::pair<Ref, double>>> rows;
    for (auto& [i, j] : keys) {
      std::vector<std::pair<Ref, double>> row;
      for (auto& [c, r] : expr(i, j)) row.push_back({r, c});
      rows.push_back(row);
    }
    lincomb_into_family(*this, R, f, rows);
  };
  build(F_P0, ksym, [&](int i, int j) { return Y.Pn(0, i, j); });
  build(F_P1, kasym, [&](int i, int j) { return Y.Pn(1, i, j); });
  build(F_J, ksym, [&](int i, int j) { return Y.Jn(i, j); });
  build(F_K0, kall, [&](int i, int j) { return Y.Kn(0, i, j); });
  build(F_K1, kall, [&](int i, int j) { return Y.Kn(1, i, j); });
  for (int f : {F_A0, F_A1, F_AB0, F_AB1, F_B0, F_B1}) {
    free_buf(R.fam[f].buf);
    R.fam[f] = Family{};
  }
  R.normal = false;
}

// ================================================================ batches
void Context::resolve(const GemmBatch& b, std::vector<RawJob>& jobs, std::vector<RawTerm>& terms, int dta, int dtb,
                      int dtc) const {
  auto P = [&](const BufRef& r, int dt) -> void* {
    int id = r.buf;
    if (id < 0) id = (-id < 8) ? ph[-id] : -1;
    if (id < 0) throw std::runtime_error("resolve: unbound placeholder buffer");
    char* base = (char*)bufs[id].p[dt];
    if (!base) throw std::runtime_error("resolve: buffer missing in requested precision");
    return base + r.off * (int64_t)dtype_size(dt);
  };
  // scale of an FP8 operand (1 for other types and unscaled buffers)
  auto S = [&](const BufRef& r, int dt) -> double {
    if (dt != DT_FP8) return 1.0;
    int id = r.buf;
    if (id < 0) id = (-id < 8) ? ph[-id] : -1;
    const DevBuf& b = bufs[id];
    if (b.fp8_seg <= 0) return 1.0;
    return b.fp8_scale[(size_t)(r.off / b.fp8_seg)];
  };
  jobs.resize(b.jobs.size());
  terms.resize(b.terms.size());
  for (size_t i = 0; i < b.jobs.size(); ++i) {
    const GemmJob& j = b.jobs[i];
    jobs[i] = RawJob{P(j.C, dtc), j.m, j.n, j.ldc, j.accumulate, 0, j.tbeg, j.tend};
  }
  for (size_t i = 0; i < b.terms.size(); ++i) {
    const GemmTerm& t = b.terms[i];
    const bool ia = t.flags & TF_IDENT_A, ib = t.flags & TF_IDENT_B;
    terms[i] = RawTerm{ia ? nullptr : P(t.A, dta), ib ? nullptr : P(t.B, dtb), t.lda, t.ldb, t.k, t.flags,
                       t.alpha * (ia ? 1.0 : S(t.A, dta)) * (ib ? 1.0 : S(t.B, dtb))};
  }
}

void Context::run_batch(const GemmBatch& b, int dta, int dtb, int dtc) {
  if (b.jobs.empty()) return;
  std::vector<RawJob> j;
  std::vector<RawTerm> t;
  resolve(b, j, t, dta, dtb, dtc);
  void* h = ex->prepare(j, t, dta, dtb, dtc);
  ex->run(h);
  ex->sync();
  ex->drop(h);
}

// ================================================================ merging
namespace {
struct LKey {
  int sop, kL2, ks2, hc, id;
  bool operator<(const LKey& o) const {
    return std::tie(sop, kL2, ks2, hc, id) < std::tie(o.sop, o.kL2, o.ks2, o.hc, o.id);
  }
};
}  // namespace

static std::vector<LAtom> merge_latoms(Context& C, Block& L, const std::vector<LAtom>& atoms, int target_dn,
                                       std::vector<std::vector<std::pair<Ref, double>>>* pending,
                                       std::vector<int>* pfam) {
  std::map<LKey, std::vector<const LAtom*>> groups;
  for (auto& a : atoms) groups[LKey{a.sop, a.kL2, a.ks2, (int)a.hc, a.L.is_id() ? 1 : 0}].push_back(&a);
  std::vector<LAtom> out;
  for (auto& [key, g] : groups) {
    if (g.size() == 1 || key.id) {
      for (auto* a : g) out.push_back(*a);
      continue;
    }
    std::vector<std::pair<Ref, double>> parts;
    for (auto* a : g) parts.push_back({a->L, a->c});
    const int dn = target_dn - C.sops[key.sop].dn;
    Ref t = C.make_lincomb(L, key.kL2, dn, parts, pending, pfam);
    out.push_back(LAtom{1.0, t, key.sop, key.kL2, key.ks2, (bool)key.hc});
  }
  return out;
}

static std::vector<RAtom> merge_ratoms(Context& C, Block& R, const std::vector<RAtom>& atoms, int target_dn,
                                       std::vector<std::vector<std::pair<Ref, double>>>* pending,
                                       std::vector<int>* pfam) {
  std::map<LKey, std::vector<const RAtom*>> groups;
  for (auto& a : atoms) groups[LKey{a.sop, a.kR2, a.ks2, (int)a.hc, a.R.is_id() ? 1 : 0}].push_back(&a);
  std::vector<RAtom> out;
  for (auto& [key, g] : groups) {
    if (g.size() == 1 || key.id) {
      for (auto* a : g) out.push_back(*a);
      continue;
    }
    std::vector<std::pair<Ref, double>> parts;
    for (auto* a : g) parts.push_back({a->R, a->c});
    const int dn = target_dn - C.sops[key.sop].dn;
    Ref t = C.make_lincomb(R, key.kL2, dn, parts, pending, pfam);
    out.push_back(RAtom{1.0, key.sop, t, key.ks2, key.kL2, (bool)key.hc});
  }
  return out;
}

// ================================================================ renormalisation
namespace {
struct Target {
  int f, idx, i, j;
};

std::vector<Target> targets_of(const Block& N) {
  std::vector<Target> t;
  for (int f = 0; f < kNumFam; ++f) {
    const Family& F = N.fam[f];
    if (!F.lay || F.nops == 0) continue;
    for (size_t key = 0; key < F.index.size(); ++key) {
      int idx = F.index[key];
      if (idx < 0) continue;
      const bool pair = F.index.size() == (size_t)N.n * N.n && !(f == F_H || f == F_C || f == F_D || f == F_SL ||
                                                                  f == F_SR);
      int i = pair ? (int)(key / N.n) : (int)key;
      int j = pair ? (int)(key % N.n) : -1;
      t.push_back(Target{f, idx, i, j});
    }
  }
  return t;
}

inline double fsign(int parity, int nket) { return (parity & nket & 1) ? -1.0 : 1.0; }
}  // namespace

std::unique_ptr<Block> Context::grow_left(Block& L, const SiteTensor& A, const Bond& nb) {
  auto N = std::make_unique<Block>();
  N->left = true;
  N->b = L.b + 1;
  N->n = n;
  N->bond = nb;
  init_families(*this, *N);
  const int o = L.b;

  // atoms per target (H gets the cross terms between L and the site)
  std::vector<Target> tg = targets_of(*N);
  std::vector<std::vector<LAtom>> atoms(tg.size());
  std::vector<std::vector<std::pair<Ref, double>>> pending;
  std::vector<int> pfam;
  for (size_t t = 0; t < tg.size(); ++t) {
    std::vector<LAtom> raw;
    if (tg[t].f == F_H) {
      raw = lgrow_h(L);
    } else {
      raw = lgrow(L, tg[t].f, tg[t].i, tg[t].j);
    }
    atoms[t] = merge_latoms(*this, L, raw, fam_dn(tg[t].f), &pending, &pfam);
  }
  materialise_lincombs(L, pending, pfam);

  // rows of each new sector: A blocks (l, sigma, a)
  const int nsec_new = (int)nb.secs.size();
  std::vector<std::vector<int>> rows_of(nsec_new);
  for (size_t bi = 0; bi < A.blocks.size(); ++bi) rows_of[A.blocks[bi].s1].push_back((int)bi);

  const int64_t tbudget = (int64_t)1 << 27;
  size_t t0 = 0;
  while (t0 < tg.size()) {
    GemmBatch s1, s2;
    int64_t tsize = 0;
    size_t t1 = t0;
    std::vector<std::tuple<int64_t, int64_t>> pieces;  // unused bookkeeping
    int tbuf = -1;
    // first pass: size of the chunk
    std::vector<int64_t> need(tg.size(), 0);
    while (t1 < tg.size()) {
      const Family& F = N->fam[tg[t1].f];
      int64_t s = 0;
      for (const OpBlock& ob : F.lay->blocks)
        for (int bi : rows_of[ob.bra]) s += (int64_t)A.blocks[bi].rows * nb.secs[ob.ket].dim;
      if (t1 > t0 && tsize + s > tbudget) break;
      tsize += s;
      need[t1] = s;
      ++t1;
    }
    tbuf = new_buf(std::max<int64_t>(tsize, 1));
    int64_t toff = 0;
    for (size_t t = t0; t < t1; ++t) {
      const Target& T = tg[t];
      const Family& F = N->fam[T.f];
      const int k2 = F.k2;
      for (const OpBlock& ob : F.lay->blocks) {
        const Sector& sa_b = nb.secs[ob.bra];
        const Sector& sa_k = nb.secs[ob.ket];
        const int da = sa_k.dim;
        const int64_t s2_tbeg = (int64_t)s2.terms.size();
        for (int bib : rows_of[ob.bra]) {
          const auto& Ab = A.blocks[bib];  // (l', sigma', a')
          const Sector& slb = L.bond.secs[Ab.s0];
          const int sigb = Ab.sig;
          // stage 1 job: T_ (D_l' x D_a)
          GemmJob j1;
          j1.C = BufRef{tbuf, toff};
          j1.m = Ab.rows;
          j1.n = da;
          j1.ldc = da;
          j1.accumulate = 0;
          j1.tbeg = (int64_t)s1.terms.size();
          for (const LAtom& at : atoms[t]) {
            const SiteOp& so = sops[at.sop];
            const Family* LF = at.L.is_id() ? nullptr : &L.family(at.L.fam);
            for (int bik : rows_of[ob.ket]) {
              const auto& Ak = A.blocks[bik];  // (l, sigma, a)
              const Sector& slk = L.bond.secs[Ak.s0];
              const int sigk = Ak.sig;
              double r;
              int blk_idx = -1;
              int64_t lda = 0;
              int flags = 0;
              double w;
              if (!at.hc) {
                r = so.r[sigb][sigk];
                if (r == 0.0) continue;
                if (LF) {
                  blk_idx = LF->lay->find(Ab.s0, Ak.s0);
                  if (blk_idx < 0) continue;
                  lda = LF->lay->blocks[blk_idx].ld;
                } else if (Ab.s0 != Ak.s0) {
                  continue;
                }
                w = coupled_factor(slb.s2, slk.s2, at.kL2, kLocS2[sigb], kLocS2[sigk], at.ks2, sa_b.s2, sa_k.s2, k2) *
                    fsign(so.parity, slk.n);
              } else {
                r = so.r[sigk][sigb];
                if (r == 0.0) continue;
                if (LF) {
                  blk_idx = LF->lay->find(Ak.s0, Ab.s0);
                  if (blk_idx < 0) continue;
                  lda = LF->lay->blocks[blk_idx].ld;
                  flags |= TF_TRANS_A;
                } else if (Ab.s0 != Ak.s0) {
                  continue;
                }
                w = coupled_factor(slk.s2, slb.s2, at.kL2, kLocS2[sigk], kLocS2[sigb], at.ks2, sa_k.s2, sa_b.s2, k2) *
                    fsign(so.parity, slb.n);
              }
              if (w == 0.0) continue;
              GemmTerm gt;
              if (LF) {
                gt.A = BufRef{LF->buf, (int64_t)at.L.idx * LF->lay->size + LF->lay->blocks[blk_idx].off};
                gt.lda = lda;
              } else {
                flags |= TF_IDENT_A;
              }
              gt.flags = flags;
              gt.B = BufRef{A.buf, Ak.off};
              gt.ldb = Ak.cols;
              gt.k = slk.dim;
              gt.alpha = at.c * w * r;
              s1.terms.push_back(gt);
              if (LF) s1.flops += 2.0 * Ab.rows * da * slk.dim;
            }
          }
          j1.tend = (int64_t)s1.terms.size();
          if (j1.tend > j1.tbeg) {
            s1.jobs.push_back(j1);
            // stage 2 term: A(l',sigma',a')^T @ T_
            GemmTerm g2;
            g2.A = BufRef{A.buf, Ab.off};
            g2.lda = Ab.cols;
            g2.flags = TF_TRANS_A;
            g2.B = BufRef{tbuf, toff};
            g2.ldb = da;
            g2.k = Ab.rows;
            g2.alpha = 1.0;
            s2.terms.push_back(g2);
            s2.flops += 2.0 * sa_b.dim * da * Ab.rows;
          }
          toff += (int64_t)Ab.rows * da;
        }
        GemmJob j2;
        j2.C = BufRef{F.buf, (int64_t)T.idx * F.lay->size + ob.off};
        j2.m = sa_b.dim;
        j2.n = da;
        j2.ldc = ob.ld;
        j2.accumulate = 0;
        j2.tbeg = s2_tbeg;
        j2.tend = (int64_t)s2.terms.size();
        s2.jobs.push_back(j2);
      }
    }
    run_batch(s1);
    run_batch(s2);
    free_buf(tbuf);
    t0 = t1;
  }
  for (auto& t : L.tmp) free_buf(t.buf);
  L.tmp.clear();
  return N;
}

std::unique_ptr<Block> Context::grow_right(Block& R, const SiteTensor& B, const Bond& nb) {
  auto N = std::make_unique<Block>();
  N->left = false;
  N->b = R.b - 1;
  N->n = n;
  // normal pairs while the right block is the smaller side of the chain
  N->normal = R.normal && (n - N->b) <= N->b;
  if (R.normal && !N->normal) to_complementary(R);
  N->bond = nb;
  init_families(*this, *N);
  const int o = R.b - 1;

  std::vector<Target> tg = targets_of(*N);
  std::vector<std::vector<RAtom>> atoms(tg.size());
  std::vector<std::vector<std::pair<Ref, double>>> pending;
  std::vector<int> pfam;
  for (size_t t = 0; t < tg.size(); ++t) {
    std::vector<RAtom> raw;
    if (tg[t].f == F_H) {
      raw = rgrow_h(R);
    } else {
      raw = rgrow(R, tg[t].f, tg[t].i, tg[t].j);
    }
    atoms[t] = merge_ratoms(*this, R, raw, fam_dn(tg[t].f), &pending, &pfam);
  }
  materialise_lincombs(R, pending, pfam);

  // columns of each new sector c: B blocks (c, sigma, r)
  const int nsec_new = (int)nb.secs.size();
  std::vector<std::vector<int>> cols_of(nsec_new);
  for (size_t bi = 0; bi < B.blocks.size(); ++bi) cols_of[B.blocks[bi].s0].push_back((int)bi);

  const int64_t tbudget = (int64_t)1 << 27;
  size_t t0 = 0;
  while (t0 < tg.size()) {
    GemmBatch s1, s2;
    int64_t tsize = 0;
    size_t t1 = t0;
    while (t1 < tg.size()) {
      const Family& F = N->fam[tg[t1].f];
      int64_t s = 0;
      for (const OpBlock& ob : F.lay->blocks)
        for (int bi : cols_of[ob.bra]) s += (int64_t)B.blocks[bi].cols * nb.secs[ob.ket].dim;
      if (t1 > t0 && tsize + s > tbudget) break;
      tsize += s;
      ++t1;
    }
    int ubuf = new_buf(std::max<int64_t>(tsize, 1));
    int64_t uoff = 0;
    for (size_t t = t0; t < t1; ++t) {
      const Target& T = tg[t];
      const Family& F = N->fam[T.f];
      const int k2 = F.k2;
      for (const OpBlock& ob : F.lay->blocks) {
        const Sector& sc_b = nb.secs[ob.bra];
        const Sector& sc_k = nb.secs[ob.ket];
        const int dc = sc_k.dim;
        const int64_t s2_tbeg = (int64_t)s2.terms.size();
        for (int bib : cols_of[ob.bra]) {
          const auto& Bb = B.blocks[bib];  // (c', sigma', r')
          const Sector& srb = R.bond.secs[Bb.s1];
          const int sigb = Bb.sig;
          GemmJob j1;
          j1.C = BufRef{ubuf, uoff};
          j1.m = Bb.cols;  // D_r'
          j1.n = dc;
          j1.ldc = dc;
          j1.accumulate = 0;
          j1.tbeg = (int64_t)s1.terms.size();
          for (const RAtom& at : atoms[t]) {
            const SiteOp& so = sops[at.sop];
            const Family* RF = at.R.is_id() ? nullptr : &R.family(at.R.fam);
            const int rpar = RF ? (std::abs(RF->dn) & 1) : 0;
            for (int bik : cols_of[ob.ket]) {
              const auto& Bk = B.blocks[bik];  // (c, sigma, r)
              const Sector& srk = R.bond.secs[Bk.s1];
              const int sigk = Bk.sig;
              double r, w;
              int blk_idx = -1, flags = TF_TRANS_B;
              int64_t lda = 0;
              if (!at.hc) {
                r = so.r[sigb][sigk];
                if (r == 0.0) continue;
                if (RF) {
                  blk_idx = RF->lay->find(Bb.s1, Bk.s1);
                  if (blk_idx < 0) continue;
                  lda = RF->lay->blocks[blk_idx].ld;
                } else if (Bb.s1 != Bk.s1) {
                  continue;
                }
                w = coupled_factor(kLocS2[sigb], kLocS2[sigk], at.ks2, srb.s2, srk.s2, at.kR2, sc_b.s2, sc_k.s2, k2) *
                    fsign(rpar, kLocN[sigk]);
              } else {
                r = so.r[sigk][sigb];
                if (r == 0.0) continue;
                if (RF) {
                  blk_idx = RF->lay->find(Bk.s1, Bb.s1);
                  if (blk_idx < 0) continue;
                  lda = RF->lay->blocks[blk_idx].ld;
                  flags |= TF_TRANS_A;
                } else if (Bb.s1 != Bk.s1) {
                  continue;
                }
                w = coupled_factor(kLocS2[sigk], kLocS2[sigb], at.ks2, srk.s2, srb.s2, at.kR2, sc_k.s2, sc_b.s2, k2) *
                    fsign(rpar, kLocN[sigb]);
              }
              if (w == 0.0) continue;
              GemmTerm gt;
              if (RF) {
                gt.A = BufRef{RF->buf, (int64_t)at.R.idx * RF->lay->size + RF->lay->blocks[blk_idx].off};
                gt.lda = lda;
              } else {
                flags |= TF_IDENT_A;
              }
              gt.flags = flags;
              gt.B = BufRef{B.buf, Bk.off};  // (D_c x D_r) used transposed
              gt.ldb = Bk.cols;
              gt.k = srk.dim;
              gt.alpha = at.c * w * r;
              s1.terms.push_back(gt);
              if (RF) s1.flops += 2.0 * Bb.cols * dc * srk.dim;
            }
          }
          j1.tend = (int64_t)s1.terms.size();
          if (j1.tend > j1.tbeg) {
            s1.jobs.push_back(j1);
            GemmTerm g2;
            g2.A = BufRef{B.buf, Bb.off};  // (D_c' x D_r')
            g2.lda = Bb.cols;
            g2.B = BufRef{ubuf, uoff};     // (D_r' x D_c)
            g2.ldb = dc;
            g2.k = Bb.cols;
            g2.alpha = 1.0;
            s2.terms.push_back(g2);
            s2.flops += 2.0 * sc_b.dim * dc * Bb.cols;
          }
          uoff += (int64_t)Bb.cols * dc;
        }
        GemmJob j2;
        j2.C = BufRef{F.buf, (int64_t)T.idx * F.lay->size + ob.off};
        j2.m = sc_b.dim;
        j2.n = dc;
        j2.ldc = ob.ld;
        j2.accumulate = 0;
        j2.tbeg = s2_tbeg;
        j2.tend = (int64_t)s2.terms.size();
        s2.jobs.push_back(j2);
      }
    }
    run_batch(s1);
    run_batch(s2);
    free_buf(ubuf);
    t0 = t1;
  }
  for (auto& t : R.tmp) free_buf(t.buf);
  R.tmp.clear();
  return N;
}

// ================================================================ psi layout
void PsiLayout::build(const Bond& lb, const Bond& rb, int n_elec, int two_s) {
  sbs.clear();
  size = 0;
  std::vector<std::pair<int, int>> akeys, ckeys;
  for (auto& s : lb.secs)
    for (int sig = 0; sig < 3; ++sig)
      for (int sa = std::abs(s.s2 - kLocS2[sig]); sa <= s.s2 + kLocS2[sig]; sa += 2)
        if (s.dim > 0) akeys.push_back({s.n + kLocN[sig], sa});
  for (auto& s : rb.secs)
    for (int sig = 0; sig < 3; ++sig)
      for (int sc = std::abs(s.s2 - kLocS2[sig]); sc <= s.s2 + kLocS2[sig]; sc += 2)
        if (s.dim > 0) ckeys.push_back({s.n + kLocN[sig], sc});
  std::sort(akeys.begin(), akeys.end());
  akeys.erase(std::unique(akeys.begin(), akeys.end()), akeys.end());
  std::sort(ckeys.begin(), ckeys.end());
  ckeys.erase(std::unique(ckeys.begin(), ckeys.end()), ckeys.end());
  for (auto& [an, as2] : akeys)
    for (auto& [cn, cs2] : ckeys) {
      if (an + cn != n_elec || !tri2(as2, cs2, two_s)) continue;
      SB sb{an, as2, cn, cs2, 0, 0, 0, 0, 0, {}, {}};
      for (size_t il = 0; il < lb.secs.size(); ++il)
        for (int s1 = 0; s1 < 3; ++s1) {
          const Sector& s = lb.secs[il];
          if (s.n + kLocN[s1] == an && tri2(s.s2, kLocS2[s1], as2) && s.dim > 0) {
            sb.rows.push_back(Row{(int)il, s1, sb.nrows, s.dim, 0});
            sb.nrows += s.dim;
          }
        }
      for (int s2 = 0; s2 < 3; ++s2)
        for (size_t ir = 0; ir < rb.secs.size(); ++ir) {
          const Sector& s = rb.secs[ir];
          if (kLocN[s2] + s.n == cn && tri2(kLocS2[s2], s.s2, cs2) && s.dim > 0) {
            sb.cols.push_back(Col{s2, (int)ir, sb.ncols, s.dim, sb.pncols});
            sb.ncols += s.dim;
            sb.pncols += pad_up(s.dim);
          }
        }
      if (sb.nrows == 0 || sb.ncols == 0) continue;
      {
        std::vector<int> ord(sb.rows.size());
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sb.rows[x].s1 < sb.rows[y].s1; });
        int r = 0;
        for (int i : ord) {
          sb.rows[i].ir0 = r;
          r += sb.rows[i].dl;
        }
      }
      sb.off = size;
      size += (int64_t)sb.nrows * sb.ncols;
      sb.poff = psize;
      psize += (int64_t)sb.nrows * sb.pncols;
      sbs.push_back(sb);
    }
}

std::vector<int> PsiLayout::pack_map() const {
  std::vector<int> m((size_t)psize, -1);
  for (const SB& sb : sbs)
    for (const Row& rr : sb.rows)
      for (int i = 0; i < rr.dl; ++i) {
        const int64_t r = rr.r0 + i, ir = rr.ir0 + i;
        for (const Col& c : sb.cols)
          for (int q = 0; q < c.dr; ++q)
            m[(size_t)(sb.poff + ir * sb.pncols + c.pc0 + q)] = (int)(sb.off + r * sb.ncols + c.c0 + q);
      }
  return m;
}

std::vector<int> PsiLayout::unpack_map() const {
  std::vector<int> m((size_t)size, -1);
  for (const SB& sb : sbs)
    for (const Row& rr : sb.rows)
      for (int i = 0; i < rr.dl; ++i) {
        const int64_t r = rr.r0 + i, ir = rr.ir0 + i;
        for (int c = 0; c < sb.ncols; ++c) m[(size_t)(sb.off + r * sb.ncols + c)] = (int)(sb.off + ir * sb.ncols + c);
      }
  return m;
}

}  // namespace dmrg
