// Cross terms of the Hamiltonian between a left part X and a right part Y of
// the chain (normal operators on X, complementary operators on Y), written
// once for every pairing that occurs: stored block (x) site, site (x) stored
// block, and enlarged block (x) enlarged block.  Providers return operator
// expressions as lists of (coefficient, payload).
#pragma once
#include <algorithm>
#include <vector>

#include "planner.hpp"

namespace dmrg {
namespace xterms {
template <class P>
using Expr = std::vector<std::pair<double, P>>;

struct StoredLeftProv {
  const Block& L;
  std::vector<int> orbs() const {
    std::vector<int> v;
    for (int i = 0; i < L.b; ++i) v.push_back(i);
    return v;
  }
  Expr<Ref> one(int f, int i, int j = -1) const {
    int idx = L.op(f, i, j);
    if (idx < 0) return {};
    return {{1.0, Ref{f, idx}}};
  }
  Expr<Ref> C(int p) const { return one(F_C, p); }
  Expr<Ref> A(int S, int i, int j) const { return one(S ? F_A1 : F_A0, i, j); }
  Expr<Ref> B(int k, int i, int j) const { return one(k ? F_B1 : F_B0, i, j); }
  Expr<Ref> SL(int r) const { return one(F_SL, r); }
};

struct SiteRightProv {
  const Integrals& I;
  int o;
  std::vector<int> orbs() const { return {o}; }
  Expr<int> C(int r) const { return r == o ? Expr<int>{{1.0, S_C}} : Expr<int>{}; }
  Expr<int> P(int S, int i, int j) const {
    if (S) return {};
    return {{0.5 * I.G(i, o, j, o), S_DD0}};
  }
  Expr<int> Q(int k, int i, int j) const {
    const SpinConstants& sc = spin_constants();
    return {{sc.ee[k] * I.G(i, j, o, o) - sc.ex[k] * I.G(i, o, o, j), k ? S_CD1 : S_CD0}};
  }
  Expr<int> SR(int p) const { return {{I.H(p, o), S_D}, {I.G(p, o, o, o), S_U3}}; }
};

struct SiteLeftProv {
  const Integrals& I;
  int o;
  std::vector<int> orbs() const { return {o}; }
  Expr<int> C(int p) const { return p == o ? Expr<int>{{1.0, S_C}} : Expr<int>{}; }
  Expr<int> A(int S, int, int) const { return S ? Expr<int>{} : Expr<int>{{1.0, S_CC0}}; }
  Expr<int> B(int k, int, int) const { return {{1.0, k ? S_CD1 : S_CD0}}; }
  Expr<int> SL(int r) const { return {{I.G(o, o, r, o), S_T3}}; }
};

struct StoredRightProv {
  const Block& R;
  std::vector<int> orbs() const {
    std::vector<int> v;
    for (int i = R.b; i < R.n; ++i) v.push_back(i);
    return v;
  }
  Expr<Ref> one(int f, int i, int j = -1, double c = 1.0) const {
    int idx = R.op(f, i, j);
    if (idx < 0 || c == 0.0) return {};
    return {{c, Ref{f, idx}}};
  }
  const Integrals* I = nullptr;  // needed when R holds normal pairs
  // Complementary pair operators written over the normal pairs of R:
  //   P^S_ij = 1/2 sum_{s,q in R} g_iqjs [d_s d_q]^S,  J_ij = sum g_ijrs [c_r d_s]^0,
  //   K^k_ij = sum g_iqrj [c_r d_q]^k.
  Expr<Ref> Pn(int S, int i, int j) const {
    Expr<Ref> e;
    for (int s = R.b; s < R.n; ++s)
      for (int q = R.b; q < R.n; ++q) {
        if (S == 1 && s == q) continue;
        const double sg = (s > q && S == 1) ? -1.0 : 1.0;
        const double c = 0.5 * sg * I->G(i, q, j, s);
        if (c == 0.0) continue;
        const int f = S ? F_AB1 : F_AB0;
        int idx = R.op(f, std::min(s, q), std::max(s, q));
        if (idx >= 0) e.push_back({c, Ref{f, idx}});
      }
    return e;
  }
  Expr<Ref> Jn(int i, int j) const {
    Expr<Ref> e;
    for (int r = R.b; r < R.n; ++r)
      for (int s = R.b; s < R.n; ++s) {
        const double c = I->G(i, j, r, s);
        int idx = R.op(F_B0, r, s);
        if (c != 0.0 && idx >= 0) e.push_back({c, Ref{F_B0, idx}});
      }
    return e;
  }
  Expr<Ref> Kn(int k, int i, int j) const {
    Expr<Ref> e;
    const int f = k ? F_B1 : F_B0;
    for (int r = R.b; r < R.n; ++r)
      for (int q = R.b; q < R.n; ++q) {
        const double c = I->G(i, q, r, j);
        int idx = R.op(f, r, q);
        if (c != 0.0 && idx >= 0) e.push_back({c, Ref{f, idx}});
      }
    return e;
  }
  static Expr<Ref> scaled(Expr<Ref> e, double s) {
    for (auto& x : e) x.first *= s;
    return e;
  }
  Expr<Ref> C(int r) const { return one(F_C, r); }
  Expr<Ref> P(int S, int i, int j) const { return R.normal ? Pn(S, i, j) : one(S ? F_P1 : F_P0, i, j); }
  Expr<Ref> Q(int k, int i, int j) const {
    const SpinConstants& sc = spin_constants();
    Expr<Ref> e = R.normal ? scaled(Kn(k, i, j), -sc.ex[k]) : one(k ? F_K1 : F_K0, i, j, -sc.ex[k]);
    if (k == 0) {
      auto jj = R.normal ? scaled(Jn(i, j), sc.ee[0]) : one(F_J, std::min(i, j), std::max(i, j), sc.ee[0]);
      e.insert(e.end(), jj.begin(), jj.end());
    }
    return e;
  }
  Expr<Ref> SR(int p) const { return one(F_SR, p); }
};

struct CompLeftProv {  // L' = L (x) site o
  const Context& C;
  const Block& L;
  std::vector<int> orbs() const {
    std::vector<int> v;
    for (int i = 0; i <= L.b; ++i) v.push_back(i);
    return v;
  }
  Expr<LAtom> wrap(std::vector<LAtom> a) const {
    Expr<LAtom> e;
    for (auto& x : a) {
      double c = x.c;
      x.c = 1.0;
      e.push_back({c, x});
    }
    return e;
  }
  Expr<LAtom> Cc(int p) const { return wrap(C.lgrow(L, F_C, p, -1)); }
  Expr<LAtom> A(int S, int i, int j) const { return wrap(C.lgrow(L, S ? F_A1 : F_A0, i, j)); }
  Expr<LAtom> B(int k, int i, int j) const { return wrap(C.lgrow(L, k ? F_B1 : F_B0, i, j)); }
  Expr<LAtom> SL(int r) const { return wrap(C.lgrow(L, F_SL, r, -1)); }
};

struct CompRightProv {  // R' = site o (x) R
  const Context& C;
  const Block& R;
  std::vector<int> orbs() const {
    std::vector<int> v;
    for (int i = R.b - 1; i < R.n; ++i) v.push_back(i);
    return v;
  }
  Expr<RAtom> wrap(std::vector<RAtom> a, double scale = 1.0) const {
    Expr<RAtom> e;
    for (auto& x : a) {
      double c = x.c * scale;
      x.c = 1.0;
      if (c != 0.0) e.push_back({c, x});
    }
    return e;
  }
  Expr<RAtom> Cc(int r) const { return wrap(C.rgrow(R, F_C, r, -1)); }
  Expr<RAtom> P(int S, int i, int j) const { return wrap(C.rgrow(R, S ? F_P1 : F_P0, i, j)); }
  Expr<RAtom> Q(int k, int i, int j) const {
    const SpinConstants& sc = spin_constants();
    Expr<RAtom> e = wrap(C.rgrow(R, k ? F_K1 : F_K0, i, j), -sc.ex[k]);
    if (k == 0) {
      auto jj = wrap(C.rgrow(R, F_J, std::min(i, j), std::max(i, j)), sc.ee[0]);
      e.insert(e.end(), jj.begin(), jj.end());
    }
    return e;
  }
  Expr<RAtom> SR(int p) const { return wrap(C.rgrow(R, F_SR, p, -1)); }
};

// accessors that normalise the C() naming
template <class X> auto xC(const X& x, int p) { return x.C(p); }
inline auto xC(const CompLeftProv& x, int p) { return x.Cc(p); }
template <class Y> auto yC(const Y& y, int r) { return y.C(r); }
inline auto yC(const CompRightProv& y, int r) { return y.Cc(r); }

// emit(c, px, py, k2, hc) for every cross term between X (left part) and Y.
template <class XP, class YP, class Emit>
void cross_terms(const XP& X, const YP& Y, Emit emit) {
  const SpinConstants& sc = spin_constants();
  const auto xo = X.orbs(), yo = Y.orbs();
  // pair creation / annihilation: sum_{i<=j} (2 - delta_ij) ap_S [A^S_ij (x) P^S_ij]^0 + h.c.
  for (int i : xo)
    for (int j : xo) {
      if (j < i) continue;
      for (int S = 0; S < 2; ++S) {
        if (S == 1 && i == j) continue;
        auto xa = X.A(S, i, j);
        if (xa.empty()) continue;
        auto yp = Y.P(S, i, j);
        const double f = sc.ap[S] * (i == j ? 1.0 : 2.0);
        for (auto& [ca, pa] : xa)
          for (auto& [cb, pb] : yp) {
            emit(f * ca * cb, pa, pb, 2 * S, false);
            emit(f * ca * cb, pa, pb, 2 * S, true);
          }
      }
    }
  // density-density: sum_{i,j} [B^k_ij (x) Q^k_ij]^0
  for (int i : xo)
    for (int j : xo)
      for (int k = 0; k < 2; ++k) {
        auto xb = X.B(k, i, j);
        if (xb.empty()) continue;
        auto yq = Y.Q(k, i, j);
        for (auto& [ca, pa] : xb)
          for (auto& [cb, pb] : yq) emit(ca * cb, pa, pb, 2 * k, false);
      }
  // one creator on X, three operators on Y (+ one-electron hopping)
  for (int p : xo) {
    auto xc = xC(X, p);
    auto ys = Y.SR(p);
    for (auto& [ca, pa] : xc)
      for (auto& [cb, pb] : ys) {
        emit(sc.cs * ca * cb, pa, pb, 1, false);
        emit(sc.cs * ca * cb, pa, pb, 1, true);
      }
  }
  // three operators on X, one creator on Y
  for (int r : yo) {
    auto xs = X.SL(r);
    auto yc = yC(Y, r);
    for (auto& [ca, pa] : xs)
      for (auto& [cb, pb] : yc) {
        emit(sc.sc * ca * cb, pa, pb, 1, false);
        emit(sc.sc * ca * cb, pa, pb, 1, true);
      }
  }
}
}  // namespace xterms

}  // namespace dmrg
