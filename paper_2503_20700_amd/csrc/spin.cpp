#include "spin.hpp"

#include <cmath>
#include <stdexcept>

#include "su2.hpp"

namespace dmrg {

// ---------------------------------------------------------------- component space
CForm cf_leaf(int L, int pos) {
  CForm f;
  f.L = L;
  std::vector<double> up(1u << L, 0.0), dn(1u << L, 0.0);
  up[0] = 1.0;
  dn[1u << pos] = 1.0;
  f.comp[1] = up;
  f.comp[-1] = dn;
  return f;
}

CForm cf_couple(const CForm& a, int ka2, const CForm& b, int kb2, int k2) {
  CForm out;
  out.L = a.L;
  const size_t dim = 1u << a.L;
  for (int q = -k2; q <= k2; q += 2) {
    std::vector<double> v(dim, 0.0);
    for (const auto& [qa, va] : a.comp) {
      int qb = q - qa;
      auto itb = b.comp.find(qb);
      if (itb == b.comp.end()) continue;
      double c = cg2(ka2, qa, kb2, qb, k2, q);
      if (c == 0.0) continue;
      for (size_t ia = 0; ia < dim; ++ia) {
        if (va[ia] == 0.0) continue;
        for (size_t ib = 0; ib < dim; ++ib) {
          if (itb->second[ib] == 0.0) continue;
          v[ia | ib] += c * va[ia] * itb->second[ib];
        }
      }
    }
    out.comp[q] = v;
  }
  return out;
}

double cf_dot(const std::vector<double>& x, const std::vector<double>& y) {
  double s = 0.0;
  for (size_t i = 0; i < x.size(); ++i) s += x[i] * y[i];
  return s;
}

std::vector<double> cf_permute(const std::vector<double>& v, int L, const std::vector<int>& perm) {
  int inv = 0;
  for (int i = 0; i < L; ++i)
    for (int j = i + 1; j < L; ++j)
      if (perm[i] > perm[j]) ++inv;
  const double sgn = (inv & 1) ? -1.0 : 1.0;
  std::vector<double> out(v.size(), 0.0);
  for (size_t idx = 0; idx < v.size(); ++idx) {
    if (v[idx] == 0.0) continue;
    size_t nidx = 0;
    for (int p = 0; p < L; ++p)
      if ((idx >> perm[p]) & 1u) nidx |= (1u << p);
    out[nidx] += sgn * v[idx];
  }
  return out;
}

namespace {
// bit value for a projection m (doubled): +1 -> 0, -1 -> 1
inline size_t mb(int m2, int pos) { return (m2 > 0 ? 0u : 1u) << pos; }
inline double phi(int s2) { return s2 > 0 ? -1.0 : 1.0; }
}  // namespace

std::vector<double> phys_e4_pair(int L) {
  std::vector<double> v(1u << L, 0.0);
  for (int s : {1, -1})
    for (int t : {1, -1})
      v[mb(s, 0) | mb(t, 1) | mb(-t, 2) | mb(-s, 3)] += phi(t) * phi(s);
  return v;
}
std::vector<double> phys_ee(int L) {
  std::vector<double> v(1u << L, 0.0);
  for (int s : {1, -1})
    for (int t : {1, -1})
      v[mb(s, 0) | mb(-s, 1) | mb(t, 2) | mb(-t, 3)] += phi(s) * phi(t);
  return v;
}
std::vector<double> phys_exch(int L) {
  std::vector<double> v(1u << L, 0.0);
  for (int s : {1, -1})
    for (int t : {1, -1})
      v[mb(s, 0) | mb(-t, 1) | mb(t, 2) | mb(-s, 3)] += phi(t) * phi(s);
  return v;
}
std::vector<double> phys_cz(int L) {
  std::vector<double> v(1u << L, 0.0);
  for (int s : {1, -1}) v[mb(s, 0) | mb(-s, 1)] += phi(s);
  return v;
}
std::vector<double> phys_xc(int L) {
  std::vector<double> v(1u << L, 0.0);
  for (int t : {1, -1}) v[mb(-t, 0) | mb(t, 1)] += phi(t);
  return v;
}
std::vector<double> phys_t3(int L) {
  // tilde(+1/2) = sum_s phi(s) c_{p,s} d_{s',+1/2} d_{q,-s}
  std::vector<double> v(1u << L, 0.0);
  for (int s : {1, -1}) v[mb(s, 0) | mb(1, 1) | mb(-s, 2)] += phi(s);
  return v;
}
std::vector<double> phys_u3(int L) {
  // tilde(+1/2) = sum_t phi(t) c_{r,t} d_{s,-t} d_{q,+1/2}
  std::vector<double> v(1u << L, 0.0);
  for (int t : {1, -1}) v[mb(t, 0) | mb(-t, 1) | mb(1, 2)] += phi(t);
  return v;
}

namespace {
// Coupled form of a side over consecutive positions [p0, p0+n).
std::vector<std::pair<int, CForm>> side_forms(int L, int p0, int n, int k12) {
  std::vector<std::pair<int, CForm>> out;
  if (n == 1) {
    out.push_back({1, cf_leaf(L, p0)});
  } else if (n == 2) {
    for (int k : {0, 2}) out.push_back({k, cf_couple(cf_leaf(L, p0), 1, cf_leaf(L, p0 + 1), 1, k)});
  } else if (n == 3) {
    CForm a = cf_couple(cf_leaf(L, p0), 1, cf_leaf(L, p0 + 1), 1, k12);
    for (int k = (k12 > 1 ? k12 - 1 : 1 - k12); k <= k12 + 1; k += 2)
      out.push_back({k, cf_couple(a, k12, cf_leaf(L, p0 + 2), 1, k)});
  } else {
    throw std::runtime_error("side_forms: unsupported side size");
  }
  return out;
}
}  // namespace

std::map<std::pair<int, int>, double> split_coeffs(const std::vector<double>& target, int L, int k2,
                                                   const SplitSpec& s) {
  std::vector<int> perm(s.xs);
  perm.insert(perm.end(), s.ys.begin(), s.ys.end());
  if ((int)perm.size() != L) throw std::runtime_error("split_coeffs: bad split");
  std::vector<double> t = cf_permute(target, L, perm);
  const int nx = (int)s.xs.size(), ny = (int)s.ys.size();
  auto xf = side_forms(L, 0, nx, s.x_k12);
  auto yf = side_forms(L, nx, ny, s.y_k12);
  std::map<std::pair<int, int>, double> out;
  std::vector<double> resid = t;
  for (auto& [kx, fx] : xf) {
    for (auto& [ky, fy] : yf) {
      if (!tri2(kx, ky, k2)) continue;
      CForm b = cf_couple(fx, kx, fy, ky, k2);
      const auto& bv = b.comp.at(k2);
      double c = cf_dot(t, bv);
      if (std::fabs(c) < 1e-14) continue;
      out[{kx, ky}] = c;
      for (size_t i = 0; i < resid.size(); ++i) resid[i] -= c * bv[i];
    }
  }
  double r = 0.0;
  for (double x : resid) r = std::max(r, std::fabs(x));
  if (r > 1e-12) throw std::runtime_error("split_coeffs: target not spanned by the requested coupled forms");
  return out;
}

// ---------------------------------------------------------------- site operators
namespace {
using Mat4 = std::array<std::array<double, 4>, 4>;

Mat4 zero4() {
  Mat4 m{};
  return m;
}
Mat4 mul4(const Mat4& a, const Mat4& b) {
  Mat4 c = zero4();
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      if (a[i][k] != 0.0)
        for (int j = 0; j < 4; ++j) c[i][j] += a[i][k] * b[k][j];
  return c;
}
Mat4 transpose4(const Mat4& a) {
  Mat4 t = zero4();
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) t[j][i] = a[i][j];
  return t;
}
// local Fock basis: 0 = |0>, 1 = |up>, 2 = |dn>, 3 = a+_up a+_dn |0>
Mat4 adag_up() {
  Mat4 m = zero4();
  m[1][0] = 1.0;
  m[3][2] = 1.0;
  return m;
}
Mat4 adag_dn() {
  Mat4 m = zero4();
  m[2][0] = 1.0;
  m[3][1] = -1.0;
  return m;
}
// component matrices of the elementary tensors
Mat4 elem(char type, int m2) {
  if (type == 'c') return m2 > 0 ? adag_up() : adag_dn();
  // d_{+1/2} = a_dn, d_{-1/2} = -a_up
  if (m2 > 0) return transpose4(adag_dn());
  Mat4 a = transpose4(adag_up());
  for (auto& row : a)
    for (double& x : row) x = -x;
  return a;
}

// (multiplet sigma, projection m2) -> local Fock index
int fock_of(int sig, int m2) {
  if (sig == 0) return 0;
  if (sig == 2) return 3;
  return m2 > 0 ? 1 : 2;
}

SiteOp reduce(const std::string& name, const Mat4& m, int k2, int dn, int parity) {
  SiteOp op;
  op.name = name;
  op.k2 = k2;
  op.dn = dn;
  op.parity = parity;
  for (int sb = 0; sb < 3; ++sb)
    for (int sk = 0; sk < 3; ++sk) {
      double val = 0.0;
      bool set = false;
      for (int mk = -kLocS2[sk]; mk <= kLocS2[sk]; mk += 2) {
        int mb2 = mk + k2;  // component q = k2
        if (std::abs(mb2) > kLocS2[sb]) continue;
        double c = cg2(kLocS2[sk], mk, k2, k2, kLocS2[sb], mb2);
        double el = m[fock_of(sb, mb2)][fock_of(sk, mk)];
        if (c == 0.0) {
          if (std::fabs(el) > 1e-13) throw std::runtime_error("site op " + name + " is not a tensor operator");
          continue;
        }
        double r = el / c;
        if (set && std::fabs(r - val) > 1e-12) throw std::runtime_error("site op " + name + " inconsistent");
        val = r;
        set = true;
      }
      op.r[sb][sk] = val;
    }
  return op;
}

// Operator matrix of a component vector over factor types (product left to right).
Mat4 realise(const std::vector<double>& v, const std::string& types) {
  const int L = (int)types.size();
  Mat4 out = zero4();
  for (size_t idx = 0; idx < v.size(); ++idx) {
    if (v[idx] == 0.0) continue;
    Mat4 p = zero4();
    for (int i = 0; i < 4; ++i) p[i][i] = 1.0;
    for (int f = 0; f < L; ++f) p = mul4(p, elem(types[f], ((idx >> f) & 1u) ? -1 : 1));
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) out[i][j] += v[idx] * p[i][j];
  }
  return out;
}

SiteOp from_form(const std::string& name, const CForm& f, int k2, const std::string& types, int dn) {
  return reduce(name, realise(f.comp.at(k2), types), k2, dn, (int)types.size() & 1);
}

std::vector<SiteOp> build_fixed() {
  std::vector<SiteOp> ops(kNumFixedSite);
  Mat4 id = zero4();
  for (int i = 0; i < 4; ++i) id[i][i] = 1.0;
  ops[S_I] = reduce("I", id, 0, 0, 0);
  ops[S_C] = from_form("c", cf_leaf(1, 0), 1, "c", 1);
  ops[S_D] = from_form("d", cf_leaf(1, 0), 1, "d", -1);
  ops[S_CC0] = from_form("[cc]0", cf_couple(cf_leaf(2, 0), 1, cf_leaf(2, 1), 1, 0), 0, "cc", 2);
  ops[S_DD0] = from_form("[dd]0", cf_couple(cf_leaf(2, 0), 1, cf_leaf(2, 1), 1, 0), 0, "dd", -2);
  ops[S_CD0] = from_form("[cd]0", cf_couple(cf_leaf(2, 0), 1, cf_leaf(2, 1), 1, 0), 0, "cd", 0);
  ops[S_CD1] = from_form("[cd]1", cf_couple(cf_leaf(2, 0), 1, cf_leaf(2, 1), 1, 2), 2, "cd", 0);
  {
    CForm t;
    t.L = 3;
    t.comp[1] = phys_t3(3);
    ops[S_T3] = reduce("T3", realise(t.comp[1], "cdd"), 1, -1, 1);
    t.comp[1] = phys_u3(3);
    ops[S_U3] = reduce("U3", realise(t.comp[1], "cdd"), 1, -1, 1);
  }
  Mat4 nn = zero4();
  nn[3][3] = 1.0;
  ops[S_NUP_NDN] = reduce("nup*ndn", nn, 0, 0, 0);
  Mat4 n = zero4();
  n[1][1] = n[2][2] = 1.0;
  n[3][3] = 2.0;
  ops[S_N] = reduce("n", n, 0, 0, 0);
  return ops;
}
}  // namespace

const SiteOp& site_op(int id) {
  static const std::vector<SiteOp> ops = build_fixed();
  return ops.at(id);
}

SiteOp site_hamiltonian(double h_oo, double g_oooo) {
  // h n + (1/2) g sum_st a+_s a+_t a_t a_s = h n + g n_up n_dn
  SiteOp op = site_op(S_N);
  const SiteOp& nn = site_op(S_NUP_NDN);
  op.name = "Hsite";
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) op.r[i][j] = h_oo * op.r[i][j] + g_oooo * nn.r[i][j];
  return op;
}

// ---------------------------------------------------------------- derived constants
namespace {
double pick(const std::map<std::pair<int, int>, double>& m, int kx, int ky) {
  auto it = m.find({kx, ky});
  return it == m.end() ? 0.0 : it->second;
}

SpinConstants derive() {
  SpinConstants c{};
  auto two = [](int a, int b) { return SplitSpec{{a, b}, {}, -1, -1}; };
  (void)two;
  {
    auto m = split_coeffs(phys_e4_pair(4), 4, 0, SplitSpec{{0, 1}, {2, 3}});
    for (int S = 0; S < 2; ++S) c.ap[S] = pick(m, 2 * S, 2 * S);
  }
  {
    auto m = split_coeffs(phys_ee(4), 4, 0, SplitSpec{{0, 1}, {2, 3}});
    for (int k = 0; k < 2; ++k) c.ee[k] = pick(m, 2 * k, 2 * k);
  }
  {
    auto m = split_coeffs(phys_exch(4), 4, 0, SplitSpec{{0, 1}, {2, 3}});
    for (int k = 0; k < 2; ++k) c.ex[k] = pick(m, 2 * k, 2 * k);
  }
  c.cs = pick(split_coeffs(phys_cz(2), 2, 0, SplitSpec{{0}, {1}}), 1, 1);
  c.sc = pick(split_coeffs(phys_xc(2), 2, 0, SplitSpec{{0}, {1}}), 1, 1);
  for (int k = 0; k < 2; ++k) {
    CForm f = cf_couple(cf_leaf(2, 0), 1, cf_leaf(2, 1), 1, 2 * k);
    // [c_o d_j]^k -> (d_j | c_o) ;  [d_s d_o]^S -> (d_o | d_s) ; [c_r d_o]^k -> (d_o | c_r)
    c.b_swap[k] = pick(split_coeffs(f.comp.at(2 * k), 2, 2 * k, SplitSpec{{1}, {0}}), 1, 1);
    c.dd_swap[k] = c.b_swap[k];
    c.cd_swap[k] = c.b_swap[k];
  }
  const auto t3 = phys_t3(3), u3 = phys_u3(3);
  {
    auto m1 = split_coeffs(t3, 3, 1, SplitSpec{{0, 1}, {2}});
    auto m2 = split_coeffs(t3, 3, 1, SplitSpec{{0, 2}, {1}});
    auto m3 = split_coeffs(t3, 3, 1, SplitSpec{{1, 2}, {0}});
    auto m4 = split_coeffs(t3, 3, 1, SplitSpec{{0}, {1, 2}});
    auto m5 = split_coeffs(t3, 3, 1, SplitSpec{{1}, {0, 2}});
    auto m6 = split_coeffs(t3, 3, 1, SplitSpec{{2}, {0, 1}});
    for (int k = 0; k < 2; ++k) {
      c.t_p1[k] = pick(m1, 2 * k, 1);
      c.t_p2[k] = pick(m2, 2 * k, 1);
      c.t_p3[k] = pick(m3, 2 * k, 1);
      c.t_p4[k] = pick(m4, 1, 2 * k);
      c.t_p5[k] = pick(m5, 1, 2 * k);
      c.t_p6[k] = pick(m6, 1, 2 * k);
    }
  }
  {
    auto m1 = split_coeffs(u3, 3, 1, SplitSpec{{0}, {1, 2}});
    auto m2 = split_coeffs(u3, 3, 1, SplitSpec{{1}, {0, 2}});
    auto m3 = split_coeffs(u3, 3, 1, SplitSpec{{2}, {0, 1}});
    auto m4 = split_coeffs(u3, 3, 1, SplitSpec{{0, 1}, {2}});
    auto m5 = split_coeffs(u3, 3, 1, SplitSpec{{0, 2}, {1}});
    auto m6 = split_coeffs(u3, 3, 1, SplitSpec{{1, 2}, {0}});
    for (int k = 0; k < 2; ++k) {
      c.u_q1[k] = pick(m1, 1, 2 * k);
      c.u_q2[k] = pick(m2, 1, 2 * k);
      c.u_q3[k] = pick(m3, 1, 2 * k);
      c.u_q4[k] = pick(m4, 2 * k, 1);
      c.u_q5[k] = pick(m5, 2 * k, 1);
      c.u_q6[k] = pick(m6, 2 * k, 1);
    }
  }
  return c;
}
}  // namespace

const SpinConstants& spin_constants() {
  static const SpinConstants c = derive();
  return c;
}

}  // namespace dmrg
