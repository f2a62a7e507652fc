#include "su2.hpp"

#include <cmath>
#include <mutex>
#include <unordered_map>

namespace dmrg {
namespace {

constexpr int kMaxFact = 400;

const long double* fact_table() {
  static long double t[kMaxFact + 1];
  static bool init = false;
  if (!init) {
    t[0] = 1.0L;
    for (int i = 1; i <= kMaxFact; ++i) t[i] = t[i - 1] * (long double)i;
    init = true;
  }
  return t;
}

inline long double fct(int n) { return fact_table()[n]; }

// Delta(abc) for doubled spins.
inline long double tri_delta(int a, int b, int c) {
  return std::sqrt(fct((a + b - c) / 2) * fct((a - b + c) / 2) * fct((-a + b + c) / 2) /
                   fct((a + b + c) / 2 + 1));
}

struct Key9 {
  int v[9];
  bool operator==(const Key9& o) const {
    for (int i = 0; i < 9; ++i)
      if (v[i] != o.v[i]) return false;
    return true;
  }
};
struct Hash9 {
  size_t operator()(const Key9& k) const {
    uint64_t h = 1469598103934665603ULL;
    for (int i = 0; i < 9; ++i) h = (h ^ (uint64_t)(k.v[i] + 1024)) * 1099511628211ULL;
    return (size_t)h;
  }
};
using Cache = std::unordered_map<Key9, double, Hash9>;

std::mutex g_mu;

}  // namespace

double cg2(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || !tri2(j1, j2, J)) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((J + M) & 1)) return 0.0;
  static Cache cache;
  Key9 key{{j1, m1, j2, m2, J, M, 0, 0, 0}};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const int c = (j1 + j2 - J) / 2;
  long double pref = (long double)(J + 1) * fct((J + j1 - j2) / 2) * fct((J - j1 + j2) / 2) * fct(c) /
                     fct((j1 + j2 + J) / 2 + 1);
  pref *= fct((J + M) / 2) * fct((J - M) / 2) * fct((j1 - m1) / 2) * fct((j1 + m1) / 2) *
          fct((j2 - m2) / 2) * fct((j2 + m2) / 2);
  long double s = 0.0L;
  for (int k = 0; k <= c; ++k) {
    int t0 = (j1 - m1) / 2 - k, t1 = (j2 + m2) / 2 - k, t2 = (J - j2 + m1) / 2 + k, t3 = (J - j1 - m2) / 2 + k;
    if (t0 < 0 || t1 < 0 || t2 < 0 || t3 < 0) continue;
    long double term = 1.0L / (fct(k) * fct(c - k) * fct(t0) * fct(t1) * fct(t2) * fct(t3));
    s += (k & 1) ? -term : term;
  }
  double r = (double)(std::sqrt(pref) * s);
  std::lock_guard<std::mutex> lk(g_mu);
  cache.emplace(key, r);
  return r;
}

double sixj2(int a, int b, int c, int d, int e, int f) {
  if (!tri2(a, b, c) || !tri2(a, e, f) || !tri2(d, b, f) || !tri2(d, e, c)) return 0.0;
  static Cache cache;
  Key9 key{{a, b, c, d, e, f, -1, -1, -1}};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  long double pre = tri_delta(a, b, c) * tri_delta(a, e, f) * tri_delta(d, b, f) * tri_delta(d, e, c);
  int s1 = (a + b + c) / 2, s2 = (a + e + f) / 2, s3 = (d + b + f) / 2, s4 = (d + e + c) / 2;
  int p1 = (a + b + d + e) / 2, p2 = (a + c + d + f) / 2, p3 = (b + c + e + f) / 2;
  int tmin = std::max(std::max(s1, s2), std::max(s3, s4));
  int tmax = std::min(p1, std::min(p2, p3));
  long double sum = 0.0L;
  for (int t = tmin; t <= tmax; ++t) {
    long double term = fct(t + 1) / (fct(t - s1) * fct(t - s2) * fct(t - s3) * fct(t - s4) * fct(p1 - t) *
                                     fct(p2 - t) * fct(p3 - t));
    sum += (t & 1) ? -term : term;
  }
  double r = (double)(pre * sum);
  std::lock_guard<std::mutex> lk(g_mu);
  cache.emplace(key, r);
  return r;
}

double ninej2(int a, int b, int c, int d, int e, int f, int g, int h, int i) {
  if (!tri2(a, b, c) || !tri2(d, e, f) || !tri2(g, h, i) || !tri2(a, d, g) || !tri2(b, e, h) ||
      !tri2(c, f, i))
    return 0.0;
  static Cache cache;
  Key9 key{{a, b, c, d, e, f, g, h, i}};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  // {a b c; d e f; g h i} = sum_x (-1)^{2x} (2x+1) {a d g; h i x}{b e h; d x f}{c f i; x a b}
  int xmin = std::max(std::max(std::abs(a - i), std::abs(h - d)), std::abs(b - f));
  int xmax = std::min(std::min(a + i, h + d), b + f);
  long double s = 0.0L;
  for (int x = xmin; x <= xmax; x += 2) {
    long double t = (long double)(x + 1) * sixj2(a, d, g, h, i, x) * sixj2(b, e, h, d, x, f) *
                    sixj2(c, f, i, x, a, b);
    s += (x & 1) ? -t : t;  // (-1)^{2x} with x doubled -> (-1)^x
  }
  double r = (double)s;
  std::lock_guard<std::mutex> lk(g_mu);
  cache.emplace(key, r);
  return r;
}

double coupled_factor(int j1b, int j1k, int k1, int j2b, int j2k, int k2, int Jb, int Jk, int k) {
  double nj = ninej2(j1b, j1k, k1, j2b, j2k, k2, Jb, Jk, k);
  if (nj == 0.0) return 0.0;
  return std::sqrt((double)(Jk + 1) * (k + 1) * (j1b + 1) * (j2b + 1)) * nj;
}

}  // namespace dmrg
