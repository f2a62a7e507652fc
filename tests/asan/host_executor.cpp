// Host executor for the sanitizer test of the library's host code: the same
// Executor interface as the HIP executor, with plain loops over host memory.
// Test infrastructure only: it is compiled by tests/test_host_asan.py into a
// separate, sanitizer-instrumented library in a temporary directory, together
// with the host sources (planner, H*psi plan, driver, C ABI), so that
// AddressSanitizer and UndefinedBehaviorSanitizer see every host-side index
// computation.  The product library never contains or loads it.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <vector>
#include <algorithm>
#include "../../paper_2503_20700_amd/csrc/exec.hpp"

namespace dmrg {
namespace {
typedef unsigned short u16;
inline u16 f2bf(float f) {
  uint32_t u; std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffff) > 0x7f800000) return (u16)((u >> 16) | 0x40);
  u += 0x7fff + ((u >> 16) & 1);
  return (u16)(u >> 16);
}
inline float bf2f(u16 h) { uint32_t u = ((uint32_t)h) << 16; float f; std::memcpy(&f, &u, 4); return f; }
// OCP E4M3: bias 7, max 448, subnormals m * 2^-9
inline double e4m3_dec(unsigned char b) {
  const int sgn = b >> 7, e = (b >> 3) & 15, m = b & 7;
  double v = e == 0 ? m * std::ldexp(1.0, -9) : (1.0 + m / 8.0) * std::ldexp(1.0, e - 7);
  return sgn ? -v : v;
}
inline unsigned char e4m3_enc(double x) {
  // round to nearest even among all E4M3 values (saturating)
  float xf = (float)x;
  double a = std::fabs((double)xf);
  if (a > 448.0) a = 448.0;
  unsigned char best = 0;
  double bd = 1e300;
  for (int c = 0; c < 127; ++c) {  // 0x7f is NaN
    const double v = e4m3_dec((unsigned char)c);
    const double d = std::fabs(v - a);
    if (d < bd || (d == bd && (c & 1) == 0 && (best & 1))) { bd = d; best = (unsigned char)c; }
  }
  return (unsigned char)(best | (xf < 0 && best ? 0x80 : 0));
}
inline double ld(const void* p, int dt, int64_t i) {
  if (dt == DT_F64) return ((const double*)p)[i];
  if (dt == DT_F32) return ((const float*)p)[i];
  if (dt == DT_FP8) return e4m3_dec(((const unsigned char*)p)[i]);
  return bf2f(((const u16*)p)[i]);
}
inline void st(void* p, int dt, int64_t i, double v) {
  if (dt == DT_F64) ((double*)p)[i] = v;
  else if (dt == DT_F32) ((float*)p)[i] = (float)v;
  else if (dt == DT_FP8) ((unsigned char*)p)[i] = e4m3_enc(v);
  else ((u16*)p)[i] = f2bf((float)v);
}
struct Prep { std::vector<RawJob> jobs; std::vector<RawTerm> terms; int da, db, dc; };

// Graph recording: between capture_begin and capture_end the queued work
// (kernels, device copies) is kept as closures that replay() runs; calls that
// a HIP stream recording refuses (allocation, host transfers, waits,
// preparation) throw, so the Davidson iteration's recorded sequences are checked for them.
typedef std::vector<std::function<void()>> Graph;

class CpuExec : public Executor {
  Graph* rec_ = nullptr;
  void queue(std::function<void()> f) {
    if (rec_) rec_->push_back(std::move(f));
    else f();
  }
  void no_rec(const char* what) const {
    if (rec_) throw std::runtime_error(std::string("executor: ") + what + " inside a graph recording");
  }

 public:
  void* alloc(size_t b) override { no_rec("alloc"); void* p = std::malloc(b ? b : 1); if (!p) throw std::bad_alloc(); return p; }
  void release(void* p) override { no_rec("release"); std::free(p); }
  void upload(void* d, const void* s, size_t b) override { no_rec("upload"); if (b) std::memcpy(d, s, b); }
  void download(void* d, const void* s, size_t b) override { no_rec("download"); if (b) std::memcpy(d, s, b); }
  void zero(void* p, size_t b) override { queue([=] { if (b) std::memset(p, 0, b); }); }
  void copy_d2d(void* d, const void* s, size_t b) override { queue([=] { if (b) std::memmove(d, s, b); }); }
  void* prepare(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc) override {
    no_rec("prepare");
    auto* P = new Prep{jobs, terms, da, db, dc};
    return P;
  }
  bool graphs() const override { return true; }
  void capture_begin() override { no_rec("capture_begin"); rec_ = new Graph(); }
  void* capture_end() override { Graph* g = rec_; rec_ = nullptr; return g; }
  void capture_abort() override { delete rec_; rec_ = nullptr; }
  void replay(void* g) override { no_rec("replay"); for (auto& f : *(Graph*)g) f(); }
  void drop_graph(void* g) override { delete (Graph*)g; }
  void run(void* h) override { queue([=] { run_now(h); }); }
  void run_now(void* h) {
    auto* P = (Prep*)h;
    const bool low = P->da != DT_F64;
    for (size_t jj = 0; jj < P->jobs.size(); ++jj) {
      const RawJob& J = P->jobs[jj];
      std::vector<double> acc((size_t)J.m * J.n, 0.0), tmp((size_t)J.m * J.n);
      for (int64_t t = J.tbeg; t < J.tend; ++t) {
        const RawTerm& T = P->terms[t];
        std::fill(tmp.begin(), tmp.end(), 0.0);
        for (int i = 0; i < J.m; ++i)
          for (int kk = 0; kk < T.k; ++kk) {
            double a;
            if (T.flags & TF_IDENT_A) a = (i == kk) ? 1.0 : 0.0;
            else a = (T.flags & TF_TRANS_A) ? ld(T.A, P->da, (int64_t)kk * T.lda + i) : ld(T.A, P->da, (int64_t)i * T.lda + kk);
            if (a == 0.0) continue;
            for (int j = 0; j < J.n; ++j) {
              double b;
              if (T.flags & TF_IDENT_B) b = (kk == j) ? 1.0 : 0.0;
              else b = (T.flags & TF_TRANS_B) ? ld(T.B, P->db, (int64_t)j * T.ldb + kk) : ld(T.B, P->db, (int64_t)kk * T.ldb + j);
              tmp[(size_t)i * J.n + j] += a * b;
            }
          }
        for (size_t e = 0; e < acc.size(); ++e) acc[e] += (low ? (double)(float)T.alpha : T.alpha) * tmp[e];
      }
      for (int i = 0; i < J.m; ++i)
        for (int j = 0; j < J.n; ++j) {
          const int64_t o = (int64_t)i * J.ldc + j;
          double v = acc[(size_t)i * J.n + j];
          if (J.accumulate) v += ld(J.C, P->dc, o);
          st(J.C, P->dc, o, v);
        }
    }
  }
  void drop(void* h) override { delete (Prep*)h; }
  void orb_scalars(const double* Bm, int naux, int n, int nc, int na, const double* gam, double* bact,
                   double* scal) override {
    for (int L = 0; L < naux; ++L) {
      const double* B = Bm + (int64_t)L * n * n;
      double J = 0, t = 0, q = 0, r = 0;
      for (int i = 0; i < nc; ++i) J += B[i * n + i];
      for (int e = 0; e < na * na; ++e) { int a = e / na, b = e % na; double v = B[(nc + a) * n + nc + b]; bact[(int64_t)L * na * na + e] = v; t += gam[e] * v; }
      for (int i = 0; i < nc; ++i) for (int j = 0; j < nc; ++j) q += B[i * n + j] * B[j * n + i];
      for (int a = 0; a < na; ++a) for (int i = 0; i < nc; ++i) { double s = 0; for (int u = 0; u < na; ++u) s += gam[a * na + u] * B[i * n + nc + u]; r += B[(nc + a) * n + i] * s; }
      scal[4 * L] = J; scal[4 * L + 1] = t; scal[4 * L + 2] = q; scal[4 * L + 3] = r;
    }
  }
  void orb_assemble(const double* Bm, int naux, int n, int nc, int na, const double* gam, const double* scal,
                    const double* bact, const double* Y, const double* Z, double* Gm, double* e2) override {
    for (int L = 0; L < naux; ++L) {
      const double* B = Bm + (int64_t)L * n * n; double* G = Gm + (int64_t)L * n * n;
      const double J = scal[4 * L], t = scal[4 * L + 1];
      const double* y = Y + (int64_t)L * na * na; const double* z = Z + (int64_t)L * na * na;
      for (int p = 0; p < n; ++p) for (int q = 0; q < n; ++q) {
        bool pc = p < nc, qc = q < nc, pa = p >= nc && p < nc + na, qa = q >= nc && q < nc + na;
        double v = 0;
        if (pc && qc) { v = -2.0 * B[q * n + p]; if (p == q) v += 4 * J + 2 * t; }
        else if (pa && qa) { int a = p - nc, b = q - nc; v = 2 * J * gam[a * na + b] + 0.5 * (y[a * na + b] + z[a * na + b]); }
        else if (pa && qc) { int a = p - nc; double s = 0; for (int u = 0; u < na; ++u) s += gam[a * na + u] * B[q * n + nc + u]; v = -s; }
        else if (pc && qa) { int b = q - nc; double s = 0; for (int a = 0; a < na; ++a) s += gam[a * na + b] * B[(nc + a) * n + p]; v = -s; }
        G[p * n + q] = v;
      }
      double s = 0; for (int e = 0; e < na * na; ++e) s += bact[(int64_t)L * na * na + e] * y[e];
      e2[L] = 0.5 * s;
    }
  }
  void* fixed_scratch(size_t* bytes) override {
    static std::vector<char> buf((size_t)128 << 20);
    *bytes = buf.size();
    return buf.data();
  }
  void* plan_fixed(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc,
                   size_t* lb, size_t* pb) override {
    *lb = 1024; *pb = 0;
    return new Prep{jobs, terms, da, db, dc};
  }
  void place_fixed(void*, void*, void*) override {}
  void drop_fixed(void* h) override { delete (Prep*)h; }
  void sync() override { no_rec("sync"); }
  static void dots(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out) {
    for (int i = 0; i < m; ++i) { double s = 0; for (int64_t j = 0; j < n; ++j) s += V[i * ldv + j] * w[j]; out[i] = s; }
  }
  static void comb(double* y, const double* V, int64_t ldv, int m, const double* c, double sgn, int64_t n, double beta) {
    for (int64_t j = 0; j < n; ++j) { double s = beta == 0.0 ? 0.0 : beta * y[j]; for (int i = 0; i < m; ++i) s += sgn * c[i] * V[i * ldv + j]; y[j] = s; }
  }
  static void axpb(double* z, double a, const double* x, double b, const double* y, int64_t n) {
    for (int64_t j = 0; j < n; ++j) z[j] = a * x[j] + b * y[j];
  }
  static void prec(double* t, const double* r, const double* d, double theta, double eps, int64_t n) {
    for (int64_t j = 0; j < n; ++j) { double den = theta - d[j]; if (std::fabs(den) < eps) den = den < 0 ? -eps : eps; t[j] = r[j] / den; }
  }
  void multidot(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out) override {
    no_rec("multidot to the host");
    dots(V, ldv, m, w, n, out);
  }
  void combine(double* y, const double* V, int64_t ldv, int m, const double* c, int64_t n, double beta) override {
    std::vector<double> cv(c, c + m);  // host coefficients are taken at the call
    queue([=] { comb(y, V, ldv, m, cv.data(), 1.0, n, beta); });
  }
  void axpby(double* z, double a, const double* x, double b, const double* y, int64_t n) override {
    queue([=] { axpb(z, a, x, b, y, n); });
  }
  void precond(double* t, const double* r, const double* d, double theta, double eps, int64_t n) override {
    queue([=] { prec(t, r, d, theta, eps, n); });
  }
  void multidot_dev(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out) override {
    queue([=] { dots(V, ldv, m, w, n, out); });
  }
  void combine_dev(double* y, const double* V, int64_t ldv, int m, const double* c, double sgn, int64_t n,
                   double beta) override {
    queue([=] { comb(y, V, ldv, m, c, sgn, n, beta); });
  }
  void axpby_dev(double* z, double a, const double* a_dev, const double* x, double b, const double* b_dev,
                 const double* y, int64_t n) override {
    queue([=] { axpb(z, a_dev ? a * a_dev[0] : a, x, b_dev ? b * b_dev[0] : b, y, n); });
  }
  void precond_dev(double* t, const double* r, const double* d, const double* theta, double eps, int64_t n) override {
    queue([=] { prec(t, r, d, theta[0], eps, n); });
  }
  int sym_eig(double* A, double* V, const std::vector<int64_t>& offs, const std::vector<int>& sizes, int max_sweeps,
               double tol, double* worst) override {
    if (worst) *worst = 0.0;
    for (size_t q = 0; q < offs.size(); ++q) {
      double* a = A + offs[q]; double* v = V + offs[q]; const int n = sizes[q];
      for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) v[i * n + j] = i == j;
      double fro = 0; for (int i = 0; i < n * n; ++i) fro += a[i] * a[i];
      for (int sw = 0; sw < 100; ++sw) {
        double off = 0; for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) if (i != j) off += a[i * n + j] * a[i * n + j];
        if (off <= 1e-30 * fro) break;
        for (int p = 0; p < n; ++p) for (int r = p + 1; r < n; ++r) {
          const double apq = a[p * n + r]; if (apq == 0.0) continue;
          const double th = (a[r * n + r] - a[p * n + p]) / (2 * apq);
          const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
          const double c = 1 / std::sqrt(t * t + 1), s = t * c;
          for (int k = 0; k < n; ++k) { const double x = a[k * n + p], y = a[k * n + r]; a[k * n + p] = c * x - s * y; a[k * n + r] = s * x + c * y; }
          for (int k = 0; k < n; ++k) { const double x = a[p * n + k], y = a[r * n + k]; a[p * n + k] = c * x - s * y; a[r * n + k] = s * x + c * y; }
          for (int k = 0; k < n; ++k) { const double x = v[k * n + p], y = v[k * n + r]; v[k * n + p] = c * x - s * y; v[k * n + r] = s * x + c * y; }
        }
      }
    }
    (void)max_sweeps; (void)tol;
    return 0;
  }
  void pack(void* dst, int dd, const double* src, const int* idx, size_t n) override {
    queue([=] { for (size_t i = 0; i < n; ++i) st(dst, dd, i, idx[i] >= 0 ? src[idx[i]] : 0.0); });
  }
  void gather(double* dst, const void* src, int ds, const int* idx, size_t n, double a, const double* x,
              const double* mul) override {
    queue([=] {
      const double m = mul ? mul[0] : 1.0;
      for (size_t i = 0; i < n; ++i) dst[i] = m * ld(src, ds, idx[i]) + (x ? a * x[i] : 0.0);
    });
  }
  static void pow2(double m, double* out) {
    int e = 0;
    if (m > 0) (void)std::frexp(m / 448.0, &e);
    out[0] = std::ldexp(1.0, e); out[1] = std::ldexp(1.0, -e);
  }
  void fp8_scales(const double* src, int64_t nseg, int64_t seg, double* d_scale) override {
    for (int64_t y = 0; y < nseg; ++y) {
      double m = 0; for (int64_t i = 0; i < seg; ++i) if (std::isfinite(src[y * seg + i])) m = std::max(m, std::fabs(src[y * seg + i]));
      pow2(m, d_scale + 2 * y);
    }
  }
  void to_fp8(void* dst, const double* src, int64_t n, int64_t seg, const double* d_scale) override {
    for (int64_t i = 0; i < n; ++i) ((unsigned char*)dst)[i] = e4m3_enc(src[i] * d_scale[2 * (i / seg) + 1]);
  }
  void pack_fp8(void* dst, const double* src, const int* idx, size_t n, double* d_scale, const double* src_all,
                size_t n_all) override {
    queue([=] {
      double m = 0; for (size_t i = 0; i < n_all; ++i) m = std::max(m, std::fabs(src_all[i]));
      pow2(m, d_scale);
      for (size_t i = 0; i < n; ++i) ((unsigned char*)dst)[i] = idx[i] >= 0 ? e4m3_enc(src[idx[i]] * d_scale[1]) : 0;
    });
  }
  void shifted_copy_at(void* dst, int dd, const double* src, const int* idx, size_t n, double a) override {
    for (size_t i = 0; i < n; ++i) st(dst, dd, idx[i], src[idx[i]] + a);
  }
  void convert(void* dst, int dd, const void* src, int ds, size_t n) override {
    for (size_t i = 0; i < n; ++i) st(dst, dd, i, ld(src, ds, i));
  }
};
}  // namespace
Executor* make_hip_executor() { return new CpuExec(); }
}  // namespace dmrg
