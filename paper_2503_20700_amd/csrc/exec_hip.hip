// HIP executor for gfx950 (MI355X): grouped, segmented-K block GEMM on MFMA.
//
// One launch executes a list of output matrices ("jobs"); each job is split
// into 64x64 tiles and every tile is owned by one work-group (4 wavefronts of
// 64 lanes, each wave a 32x32 quadrant = 2x2 MFMA 16x16 blocks).  The tile loops
// over all products of its job (K concatenated over products), staging 64xK
// slabs of A and B through LDS, and writes (or accumulates into) C once, so
// there are no atomics and the summation order is fixed.
//
// Arithmetic paths:
//   F64  : v_mfma_f64_16x16x4f64, operands and accumulation in FP64
//   F32  : v_mfma_f32_16x16x4f32, FP32 operands, FP32 accumulation
//   BF16 : v_mfma_f32_16x16x32_bf16, BF16 operands (RNE), FP32 accumulation
// Operands may be stored in a wider type than the arithmetic (they are
// rounded while being staged into LDS); outputs are written in their own type.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <type_traits>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "exec.hpp"

namespace dmrg {
namespace {

#define HIP_OK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int TM = 64, TN = 64;

__device__ __forceinline__ u16 f2bf(float f) {
  unsigned int b = __float_as_uint(f);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (u16)((b >> 16) | 0x40);  // quiet NaN
  b += 0x7fffu + ((b >> 16) & 1u);
  return (u16)(b >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float(((unsigned int)h) << 16); }

template <int DT>
__device__ __forceinline__ double ldv(const void* p, long long i) {
  if constexpr (DT == DT_F64) return ((const double*)p)[i];
  else if constexpr (DT == DT_F32) return (double)((const float*)p)[i];
  else return (double)bf2f(((const u16*)p)[i]);
}
template <int DT>
__device__ __forceinline__ float ldf(const void* p, long long i) {
  if constexpr (DT == DT_F64) return (float)((const double*)p)[i];
  else if constexpr (DT == DT_F32) return ((const float*)p)[i];
  else return bf2f(((const u16*)p)[i]);
}
template <int DT, typename V>
__device__ __forceinline__ void stv(void* p, long long i, V v) {
  if constexpr (DT == DT_F64) ((double*)p)[i] = (double)v;
  else if constexpr (DT == DT_F32) ((float*)p)[i] = (float)v;
  else ((u16*)p)[i] = f2bf((float)v);
}

// Row of accumulator element v held by lane group lg (= lane / 16) inside a
// 16x16 MFMA output block; the column is lane % 16.  The FP64 instruction
// interleaves rows across lane groups, the FP32-accumulating ones do not.
template <int MODE>
__device__ __forceinline__ int acc_row(int lg, int v) {
  if constexpr (MODE == DT_F64) return 4 * v + lg;
  else return 4 * lg + v;
}

// MODE: DT_F64 / DT_F32 / DT_BF16 arithmetic; DA/DB/DC storage types.
template <int MODE, int DA, int DB, int DC>
__global__ __launch_bounds__(256) void gemm_kernel(const RawJob* __restrict__ jobs, const RawTerm* __restrict__ terms,
                                                   const int* __restrict__ tiles) {
  using acc_t = typename std::conditional<MODE == DT_F64, d4, f4>::type;
  using sc_t = typename std::conditional<MODE == DT_F64, double, float>::type;
  constexpr int KT = (MODE == DT_BF16) ? 32 : 16;
  // F64/F32: LDS k-major [KT][TM+1]; BF16: row-major [TM][KT+8] of bf16 bits
  constexpr int LDS_A = (MODE == DT_BF16) ? TM * (KT + 8) * 2 : KT * (TM + 1) * (MODE == DT_F64 ? 8 : 4);
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * LDS_A];
  unsigned char* sA = smem;
  unsigned char* sB = smem + LDS_A;

  const int tid = threadIdx.x;
  const int job = tiles[3 * blockIdx.x], ti = tiles[3 * blockIdx.x + 1], tj = tiles[3 * blockIdx.x + 2];
  const RawJob J = jobs[job];
  const int m0 = ti * TM, n0 = tj * TN;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lg = lane >> 4;

  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0;

  for (long long t = J.tbeg; t < J.tend; ++t) {
    const RawTerm T = terms[t];
    const int K = T.k;
    if (T.flags & (TF_IDENT_A | TF_IDENT_B)) {
      // C += alpha * (the other operand): read it at this lane's accumulator positions.
      const bool ia = T.flags & TF_IDENT_A;
      const void* P = ia ? T.B : T.A;
      const long long ld = ia ? T.ldb : T.lda;
      const bool tr = ia ? (T.flags & TF_TRANS_B) : (T.flags & TF_TRANS_A);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = m0 + wm + a * 16 + acc_row<MODE>(lg, v);
            const int col = n0 + wn + b * 16 + lr;
            if (row < J.m && col < J.n) {
              const long long idx = tr ? (long long)col * ld + row : (long long)row * ld + col;
              const double x = ia ? ldv<DB>(P, idx) : ldv<DA>(P, idx);
              acc[a][b][v] += (sc_t)(T.alpha * x);
            }
          }
      continue;
    }
    const bool ta = T.flags & TF_TRANS_A, tb = T.flags & TF_TRANS_B;
    const sc_t alpha = (sc_t)T.alpha;
    for (int k0 = 0; k0 < K; k0 += KT) {
      // ---- stage A (TM x KT) and B (KT x TN) into LDS
      constexpr int PER = TM * KT / 256;
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int idx = tid + 256 * r;
        int i, kk;
        if (!ta) { i = idx / KT; kk = idx % KT; } else { kk = idx / TM; i = idx % TM; }
        const int gi = m0 + i, gk = k0 + kk;
        sc_t v = 0;
        if (gi < J.m && gk < K) {
          const long long g = ta ? (long long)gk * T.lda + gi : (long long)gi * T.lda + gk;
          if constexpr (MODE == DT_F64) v = (sc_t)ldv<DA>(T.A, g) * alpha;
          else v = ldf<DA>(T.A, g) * alpha;
        }
        if constexpr (MODE == DT_BF16) ((u16*)sA)[i * (KT + 8) + kk] = f2bf(v);
        else ((sc_t*)sA)[kk * (TM + 1) + i] = v;
      }
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int idx = tid + 256 * r;
        int j, kk;
        if (!tb) { kk = idx / TN; j = idx % TN; } else { j = idx / KT; kk = idx % KT; }
        const int gj = n0 + j, gk = k0 + kk;
        sc_t v = 0;
        if (gj < J.n && gk < K) {
          const long long g = tb ? (long long)gj * T.ldb + gk : (long long)gk * T.ldb + gj;
          if constexpr (MODE == DT_F64) v = (sc_t)ldv<DB>(T.B, g);
          else v = ldf<DB>(T.B, g);
        }
        if constexpr (MODE == DT_BF16) ((u16*)sB)[j * (KT + 8) + kk] = f2bf(v);
        else ((sc_t*)sB)[kk * (TN + 1) + j] = v;
      }
      __syncthreads();
      // ---- MFMA
      if constexpr (MODE == DT_BF16) {
        bf8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = *(const bf8*)&((const u16*)sA)[(wm + a * 16 + lr) * (KT + 8) + 8 * lg];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = *(const bf8*)&((const u16*)sB)[(wn + b * 16 + lr) * (KT + 8) + 8 * lg];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
      } else {
#pragma unroll
        for (int kk = 0; kk < KT; kk += 4) {
          const sc_t* A_ = (const sc_t*)sA;
          const sc_t* B_ = (const sc_t*)sB;
          sc_t a0 = A_[(kk + lg) * (TM + 1) + wm + lr];
          sc_t a1 = A_[(kk + lg) * (TM + 1) + wm + 16 + lr];
          sc_t b0 = B_[(kk + lg) * (TN + 1) + wn + lr];
          sc_t b1 = B_[(kk + lg) * (TN + 1) + wn + 16 + lr];
          if constexpr (MODE == DT_F64) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
          } else {
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
  }
  // ---- write back (row = 4*lg + v, col = lr inside each 16x16 block)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + a * 16 + acc_row<MODE>(lg, v);
        const int col = n0 + wn + b * 16 + lr;
        if (row < J.m && col < J.n) {
          const long long o = (long long)row * J.ldc + col;
          if (J.accumulate) {
            if constexpr (DC == DT_F64) ((double*)J.C)[o] += (double)acc[a][b][v];
            else stv<DC>(J.C, o, ldv<DC>(J.C, o) + (double)acc[a][b][v]);
          } else {
            stv<DC>(J.C, o, acc[a][b][v]);
          }
        }
      }
}

template <int DS, int DD>
__global__ void convert_kernel(void* dst, const void* src, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    stv<DD>(dst, i, ldv<DS>(src, i));
}

// ---- FP64 vector kernels (Davidson).  Grid-stride loops, fixed reduction order.
constexpr int kDotBlocks = 1024;

__global__ __launch_bounds__(256) void multidot_partial(const double* __restrict__ V, long long ldv, int m,
                                                         const double* __restrict__ w, long long n,
                                                         double* __restrict__ part) {
  __shared__ double red[256];
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) s += V[i * ldv + j] * w[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)i * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void multidot_final(const double* __restrict__ part, int nb, int m,
                                                       double* __restrict__ out) {
  __shared__ double red[256];
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) s += part[(long long)i * nb + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
    __syncthreads();
  }
}

struct Coef64 {
  double c[64];
};

__global__ void combine_kernel(double* __restrict__ y, const double* __restrict__ V, long long ldv, int m, Coef64 c,
                               long long n, double beta) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
    double s = (beta == 0.0) ? 0.0 : beta * y[j];
    for (int i = 0; i < m; ++i) s += c.c[i] * V[i * ldv + j];
    y[j] = s;
  }
}

__global__ void axpby_kernel(double* z, double a, const double* x, double b, const double* y, long long n) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
    z[j] = a * x[j] + b * y[j];
}

__global__ void precond_kernel(double* t, const double* r, const double* d, double theta, double eps, long long n) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
    double den = theta - d[j];
    if (fabs(den) < eps) den = den < 0 ? -eps : eps;
    t[j] = r[j] / den;
  }
}

// ---- batched parallel Jacobi eigensolver (one work-group per matrix)
// Round-robin (circle) ordering over np = n rounded up to even "players":
// in round r player 0 meets player (r % (np-1)) + 1 ... every round pairs are
// disjoint, so all row rotations and then all column rotations of a round
// compose to J^T A J with J the product of the round's plane rotations.
__device__ __forceinline__ void rr_pair(int t, int r, int np, int& p, int& q) {
  const int m = np - 1;
  if (t == 0) {
    p = np - 1;
    q = r % m;
  } else {
    p = (r + t) % m;
    q = (r - t + m) % m;
  }
  if (p > q) {
    int x = p;
    p = q;
    q = x;
  }
}

__global__ __launch_bounds__(256) void jacobi_kernel(double* __restrict__ Aall, double* __restrict__ Vall,
                                                     const long long* __restrict__ offs, const int* __restrict__ sizes,
                                                     int max_sweeps, double tol) {
  const int n = sizes[blockIdx.x];
  double* A = Aall + offs[blockIdx.x];
  double* V = Vall + offs[blockIdx.x];
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double red[256];
  __shared__ double cs[512], sn[512];
  __shared__ int pp[512], qq[512];
  __shared__ double stop_flag;
  for (long long i = tid; i < (long long)n * n; i += nt) V[i] = ((i / n) == (i % n)) ? 1.0 : 0.0;
  if (n <= 1) return;
  const int np = n + (n & 1);
  const int npairs = np / 2;
  __syncthreads();
  // ||A||_F^2
  double fs = 0.0;
  for (long long i = tid; i < (long long)n * n; i += nt) fs += A[i] * A[i];
  red[tid] = fs;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double fro2 = red[0];
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0;
    for (long long i = tid; i < (long long)n * n; i += nt)
      if ((i / n) != (i % n)) off += A[i] * A[i];
    red[tid] = off;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) stop_flag = (red[0] <= tol * tol * fro2) ? 1.0 : 0.0;
    __syncthreads();
    if (stop_flag != 0.0) break;
    for (int r = 0; r < np - 1; ++r) {
      // rotation angles for this round (pairs processed in slices of 512)
      for (int t0 = 0; t0 < npairs; t0 += 512) {
        const int cnt = min(512, npairs - t0);
        for (int t = tid; t < cnt; t += nt) {
          int p, q;
          rr_pair(t0 + t, r, np, p, q);
          double c = 1.0, s = 0.0;
          if (q < n) {
            const double apq = A[(long long)p * n + q];
            if (apq != 0.0) {
              const double app = A[(long long)p * n + p], aqq = A[(long long)q * n + q];
              const double tau = (aqq - app) / (2.0 * apq);
              const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + tt * tt);
              s = tt * c;
            }
          }
          cs[t] = c;
          sn[t] = s;
          pp[t] = p;
          qq[t] = (q < n) ? q : -1;
        }
        __syncthreads();
        // rows p, q of A
        for (long long i = tid; i < (long long)cnt * n; i += nt) {
          const int t = (int)(i / n), k = (int)(i % n);
          if (qq[t] < 0 || sn[t] == 0.0) continue;
          const long long ip = (long long)pp[t] * n + k, iq = (long long)qq[t] * n + k;
          const double a = A[ip], b = A[iq];
          A[ip] = cs[t] * a - sn[t] * b;
          A[iq] = sn[t] * a + cs[t] * b;
        }
        __syncthreads();
        // columns p, q of A and of V
        for (long long i = tid; i < (long long)cnt * n; i += nt) {
          const int t = (int)(i / n), k = (int)(i % n);
          if (qq[t] < 0 || sn[t] == 0.0) continue;
          const long long ip = (long long)k * n + pp[t], iq = (long long)k * n + qq[t];
          double a = A[ip], b = A[iq];
          A[ip] = cs[t] * a - sn[t] * b;
          A[iq] = sn[t] * a + cs[t] * b;
          a = V[ip];
          b = V[iq];
          V[ip] = cs[t] * a - sn[t] * b;
          V[iq] = sn[t] * a + cs[t] * b;
        }
        __syncthreads();
      }
    }
  }
}

struct Prepared {
  RawJob* d_jobs = nullptr;
  RawTerm* d_terms = nullptr;
  int* d_tiles = nullptr;
  long long ntiles = 0;
  int mode = DT_F64, da = DT_F64, db = DT_F64, dc = DT_F64;
};

using KernelFn = void (*)(const RawJob*, const RawTerm*, const int*);

KernelFn pick(int mode, int da, int db, int dc) {
#define K_(M, A, B, C) \
  if (mode == M && da == A && db == B && dc == C) return gemm_kernel<M, A, B, C>;
  K_(DT_F64, DT_F64, DT_F64, DT_F64)
  K_(DT_F32, DT_F32, DT_F32, DT_F32)
  K_(DT_BF16, DT_BF16, DT_BF16, DT_BF16)
  K_(DT_BF16, DT_BF16, DT_BF16, DT_F32)
#undef K_
  throw std::runtime_error("executor: unsupported dtype combination");
}

class HipExec : public Executor {
 public:
  HipExec() { HIP_OK(hipStreamCreate(&stream_)); }
  ~HipExec() override {
    if (dot_part_) (void)hipFree(dot_part_);
    if (dot_out_) (void)hipFree(dot_out_);
    for (auto& e : events_) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    if (stream_) (void)hipStreamDestroy(stream_);
  }
  void* alloc(size_t bytes) override {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    return p;
  }
  void release(void* p) override {
    if (p) HIP_OK(hipFree(p));
  }
  void upload(void* d, const void* s, size_t b) override {
    if (b) HIP_OK(hipMemcpyAsync(d, s, b, hipMemcpyHostToDevice, stream_));
    HIP_OK(hipStreamSynchronize(stream_));
  }
  void download(void* d, const void* s, size_t b) override {
    if (b) HIP_OK(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToHost, stream_));
    HIP_OK(hipStreamSynchronize(stream_));
  }
  void zero(void* p, size_t b) override {
    if (b) HIP_OK(hipMemsetAsync(p, 0, b, stream_));
  }
  void copy_d2d(void* d, const void* s, size_t b) override {
    if (b) HIP_OK(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, stream_));
  }
  void* prepare(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc) override {
    auto* P = new Prepared();
    P->da = da;
    P->db = db;
    P->dc = dc;
    P->mode = (da == DT_F64) ? DT_F64 : (da == DT_F32 ? DT_F32 : DT_BF16);
    std::vector<int> tiles;
    for (size_t j = 0; j < jobs.size(); ++j) {
      const int tm = (jobs[j].m + TM - 1) / TM, tn = (jobs[j].n + TN - 1) / TN;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          tiles.push_back((int)j);
          tiles.push_back(a);
          tiles.push_back(b);
        }
    }
    P->ntiles = (long long)tiles.size() / 3;
    if (P->ntiles) {
      P->d_jobs = (RawJob*)alloc(jobs.size() * sizeof(RawJob));
      P->d_terms = (RawTerm*)alloc(std::max<size_t>(terms.size(), 1) * sizeof(RawTerm));
      P->d_tiles = (int*)alloc(tiles.size() * sizeof(int));
      upload(P->d_jobs, jobs.data(), jobs.size() * sizeof(RawJob));
      if (!terms.empty()) upload(P->d_terms, terms.data(), terms.size() * sizeof(RawTerm));
      upload(P->d_tiles, tiles.data(), tiles.size() * sizeof(int));
    }
    pick(P->mode, da, db, dc);  // validate
    return P;
  }
  void run(void* h) override {
    auto* P = (Prepared*)h;
    if (!P->ntiles) return;
    KernelFn k = pick(P->mode, P->da, P->db, P->dc);
    const long long maxg = 0x7fffffffLL;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing_) {
      HIP_OK(hipEventCreate(&e0));
      HIP_OK(hipEventCreate(&e1));
      HIP_OK(hipEventRecord(e0, stream_));
    }
    for (long long t0 = 0; t0 < P->ntiles; t0 += maxg) {
      const long long nt = std::min(maxg, P->ntiles - t0);
      hipLaunchKernelGGL(k, dim3((unsigned)nt), dim3(256), 0, stream_, P->d_jobs, P->d_terms, P->d_tiles + 3 * t0);
    }
    HIP_OK(hipGetLastError());
    if (timing_) {
      HIP_OK(hipEventRecord(e1, stream_));
      events_.push_back({e0, e1});
    }
  }
  void timing(bool on) override {
    sync();
    for (auto& e : events_) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    events_.clear();
    timing_ = on;
  }
  std::pair<double, long long> kernel_time() override {
    sync();
    double tot = 0.0;
    for (auto& e : events_) {
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
    }
    return {tot, (long long)events_.size()};
  }
  void drop(void* h) override {
    auto* P = (Prepared*)h;
    if (!P) return;
    HIP_OK(hipStreamSynchronize(stream_));
    release(P->d_jobs);
    release(P->d_terms);
    release(P->d_tiles);
    delete P;
  }
  void sync() override { HIP_OK(hipStreamSynchronize(stream_)); }
  void convert(void* dst, int dd, const void* src, int ds, size_t n) override {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
#define C_(S, D) \
  if (ds == S && dd == D) { hipLaunchKernelGGL((convert_kernel<S, D>), dim3(grid), dim3(256), 0, stream_, dst, src, (long long)n); HIP_OK(hipGetLastError()); return; }
    C_(DT_F64, DT_F32) C_(DT_F64, DT_BF16) C_(DT_F32, DT_F64) C_(DT_BF16, DT_F64) C_(DT_F32, DT_BF16) C_(DT_BF16, DT_F32)
#undef C_
    throw std::runtime_error("executor: unsupported conversion");
  }
  void multidot(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out_host) override {
    if (m <= 0) return;
    if (m > 64) throw std::runtime_error("multidot: m > 64");
    if (!dot_part_) {
      dot_part_ = (double*)alloc(sizeof(double) * kDotBlocks * 64);
      dot_out_ = (double*)alloc(sizeof(double) * 64);
    }
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 255) / 256));
    hipLaunchKernelGGL(multidot_partial, dim3(nb), dim3(256), 0, stream_, V, (long long)ldv, m, w, (long long)n,
                       dot_part_);
    hipLaunchKernelGGL(multidot_final, dim3(1), dim3(256), 0, stream_, dot_part_, nb, m, dot_out_);
    HIP_OK(hipGetLastError());
    download(out_host, dot_out_, sizeof(double) * m);
  }
  void combine(double* y, const double* V, int64_t ldv, int m, const double* c_host, int64_t n, double beta) override {
    if (m > 64) throw std::runtime_error("combine: m > 64");
    Coef64 c{};
    for (int i = 0; i < m; ++i) c.c[i] = c_host[i];
    hipLaunchKernelGGL(combine_kernel, dim3(grid1(n)), dim3(256), 0, stream_, y, V, (long long)ldv, m, c, (long long)n,
                       beta);
    HIP_OK(hipGetLastError());
  }
  void axpby(double* z, double a, const double* x, double b, const double* y, int64_t n) override {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid1(n)), dim3(256), 0, stream_, z, a, x, b, y, (long long)n);
    HIP_OK(hipGetLastError());
  }
  void precond(double* t, const double* r, const double* d, double theta, double eps, int64_t n) override {
    hipLaunchKernelGGL(precond_kernel, dim3(grid1(n)), dim3(256), 0, stream_, t, r, d, theta, eps, (long long)n);
    HIP_OK(hipGetLastError());
  }
  void sym_eig(double* A, double* V, const std::vector<int64_t>& offs, const std::vector<int>& sizes, int max_sweeps,
               double tol) override {
    if (offs.empty()) return;
    long long* d_off = (long long*)alloc(offs.size() * sizeof(long long));
    int* d_sz = (int*)alloc(sizes.size() * sizeof(int));
    upload(d_off, offs.data(), offs.size() * sizeof(long long));
    upload(d_sz, sizes.data(), sizes.size() * sizeof(int));
    hipLaunchKernelGGL(jacobi_kernel, dim3((unsigned)offs.size()), dim3(256), 0, stream_, A, V, d_off, d_sz,
                       max_sweeps, tol);
    HIP_OK(hipGetLastError());
    sync();
    release(d_off);
    release(d_sz);
  }
  hipStream_t stream() const { return stream_; }

 private:
  static unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }
  double* dot_part_ = nullptr;
  double* dot_out_ = nullptr;
  hipStream_t stream_ = nullptr;
  bool timing_ = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events_;
};

}  // namespace

Executor* make_hip_executor() { return new HipExec(); }

}  // namespace dmrg
