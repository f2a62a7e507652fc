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

#include <algorithm>
#include <chrono>
#include <limits>
#include <map>
#include <tuple>
#include <mutex>
#include <unordered_map>
#include <cstdio>
#include <type_traits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
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

// FP32 -> BF16, round to nearest even (hardware conversion on gfx950).
__device__ __forceinline__ u16 f2bf(float f) { return __builtin_bit_cast(u16, (__bf16)f); }
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float(((unsigned int)h) << 16); }

// FP8 (OCP E4M3) storage.  Every E4M3 value is exactly a BF16 value, so FP8
// operands are widened to BF16 as they are loaded and multiplied on the BF16
// MFMA; the FP8 copies halve the operand bytes the kernels move.
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned bf16x2_of(f2v f) { return (unsigned)f2bf(f[0]) | ((unsigned)f2bf(f[1]) << 16); }
__device__ __forceinline__ uint4 fp8x8_to_bf16x8(uint2 x) {
  return make_uint4(bf16x2_of(__builtin_amdgcn_cvt_pk_f32_fp8((int)x.x, false)),
                    bf16x2_of(__builtin_amdgcn_cvt_pk_f32_fp8((int)x.x, true)),
                    bf16x2_of(__builtin_amdgcn_cvt_pk_f32_fp8((int)x.y, false)),
                    bf16x2_of(__builtin_amdgcn_cvt_pk_f32_fp8((int)x.y, true)));
}
__device__ __forceinline__ float fp8_to_f(unsigned char b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }
// round to nearest even E4M3, saturating at +-448
__device__ __forceinline__ unsigned char f_to_fp8(float v) {
  v = fminf(fmaxf(v, -448.f), 448.f);
  return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xff);
}

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

// Storage element of each dtype and its conversion to the arithmetic type.
template <int DT> struct raw_of;
template <> struct raw_of<DT_F64> { using T = double; };
template <> struct raw_of<DT_F32> { using T = float; };
template <> struct raw_of<DT_BF16> { using T = u16; };
template <int DT, typename S>
__device__ __forceinline__ S raw_to(typename raw_of<DT>::T r) {
  if constexpr (DT == DT_BF16) return (S)bf2f(r);
  else return (S)r;
}

// One unit of work of a launch: output tile (ti, tj) of job `job`, summing the
// products [tbeg, tend) of that job.  slot < 0: the item owns the tile and
// writes C; otherwise it writes its partial sum to partial slot `slot` and a
// reduction launch adds the job's slots in order (deterministic split-K).
struct WorkItem {
  int job, ti, tj, tbeg, tend, slot;
  int dense0;     // first product in [tbeg, tend) that is not an identity (tend if none)
  int has_ident;  // the range holds identity products
};
struct RedItem {
  int job, ti, tj, slot0, nslot, pad;
};

// MODE: DT_F64 / DT_F32 / DT_BF16 arithmetic; A and B are stored in the
// arithmetic type, C in DC.
//
// The K loop runs over the flattened (product, K slab) sequence of the item
// and is software-pipelined: the global loads of the next slab (which may
// belong to the next product) are issued into registers before the MFMAs of
// the current slab, and LDS is double-buffered, so each K step has a single
// barrier.  In the FP32/BF16 paths each product is accumulated on its own and
// added to the tile with its weight alpha (in FP32) when its last slab is
// done, so operands are staged unscaled (BF16 bits are copied unchanged and
// the weight is not rounded into the operand); the FP64 path scales A by
// alpha while staging it.
//
// Operands flagged TF_PAD_A / TF_PAD_B (and 16-byte aligned, with a row
// stride that keeps every row 16-byte aligned) have rows padded to a multiple
// of 8 elements; they are staged with 16-byte vector loads along their
// contiguous dimension, masking the elements past the logical extent.  Other
// operands are staged element by element.
enum { LD_SCALAR = 0, LD_VEC_K = 1, LD_VEC_MN = 2 };

// Zero the elements of a 16-byte vector of ES-byte elements from index nvalid on.
template <int ES>
__device__ __forceinline__ uint4 keep_first(uint4 x, int nvalid) {
  unsigned w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    unsigned m;
    if constexpr (ES == 2) m = (2 * d < nvalid ? 0x0000ffffu : 0u) | (2 * d + 1 < nvalid ? 0xffff0000u : 0u);
    else if constexpr (ES == 4) m = d < nvalid ? 0xffffffffu : 0u;
    else m = (d / 2) < nvalid ? 0xffffffffu : 0u;
    w[d] &= m;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

template <int MODE, int DC, int KT>
__global__ __launch_bounds__(256) void gemm_kernel(const RawJob* __restrict__ jobs, const RawTerm* __restrict__ terms,
                                                   const WorkItem* __restrict__ items, void* __restrict__ part) {
  using acc_t = typename std::conditional<MODE == DT_F64, d4, f4>::type;
  using sc_t = typename std::conditional<MODE == DT_F64, double, float>::type;
  using el_t = typename raw_of<MODE>::T;
  static_assert(MODE == DT_BF16 ? (KT % 32 == 0) : (KT == 16), "K slab: multiple of 32 (BF16) or 16");
  constexpr int VW = 16 / (int)sizeof(el_t);  // elements per 16-byte vector
  constexpr int PER = TM * KT / 256;           // elements of each operand per thread and slab
  constexpr int NV = PER / VW;                 // 16-byte vectors per thread and slab
  static_assert(NV * VW == PER && NV >= 1, "slab must split into whole vectors");
  // BF16: LDS row-major [TM][KT+8] (k contiguous, MFMA operand layout);
  // F32/F64: LDS k-major [KT][TM+1]
  constexpr int LDA_S = (MODE == DT_BF16) ? KT + 8 : TM + 1;
  constexpr int LDS_A = (MODE == DT_BF16) ? TM * (KT + 8) * 2 : KT * (TM + 1) * (int)sizeof(el_t);
  __shared__ __attribute__((aligned(16))) unsigned char smem[4 * LDS_A];

  const int tid = threadIdx.x;
  WorkItem W;       // the work item of this work-group
  RawJob J;
  int m0 = 0, n0 = 0;
  int lmm = 0, lnn = 0, lm0 = 0, ln0 = 0;  // extents and origin of the tile being loaded
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lg = lane >> 4;

  acc_t acc[2][2], accp[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = accp[a][b][v] = 0;

  // ---- identity products: C += alpha * (the other operand), read at this
  // lane's accumulator positions.
  auto identity_pass = [&]() {
    for (int t = W.tbeg; t < W.tend; ++t) {
      const int fl = terms[t].flags;
      if (!(fl & (TF_IDENT_A | TF_IDENT_B))) continue;
      const RawTerm T = terms[t];
      const bool ia = fl & TF_IDENT_A;
      const void* P = ia ? T.B : T.A;
      const long long ld = ia ? T.ldb : T.lda;
      const bool tr = ia ? (fl & TF_TRANS_B) : (fl & TF_TRANS_A);
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
              acc[a][b][v] += (sc_t)(T.alpha * ldv<MODE>(P, idx));
            }
          }
    }
  };

  auto next_dense = [&](int t, int tend) {
    while (t < tend && (terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) ++t;
    return t;
  };
  union Regs {
    uint4 v[NV];
    el_t e[PER];
  };
  Regs ra, rb;
  int amode = LD_SCALAR, bmode = LD_SCALAR, rflags = 0;
  constexpr bool kScaleA = (MODE == DT_F64);  // weight applied to A while staging
  sc_t ralpha = 1;

  auto vec_ok = [](const void* p, long long ld) {
    return (((unsigned long long)p & 15ull) == 0) && (((ld * (long long)sizeof(el_t)) & 15ll) == 0);
  };
  // Fill the registers with slab k0 of product t.
  auto load = [&](int t, int k0) {
    const RawTerm T = terms[t];
    const int K = T.k;
    const bool ta = T.flags & TF_TRANS_A, tb = T.flags & TF_TRANS_B;
    rflags = T.flags;
    if constexpr (kScaleA) ralpha = (sc_t)T.alpha;
    const el_t* A = (const el_t*)T.A;
    const el_t* B = (const el_t*)T.B;
    amode = ((T.flags & TF_PAD_A) && vec_ok(T.A, T.lda)) ? (ta ? LD_VEC_MN : LD_VEC_K) : LD_SCALAR;
    bmode = ((T.flags & TF_PAD_B) && vec_ok(T.B, T.ldb)) ? (tb ? LD_VEC_K : LD_VEC_MN) : LD_SCALAR;
    // ---- A (TM x KT)
    if (amode == LD_VEC_K) {  // rows i, vectors along k
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int i = gv / (KT / VW), kv = (gv % (KT / VW)) * VW;
        const int gi = lm0 + i, gk = k0 + kv;
        ra.v[v] = make_uint4(0, 0, 0, 0);
        if (gi < lmm && gk < K) {
          ra.v[v] = *(const uint4*)(A + (long long)gi * T.lda + gk);
          if (K - gk < VW) ra.v[v] = keep_first<sizeof(el_t)>(ra.v[v], K - gk);
        }
      }
    } else if (amode == LD_VEC_MN) {  // rows k, vectors along i
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int kk = gv / (TM / VW), iv = (gv % (TM / VW)) * VW;
        const int gi = lm0 + iv, gk = k0 + kk;
        ra.v[v] = make_uint4(0, 0, 0, 0);
        if (gi < lmm && gk < K) {
          ra.v[v] = *(const uint4*)(A + (long long)gk * T.lda + gi);
          if (lmm - gi < VW) ra.v[v] = keep_first<sizeof(el_t)>(ra.v[v], lmm - gi);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int idx = tid + 256 * r;
        int i, kk;
        if (!ta) { i = idx / KT; kk = idx % KT; } else { kk = idx / TM; i = idx % TM; }
        const int gi = lm0 + i, gk = k0 + kk;
        ra.e[r] = (el_t)0;
        if (gi < lmm && gk < K) ra.e[r] = A[ta ? (long long)gk * T.lda + gi : (long long)gi * T.lda + gk];
      }
    }
    // ---- B (KT x TN)
    if (bmode == LD_VEC_K) {  // stored transposed: rows j, vectors along k
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int j = gv / (KT / VW), kv = (gv % (KT / VW)) * VW;
        const int gj = ln0 + j, gk = k0 + kv;
        rb.v[v] = make_uint4(0, 0, 0, 0);
        if (gj < lnn && gk < K) {
          rb.v[v] = *(const uint4*)(B + (long long)gj * T.ldb + gk);
          if (K - gk < VW) rb.v[v] = keep_first<sizeof(el_t)>(rb.v[v], K - gk);
        }
      }
    } else if (bmode == LD_VEC_MN) {  // rows k, vectors along j
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int kk = gv / (TN / VW), jv = (gv % (TN / VW)) * VW;
        const int gj = ln0 + jv, gk = k0 + kk;
        rb.v[v] = make_uint4(0, 0, 0, 0);
        if (gj < lnn && gk < K) {
          rb.v[v] = *(const uint4*)(B + (long long)gk * T.ldb + gj);
          if (lnn - gj < VW) rb.v[v] = keep_first<sizeof(el_t)>(rb.v[v], lnn - gj);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int idx = tid + 256 * r;
        int j, kk;
        if (!tb) { kk = idx / TN; j = idx % TN; } else { j = idx / KT; kk = idx % KT; }
        const int gj = ln0 + j, gk = k0 + kk;
        rb.e[r] = (el_t)0;
        if (gj < lnn && gk < K) rb.e[r] = B[tb ? (long long)gj * T.ldb + gk : (long long)gk * T.ldb + gj];
      }
    }
  };
  // Element (i, k) of the A slab / (k, j) of the B slab into LDS.
  auto putA = [&](el_t* sA, int i, int kk, el_t x) {
    if constexpr (MODE == DT_BF16) sA[i * LDA_S + kk] = x;
    else if constexpr (kScaleA) sA[kk * LDA_S + i] = x * ralpha;
    else sA[kk * LDA_S + i] = x;
  };
  auto putB = [&](el_t* sB, int j, int kk, el_t x) {
    if constexpr (MODE == DT_BF16) sB[j * LDA_S + kk] = x;
    else sB[kk * LDA_S + j] = x;
  };
  auto store = [&](unsigned char* sAb, unsigned char* sBb) {
    el_t* sA = (el_t*)sAb;
    el_t* sB = (el_t*)sBb;
    if (amode == LD_VEC_K) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int i = gv / (KT / VW), kv = (gv % (KT / VW)) * VW;
        if constexpr (MODE == DT_BF16) {
          *(uint4*)(sA + i * LDA_S + kv) = ra.v[v];
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) putA(sA, i, kv + q, ra.e[v * VW + q]);
        }
      }
    } else if (amode == LD_VEC_MN) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int kk = gv / (TM / VW), iv = (gv % (TM / VW)) * VW;
#pragma unroll
        for (int q = 0; q < VW; ++q) putA(sA, iv + q, kk, ra.e[v * VW + q]);
      }
    } else {
      const bool ta = rflags & TF_TRANS_A;
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int idx = tid + 256 * r;
        int i, kk;
        if (!ta) { i = idx / KT; kk = idx % KT; } else { kk = idx / TM; i = idx % TM; }
        putA(sA, i, kk, ra.e[r]);
      }
    }
    // B: the LDS layout of B^T equals that of A (rows j)
    if (bmode == LD_VEC_K) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int j = gv / (KT / VW), kv = (gv % (KT / VW)) * VW;
        if constexpr (MODE == DT_BF16) {
          *(uint4*)(sB + j * LDA_S + kv) = rb.v[v];
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) putB(sB, j, kv + q, rb.e[v * VW + q]);
        }
      }
    } else if (bmode == LD_VEC_MN) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int gv = tid + 256 * v;
        const int kk = gv / (TN / VW), jv = (gv % (TN / VW)) * VW;
#pragma unroll
        for (int q = 0; q < VW; ++q) putB(sB, jv + q, kk, rb.e[v * VW + q]);
      }
    } else {
      const bool tb = rflags & TF_TRANS_B;
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int idx = tid + 256 * r;
        int j, kk;
        if (!tb) { kk = idx / TN; j = idx % TN; } else { j = idx / KT; kk = idx % KT; }
        putB(sB, j, kk, rb.e[r]);
      }
    }
  };
  auto compute = [&](const unsigned char* sA, const unsigned char* sB) {
    if constexpr (MODE == DT_BF16) {
#pragma unroll
      for (int kk = 0; kk < KT; kk += 32) {
        bf8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
          av[a] = *(const bf8*)&((const u16*)sA)[(wm + a * 16 + lr) * LDA_S + kk + 8 * lg];
#pragma unroll
        for (int b = 0; b < 2; ++b)
          bv[b] = *(const bf8*)&((const u16*)sB)[(wn + b * 16 + lr) * LDA_S + kk + 8 * lg];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            accp[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], accp[a][b], 0, 0, 0);
      }
    } else {
      const sc_t* A_ = (const sc_t*)sA;
      const sc_t* B_ = (const sc_t*)sB;
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        const sc_t a0 = A_[(kk + lg) * LDA_S + wm + lr];
        const sc_t a1 = A_[(kk + lg) * LDA_S + wm + 16 + lr];
        const sc_t b0 = B_[(kk + lg) * LDA_S + wn + lr];
        const sc_t b1 = B_[(kk + lg) * LDA_S + wn + 16 + lr];
        if constexpr (MODE == DT_F64) {
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        } else {
          accp[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, accp[0][0], 0, 0, 0);
          accp[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, accp[0][1], 0, 0, 0);
          accp[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, accp[1][0], 0, 0, 0);
          accp[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, accp[1][1], 0, 0, 0);
        }
      }
    }
  };

  // ---- write back the finished item (C, or its partial slot)
  auto write_back = [&]() {
    if (W.slot >= 0) {
      sc_t* P = (sc_t*)part + (long long)W.slot * (TM * TN);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            P[(wm + a * 16 + acc_row<MODE>(lg, v)) * TN + wn + b * 16 + lr] = acc[a][b][v];
      return;
    }
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

  };
  auto set_load_tile = [&](const WorkItem& w, const RawJob& j) {
    lmm = j.m;
    lnn = j.n;
    lm0 = w.ti * TM;
    ln0 = w.tj * TN;
  };
  {
    W = items[blockIdx.x];
    J = jobs[W.job];
    m0 = W.ti * TM;
    n0 = W.tj * TN;
    int t = next_dense(W.tbeg, W.tend), k0 = 0;
    if (t < W.tend) {
      set_load_tile(W, J);
      load(t, 0);
    }
    identity_pass();
    int buf = 0;
    while (t < W.tend) {
      unsigned char* sA = smem + buf * 2 * LDS_A;
      unsigned char* sB = sA + LDS_A;
      store(sA, sB);
      __syncthreads();
      const RawTerm& Tc = terms[t];
      const int Kc = Tc.k;
      const sc_t alpha = (sc_t)Tc.alpha;
      int t2 = t, k2 = k0 + KT;
      const bool last = k2 >= Kc;
      if (last) {
        t2 = next_dense(t + 1, W.tend);
        k2 = 0;
      }
      if (t2 < W.tend) load(t2, k2);
      compute(sA, sB);
      if (!kScaleA && last) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              acc[a][b][v] += alpha * accp[a][b][v];
              accp[a][b][v] = 0;
            }
      }
      buf ^= 1;
      t = t2;
      k0 = k2;
    }
    write_back();
  }
}


// BF16 kernel for launches whose dense products all have padded, 16-byte
// aligned operands (the two stages of H*psi).  Same work items and MFMA
// layout as gemm_kernel, with output tiles of BM x BN (64 or 128 each; four
// waves in a 2 x 2 grid, each owning a (BM/2) x (BN/2) quadrant) and a lean
// K loop:
//   * each thread keeps a pointer cursor per operand vector for the product
//     being loaded, set once per product and advanced by one slab per step;
//   * every thread owns fixed 16-byte vectors of each slab (rows along the
//     operand's contiguous dimension), with LDS offsets fixed per thread;
//   * LDS rows hold their four 8-element k groups in the order
//     g ^ ((row >> 4) & 3), so rows 16 apart (same banks at the 80-byte row
//     stride) use different banks for transposed stores;
//   * product weights use a scaled frame: the accumulator holds the partial
//     sum divided by the weight of the product being multiplied, rescaled by
//     w_prev / w_next (FP32) when a new product starts and by the last weight
//     before write-back, so no second accumulator is needed.
// The kernel is latency bound (short K per product, one slab in flight), so
// the register budget is capped to keep more waves resident: 7 per SIMD for
// 64 x 64 tiles and 4 for the larger ones, the most that compile without
// spilling to scratch.
// Identity products of a work item of the padded BF16 kernels: acc +=
// alpha * (the other operand) over the tile, in the unscaled frame (before
// any dense product).  Wave quadrant (wm, wn), MFMA lane coordinates lr, lg.
template <int BM, int BN, bool AF8, bool BF8>
__device__ __forceinline__ void tile_identity_products(f4 (&acc)[BM / 32][BN / 32], const WorkItem& W, const RawJob& J,
                                                       const RawTerm* __restrict__ terms, int m0, int n0, int wm,
                                                       int wn, int lr, int lg) {
  constexpr int FA = BM / 32, FB = BN / 32;
  for (int t = W.tbeg; t < W.tend; ++t) {
    const int fl = terms[t].flags;
    if (!(fl & (TF_IDENT_A | TF_IDENT_B))) continue;
    const RawTerm T = terms[t];
    const bool ia = fl & TF_IDENT_A;
    const void* P = ia ? T.B : T.A;
    const bool f8 = ia ? BF8 : AF8;
    const long long ld = ia ? T.ldb : T.lda;
    const bool tr = ia ? (fl & TF_TRANS_B) : (fl & TF_TRANS_A);
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = m0 + wm + a * 16 + 4 * lg + v;
          const int col = n0 + wn + b * 16 + lr;
          if (row < J.m && col < J.n) {
            const long long e = tr ? (long long)col * ld + row : (long long)row * ld + col;
            acc[a][b][v] += (float)T.alpha * (f8 ? fp8_to_f(((const unsigned char*)P)[e]) : bf2f(((const u16*)P)[e]));
          }
        }
  }
}

// Write-back of a BM x BN tile of the padded BF16 kernels: into C (BF16
// output tiles with aligned rows staged through smem and stored as 16-byte
// vectors), or into the item's partial slot.  smem must hold BM x BN u16 and
// may still be read by other waves on entry.
template <int DC, int BM, int BN>
__device__ __forceinline__ void tile_store(const f4 (&acc)[BM / 32][BN / 32], const WorkItem& W, const RawJob& J,
                                           u16* smem, void* __restrict__ part, int m0, int n0, int wm, int wn,
                                           int lr, int lg, int tid) {
  constexpr int FA = BM / 32, FB = BN / 32;
  if constexpr (DC == DT_BF16) {
    if (W.slot < 0 && !J.accumulate && (((uintptr_t)J.C) & 15) == 0 && (J.ldc & 7) == 0 && (J.n & 7) == 0) {
      __syncthreads();  // every wave is done reading the last slab
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) smem[(wm + a * 16 + 4 * lg + v) * BN + wn + b * 16 + lr] = f2bf(acc[a][b][v]);
      __syncthreads();
      constexpr int VPR = BN / 8;  // vectors per tile row
#pragma unroll
      for (int i = tid; i < BM * VPR; i += 256) {
        const int r = i / VPR, c8 = (i % VPR) * 8;
        if (m0 + r < J.m && n0 + c8 < J.n)
          *(uint4*)((u16*)J.C + (long long)(m0 + r) * J.ldc + n0 + c8) = *(const uint4*)(smem + r * BN + c8);
      }
      return;
    }
  }
  if (W.slot >= 0) {
    float* P = (float*)part + (long long)W.slot * (BM * BN);
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(wm + a * 16 + 4 * lg + v) * BN + wn + b * 16 + lr] = acc[a][b][v];
    return;
  }
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + a * 16 + 4 * lg + v;
        const int col = n0 + wn + b * 16 + lr;
        if (row < J.m && col < J.n) {
          const long long o = (long long)row * J.ldc + col;
          if (J.accumulate) stv<DC>(J.C, o, ldv<DC>(J.C, o) + (double)acc[a][b][v]);
          else stv<DC>(J.C, o, acc[a][b][v]);
        }
      }
}

template <int DC, int BM, int BN, bool AF8 = false, bool BF8 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BM * BN > 8192 ? 2 : (BM * BN > 4096 ? 4 : 7)))) void gemm_bf16_padded(const RawJob* __restrict__ jobs,
                                                        const RawTerm* __restrict__ terms,
                                                        const WorkItem* __restrict__ items, void* __restrict__ part) {
  constexpr int KT = 32, LS = KT + 8;     // LDS row stride in bf16 elements (80 bytes)
  constexpr int NA = BM / 64, NB = BN / 64;  // 16-byte vectors per thread per slab
  constexpr int FA = BM / 32, FB = BN / 32;  // 16x16 MFMA blocks per wave along m / n
  // two A and two B slab buffers; after the K loop the same memory stages
  // a BF16 output tile (BM x BN <= 2 (BM + BN) LS elements)
  __shared__ __attribute__((aligned(16))) u16 smem[2 * (BM + BN) * LS];
  static_assert(BM * BN <= 2 * (BM + BN) * LS, "output tile must fit the slab buffers");
  // buffer b: A slab at smem + b * BM * LS, B slab at smem + (2 BM + b BN) * LS
  const int tid = threadIdx.x;
  const WorkItem W = items[blockIdx.x];
  const RawJob J = jobs[W.job];
  const int m0 = W.ti * BM, n0 = W.tj * BN;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int lr = lane & 15, lg = lane >> 4;

  f4 acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  // identity products, in the unscaled frame
  if (W.has_ident) tile_identity_products<BM, BN, AF8, BF8>(acc, W, J, terms, m0, n0, wm, wn, lr, lg);
  auto lds_at = [](int j, int k) { return j * LS + 8 * ((k >> 3) ^ ((j >> 4) & 3)) + (k & 7); };
  // thread roles for vector v of an operand with R rows (R = BM or BN):
  //   "K":  row (tid + 256 v) >> 2, k offset ((tid + 256 v) & 3) * 8
  //   "MN": k row (tid + 256 v) / (R / 8), offset ((tid + 256 v) % (R / 8)) * 8 along m (n)
  const int kvK = (tid & 3) * 8;
  int offAK[NA], offBK[NB], offAM[NA][8], offBM[NB][8], kAM[NA], vAM[NA], kBM[NB], vBM[NB];
#pragma unroll
  for (int v = 0; v < NA; ++v) {
    const int vi = tid + 256 * v;
    offAK[v] = lds_at(vi >> 2, kvK);
    kAM[v] = vi / (BM / 8);
    vAM[v] = (vi % (BM / 8)) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) offAM[v][q] = lds_at(vAM[v] + q, kAM[v]);
  }
#pragma unroll
  for (int v = 0; v < NB; ++v) {
    const int vi = tid + 256 * v;
    offBK[v] = lds_at(vi >> 2, kvK);
    kBM[v] = vi / (BN / 8);
    vBM[v] = (vi % (BN / 8)) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) offBM[v][q] = lds_at(vBM[v] + q, kBM[v]);
  }

  // load cursor (product whose slabs are being loaded), in bytes; FP8
  // operands have 1-byte elements
  constexpr int ESA = AF8 ? 1 : 2, ESB = BF8 ? 1 : 2;
  const unsigned char* pa[NA];
  const unsigned char* pb[NB];
  long long stepA = 0, stepB = 0;
  bool aK = true, bK = true;
  bool okA[NA], okB[NB];
  int nvA[NA], nvB[NB];
  auto begin = [&](const RawTerm& T) {
    aK = !(T.flags & TF_TRANS_A);  // A stored m x k (k contiguous)
    bK = (T.flags & TF_TRANS_B);   // B stored n x k (k contiguous)
    const unsigned char* A = (const unsigned char*)T.A;
    const unsigned char* B = (const unsigned char*)T.B;
#pragma unroll
    for (int v = 0; v < NA; ++v) {
      const int vi = tid + 256 * v;
      if (aK) {
        okA[v] = m0 + (vi >> 2) < J.m;
        pa[v] = A + ((long long)(m0 + (vi >> 2)) * T.lda + kvK) * ESA;
      } else {
        nvA[v] = min(max(J.m - (m0 + vAM[v]), 0), 8);
        pa[v] = A + ((long long)kAM[v] * T.lda + m0 + vAM[v]) * ESA;
      }
    }
    stepA = (aK ? KT : (long long)KT * T.lda) * ESA;
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      const int vi = tid + 256 * v;
      if (bK) {
        okB[v] = n0 + (vi >> 2) < J.n;
        pb[v] = B + ((long long)(n0 + (vi >> 2)) * T.ldb + kvK) * ESB;
      } else {
        nvB[v] = min(max(J.n - (n0 + vBM[v]), 0), 8);
        pb[v] = B + ((long long)kBM[v] * T.ldb + n0 + vBM[v]) * ESB;
      }
    }
    stepB = (bK ? KT : (long long)KT * T.ldb) * ESB;
  };
  uint4 ra[NA], rb[NB];
  const uint4 z4 = make_uint4(0, 0, 0, 0);
  // 8 elements at p: a 16-byte vector of BF16, or 8 FP8 bytes widened to BF16
  auto vec8 = [&](const unsigned char* p, bool f8) -> uint4 {
    if (f8) return fp8x8_to_bf16x8(*(const uint2*)p);
    return *(const uint4*)p;
  };
  auto load = [&](int K, int k0) {
    const int nvk = K - (k0 + kvK);  // valid k in this thread's vector ("K" role)
#pragma unroll
    for (int v = 0; v < NA; ++v) {
      if (aK) {
        ra[v] = (okA[v] && nvk > 0) ? vec8(pa[v], AF8) : z4;
        if (nvk < 8) ra[v] = keep_first<2>(ra[v], nvk);
      } else {
        ra[v] = (k0 + kAM[v] < K && nvA[v] > 0) ? vec8(pa[v], AF8) : z4;
        if (nvA[v] < 8) ra[v] = keep_first<2>(ra[v], nvA[v]);
      }
      pa[v] += stepA;
    }
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      if (bK) {
        rb[v] = (okB[v] && nvk > 0) ? vec8(pb[v], BF8) : z4;
        if (nvk < 8) rb[v] = keep_first<2>(rb[v], nvk);
      } else {
        rb[v] = (k0 + kBM[v] < K && nvB[v] > 0) ? vec8(pb[v], BF8) : z4;
        if (nvB[v] < 8) rb[v] = keep_first<2>(rb[v], nvB[v]);
      }
      pb[v] += stepB;
    }
  };
  bool sK_A = true, sK_B = true;  // layout of the registers being stored
  auto store = [&](u16* sA, u16* sB) {
#pragma unroll
    for (int v = 0; v < NA; ++v) {
      if (sK_A) {
        *(uint4*)(sA + offAK[v]) = ra[v];
      } else {
        const unsigned w[4] = {ra[v].x, ra[v].y, ra[v].z, ra[v].w};
#pragma unroll
        for (int q = 0; q < 8; ++q) sA[offAM[v][q]] = (u16)(w[q >> 1] >> (16 * (q & 1)));
      }
    }
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      if (sK_B) {
        *(uint4*)(sB + offBK[v]) = rb[v];
      } else {
        const unsigned w[4] = {rb[v].x, rb[v].y, rb[v].z, rb[v].w};
#pragma unroll
        for (int q = 0; q < 8; ++q) sB[offBM[v][q]] = (u16)(w[q >> 1] >> (16 * (q & 1)));
      }
    }
  };
  int rdA[FA], rdB[FB];
#pragma unroll
  for (int a = 0; a < FA; ++a) rdA[a] = lds_at(wm + a * 16 + lr, 8 * lg);
#pragma unroll
  for (int b = 0; b < FB; ++b) rdB[b] = lds_at(wn + b * 16 + lr, 8 * lg);

  auto next_dense = [&](int t) {
    while (t < W.tend && (terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) ++t;
    return t;
  };
  int t = W.dense0, k0 = 0;
  int Kc = 0;
  float alpha = 1.f, scale = 1.f;  // weight of product t; current frame of acc
  if (t < W.tend) {
    const RawTerm T = terms[t];
    Kc = T.k;
    alpha = (float)T.alpha;
    begin(T);
    load(Kc, 0);
    sK_A = aK;
    sK_B = bK;
  }
  int buf = 0;
  while (t < W.tend) {
    u16* sA = smem + buf * (BM * LS);
    u16* sB = smem + (2 * BM + buf * BN) * LS;
    store(sA, sB);
    __syncthreads();
    // next slab: same product, or the first slab of the next dense product
    int t2 = t, k2 = k0 + KT, K2 = Kc;
    float alpha2 = alpha;
    if (k2 >= Kc) {
      t2 = next_dense(t + 1);
      k2 = 0;
      if (t2 < W.tend) {
        const RawTerm T = terms[t2];
        K2 = T.k;
        alpha2 = (float)T.alpha;
        begin(T);
      }
    }
    if (t2 < W.tend) load(K2, k2);
    if (k0 == 0 && alpha != scale) {
      // product t starts: move the accumulator into its frame
      const float r = scale / alpha;
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] *= r;
      scale = alpha;
    }
    bf8 av[FA], bv[FB];
#pragma unroll
    for (int a = 0; a < FA; ++a) av[a] = *(const bf8*)(sA + rdA[a]);
#pragma unroll
    for (int b = 0; b < FB; ++b) bv[b] = *(const bf8*)(sB + rdB[b]);
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    sK_A = aK;
    sK_B = bK;
    buf ^= 1;
    t = t2;
    k0 = k2;
    Kc = K2;
    alpha = alpha2;
  }
  if (scale != 1.f) {
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b) acc[a][b] *= scale;
  }
  tile_store<DC, BM, BN>(acc, W, J, smem, part, m0, n0, wm, wn, lr, lg, tid);
}

// 16 bytes per lane from global memory straight into LDS: lane l of the
// wave writes LDS bytes [lds + 16 l, lds + 16 l + 16) (lds: wave-uniform
// byte address).  Written as inline assembly so that the compiler, which
// cannot tell the pipeline stages apart, does not add its own wait for every
// outstanding LDS write before each LDS read; the kernel orders them itself
// with pipe_wait_barrier.  No register is written, so nothing is left in
// flight behind the compiler's back.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // m0 is set here on purpose
__device__ __forceinline__ void lds_dma16(const void* g, unsigned lds) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(lds), "v"(g) : "m0");
}
#pragma clang diagnostic pop
// Wait until at most N of this wave's vector-memory operations are in
// flight and its LDS reads are done, then a work-group barrier (and a
// compiler memory barrier).
template <int N>
__device__ __forceinline__ void pipe_wait_barrier() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Padded BF16 grouped GEMM with an S-stage LDS pipeline: the same work items,
// products, scaled accumulator frame, identity products and write-back as
// gemm_bf16_padded, but every operand slab (32 k wide) is copied from global
// memory into its own LDS stage by LDS DMA (no staging registers), S - 1
// slabs ahead of the MFMAs, so each work-group keeps several slabs in
// flight.  LDS layouts per stage and operand (R = BM or BN rows):
//   * stored along k (A not transposed, B transposed): R rows of 32 k in
//     four 16-byte chunks, chunk q of row r at slot q ^ ((r >> 2) & 3);
//   * stored along m or n: 32 k rows of R elements in R / 8 chunks, chunk q
//     of k row k at slot q ^ ((k >> 3) & (R / 8 - 1)) (the four k groups of
//     an MFMA operand in different banks), read with the gfx950 transposing
//     LDS read.
// Each wave copies R / 64 consecutive 1 KB pieces of each operand slab.
// Lanes outside the operand (rows past m or n, k chunks past K) copy the
// operand's first 16 bytes instead, so every wave issues the same number of
// copies per slab and the waits count them exactly; those LDS cells only
// reach rows and columns that are not written back (past m or n), or are
// zeroed in registers (k past K) before the MFMA.
template <int DC, int BM, int BN, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    S == 2 ? (BM * BN > 4096 ? 5 : 7) : (BM * BN > 8192 ? 2 : (BM * BN > 4096 ? 3 : 5))))) void gemm_bf16_pipe(
    const RawJob* __restrict__ jobs, const RawTerm* __restrict__ terms, const WorkItem* __restrict__ items,
    void* __restrict__ part) {
  constexpr int KT = 32;
  constexpr int FA = BM / 32, FB = BN / 32;  // 16x16 MFMA blocks per wave along m / n
  constexpr int NA = BM / 64, NB = BN / 64;  // 1 KB copies per wave per slab
  constexpr int NI = NA + NB;
  constexpr int SA = BM * KT, STG = (BM + BN) * KT;  // u16 elements: A part of a stage, a stage
  static_assert(S >= 2 && S <= 4, "pipeline depth");
  __shared__ __attribute__((aligned(16))) u16 smem[S * STG];
  static_assert(BM * BN <= S * STG, "output tile must fit the stages");
  const int tid = threadIdx.x;
  const WorkItem W = items[blockIdx.x];
  const RawJob J = jobs[W.job];
  const int m0 = W.ti * BM, n0 = W.tj * BN;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int lr = lane & 15, lg = lane >> 4;

  f4 acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  if (W.has_ident) tile_identity_products<BM, BN, false, false>(acc, W, J, terms, m0, n0, wm, wn, lr, lg);

  // Product records are read through the constant address space, which
  // makes the compiler use scalar loads for them (counted apart from the
  // vector-memory operations the pipeline waits on): a vector load of a
  // record inside the K loop would come with a wait for every slab in
  // flight.
  typedef const __attribute__((address_space(4))) RawTerm CTerm;
  CTerm* cterms = (CTerm*)(uintptr_t)terms;
  auto next_dense = [&](int t) {
    while (t < W.tend && ((cterms[t].flags & (TF_IDENT_A | TF_IDENT_B)) || cterms[t].k <= 0)) ++t;
    return t;
  };
  const unsigned lds0 = (unsigned)(uintptr_t)smem;
  // ---- loader: product tl, slab kl
  int tl = next_dense(W.dense0), kl = 0;
  const u16* LA = nullptr;
  const u16* LB = nullptr;
  long long lda = 0, ldb = 0;
  int lK = 0;
  bool laK = true, lbK = true;
  auto load_term = [&]() {
    CTerm& T = cterms[tl];
    LA = (const u16*)T.A;
    LB = (const u16*)T.B;
    lda = T.lda;
    ldb = T.ldb;
    lK = T.k;
    const int fl = T.flags;
    laK = !(fl & TF_TRANS_A);  // A stored m x k
    lbK = (fl & TF_TRANS_B);   // B stored n x k
  };
  if (tl < W.tend) load_term();
  // one operand's copies of slab kl into LDS byte address dst
  auto copy_operand = [&](const u16* P, long long ld, bool alongK, int R, int r0, int ext, int nv, unsigned dst) {
    for (int v = 0; v < nv; ++v) {
      const int c = wave * nv + v;  // 1 KB piece of the slab
      const int pz = c * 64 + lane;  // 16-byte slot
      const u16* g = P;
      if (alongK) {
        const int row = pz >> 2, q = (pz & 3) ^ ((row >> 2) & 3);
        if (r0 + row < ext && kl + 8 * q < lK) g = P + (long long)(r0 + row) * ld + kl + 8 * q;
      } else {
        const int cpr = R / 8, kr = pz / cpr, q = (pz % cpr) ^ ((kr >> 3) & (cpr - 1));
        if (kl + kr < lK && r0 + 8 * q < ext) g = P + (long long)(kl + kr) * ld + r0 + 8 * q;
      }
      lds_dma16(g, __builtin_amdgcn_readfirstlane(dst + c * 1024));
    }
  };
  auto issue = [&](int st) {
    const unsigned base = lds0 + (unsigned)(st * STG) * 2u;
    copy_operand(LA, lda, laK, BM, m0, J.m, NA, base);
    copy_operand(LB, ldb, lbK, BN, n0, J.n, NB, base + SA * 2u);
    kl += KT;
    if (kl >= lK) {
      tl = next_dense(tl + 1);
      kl = 0;
      if (tl < W.tend) load_term();
    }
  };
  int issued = 0;
#pragma unroll
  for (int s0 = 0; s0 < S - 1; ++s0)
    if (tl < W.tend) {
      issue(s0);
      ++issued;
    }
  // ---- consumer: product tc, slab kc
  int tc = next_dense(W.dense0), kc = 0, cK = 0;
  bool caK = true, cbK = true;
  float alpha = 1.f, scale = 1.f;
  auto use_term = [&]() {
    CTerm& T = cterms[tc];
    cK = T.k;
    const int fl = T.flags;
    caK = !(fl & TF_TRANS_A);
    cbK = (fl & TF_TRANS_B);
    alpha = (float)T.alpha;
  };
  if (tc < W.tend) use_term();
  // LDS element offsets of this lane's MFMA operands (k group lg)
  auto offK = [&](int r) { return r * KT + 8 * (lg ^ ((r >> 2) & 3)); };
  auto offMN = [&](int R, int k, int r) { return k * R + 8 * ((r >> 3) ^ ((k >> 3) & (R / 8 - 1))) + (r & 7); };
  // Operand stored along m / n: ds_read_b64_tr_b16 over each group of 16
  // lanes returns to lane i the value j of the 4-element run addressed by
  // lane 4 j + (i >> 2), element i & 3.  Lane q of k group lg addresses the
  // run at k row 8 lg + (q >> 2) (+ 4 for the upper half) and column
  // c0 + 4 (q & 3), so lane (lr, lg) receives column c0 + lr at k rows
  // 8 lg .. 8 lg + 7: its MFMA operand, in two reads instead of eight.
  typedef short s4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) s4 lds_s4;
  auto frag_mn = [&](const u16* sX, int R, int c0) -> bf8 {
    const int k1 = 8 * lg + (lr >> 2), c = c0 + 4 * (lr & 3);
    const s4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(sX + offMN(R, k1, c)));
    const s4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(sX + offMN(R, k1 + 4, c)));
    return __builtin_bit_cast(bf8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
  };
  int i = 0;
  while (tc < W.tend) {
    const int st = i % S;
    const int ahead = issued - i - 1;  // slabs issued after slab i, 0 .. S - 2
    if (S >= 4 && ahead >= 2) pipe_wait_barrier<2 * NI>();
    else if (S >= 3 && ahead >= 1) pipe_wait_barrier<NI>();
    else pipe_wait_barrier<0>();
    if (tl < W.tend) {
      issue(issued % S);  // the stage slab i - 1 used; every wave is past it
      ++issued;
    }
    if (kc == 0 && alpha != scale) {  // product tc starts: move acc into its frame
      const float r = scale / alpha;
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] *= r;
      scale = alpha;
    }
    const u16* sA = smem + st * STG;
    const u16* sB = sA + SA;
    bf8 av[FA], bv[FB];
#pragma unroll
    for (int a = 0; a < FA; ++a) {
      const int r = wm + a * 16 + lr;
      if (caK) av[a] = *(const bf8*)(sA + offK(r));
      else av[a] = frag_mn(sA, BM, wm + a * 16);
    }
#pragma unroll
    for (int b = 0; b < FB; ++b) {
      const int r = wn + b * 16 + lr;
      if (cbK) bv[b] = *(const bf8*)(sB + offK(r));
      else bv[b] = frag_mn(sB, BN, wn + b * 16);
    }
    const int nvk = cK - kc - 8 * lg;  // valid k of this lane's eight
    if (nvk < 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j >= nvk) {
#pragma unroll
          for (int a = 0; a < FA; ++a) av[a][j] = (__bf16)0.f;
#pragma unroll
          for (int b = 0; b < FB; ++b) bv[b][j] = (__bf16)0.f;
        }
    }
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    ++i;
    kc += KT;
    if (kc >= cK) {
      tc = next_dense(tc + 1);
      kc = 0;
      if (tc < W.tend) use_term();
    }
  }
  if (scale != 1.f) {
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b) acc[a][b] *= scale;
  }
  tile_store<DC, BM, BN>(acc, W, J, smem, part, m0, n0, wm, wn, lr, lg, tid);
}

// FP64 counterpart of gemm_bf16_pipe for padded launches: slabs of 16 k
// (16-byte LDS DMA pieces of two doubles), S stages, v_mfma_f64_16x16x4f64
// with 2 x 2 blocks per wave (64 x 64 tile) or 4 x 2 / 2 x 4 (128 x 64,
// 64 x 128).  MFMA step s of a slab takes k = 4 lg + s from lane group lg,
// so a lane's four k values of an operand stored along k are one 32-byte
// run.  LDS layouts per stage and operand (R rows):
//   * along k: R rows of 16 doubles in eight 16-byte chunks, chunk q of row r
//     at slot q ^ (r & 7), read as two 16-byte vectors;
//   * along m or n: 16 k rows of R doubles in R / 2 chunks, chunk q of k row
//     k at slot q ^ (((k >> 2) & 3) << 3), read as four 8-byte values.
// Product weights multiply A as it is read from LDS (as in gemm_kernel).
// Same copy / wait / masking rules as gemm_bf16_pipe.
template <int BM, int BN, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == 2 ? 4 : 3))) void gemm_f64_pipe(
    const RawJob* __restrict__ jobs, const RawTerm* __restrict__ terms, const WorkItem* __restrict__ items,
    void* __restrict__ part) {
  constexpr int KT = 16;
  constexpr int FA = BM / 32, FB = BN / 32;
  constexpr int NA = BM / 32, NB = BN / 32;  // 1 KB copies per wave per slab (R / 8 pieces over 4 waves)
  constexpr int NI = NA + NB;
  constexpr int SA = BM * KT, STG = (BM + BN) * KT;  // doubles
  static_assert(S >= 2 && S <= 3, "pipeline depth");
  __shared__ __attribute__((aligned(16))) double smem[S * STG];
  const int tid = threadIdx.x;
  const WorkItem W = items[blockIdx.x];
  const RawJob J = jobs[W.job];
  const int m0 = W.ti * BM, n0 = W.tj * BN;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int lr = lane & 15, lg = lane >> 4;

  d4 acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  if (W.has_ident)
    for (int t = W.tbeg; t < W.tend; ++t) {
      const int fl = terms[t].flags;
      if (!(fl & (TF_IDENT_A | TF_IDENT_B))) continue;
      const RawTerm T = terms[t];
      const bool ia = fl & TF_IDENT_A;
      const double* P = (const double*)(ia ? T.B : T.A);
      const long long ld = ia ? T.ldb : T.lda;
      const bool tr = ia ? (fl & TF_TRANS_B) : (fl & TF_TRANS_A);
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = m0 + wm + a * 16 + 4 * v + lg, col = n0 + wn + b * 16 + lr;
            if (row < J.m && col < J.n) acc[a][b][v] += T.alpha * P[tr ? (long long)col * ld + row : (long long)row * ld + col];
          }
    }

  typedef const __attribute__((address_space(4))) RawTerm CTerm;
  CTerm* cterms = (CTerm*)(uintptr_t)terms;
  auto next_dense = [&](int t) {
    while (t < W.tend && ((cterms[t].flags & (TF_IDENT_A | TF_IDENT_B)) || cterms[t].k <= 0)) ++t;
    return t;
  };
  const unsigned lds0 = (unsigned)(uintptr_t)smem;
  int tl = next_dense(W.dense0), kl = 0;
  const double* LA = nullptr;
  const double* LB = nullptr;
  long long lda = 0, ldb = 0;
  int lK = 0;
  bool laK = true, lbK = true;
  auto load_term = [&]() {
    CTerm& T = cterms[tl];
    LA = (const double*)T.A;
    LB = (const double*)T.B;
    lda = T.lda;
    ldb = T.ldb;
    lK = T.k;
    const int fl = T.flags;
    laK = !(fl & TF_TRANS_A);
    lbK = (fl & TF_TRANS_B);
  };
  if (tl < W.tend) load_term();
  auto copy_operand = [&](const double* P, long long ld, bool alongK, int R, int r0, int ext, int nv, unsigned dst) {
    for (int v = 0; v < nv; ++v) {
      const int c = wave * nv + v;
      const int pz = c * 64 + lane;
      const double* g = P;
      if (alongK) {
        const int row = pz >> 3, q = (pz & 7) ^ (row & 7);
        if (r0 + row < ext && kl + 2 * q < lK) g = P + (long long)(r0 + row) * ld + kl + 2 * q;
      } else {
        const int cpr = R / 2, kr = pz / cpr, q = (pz % cpr) ^ (((kr >> 2) & 3) << 3);
        if (kl + kr < lK && r0 + 2 * q < ext) g = P + (long long)(kl + kr) * ld + r0 + 2 * q;
      }
      lds_dma16(g, __builtin_amdgcn_readfirstlane(dst + c * 1024));
    }
  };
  auto issue = [&](int st) {
    const unsigned base = lds0 + (unsigned)(st * STG) * 8u;
    copy_operand(LA, lda, laK, BM, m0, J.m, NA, base);
    copy_operand(LB, ldb, lbK, BN, n0, J.n, NB, base + SA * 8u);
    kl += KT;
    if (kl >= lK) {
      tl = next_dense(tl + 1);
      kl = 0;
      if (tl < W.tend) load_term();
    }
  };
  int issued = 0;
#pragma unroll
  for (int s0 = 0; s0 < S - 1; ++s0)
    if (tl < W.tend) {
      issue(s0);
      ++issued;
    }
  int tc = next_dense(W.dense0), kc = 0, cK = 0;
  bool caK = true, cbK = true;
  double alpha = 1.0;
  auto use_term = [&]() {
    CTerm& T = cterms[tc];
    cK = T.k;
    const int fl = T.flags;
    caK = !(fl & TF_TRANS_A);
    cbK = (fl & TF_TRANS_B);
    alpha = T.alpha;
  };
  if (tc < W.tend) use_term();
  // this lane's four values (k = 4 lg + s) of row / column r
  auto frag = [&](const double* sX, bool alongK, int R, int r, double (&f)[4]) {
    if (alongK) {
      const double2 u = *(const double2*)(sX + r * KT + 2 * ((2 * lg) ^ (r & 7)));
      const double2 w = *(const double2*)(sX + r * KT + 2 * ((2 * lg + 1) ^ (r & 7)));
      f[0] = u.x;
      f[1] = u.y;
      f[2] = w.x;
      f[3] = w.y;
    } else {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int k = 4 * lg + s2;
        f[s2] = sX[k * R + 2 * ((r >> 1) ^ (lg << 3)) + (r & 1)];
      }
    }
  };
  int i = 0;
  while (tc < W.tend) {
    const int st = i % S;
    const int ahead = issued - i - 1;
    if (S >= 3 && ahead >= 1) pipe_wait_barrier<NI>();
    else pipe_wait_barrier<0>();
    if (tl < W.tend) {
      issue(issued % S);
      ++issued;
    }
    const double* sA = smem + st * STG;
    const double* sB = sA + SA;
    double af[FA][4], bf[FB][4];
#pragma unroll
    for (int a = 0; a < FA; ++a) frag(sA, caK, BM, wm + a * 16 + lr, af[a]);
#pragma unroll
    for (int b = 0; b < FB; ++b) frag(sB, cbK, BN, wn + b * 16 + lr, bf[b]);
    const int nvk = cK - kc - 4 * lg;  // valid k of this lane's four
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const bool ok = s2 < nvk;
#pragma unroll
      for (int a = 0; a < FA; ++a) af[a][s2] = ok ? af[a][s2] * alpha : 0.0;
#pragma unroll
      for (int b = 0; b < FB; ++b) bf[b][s2] = ok ? bf[b][s2] : 0.0;
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][s2], bf[b][s2], acc[a][b], 0, 0, 0);
    ++i;
    kc += KT;
    if (kc >= cK) {
      tc = next_dense(tc + 1);
      kc = 0;
      if (tc < W.tend) use_term();
    }
  }
  // write back: C (FP64, rows 4 v + lg of each 16 x 16 block), or the partial slot
  if (W.slot >= 0) {
    double* P = (double*)part + (long long)W.slot * (BM * BN);
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(wm + a * 16 + 4 * v + lg) * BN + wn + b * 16 + lr] = acc[a][b][v];
    return;
  }
  double* C = (double*)J.C;
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + a * 16 + 4 * v + lg, col = n0 + wn + b * 16 + lr;
        if (row < J.m && col < J.n) {
          const long long o = (long long)row * J.ldc + col;
          if (J.accumulate) C[o] += acc[a][b][v];
          else C[o] = acc[a][b][v];
        }
      }
}

// BF16 kernel for padded launches dominated by small blocks (many output
// matrices of a few rows or columns, where a 64 x 64 tile is mostly empty):
// each wave owns one 32 x 32 output tile (2 x 2 blocks of
// v_mfma_f32_16x16x32_bf16) and the four waves of a work-group serve four
// independent work items.  Operands go from memory straight into the MFMA
// registers -- one 16-byte vector per lane and block where the operand is
// contiguous along k, eight 2-byte loads where it is contiguous along m (n)
// -- so there is no LDS and no barrier; the next slab is loaded before the
// current one is multiplied.  Product weights use the scaled accumulator
// frame of gemm_bf16_padded.  Same work items, split-K slots and reduction as
// the other kernels, with bm = bn = 32.  The register budget is capped at 6
// waves per SIMD, the most that compiles without scratch.
template <int DC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void gemm_bf16_wave(const RawJob* __restrict__ jobs, const RawTerm* __restrict__ terms,
                                                      const WorkItem* __restrict__ items, void* __restrict__ part,
                                                      long long nitems) {
  constexpr int T = 32, KT = 32;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const long long it = (long long)blockIdx.x * 4 + wv;
  if (it >= nitems) return;  // whole wave; the kernel has no barrier
  const WorkItem W = items[it];
  const RawJob J = jobs[W.job];
  const int m0 = W.ti * T, n0 = W.tj * T;
  const int lr = lane & 15, lg = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  // identity products, in the unscaled frame
  if (W.has_ident)
    for (int t = W.tbeg; t < W.tend; ++t) {
      const int fl = terms[t].flags;
      if (!(fl & (TF_IDENT_A | TF_IDENT_B))) continue;
      const RawTerm Ti = terms[t];
      const bool ia = fl & TF_IDENT_A;
      const u16* P = (const u16*)(ia ? Ti.B : Ti.A);
      const long long ld = ia ? Ti.ldb : Ti.lda;
      const bool tr = ia ? (fl & TF_TRANS_B) : (fl & TF_TRANS_A);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = m0 + a * 16 + 4 * lg + v, col = n0 + b * 16 + lr;
            if (row < J.m && col < J.n)
              acc[a][b][v] += (float)Ti.alpha * bf2f(P[tr ? (long long)col * ld + row : (long long)row * ld + col]);
          }
    }
  // slab k0 of product Tm into this lane's operand registers: k = k0 + 8 lg + j
  auto fetch = [&](const RawTerm& Tm, int k0, uint4 (&ra)[2], uint4 (&rb)[2]) {
    const int kb = k0 + 8 * lg, nk = Tm.k - kb;
    const u16* A = (const u16*)Tm.A;
    const u16* B = (const u16*)Tm.B;
    const bool aK = !(Tm.flags & TF_TRANS_A);  // A stored m x k
    const bool bK = (Tm.flags & TF_TRANS_B);   // B stored n x k
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int r = m0 + a * 16 + lr;
      ra[a] = make_uint4(0, 0, 0, 0);
      if (r < J.m && nk > 0) {
        if (aK) {
          ra[a] = *(const uint4*)(A + (long long)r * Tm.lda + kb);
          if (nk < 8) ra[a] = keep_first<2>(ra[a], nk);
        } else {
          unsigned w[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const unsigned lo = (2 * q < nk) ? A[(long long)(kb + 2 * q) * Tm.lda + r] : 0u;
            const unsigned hi = (2 * q + 1 < nk) ? A[(long long)(kb + 2 * q + 1) * Tm.lda + r] : 0u;
            w[q] = lo | (hi << 16);
          }
          ra[a] = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = n0 + b * 16 + lr;
      rb[b] = make_uint4(0, 0, 0, 0);
      if (c < J.n && nk > 0) {
        if (bK) {
          rb[b] = *(const uint4*)(B + (long long)c * Tm.ldb + kb);
          if (nk < 8) rb[b] = keep_first<2>(rb[b], nk);
        } else {
          unsigned w[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const unsigned lo = (2 * q < nk) ? B[(long long)(kb + 2 * q) * Tm.ldb + c] : 0u;
            const unsigned hi = (2 * q + 1 < nk) ? B[(long long)(kb + 2 * q + 1) * Tm.ldb + c] : 0u;
            w[q] = lo | (hi << 16);
          }
          rb[b] = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
    }
  };
  auto next_dense = [&](int t) {
    while (t < W.tend && (terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) ++t;
    return t;
  };
  uint4 ra[2], rb[2], na[2], nb[2];
  int t = W.dense0, k0 = 0;
  float scale = 1.f;  // acc holds the partial sum divided by scale
  RawTerm Tc;
  if (t < W.tend) {
    Tc = terms[t];
    fetch(Tc, 0, ra, rb);
  }
  while (t < W.tend) {
    int t2 = t, k2 = k0 + KT;
    RawTerm Tn = Tc;
    if (k2 >= Tc.k) {
      t2 = next_dense(t + 1);
      k2 = 0;
      if (t2 < W.tend) Tn = terms[t2];
    }
    if (t2 < W.tend) fetch(Tn, k2, na, nb);
    const float alpha = (float)Tc.alpha;
    if (k0 == 0 && alpha != scale) {
      // product t starts: move the accumulator into its frame
      const float r = scale / alpha;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] *= r;
      scale = alpha;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ra[a]),
                                                            __builtin_bit_cast(bf8, rb[b]), acc[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      ra[a] = na[a];
      rb[a] = nb[a];
    }
    t = t2;
    k0 = k2;
    Tc = Tn;
  }
  if (scale != 1.f) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] *= scale;
  }
  if (W.slot >= 0) {
    float* P = (float*)part + (long long)W.slot * (T * T);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(a * 16 + 4 * lg + v) * T + b * 16 + lr] = acc[a][b][v];
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + a * 16 + 4 * lg + v, col = n0 + b * 16 + lr;
        if (row < J.m && col < J.n) {
          const long long o = (long long)row * J.ldc + col;
          if (J.accumulate) stv<DC>(J.C, o, ldv<DC>(J.C, o) + (double)acc[a][b][v]);
          else stv<DC>(J.C, o, acc[a][b][v]);
        }
      }
}

// FP64 counterpart of gemm_bf16_wave for launches of mostly small blocks:
// one wave per 32 x 32 output tile (2 x 2 blocks of v_mfma_f64_16x16x4f64),
// four independent work items per work-group, K slabs of 16.  Each lane
// loads its operand elements (row or column lr, k = k0 + 4 s + lg) directly;
// 8-byte loads need no padding or alignment, so any FP64 launch qualifies.
// The product weight multiplies A as it is loaded, as in gemm_kernel.  The
// register cap keeps 4 waves per SIMD (127 VGPRs, no scratch).
template <int DUMMY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gemm_f64_wave(const RawJob* __restrict__ jobs, const RawTerm* __restrict__ terms,
                                                     const WorkItem* __restrict__ items, void* __restrict__ part,
                                                     long long nitems) {
  constexpr int T = 32, KT = 16;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const long long it = (long long)blockIdx.x * 4 + wv;
  if (it >= nitems) return;  // whole wave; the kernel has no barrier
  const WorkItem W = items[it];
  const RawJob J = jobs[W.job];
  const int m0 = W.ti * T, n0 = W.tj * T;
  const int lr = lane & 15, lg = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  if (W.has_ident)
    for (int t = W.tbeg; t < W.tend; ++t) {
      const int fl = terms[t].flags;
      if (!(fl & (TF_IDENT_A | TF_IDENT_B))) continue;
      const RawTerm Ti = terms[t];
      const bool ia = fl & TF_IDENT_A;
      const double* P = (const double*)(ia ? Ti.B : Ti.A);
      const long long ld = ia ? Ti.ldb : Ti.lda;
      const bool tr = ia ? (fl & TF_TRANS_B) : (fl & TF_TRANS_A);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = m0 + a * 16 + acc_row<DT_F64>(lg, v), col = n0 + b * 16 + lr;
            if (row < J.m && col < J.n)
              acc[a][b][v] += Ti.alpha * P[tr ? (long long)col * ld + row : (long long)row * ld + col];
          }
    }
  // slab k0 of product Tm: ra[a][s] = alpha A(m0 + 16 a + lr, k0 + 4 s + lg),
  // rb[b][s] = B(k0 + 4 s + lg, n0 + 16 b + lr), zero outside the matrices
  auto fetch = [&](const RawTerm& Tm, int k0, double (&ra)[2][4], double (&rb)[2][4]) {
    const double* A = (const double*)Tm.A;
    const double* B = (const double*)Tm.B;
    const bool ta = Tm.flags & TF_TRANS_A, tb = Tm.flags & TF_TRANS_B;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int r = m0 + a * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 4 * q + lg;
        ra[a][q] = (r < J.m && k < Tm.k) ? Tm.alpha * A[ta ? (long long)k * Tm.lda + r : (long long)r * Tm.lda + k] : 0.0;
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = n0 + b * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 4 * q + lg;
        rb[b][q] = (c < J.n && k < Tm.k) ? B[tb ? (long long)c * Tm.ldb + k : (long long)k * Tm.ldb + c] : 0.0;
      }
    }
  };
  auto next_dense = [&](int t) {
    while (t < W.tend && (terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) ++t;
    return t;
  };
  double ra[2][4], rb[2][4], na[2][4], nb[2][4];
  int t = W.dense0, k0 = 0;
  RawTerm Tc;
  if (t < W.tend) {
    Tc = terms[t];
    fetch(Tc, 0, ra, rb);
  }
  while (t < W.tend) {
    int t2 = t, k2 = k0 + KT;
    RawTerm Tn = Tc;
    if (k2 >= Tc.k) {
      t2 = next_dense(t + 1);
      k2 = 0;
      if (t2 < W.tend) Tn = terms[t2];
    }
    if (t2 < W.tend) fetch(Tn, k2, na, nb);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[a][q], rb[b][q], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ra[a][q] = na[a][q];
        rb[a][q] = nb[a][q];
      }
    t = t2;
    k0 = k2;
    Tc = Tn;
  }
  if (W.slot >= 0) {
    double* P = (double*)part + (long long)W.slot * (T * T);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(a * 16 + acc_row<DT_F64>(lg, v)) * T + b * 16 + lr] = acc[a][b][v];
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + a * 16 + acc_row<DT_F64>(lg, v), col = n0 + b * 16 + lr;
        if (row < J.m && col < J.n) {
          const long long o = (long long)row * J.ldc + col;
          double* C = (double*)J.C;
          if (J.accumulate) C[o] += acc[a][b][v];
          else C[o] = acc[a][b][v];
        }
      }
}

// Sum of the partial tiles (bm x bn values each) of split items, in slot
// order, into C.
template <int MODE, int DC>
__global__ __launch_bounds__(256) void reduce_kernel(const RawJob* __restrict__ jobs, const RedItem* __restrict__ items,
                                                     const void* __restrict__ part, int bm, int bn) {
  using sc_t = typename std::conditional<MODE == DT_F64, double, float>::type;
  const RedItem R = items[blockIdx.x];
  const RawJob J = jobs[R.job];
  const long long tile = (long long)bm * bn;
  const sc_t* P = (const sc_t*)part + (long long)R.slot0 * tile;
  for (int e = threadIdx.x; e < bm * bn; e += 256) {
    const int row = R.ti * bm + e / bn, col = R.tj * bn + e % bn;
    if (row >= J.m || col >= J.n) continue;
    sc_t s = 0;
    for (int q = 0; q < R.nslot; ++q) s += P[(long long)q * tile + e];
    const long long o = (long long)row * J.ldc + col;
    if (J.accumulate) {
      if constexpr (DC == DT_F64) ((double*)J.C)[o] += (double)s;
      else stv<DC>(J.C, o, ldv<DC>(J.C, o) + (double)s);
    } else {
      stv<DC>(J.C, o, s);
    }
  }
}

template <int DD>
__global__ void pack_kernel(void* dst, const double* __restrict__ src, const int* __restrict__ idx, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int j = idx[i];
    stv<DD>(dst, i, j >= 0 ? src[j] : 0.0);
  }
}

// bytes of zeros: 16-byte vectors, then the tail (stream-ordered clear that a
// graph may record, unlike a memset node)
__global__ void fill_zero_kernel(unsigned char* p, long long nbytes) {
  const long long nv = nbytes >> 4;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nv; i += (long long)gridDim.x * blockDim.x)
    ((uint4*)p)[i] = make_uint4(0, 0, 0, 0);
  const long long t = (nv << 4) + blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < nbytes && blockIdx.x == 0 && threadIdx.x < 16) p[t] = 0;
}

template <int DS>
__global__ void gather_kernel(double* __restrict__ dst, const void* __restrict__ src, const int* __restrict__ idx,
                              long long n, double a, const double* __restrict__ x, const double* __restrict__ mul) {
  const double m = mul ? mul[0] : 1.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = x ? m * ldv<DS>(src, idx[i]) + a * x[i] : m * ldv<DS>(src, idx[i]);
}

// ---- FP8 copies.  Power-of-two scales s, chosen so that max|x| / s <= 448
// (the largest finite E4M3 value): the stored values are x / s rounded to
// E4M3, and s is applied exactly in FP32/FP64 elsewhere.
__global__ __launch_bounds__(256) void absmax_partial(const double* __restrict__ x, long long n, long long stride,
                                                      double* __restrict__ part) {
  // one work-group per (segment blockIdx.y, slice blockIdx.x) of the segments [y*stride, y*stride + n)
  __shared__ double red[256];
  const double* p = x + (long long)blockIdx.y * stride;
  double m = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) m = fmax(m, fabs(p[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// scale[y] = (s, 1/s) of segment y from its gridDim-wide partial maxima
// Segments whose largest magnitude is at most `floor` keep the scale 1 (their
// elements then round to E4M3 as they are, which flushes values far below
// its smallest subnormal 2^-9 to zero).
__global__ void pow2_scale(const double* __restrict__ part, int nb, int nseg, double* __restrict__ scale,
                           double floor) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= nseg) return;
  double m = 0.0;
  for (int i = 0; i < nb; ++i) m = fmax(m, part[(long long)y * nb + i]);
  int e = 0;
  if (m > floor) {
    (void)frexp(m / 448.0, &e);  // m / 448 = f * 2^e, f in [0.5, 1): m / 2^e <= 448
  }
  scale[2 * y] = ldexp(1.0, e);
  scale[2 * y + 1] = ldexp(1.0, -e);
}

__global__ void to_fp8_kernel(unsigned char* __restrict__ dst, const double* __restrict__ src, long long n,
                              long long seg, const double* __restrict__ scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = f_to_fp8((float)(src[i] * scale[2 * (i / seg) + 1]));
}

__global__ void pack_fp8_kernel(unsigned char* __restrict__ dst, const double* __restrict__ src,
                                const int* __restrict__ idx, long long n, const double* __restrict__ scale) {
  const double inv = scale[1];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int j = idx[i];
    dst[i] = j >= 0 ? f_to_fp8((float)(src[j] * inv)) : (unsigned char)0;
  }
}

template <int DD>
__global__ void shifted_copy_kernel(void* __restrict__ dst, const double* __restrict__ src,
                                    const int* __restrict__ idx, long long n, double a) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    stv<DD>(dst, idx[i], src[idx[i]] + a);
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

// The scalar arguments come from the kernel arguments, or (a non-null device
// pointer: launches recorded into a graph) from device memory.
__global__ __launch_bounds__(256) void combine_kernel(double* __restrict__ y, const double* __restrict__ V,
                                                      long long ldv, int m, Coef64 c, const double* c_dev, double sgn,
                                                      long long n, double beta) {
  __shared__ double cs[64];
  if ((int)threadIdx.x < m) cs[threadIdx.x] = c_dev ? sgn * c_dev[threadIdx.x] : c.c[threadIdx.x];
  __syncthreads();
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
    double s = (beta == 0.0) ? 0.0 : beta * y[j];
    for (int i = 0; i < m; ++i) s += cs[i] * V[i * ldv + j];
    y[j] = s;
  }
}

__global__ void axpby_kernel(double* z, double a, const double* a_dev, const double* x, double b, const double* b_dev,
                             const double* y, long long n) {
  if (a_dev) a *= a_dev[0];
  if (b_dev) b *= b_dev[0];
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
    z[j] = a * x[j] + b * y[j];
}

__global__ void precond_kernel(double* t, const double* r, const double* d, double theta, const double* theta_dev,
                               double eps, long long n) {
  if (theta_dev) theta = theta_dev[0];
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
    double den = theta - d[j];
    if (fabs(den) < eps) den = den < 0 ? -eps : eps;
    t[j] = r[j] / den;
  }
}

// ---- orbital-rotation energy terms and their gradient (one work-group per
// auxiliary index L; n x n matrices, orbitals ordered core, active, virtual)
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(256) void orb_scalars_kernel(const double* __restrict__ Bm, int n, int nc, int na,
                                                          const double* __restrict__ gam, double* __restrict__ bact,
                                                          double* __restrict__ scal) {
  __shared__ double red[256];
  const int L = blockIdx.x;
  const double* B = Bm + (long long)L * n * n;
  double J = 0.0, t = 0.0, q = 0.0, r = 0.0;
  for (int i = threadIdx.x; i < nc; i += 256) J += B[(long long)i * n + i];
  for (int e = threadIdx.x; e < na * na; e += 256) {
    const int a = e / na, b = e % na;
    const double v = B[(long long)(nc + a) * n + nc + b];
    bact[(long long)L * na * na + e] = v;
    t += gam[e] * v;
  }
  for (int e = threadIdx.x; e < nc * nc; e += 256) {
    const int i = e / nc, j = e % nc;
    q += B[(long long)i * n + j] * B[(long long)j * n + i];
  }
  // r = sum_{t,i} B_{c+t,i} (sum_u gam_tu B_{i,c+u})
  for (int e = threadIdx.x; e < na * nc; e += 256) {
    const int a = e / nc, i = e % nc;
    double s = 0.0;
    for (int u = 0; u < na; ++u) s += gam[a * na + u] * B[(long long)i * n + nc + u];
    r += B[(long long)(nc + a) * n + i] * s;
  }
  J = block_sum(J, red);
  t = block_sum(t, red);
  q = block_sum(q, red);
  r = block_sum(r, red);
  if (threadIdx.x == 0) {
    scal[4 * L + 0] = J;
    scal[4 * L + 1] = t;
    scal[4 * L + 2] = q;
    scal[4 * L + 3] = r;
  }
}

__global__ __launch_bounds__(256) void orb_assemble_kernel(const double* __restrict__ Bm, int n, int nc, int na,
                                                           const double* __restrict__ gam,
                                                           const double* __restrict__ scal,
                                                           const double* __restrict__ bact,
                                                           const double* __restrict__ Y, const double* __restrict__ Z,
                                                           double* __restrict__ Gm, double* __restrict__ e2) {
  __shared__ double red[256];
  const int L = blockIdx.x;
  const long long nn = (long long)n * n;
  const double* B = Bm + L * nn;
  double* G = Gm + L * nn;
  const double J = scal[4 * L + 0], t = scal[4 * L + 1];
  const double* y = Y + (long long)L * na * na;
  const double* z = Z + (long long)L * na * na;
  for (long long e = threadIdx.x; e < nn; e += 256) {
    const int p = (int)(e / n), q = (int)(e % n);
    const bool pc = p < nc, qc = q < nc;
    const bool pa = p >= nc && p < nc + na, qa = q >= nc && q < nc + na;
    double v = 0.0;
    if (pc && qc) {
      v = -2.0 * B[(long long)q * n + p];  // d(-q)/dB_pq
      if (p == q) v += 4.0 * J + 2.0 * t;   // d(2J^2 + 2Jt)/dB_ii
    } else if (pa && qa) {
      const int a = p - nc, b = q - nc;
      v = 2.0 * J * gam[a * na + b] + 0.5 * (y[a * na + b] + z[a * na + b]);
    } else if (pa && qc) {  // d(-r)/dB_{c+t,i} = -sum_u gam_tu B_{i,c+u}
      const int a = p - nc;
      double s = 0.0;
      for (int u = 0; u < na; ++u) s += gam[a * na + u] * B[(long long)q * n + nc + u];
      v = -s;
    } else if (pc && qa) {  // d(-r)/dB_{i,c+u} = -sum_t gam_tu B_{c+t,i}
      const int b = q - nc;
      double s = 0.0;
      for (int a = 0; a < na; ++a) s += gam[a * na + b] * B[(long long)(nc + a) * n + p];
      v = -s;
    }
    G[e] = v;
  }
  double s = 0.0;
  for (int e = threadIdx.x; e < na * na; e += 256) s += bact[(long long)L * na * na + e] * y[e];
  s = block_sum(s, red);
  if (threadIdx.x == 0) e2[L] = 0.5 * s;
}

// ---- batched two-sided Jacobi eigensolver, parallel over the whole GPU
// Round-robin (circle) ordering over np = n rounded up to even "players":
// in round r player 0 meets player (r % (np-1)) + 1 ... every round pairs are
// disjoint, so all row rotations and then all column rotations of a round
// compose to R A R^T with R the product of the round's plane rotations.  A
// round is two launches over all matrices of the batch: the rotation angles
// of every pair, then the update of every 2x2 block (pair t rows, pair u
// columns) of A and every (row, pair) of V.  np-1 rounds make one sweep.
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

struct JacMat {
  long long off;        // element offset of the matrix (and of its V)
  long long blk_base;   // first 2x2-block work index
  long long vrow_base;  // first (row, pair) work index of V
  int n, np, pair_base, pad;
};

__device__ __forceinline__ int jac_find(const JacMat* __restrict__ M, int nm, long long g, int which) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const long long b = which == 0 ? (long long)M[mid].pair_base : (which == 1 ? M[mid].blk_base : M[mid].vrow_base);
    if (b <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void jac_identity(double* __restrict__ V, const JacMat* __restrict__ M) {
  const JacMat m = M[blockIdx.x];
  double* v = V + m.off;
  for (long long i = threadIdx.x; i < (long long)m.n * m.n; i += blockDim.x) v[i] = (i / m.n == i % m.n) ? 1.0 : 0.0;
}

// out[2*i] = off-diagonal sum of squares, out[2*i+1] = total, matrix i
__global__ __launch_bounds__(256) void jac_norms(const double* __restrict__ A, const JacMat* __restrict__ M,
                                                 double* __restrict__ out) {
  __shared__ double r0[256], r1[256];
  const JacMat m = M[blockIdx.x];
  const double* a = A + m.off;
  double off = 0.0, tot = 0.0;
  for (long long i = threadIdx.x; i < (long long)m.n * m.n; i += blockDim.x) {
    const double x = a[i] * a[i];
    tot += x;
    if (i / m.n != i % m.n) off += x;
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = r0[0];
    out[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ __launch_bounds__(256) void jac_angles(const double* __restrict__ A, const JacMat* __restrict__ M, int nm,
                                                  int npairs_total, int r, double* __restrict__ cs,
                                                  double* __restrict__ sn, int* __restrict__ pp, int* __restrict__ qq) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npairs_total) return;
  const JacMat m = M[jac_find(M, nm, g, 0)];
  const int t = g - m.pair_base;
  double c = 1.0, s = 0.0;
  int p = 0, q = -1;
  if (r < m.np - 1) {
    rr_pair(t, r, m.np, p, q);
    if (q >= m.n) q = -1;
    if (q >= 0) {
      const double* a = A + m.off;
      const double apq = a[(long long)p * m.n + q];
      if (apq != 0.0) {
        const double app = a[(long long)p * m.n + p], aqq = a[(long long)q * m.n + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        c = 1.0 / sqrt(1.0 + tt * tt);
        s = tt * c;
      }
    }
  } else {
    p = -1;  // this matrix has finished its rounds of the sweep
  }
  cs[g] = c;
  sn[g] = s;
  pp[g] = p;
  qq[g] = q;
}

// Work items [0, nblk): 2x2 blocks of A; [nblk, nblk + nvrow): (row, pair) of V.
__global__ __launch_bounds__(256) void jac_apply(double* __restrict__ A, double* __restrict__ V,
                                                 const JacMat* __restrict__ M, int nm, long long nblk, long long nvrow,
                                                 const double* __restrict__ cs, const double* __restrict__ sn,
                                                 const int* __restrict__ pp, const int* __restrict__ qq) {
  const long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (g < nblk) {
    const JacMat m = M[jac_find(M, nm, g, 1)];
    const int npairs = m.np >> 1;
    const long long L = g - m.blk_base;
    const int t = (int)(L / npairs), u = (int)(L % npairs);
    const int it = m.pair_base + t, iu = m.pair_base + u;
    const int pt = pp[it], qt = qq[it], pu = pp[iu], qu = qq[iu];
    if (pt < 0) return;  // matrix idle in this round
    if (sn[it] == 0.0 && sn[iu] == 0.0) return;
    double* a = A + m.off;
    const long long n = m.n;
    const double ct = cs[it], st = sn[it], cu = cs[iu], su = sn[iu];
    // block rows {pt, qt}, cols {pu, qu}; missing indices (q = -1) are absent
    double b00 = a[pt * n + pu];
    double b01 = qu >= 0 ? a[pt * n + qu] : 0.0;
    double b10 = qt >= 0 ? a[qt * n + pu] : 0.0;
    double b11 = (qt >= 0 && qu >= 0) ? a[qt * n + qu] : 0.0;
    // rows: p' = c p - s q, q' = s p + c q
    double r00 = ct * b00 - st * b10, r01 = ct * b01 - st * b11;
    double r10 = st * b00 + ct * b10, r11 = st * b01 + ct * b11;
    // columns likewise
    b00 = cu * r00 - su * r01;
    b01 = su * r00 + cu * r01;
    b10 = cu * r10 - su * r11;
    b11 = su * r10 + cu * r11;
    a[pt * n + pu] = b00;
    if (qu >= 0) a[pt * n + qu] = b01;
    if (qt >= 0) a[qt * n + pu] = b10;
    if (qt >= 0 && qu >= 0) a[qt * n + qu] = b11;
    return;
  }
  const long long h = g - nblk;
  if (h >= nvrow) return;
  const JacMat m = M[jac_find(M, nm, h, 2)];
  const int npairs = m.np >> 1;
  const long long L = h - m.vrow_base;
  const long long i = L / npairs;
  const int iu = m.pair_base + (int)(L % npairs);
  const int pu = pp[iu], qu = qq[iu];
  if (pu < 0 || qu < 0 || sn[iu] == 0.0) return;
  double* v = V + m.off + i * m.n;
  const double cu = cs[iu], su = sn[iu];
  const double x = v[pu], y = v[qu];
  v[pu] = cu * x - su * y;
  v[qu] = su * x + cu * y;
}

// Work-groups per launch of the grouped kernels: 256 threads each, and the
// grid's work-item count must fit 32 bits.
constexpr long long kMaxGroups = 1LL << 23;

// Fixed device scratch of the allocation-free H*psi entry point
// (dmrg_hpsi_dev_noalloc): one call's task lists, padded operand copy of psi,
// psi' accumulator, intermediates and partial tiles.  Every GPU the library
// runs on holds one copy until the process ends; all contexts on a device
// share it.  Host code reaches it only through the address returned by
// hipGetSymbolAddress (fixed_scratch_address), never through its name.
constexpr size_t kFixedScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device and kept.
void* fixed_scratch_address() {
  static std::mutex mu;
  static std::map<int, void*> addr;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw std::runtime_error("executor: fixed scratch has no device address");
  addr[dev] = p;
  return p;
}

struct Prepared {
  RawJob* d_jobs = nullptr;
  RawTerm* d_terms = nullptr;
  WorkItem* d_items = nullptr;
  RedItem* d_reds = nullptr;
  long long nitems = 0, nreds = 0, nslots = 0;
  int mode = DT_F64, da = DT_F64, db = DT_F64, dc = DT_F64, kt = 16;
  bool padded = false;  // BF16 launch served by gemm_bf16_padded
  bool wave = false;    // ... or by gemm_bf16_wave (32 x 32 tile per wave)
  bool pipe = false;    // ... or by gemm_bf16_pipe (LDS DMA pipeline)
  int stages = 0;       // its LDS stages (0: the default for the tile)
  bool pad64 = false;   // FP64 launch whose operands suit gemm_f64_pipe
  int bm = TM, bn = TN;  // output tile of the launch
  void* part = nullptr;  // partial tiles of a fixed-scratch launch (else the executor's)
  // fixed-scratch launches: task lists kept on the host until placed
  std::vector<RawJob> h_jobs;
  std::vector<RawTerm> h_terms;
  std::vector<WorkItem> h_items;
  std::vector<RedItem> h_reds;
};

using KernelFn = void (*)(const RawJob*, const RawTerm*, const WorkItem*, void*);
using WaveFn = void (*)(const RawJob*, const RawTerm*, const WorkItem*, void*, long long);
using ReduceFn = void (*)(const RawJob*, const RedItem*, const void*, int, int);

KernelFn pick(int mode, int da, int db, int dc, int kt) {
  if (da != mode || db != mode) throw std::runtime_error("executor: operands must be stored in the arithmetic type");
  if (mode == DT_F64 && dc == DT_F64) return gemm_kernel<DT_F64, DT_F64, 16>;
  if (mode == DT_F32 && dc == DT_F32) return gemm_kernel<DT_F32, DT_F32, 16>;
  if (mode == DT_BF16 && dc == DT_BF16) return kt == 64 ? gemm_kernel<DT_BF16, DT_BF16, 64> : gemm_kernel<DT_BF16, DT_BF16, 32>;
  if (mode == DT_BF16 && dc == DT_F32) return kt == 64 ? gemm_kernel<DT_BF16, DT_F32, 64> : gemm_kernel<DT_BF16, DT_F32, 32>;
  throw std::runtime_error("executor: unsupported dtype combination");
}

KernelFn pick_padded(int dc, int bm, int bn, bool af8 = false, bool bf8 = false) {
#define P_(D, M, N, FA, FB) \
  if (dc == D && bm == M && bn == N && af8 == FA && bf8 == FB) return gemm_bf16_padded<D, M, N, FA, FB>;
  P_(DT_BF16, 64, 64, false, false) P_(DT_BF16, 64, 128, false, false) P_(DT_BF16, 128, 64, false, false)
  P_(DT_F32, 64, 64, false, false) P_(DT_F32, 64, 128, false, false) P_(DT_F32, 128, 64, false, false)
  P_(DT_BF16, 128, 128, false, false) P_(DT_F32, 128, 128, false, false)
  // FP8 operands: stage L (operator blocks and psi in FP8, X out in BF16),
  // stage R (X in BF16, operator blocks in FP8, psi' out in FP32)
  P_(DT_BF16, 64, 64, true, true) P_(DT_BF16, 64, 128, true, true) P_(DT_BF16, 128, 64, true, true)
  P_(DT_F32, 64, 64, false, true) P_(DT_F32, 64, 128, false, true) P_(DT_F32, 128, 64, false, true)
  // (and the self-test's FP8 x FP8 into FP32)
  P_(DT_F32, 64, 64, true, true) P_(DT_F32, 64, 128, true, true) P_(DT_F32, 128, 64, true, true)
#undef P_
  throw std::runtime_error("executor: unsupported tile shape or FP8 operand combination");
}

// The LDS-pipelined kernel for a tile (BF16 operands only); the stage count
// keeps the LDS of a work-group at 32-48 KB.
// Two stages (16-24 KB) let more work-groups share a CU, for launches whose
// items are a few slabs long.
KernelFn pick_pipe(int dc, int bm, int bn, int stages = 0) {
#define P_(D, M, N, S, SS) \
  if (dc == D && bm == M && bn == N && (stages == 0 ? SS == 0 : stages == S)) return gemm_bf16_pipe<D, M, N, S>;
  P_(DT_BF16, 64, 64, 4, 0) P_(DT_BF16, 64, 128, 3, 0) P_(DT_BF16, 128, 64, 3, 0) P_(DT_BF16, 128, 128, 3, 0)
  P_(DT_F32, 64, 64, 4, 0) P_(DT_F32, 64, 128, 3, 0) P_(DT_F32, 128, 64, 3, 0) P_(DT_F32, 128, 128, 3, 0)
  P_(DT_BF16, 64, 64, 2, 1) P_(DT_BF16, 64, 128, 2, 1) P_(DT_BF16, 128, 64, 2, 1)
  P_(DT_F32, 64, 64, 2, 1) P_(DT_F32, 64, 128, 2, 1) P_(DT_F32, 128, 64, 2, 1)
#undef P_
  throw std::runtime_error("executor: unsupported tile shape for the pipelined kernel");
}

KernelFn pick_pipe_f64(int bm, int bn, int stages) {
  if (bm == 64 && bn == 64 && stages == 3) return gemm_f64_pipe<64, 64, 3>;
  if (bm == 64 && bn == 64 && stages == 2) return gemm_f64_pipe<64, 64, 2>;
  if (bm == 128 && bn == 64 && stages == 2) return gemm_f64_pipe<128, 64, 2>;
  if (bm == 64 && bn == 128 && stages == 2) return gemm_f64_pipe<64, 128, 2>;
  throw std::runtime_error("executor: unsupported tile for the FP64 pipelined kernel");
}

// Output tile of a padded BF16 launch.  Candidates 64x64, 64x128 and 128x64:
// among those whose padded MFMA work (tiles x tile area x K rounded to 32)
// is within 10 % of the smallest, the one with the fewest tiles (less fixed
// cost per item, more reuse of each staged slab).  DMRG_TILE=MxN overrides
// (also 128x128, which only the tuner picks otherwise).
void choose_tile(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int& bm, int& bn) {
  const int cand[3][2] = {{64, 64}, {64, 128}, {128, 64}};
  if (const char* e = std::getenv("DMRG_TILE")) {
    if (std::string(e) == "128x128") {
      bm = bn = 128;
      return;
    }
    for (auto& c : cand)
      if (std::string(e) == std::to_string(c[0]) + "x" + std::to_string(c[1])) {
        bm = c[0];
        bn = c[1];
        return;
      }
  }
  double work[3] = {0, 0, 0}, tiles[3] = {0, 0, 0};
  for (const RawJob& J : jobs) {
    double kpad = 0.0;
    for (int64_t t = J.tbeg; t < J.tend; ++t)
      if (!(terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) kpad += (double)((terms[t].k + 31) / 32 * 32);
    for (int c = 0; c < 3; ++c) {
      const double nt = (double)((J.m + cand[c][0] - 1) / cand[c][0]) * (double)((J.n + cand[c][1] - 1) / cand[c][1]);
      tiles[c] += nt;
      work[c] += nt * cand[c][0] * cand[c][1] * kpad;
    }
  }
  const double wmin = std::min(work[0], std::min(work[1], work[2]));
  int best = 0;
  for (int c = 1; c < 3; ++c)
    if (work[c] <= 1.1 * wmin && (work[best] > 1.1 * wmin || tiles[c] < tiles[best])) best = c;
  bm = cand[best][0];
  bn = cand[best][1];
}

// Whether a launch goes to a wave kernel (gemm_bf16_wave for padded BF16,
// gemm_f64_wave for FP64): when its padded MFMA work with 32 x 32 tiles (one
// wave each) is below 0.6 of that with 64 x 64 tiles, i.e. when most 64 x 64
// tiles would be largely empty.  kt: the K slab the padding is counted in.
// DMRG_WAVE=0 / 1 forces the choice.
bool choose_wave(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int kt) {
  if (const char* e = std::getenv("DMRG_WAVE")) return std::atoi(e) != 0;
  double w32 = 0.0, w64 = 0.0;
  for (const RawJob& J : jobs) {
    double kpad = 0.0;
    for (int64_t t = J.tbeg; t < J.tend; ++t)
      if (!(terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) kpad += (double)((terms[t].k + kt - 1) / kt * kt);
    w32 += (double)((J.m + 31) / 32) * (double)((J.n + 31) / 32) * 1024.0 * kpad;
    w64 += (double)((J.m + 63) / 64) * (double)((J.n + 63) / 64) * 4096.0 * kpad;
  }
  return w32 < 0.6 * w64;
}

WaveFn pick_wave(int mode, int dc) {
  if (mode == DT_F64 && dc == DT_F64) return gemm_f64_wave<0>;
  if (mode != DT_BF16) throw std::runtime_error("executor: unsupported wave-kernel mode");
  if (dc == DT_BF16) return gemm_bf16_wave<DT_BF16>;
  if (dc == DT_F32) return gemm_bf16_wave<DT_F32>;
  throw std::runtime_error("executor: unsupported wave-kernel output type");
}

// K slab of a BF16 launch: 64 when that pads the products' K by at most 1/8
// more than slabs of 32 would (long products), else 32 (short products, e.g.
// the K pieces of stage R).  DMRG_BF16_KT=32|64 overrides.
int choose_kt_bf16(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms) {
  if (const char* e = std::getenv("DMRG_BF16_KT")) {
    const int v = std::atoi(e);
    if (v == 32 || v == 64) return v;
  }
  double p32 = 0.0, p64 = 0.0;
  for (const RawJob& J : jobs) {
    const double tiles = (double)((J.m + TM - 1) / TM) * (double)((J.n + TN - 1) / TN);
    for (int64_t t = J.tbeg; t < J.tend; ++t) {
      if (terms[t].flags & (TF_IDENT_A | TF_IDENT_B)) continue;
      p32 += tiles * (double)((terms[t].k + 31) / 32 * 32);
      p64 += tiles * (double)((terms[t].k + 63) / 64 * 64);
    }
  }
  return (p64 <= 1.125 * p32) ? 64 : 32;
}
ReduceFn pick_reduce(int mode, int dc) {
  if (mode == DT_F64 && dc == DT_F64) return reduce_kernel<DT_F64, DT_F64>;
  if (mode != DT_F64 && dc == DT_F32) return reduce_kernel<DT_F32, DT_F32>;
  if (mode != DT_F64 && dc == DT_BF16) return reduce_kernel<DT_F32, DT_BF16>;
  throw std::runtime_error("executor: unsupported reduction dtype");
}

// Work decomposition of one launch.  The cost of a tile is its number of K
// steps (one per KT slice of each dense product, half a step per identity
// product).  Tiles whose cost exceeds a target are cut between products into
// several items that write partial tiles; the target is chosen so that the
// launch has at least ~min_items items (16k work-groups fill 256 CUs several
// times over; the wave kernels take four items per work-group and ask for
// 64k) but never below min_steps (64: a floor of 16 for the wave kernels
// added reduction work and gained nothing; 400 for the pipelined kernels).
// Items are issued heaviest first (longest processing time first), which
// bounds the tail of the launch, then grouped by shared A slab per XCD.
void plan_items(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int kt, int bm, int bn,
                double min_items, double min_steps, std::vector<WorkItem>& items, std::vector<RedItem>& reds,
                long long& nslots) {
  std::vector<double> pcost(terms.size());
  for (size_t t = 0; t < terms.size(); ++t)
    pcost[t] = (terms[t].flags & (TF_IDENT_A | TF_IDENT_B)) ? 0.5 : (double)((terms[t].k + kt - 1) / kt);
  double total = 0.0;
  for (const RawJob& J : jobs) {
    double c = 0.0;
    for (int64_t t = J.tbeg; t < J.tend; ++t) c += pcost[t];
    total += c * (double)((J.m + bm - 1) / bm) * (double)((J.n + bn - 1) / bn);
  }
  double target = std::max(min_steps, total / min_items);
  // DMRG_SPLIT_STEPS overrides the target (tuning and tests of the split path)
  if (const char* e = std::getenv("DMRG_SPLIT_STEPS")) {
    const double v = std::atof(e);
    if (v > 0.0) target = v;
  }
  std::vector<std::pair<double, WorkItem>> work;
  nslots = 0;
  reds.clear();
  for (size_t j = 0; j < jobs.size(); ++j) {
    const RawJob& J = jobs[j];
    if (J.m <= 0 || J.n <= 0) continue;
    // cut points of the product list (shared by all tiles of the job)
    std::vector<std::pair<int, int>> segs;
    std::vector<double> scost;
    double c = 0.0;
    int64_t s0 = J.tbeg;
    for (int64_t t = J.tbeg; t < J.tend; ++t) {
      c += pcost[t];
      if (c >= target && t + 1 < J.tend) {
        segs.push_back({(int)s0, (int)(t + 1)});
        scost.push_back(c);
        s0 = t + 1;
        c = 0.0;
      }
    }
    segs.push_back({(int)s0, (int)J.tend});
    scost.push_back(c);
    const int tm = (J.m + bm - 1) / bm, tn = (J.n + bn - 1) / bn;
    // per segment: first dense product and whether identities occur
    std::vector<int> d0(segs.size()), hid(segs.size());
    for (size_t q = 0; q < segs.size(); ++q) {
      d0[q] = segs[q].second;
      hid[q] = 0;
      for (int t = segs[q].first; t < segs[q].second; ++t) {
        if (terms[t].flags & (TF_IDENT_A | TF_IDENT_B)) hid[q] = 1;
        else if (d0[q] == segs[q].second) d0[q] = t;
      }
    }
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) {
        if (segs.size() == 1) {
          work.push_back({scost[0], WorkItem{(int)j, a, b, segs[0].first, segs[0].second, -1, d0[0], hid[0]}});
          continue;
        }
        reds.push_back(RedItem{(int)j, a, b, (int)nslots, (int)segs.size(), 0});
        for (size_t q = 0; q < segs.size(); ++q)
          work.push_back({scost[q], WorkItem{(int)j, a, b, segs[q].first, segs[q].second, (int)(nslots + q), d0[q],
                                             hid[q]}});
        nslots += (long long)segs.size();
      }
  }
  std::stable_sort(work.begin(), work.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  items.resize(work.size());
  for (size_t i = 0; i < work.size(); ++i) items[i] = work[i].second;
  {
    // Items that read the same A slab (same job, output row tile and product
    // segment) as consecutive work-groups of one XCD, so that they meet in
    // its L2: work-group i runs on XCD i mod 8, so each group goes whole to
    // the XCD queue with the least work so far, and the queues are
    // interleaved.  Groups keep the LPT order of their first item.  At
    // CAS(82,82): BF16 H*psi 308 -> 304 ms, FP64 1660 -> 1621 ms.
    // DMRG_XCD_GROUP=0 keeps the plain LPT order.
    const char* e = std::getenv("DMRG_XCD_GROUP");
    if (!(e && std::atoi(e) == 0) && items.size() > 64) {
      constexpr int kXcd = 8;
      // group by (job, row tile, segment start) with a sort, not a map: a
      // stage-L launch has about a million items
      struct K {
        int job, ti, tbeg;
        size_t pos;
      };
      std::vector<K> keys(work.size());
      for (size_t i = 0; i < work.size(); ++i) {
        const WorkItem& w = work[i].second;
        keys[i] = K{w.job, w.ti, w.tbeg, i};
      }
      std::sort(keys.begin(), keys.end(), [](const K& a, const K& b) {
        if (a.job != b.job) return a.job < b.job;
        if (a.ti != b.ti) return a.ti < b.ti;
        if (a.tbeg != b.tbeg) return a.tbeg < b.tbeg;
        return a.pos < b.pos;
      });
      // groups as [begin, end) ranges of keys, ordered by their first LPT position
      std::vector<std::pair<size_t, size_t>> grp;
      for (size_t i = 0; i < keys.size();) {
        size_t j = i + 1;
        while (j < keys.size() && keys[j].job == keys[i].job && keys[j].ti == keys[i].ti && keys[j].tbeg == keys[i].tbeg)
          ++j;
        grp.push_back({i, j});
        i = j;
      }
      std::sort(grp.begin(), grp.end(), [&](const auto& a, const auto& b) { return keys[a.first].pos < keys[b.first].pos; });
      std::vector<std::vector<WorkItem>> q(kXcd);
      std::vector<double> load(kXcd, 0.0);
      for (const auto& gr : grp) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (size_t i = gr.first; i < gr.second; ++i) {
          q[x].push_back(work[keys[i].pos].second);
          load[x] += work[keys[i].pos].first;
        }
      }
      size_t pos = 0;
      for (size_t r = 0; pos < items.size(); ++r)
        for (int x = 0; x < kXcd; ++x)
          if (r < q[x].size()) items[pos++] = q[x][r];
    }
  }
}

// Wall-clock accumulator for one category of executor calls.
struct HostTimer {
  double s = 0.0;
  long long n = 0;
};
struct Scope {
  HostTimer& t;
  std::chrono::steady_clock::time_point t0;
  explicit Scope(HostTimer& x) : t(x), t0(std::chrono::steady_clock::now()) {}
  ~Scope() {
    t.s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    t.n++;
  }
};

class HipExec : public Executor {
 public:
  HipExec() {
    HIP_OK(hipStreamCreate(&stream_));
    fixed_ = fixed_scratch_address();
  }
  ~HipExec() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (auto& b : size_of_) (void)hipFree(b.first);  // live and cached blocks
    size_of_.clear();
    free_.clear();
    for (auto& e : events_) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : order_ev_)
      if (e) (void)hipEventDestroy(e);
    if (stream_) (void)hipStreamDestroy(stream_);
  }
  void wait_for(void* s) override {
    hipEvent_t e = order_event(0);
    HIP_OK(hipEventRecord(e, (hipStream_t)s));
    HIP_OK(hipStreamWaitEvent(stream_, e, 0));
  }
  void signal(void* s) override {
    hipEvent_t e = order_event(1);
    HIP_OK(hipEventRecord(e, stream_));
    HIP_OK(hipStreamWaitEvent((hipStream_t)s, e, 0));
  }
  // Device memory is cached: released blocks go to a free list keyed by size
  // and are handed out again for requests they fit (within 1/8 slack), so a
  // sweep does not pay hipMalloc/hipFree for every operator family and task
  // list.  All device work is ordered on the executor's one stream, so a
  // block reused by a later call is only touched after earlier work on it.
  // When hipMalloc fails the cache is returned to the runtime and the
  // allocation retried once.
  void* alloc(size_t bytes) override {
    Scope sc(t_alloc_);
    const size_t s = round_size(bytes);
    auto it = free_.lower_bound(s);
    if (it != free_.end() && it->first <= s + s / 8) {
      void* p = it->second;
      cached_ -= it->first;
      free_.erase(it);
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, s) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      if (hipMalloc(&p, s) != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
      }
    }
    size_of_[p] = s;
    return p;
  }
  void release(void* p) override {
    Scope sc(t_free_);
    if (!p) return;
    auto it = size_of_.find(p);
    if (it == size_of_.end()) throw std::runtime_error("executor: release of an unknown pointer");
    free_.insert({it->second, p});
    cached_ += it->second;
    if (cached_ > kCacheCap) {
      // keep the cache bounded: return the largest blocks to the runtime
      HIP_OK(hipStreamSynchronize(stream_));
      while (cached_ > kCacheCap / 2 && !free_.empty()) {
        auto last = std::prev(free_.end());
        cached_ -= last->first;
        size_of_.erase(last->second);
        (void)hipFree(last->second);
        free_.erase(last);
      }
    }
  }
  // Return every cached block to the runtime.
  void trim() {
    if (free_.empty()) return;
    HIP_OK(hipStreamSynchronize(stream_));
    for (auto& f : free_) {
      size_of_.erase(f.second);
      (void)hipFree(f.second);
    }
    free_.clear();
    cached_ = 0;
  }
  void upload(void* d, const void* s, size_t b) override {
    Scope sc(t_up_);
    if (b) HIP_OK(hipMemcpyAsync(d, s, b, hipMemcpyHostToDevice, stream_));
    HIP_OK(hipStreamSynchronize(stream_));
  }
  void download(void* d, const void* s, size_t b) override {
    Scope sc(t_down_);
    if (b) HIP_OK(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToHost, stream_));
    HIP_OK(hipStreamSynchronize(stream_));
  }
  void zero(void* p, size_t b) override {
    if (!b) return;
    if (capturing_) {
      // the buffers cleared here are hipMalloc'ed, so 16-byte aligned
      if ((uintptr_t)p & 15) throw std::runtime_error("executor: unaligned clear in a captured graph");
      const unsigned grid = (unsigned)std::min<size_t>((b / 16 + 255) / 256 + 1, 65536);
      hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, stream_, (unsigned char*)p, (long long)b);
      HIP_OK(hipGetLastError());
    } else {
      HIP_OK(hipMemsetAsync(p, 0, b, stream_));
    }
  }
  bool graphs() const override { return true; }
  void capture_begin() override {
    dot_buffers();  // allocated outside the recording
    HIP_OK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    capturing_ = true;
  }
  void* capture_end() override {
    capturing_ = false;
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamEndCapture(stream_, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_OK(r);
    return (void*)e;
  }
  void capture_abort() override {
    if (!capturing_) return;
    capturing_ = false;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(stream_, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
  }
  void replay(void* e) override { HIP_OK(hipGraphLaunch((hipGraphExec_t)e, stream_)); }
  void drop_graph(void* e) override {
    if (e) (void)hipGraphExecDestroy((hipGraphExec_t)e);
  }
  long long scratch_generation() const override { return part_gen_; }
  bool timing_on() const override { return timing_; }
  void copy_d2d(void* d, const void* s, size_t b) override {
    if (b) HIP_OK(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, stream_));
  }
  // Kernel choice and work items of a launch (host only).
  // cfg (padded BF16 launches only): 0 the static rule (choose_wave /
  // choose_tile), 1..3 the tiles 64x64, 64x128, 128x64, 4 the wave kernel,
  // 5 the tile 128x128, 6..9 the LDS-pipelined kernel with tiles 64x64,
  // 64x128, 128x64, 128x128, 10..12 the same with two stages and tiles
  // 64x64, 64x128, 128x64 (5..12: BF16 operands only).
  Prepared* configure(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc,
                      std::vector<WorkItem>& items, std::vector<RedItem>& reds, int cfg = 0) {
    auto* P = new Prepared();
    P->da = da;
    P->db = db;
    P->dc = dc;
    const bool f8 = da == DT_FP8 || db == DT_FP8;
    P->mode = (da == DT_F64) ? DT_F64 : (da == DT_F32 ? DT_F32 : DT_BF16);
    if (P->mode == DT_BF16 && (dc == DT_BF16 || dc == DT_F32)) {
      bool ok = true;
      // vector loads: 16-byte aligned BF16 rows, 8-byte aligned FP8 rows
      const uintptr_t ma = da == DT_FP8 ? 7 : 15, mb = db == DT_FP8 ? 7 : 15;
      double wmin = HUGE_VAL, wmax = 0.0;
      for (const RawTerm& T : terms) {
        if (T.flags & (TF_IDENT_A | TF_IDENT_B)) continue;
        const double aw = std::fabs(T.alpha);
        if (!(T.flags & TF_PAD_A) || !(T.flags & TF_PAD_B) || ((uintptr_t)T.A & ma) || ((uintptr_t)T.B & mb) ||
            (T.lda & 7) || (T.ldb & 7) || !(aw >= 1e-30 && aw <= 1e30)) {
          ok = false;
          break;
        }
        wmin = std::min(wmin, aw);
        wmax = std::max(wmax, aw);
      }
      // The scaled-frame accumulation divides the running sum by the weight
      // in flight and multiplies it by weight ratios, in FP32: weights within
      // 1e-30..1e30 and ratios up to 1e30 keep both far inside FP32 range
      // (the FP8 scales of the operands are folded into the weights, which
      // makes them small).
      if (ok && wmax > 0.0 && wmax > 1e30 * wmin) ok = false;
      P->padded = ok && (f8 || !std::getenv("DMRG_NO_PADDED_KERNEL"));
    }
    if (P->mode == DT_F64 && db == DT_F64 && dc == DT_F64) {
      // 16-byte LDS DMA pieces: padded rows, 16-byte aligned, even strides
      bool ok = true;
      for (const RawTerm& T : terms) {
        if (T.flags & (TF_IDENT_A | TF_IDENT_B)) continue;
        if (!(T.flags & TF_PAD_A) || !(T.flags & TF_PAD_B) || ((uintptr_t)T.A & 15) || ((uintptr_t)T.B & 15) ||
            (T.lda & 1) || (T.ldb & 1)) {
          ok = false;
          break;
        }
      }
      P->pad64 = ok;
      if (ok && cfg == 0) {  // forced from the environment (tests, experiments)
        const char* e = std::getenv("DMRG_TILE");
        if (e && std::string(e).rfind("f64pipe", 0) == 0) {
          const std::string t(e + 7);
          cfg = t == "64x64" ? 20 : t == "2s64x64" ? 21 : t == "2s128x64" ? 22 : t == "2s64x128" ? 23 : 0;
          if (!cfg)
            throw std::runtime_error("executor: DMRG_TILE=f64pipeMxN takes 64x64, 2s64x64, 2s128x64 or 2s64x128");
        }
      }
    }
    if (cfg >= 20 && !P->pad64) cfg = 0;
    if (f8 && !P->padded) {
      delete P;
      throw std::runtime_error(
          "executor: FP8 operands need padded, aligned operands and weights within 1e-30..1e30 (ratios up to 1e30)");
    }
    if (f8 && cfg >= 4) cfg = 1;  // FP8 operands: the three smaller register-staged tiles only
    if (P->padded && cfg == 0 && !f8) {  // forced from the environment (tests, experiments)
      const char* e = std::getenv("DMRG_TILE");
      if (e && std::string(e).rfind("pipe", 0) == 0) {
        const std::string t(e + 4);
        cfg = t == "64x64" ? 6 : t == "64x128" ? 7 : t == "128x64" ? 8 : t == "128x128" ? 9 : t == "2s64x64" ? 10
            : t == "2s64x128" ? 11 : t == "2s128x64" ? 12 : 0;
        if (!cfg)
          throw std::runtime_error(
              "executor: DMRG_TILE=pipeMxN takes 64x64, 64x128, 128x64, 128x128 (or 2sMxN: two stages)");
      }
    }
    P->kt = P->padded ? 32 : (P->mode == DT_BF16 ? choose_kt_bf16(jobs, terms) : 16);
    if (cfg >= 20) {  // FP64 pipelined tiles: 64x64 (3 stages), 64x64, 128x64, 64x128 (2 stages)
      static const int t64[4][3] = {{64, 64, 3}, {64, 64, 2}, {128, 64, 2}, {64, 128, 2}};
      P->pipe = true;
      P->bm = t64[cfg - 20][0];
      P->bn = t64[cfg - 20][1];
      P->stages = t64[cfg - 20][2];
    } else if (P->padded && cfg > 0) {
      static const int tiles[12][2] = {{64, 64}, {64, 128}, {128, 64}, {32, 32}, {128, 128}, {64, 64},
                                       {64, 128}, {128, 64}, {128, 128}, {64, 64}, {64, 128}, {128, 64}};
      P->wave = cfg == 4;
      P->pipe = cfg >= 6;
      P->stages = cfg >= 10 ? 2 : 0;
      P->bm = tiles[cfg - 1][0];
      P->bn = tiles[cfg - 1][1];
    } else if (P->padded) {
      P->wave = !f8 && choose_wave(jobs, terms, 32);
      if (P->wave) P->bm = P->bn = 32;
      else choose_tile(jobs, terms, P->bm, P->bn);
    } else if (P->mode == DT_F64 && dc == DT_F64 && !std::getenv("DMRG_NO_F64_WAVE")) {
      P->wave = choose_wave(jobs, terms, 16);
      if (P->wave) {
        P->bm = P->bn = 32;
      } else if (P->pad64 && !(std::getenv("DMRG_PIPE") && std::atoi(std::getenv("DMRG_PIPE")) == 0)) {
        // the two-stage 64 x 64 pipelined tile: what the tuner chose for every
        // FP64 H*psi launch class of the CAS(32,32) and CAS(82,82) workloads
        P->pipe = true;
        P->bm = P->bn = 64;
        P->stages = 2;
      }
    }
    try {
      if (!f8) pick(P->mode, da, db, dc, P->kt);  // validate
      if (terms.size() > (size_t)0x7fffffff) throw std::runtime_error("executor: too many products in one launch");
      // the pipelined kernels keep several slabs in flight per work-group and
      // pay for the partial tiles of split items: longer product segments
      // (at least 400 slabs) measured best for them at CAS(82,82) (BF16
      // H*psi 304 -> 294 ms against the 64-slab floor; 160 slabs 306 ms,
      // 800 slabs 300 ms, 1600 slabs 308 ms)
      plan_items(jobs, terms, P->kt, P->bm, P->bn, P->wave ? 65536.0 : 16384.0, P->pipe ? 400.0 : 64.0, items, reds,
                 P->nslots);
      P->nitems = (long long)items.size();
      P->nreds = (long long)reds.size();
      if (P->nreds) pick_reduce(P->mode, dc);
    } catch (...) {
      delete P;
      throw;
    }
    return P;
  }
  size_t part_need(const Prepared* P) const {
    return (size_t)P->nslots * P->bm * P->bn * (P->mode == DT_F64 ? 8 : 4);
  }
  void* prepare(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc) override {
    return prepare_cfg(jobs, terms, da, db, dc, 0);
  }
  // Measured choice of the kernel configuration of a padded BF16 launch:
  // every candidate (four LDS tiles, the wave kernel; the three smaller
  // tiles for FP8 operands) is prepared and timed
  // on the launch itself (one warm-up and one timed run; the launch's outputs
  // are scratch that the caller clears or overwrites before real use), and
  // the fastest kept.  Choices are cached per launch class -- operand and
  // output types and the log2 buckets of the padded MFMA work, the job count
  // and the mean m, n and K -- so launches of one shape are timed once per
  // process; DMRG_TUNE_FILE names a file that keeps the cache across
  // processes, DMRG_TUNE=0 falls back to the static rule.
  void* prepare_tuned(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db,
                      int dc) override {
    const bool f8 = da == DT_FP8 || db == DT_FP8;
    const bool lowp = (da == DT_BF16 || da == DT_FP8) && (db == DT_BF16 || db == DT_FP8) &&
                      (dc == DT_BF16 || dc == DT_F32);
    const bool f64 = da == DT_F64 && db == DT_F64 && dc == DT_F64;
    const bool no_pipe = std::getenv("DMRG_PIPE") && std::atoi(std::getenv("DMRG_PIPE")) == 0;
    // FP64 launches take the static rule (which picks the pipelined tile the
    // tuner chose for every FP64 class measured) unless DMRG_TUNE_F64 is set:
    // timing five FP64 candidates costs seconds per block of a sweep
    if ((!lowp && !f64) || jobs.empty() || (std::getenv("DMRG_TUNE") && std::atoi(std::getenv("DMRG_TUNE")) == 0) ||
        std::getenv("DMRG_TILE") || std::getenv("DMRG_WAVE") || std::getenv("DMRG_NO_PADDED_KERNEL") ||
        (f64 && (no_pipe || std::getenv("DMRG_NO_F64_WAVE") || !std::getenv("DMRG_TUNE_F64"))))
      return prepare(jobs, terms, da, db, dc);
    // candidates: BF16 / FP8 padded launches 1..12 (FP8 1..3); FP64 launches
    // the static rule (gemm_kernel or gemm_f64_wave) and the pipelined tiles
    std::vector<int> cands;
    if (f64) cands = {0, 20, 21, 22, 23};
    else
      for (int c = 1; c <= (f8 ? 3 : no_pipe ? 5 : 12); ++c) cands.push_back(c);
    const std::string key = tune_key(jobs, terms, da, db, dc);
    std::lock_guard<std::mutex> lock(tune_mu());
    load_tune_file();
    auto it = tune_map().find(key);
    if (it != tune_map().end()) return prepare_cfg(jobs, terms, da, db, dc, it->second);
    int best = 0;
    float best_ms = 0.0f;
    void* keep = nullptr;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    for (int cfg : cands) {
      void* h = prepare_cfg(jobs, terms, da, db, dc, cfg);
      if (!(f64 ? ((Prepared*)h)->pad64 : ((Prepared*)h)->padded)) {  // no choice to make
        HIP_OK(hipEventDestroy(e0));
        HIP_OK(hipEventDestroy(e1));
        if (keep) drop(keep);
        return h;
      }
      const bool was = timing_;
      timing_ = false;
      run(h);  // warm-up
      HIP_OK(hipEventRecord(e0, stream_));
      run(h);
      HIP_OK(hipEventRecord(e1, stream_));
      timing_ = was;
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      if (!keep || ms < best_ms) {
        if (keep) drop(keep);
        keep = h;
        best = cfg;
        best_ms = ms;
      } else {
        drop(h);
      }
    }
    HIP_OK(hipEventDestroy(e0));
    HIP_OK(hipEventDestroy(e1));
    tune_map()[key] = best;
    ++tuned_count();
    save_tune_file(key, best);
    return keep;
  }
  std::string tuner_report() const override {
    std::lock_guard<std::mutex> lock(tune_mu());
    static const std::pair<int, const char*> names[] = {
        {1, "64x64"}, {2, "64x128"}, {3, "128x64"}, {4, "wave32x32"}, {5, "128x128"}, {6, "pipe64x64"},
        {7, "pipe64x128"}, {8, "pipe128x64"}, {9, "pipe128x128"}, {10, "pipe2s64x64"}, {11, "pipe2s64x128"},
        {12, "pipe2s128x64"}, {0, "f64_static"}, {20, "f64pipe64x64"}, {21, "f64pipe2s64x64"},
        {22, "f64pipe2s128x64"}, {23, "f64pipe2s64x128"}};
    std::map<int, int> cnt;
    for (auto& kv : tune_map()) cnt[kv.second]++;
    std::string b = "{\"classes\": " + std::to_string(tune_map().size()) +
                    ", \"timed_here\": " + std::to_string(tuned_count());
    for (auto& nm : names) b += std::string(", \"") + nm.second + "\": " + std::to_string(cnt[nm.first]);
    b += "}";
    return b;
  }
  void* prepare_cfg(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc,
                    int cfg) {
    Scope sc(t_prep_);
    std::vector<WorkItem> items;
    std::vector<RedItem> reds;
    Prepared* P = configure(jobs, terms, da, db, dc, items, reds, cfg);
    if (P->nitems) {
      P->d_jobs = (RawJob*)alloc(jobs.size() * sizeof(RawJob));
      P->d_terms = (RawTerm*)alloc(std::max<size_t>(terms.size(), 1) * sizeof(RawTerm));
      P->d_items = (WorkItem*)alloc(items.size() * sizeof(WorkItem));
      upload(P->d_jobs, jobs.data(), jobs.size() * sizeof(RawJob));
      if (!terms.empty()) upload(P->d_terms, terms.data(), terms.size() * sizeof(RawTerm));
      upload(P->d_items, items.data(), items.size() * sizeof(WorkItem));
      if (P->nreds) {
        P->d_reds = (RedItem*)alloc(reds.size() * sizeof(RedItem));
        upload(P->d_reds, reds.data(), reds.size() * sizeof(RedItem));
      }
    }
    const size_t need = part_need(P);
    if (need > part_bytes_) {
      sync();
      if (part_) release(part_);
      part_ = nullptr;
      part_bytes_ = 0;
      part_ = alloc(need);
      part_bytes_ = need;
      ++part_gen_;  // graphs recorded against the old buffer are stale
    }
    return P;
  }
  void run(void* h) override {
    auto* P = (Prepared*)h;
    if (!P->nitems) return;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing_) {
      HIP_OK(hipEventCreate(&e0));
      HIP_OK(hipEventCreate(&e1));
      HIP_OK(hipEventRecord(e0, stream_));
    }
    // One work-group per item; the hardware dispatcher balances the load.  A
    // dispatch counts its work-items in 32 bits, so a launch of more than
    // kMaxGroups items is issued as several launches over consecutive items.
    const long long maxg = kMaxGroups;
    if (P->wave) {
      // four items per work-group, one per wave
      WaveFn k = pick_wave(P->mode, P->dc);
      for (long long t0 = 0; t0 < P->nitems; t0 += 4 * maxg) {
        const long long nt = std::min(4 * maxg, P->nitems - t0);
        hipLaunchKernelGGL(k, dim3((unsigned)((nt + 3) / 4)), dim3(256), 0, stream_, P->d_jobs, P->d_terms,
                           P->d_items + t0, P->part ? P->part : part_, nt);
      }
    } else {
      KernelFn k = P->pipe     ? (P->mode == DT_F64 ? pick_pipe_f64(P->bm, P->bn, P->stages)
                                                    : pick_pipe(P->dc, P->bm, P->bn, P->stages))
                   : P->padded ? pick_padded(P->dc, P->bm, P->bn, P->da == DT_FP8, P->db == DT_FP8)
                               : pick(P->mode, P->da, P->db, P->dc, P->kt);
      for (long long t0 = 0; t0 < P->nitems; t0 += maxg) {
        const long long nt = std::min(maxg, P->nitems - t0);
        hipLaunchKernelGGL(k, dim3((unsigned)nt), dim3(256), 0, stream_, P->d_jobs, P->d_terms, P->d_items + t0,
                           P->part ? P->part : part_);
      }
    }
    HIP_OK(hipGetLastError());
    if (P->nreds) {
      ReduceFn r = pick_reduce(P->mode, P->dc);
      for (long long t0 = 0; t0 < P->nreds; t0 += maxg) {
        const long long nt = std::min(maxg, P->nreds - t0);
        hipLaunchKernelGGL(r, dim3((unsigned)nt), dim3(256), 0, stream_, P->d_jobs, P->d_reds + t0,
                           P->part ? P->part : part_, P->bm, P->bn);
      }
      HIP_OK(hipGetLastError());
    }
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
    release(P->d_items);
    release(P->d_reds);
    delete P;
  }
  void orb_scalars(const double* B, int naux, int n, int nc, int na, const double* gam, double* bact,
                   double* scal) override {
    if (naux <= 0) return;
    hipLaunchKernelGGL(orb_scalars_kernel, dim3(naux), dim3(256), 0, stream_, B, n, nc, na, gam, bact, scal);
    HIP_OK(hipGetLastError());
  }
  void orb_assemble(const double* B, int naux, int n, int nc, int na, const double* gam, const double* scal,
                    const double* bact, const double* Y, const double* Z, double* G, double* e2) override {
    if (naux <= 0) return;
    hipLaunchKernelGGL(orb_assemble_kernel, dim3(naux), dim3(256), 0, stream_, B, n, nc, na, gam, scal, bact, Y, Z,
                       G, e2);
    HIP_OK(hipGetLastError());
  }
  void* fixed_scratch(size_t* bytes) override {
    *bytes = kFixedScratchBytes;
    return fixed_;
  }
  void* plan_fixed(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db, int dc,
                   size_t* list_bytes, size_t* part_bytes) override {
    Scope sc(t_prep_);
    std::vector<WorkItem> items;
    std::vector<RedItem> reds;
    Prepared* P = configure(jobs, terms, da, db, dc, items, reds);
    P->h_jobs = jobs;
    P->h_terms = terms;
    P->h_items.swap(items);
    P->h_reds.swap(reds);
    *list_bytes = fixed_layout(P, nullptr);
    *part_bytes = part_need(P);
    return P;
  }
  void place_fixed(void* h, void* dev, void* part) override {
    auto* P = (Prepared*)h;
    fixed_layout(P, (char*)dev);
    P->part = part;
    if (!P->nitems) return;
    upload(P->d_jobs, P->h_jobs.data(), P->h_jobs.size() * sizeof(RawJob));
    if (!P->h_terms.empty()) upload(P->d_terms, P->h_terms.data(), P->h_terms.size() * sizeof(RawTerm));
    upload(P->d_items, P->h_items.data(), P->h_items.size() * sizeof(WorkItem));
    if (P->nreds) upload(P->d_reds, P->h_reds.data(), P->h_reds.size() * sizeof(RedItem));
  }
  void drop_fixed(void* h) override { delete (Prepared*)h; }
  void sync() override {
    Scope sc(t_sync_);
    HIP_OK(hipStreamSynchronize(stream_));
  }
  std::string host_profile() const override {
    char b[512];
    std::snprintf(b, sizeof b,
                  "alloc %.2fs/%lld free %.2fs/%lld upload %.2fs/%lld download %.2fs/%lld prepare %.2fs/%lld "
                  "sync %.2fs/%lld",
                  t_alloc_.s, t_alloc_.n, t_free_.s, t_free_.n, t_up_.s, t_up_.n, t_down_.s, t_down_.n, t_prep_.s,
                  t_prep_.n, t_sync_.s, t_sync_.n);
    return b;
  }
  void pack(void* dst, int dd, const double* src, const int* idx, size_t n) override {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    if (dd == DT_F64) hipLaunchKernelGGL((pack_kernel<DT_F64>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, (long long)n);
    else if (dd == DT_F32) hipLaunchKernelGGL((pack_kernel<DT_F32>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, (long long)n);
    else if (dd == DT_BF16) hipLaunchKernelGGL((pack_kernel<DT_BF16>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, (long long)n);
    else throw std::runtime_error("executor: unsupported pack dtype");
    HIP_OK(hipGetLastError());
  }
  void gather(double* dst, const void* src, int ds, const int* idx, size_t n, double a, const double* x,
              const double* mul) override {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    const long long nn = (long long)n;
    if (ds == DT_F64) hipLaunchKernelGGL((gather_kernel<DT_F64>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, nn, a, x, mul);
    else if (ds == DT_F32) hipLaunchKernelGGL((gather_kernel<DT_F32>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, nn, a, x, mul);
    else if (ds == DT_BF16) hipLaunchKernelGGL((gather_kernel<DT_BF16>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, nn, a, x, mul);
    else throw std::runtime_error("executor: unsupported gather dtype");
    HIP_OK(hipGetLastError());
  }
  void fp8_scales(const double* src, int64_t nseg, int64_t seg, double* d_scale) override {
    if (nseg <= 0) return;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(64, (seg + 255) / 256));
    double* part = (double*)alloc((size_t)nseg * nb * sizeof(double));
    for (int64_t y0 = 0; y0 < nseg; y0 += 65535) {
      const int ny = (int)std::min<int64_t>(65535, nseg - y0);
      hipLaunchKernelGGL(absmax_partial, dim3(nb, ny), dim3(256), 0, stream_, src + y0 * seg, (long long)seg,
                         (long long)seg, part + y0 * nb);
    }
    // Operator segments of at most 1e-13 (round-off of the FP64 block
    // build; operators are in Hartree units) are flushed to zero: far below
    // the E4M3 resolution of any product they enter, and a scale that small
    // would push the folded product weights out of the kernel's range.
    hipLaunchKernelGGL(pow2_scale, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, stream_, part, nb, (int)nseg,
                       d_scale, 1e-13);
    HIP_OK(hipGetLastError());
    sync();
    release(part);
  }
  void to_fp8(void* dst, const double* src, int64_t n, int64_t seg, const double* d_scale) override {
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(to_fp8_kernel, dim3(grid), dim3(256), 0, stream_, (unsigned char*)dst, src, (long long)n,
                       (long long)seg, d_scale);
    HIP_OK(hipGetLastError());
  }
  void pack_fp8(void* dst, const double* src, const int* idx, size_t n, double* d_scale, const double* src_all,
                size_t n_all) override {
    if (!n) return;
    // scale of the whole source vector (one segment), then the packed copy
    const int nb = (int)std::max<size_t>(1, std::min<size_t>(1024, (n_all + 255) / 256));
    if (!fp8_part_) fp8_part_ = (double*)alloc(1024 * sizeof(double));
    hipLaunchKernelGGL(absmax_partial, dim3(nb, 1), dim3(256), 0, stream_, src_all, (long long)n_all, (long long)n_all,
                       fp8_part_);
    hipLaunchKernelGGL(pow2_scale, dim3(1), dim3(1), 0, stream_, fp8_part_, nb, 1, d_scale, 0.0);
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(pack_fp8_kernel, dim3(grid), dim3(256), 0, stream_, (unsigned char*)dst, src, idx, (long long)n,
                       d_scale);
    HIP_OK(hipGetLastError());
  }
  void shifted_copy_at(void* dst, int dd, const double* src, const int* idx, size_t n, double a) override {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    const long long nn = (long long)n;
    if (dd == DT_F32) hipLaunchKernelGGL((shifted_copy_kernel<DT_F32>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, nn, a);
    else if (dd == DT_BF16) hipLaunchKernelGGL((shifted_copy_kernel<DT_BF16>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, nn, a);
    else if (dd == DT_F64) hipLaunchKernelGGL((shifted_copy_kernel<DT_F64>), dim3(grid), dim3(256), 0, stream_, dst, src, idx, nn, a);
    else throw std::runtime_error("executor: unsupported shifted copy dtype");
    HIP_OK(hipGetLastError());
  }
  void convert(void* dst, int dd, const void* src, int ds, size_t n) override {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
#define C_(S, D) \
  if (ds == S && dd == D) { hipLaunchKernelGGL((convert_kernel<S, D>), dim3(grid), dim3(256), 0, stream_, dst, src, (long long)n); HIP_OK(hipGetLastError()); return; }
    C_(DT_F64, DT_F32) C_(DT_F64, DT_BF16) C_(DT_F32, DT_F64) C_(DT_BF16, DT_F64) C_(DT_F32, DT_BF16) C_(DT_BF16, DT_F32)
#undef C_
    throw std::runtime_error("executor: unsupported conversion");
  }
  void dot_buffers() {
    if (!dot_part_) {
      dot_part_ = (double*)alloc(sizeof(double) * kDotBlocks * 64);
      dot_out_ = (double*)alloc(sizeof(double) * 64);
    }
  }
  void multidot_dev(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out_dev) override {
    if (m <= 0) return;
    if (m > 64) throw std::runtime_error("multidot: m > 64");
    if (!dot_part_ && capturing_) throw std::runtime_error("multidot: first use inside a graph recording");
    dot_buffers();
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 255) / 256));
    hipLaunchKernelGGL(multidot_partial, dim3(nb), dim3(256), 0, stream_, V, (long long)ldv, m, w, (long long)n,
                       dot_part_);
    hipLaunchKernelGGL(multidot_final, dim3(1), dim3(256), 0, stream_, dot_part_, nb, m, out_dev);
    HIP_OK(hipGetLastError());
  }
  void multidot(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out_host) override {
    if (m <= 0) return;
    dot_buffers();
    multidot_dev(V, ldv, m, w, n, dot_out_);
    download(out_host, dot_out_, sizeof(double) * m);
  }
  void combine(double* y, const double* V, int64_t ldv, int m, const double* c_host, int64_t n, double beta) override {
    if (m > 64) throw std::runtime_error("combine: m > 64");
    Coef64 c{};
    for (int i = 0; i < m; ++i) c.c[i] = c_host[i];
    hipLaunchKernelGGL(combine_kernel, dim3(grid1(n)), dim3(256), 0, stream_, y, V, (long long)ldv, m, c,
                       (const double*)nullptr, 1.0, (long long)n, beta);
    HIP_OK(hipGetLastError());
  }
  void combine_dev(double* y, const double* V, int64_t ldv, int m, const double* c_dev, double sgn, int64_t n,
                   double beta) override {
    if (m > 64) throw std::runtime_error("combine: m > 64");
    hipLaunchKernelGGL(combine_kernel, dim3(grid1(n)), dim3(256), 0, stream_, y, V, (long long)ldv, m, Coef64{}, c_dev,
                       sgn, (long long)n, beta);
    HIP_OK(hipGetLastError());
  }
  void axpby(double* z, double a, const double* x, double b, const double* y, int64_t n) override {
    axpby_dev(z, a, nullptr, x, b, nullptr, y, n);
  }
  void axpby_dev(double* z, double a, const double* a_dev, const double* x, double b, const double* b_dev,
                 const double* y, int64_t n) override {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid1(n)), dim3(256), 0, stream_, z, a, a_dev, x, b, b_dev, y, (long long)n);
    HIP_OK(hipGetLastError());
  }
  void precond(double* t, const double* r, const double* d, double theta, double eps, int64_t n) override {
    hipLaunchKernelGGL(precond_kernel, dim3(grid1(n)), dim3(256), 0, stream_, t, r, d, theta, (const double*)nullptr,
                       eps, (long long)n);
    HIP_OK(hipGetLastError());
  }
  void precond_dev(double* t, const double* r, const double* d, const double* theta_dev, double eps,
                   int64_t n) override {
    hipLaunchKernelGGL(precond_kernel, dim3(grid1(n)), dim3(256), 0, stream_, t, r, d, 0.0, theta_dev, eps,
                       (long long)n);
    HIP_OK(hipGetLastError());
  }
  int sym_eig(double* A, double* V, const std::vector<int64_t>& offs, const std::vector<int>& sizes, int max_sweeps,
              double tol, double* worst) override {
    if (worst) *worst = 0.0;
    if (offs.empty()) return 0;
    auto thr2 = [&](int i) {
      const double t = std::max(tol, 4.0 * sizes[i] * std::numeric_limits<double>::epsilon());
      return t * t;
    };
    const int nall = (int)offs.size();
    // per-matrix descriptors of a list of matrices (bases for the work indices)
    auto describe = [&](const std::vector<int>& ids, std::vector<JacMat>& M, long long& npair, long long& nblk,
                        long long& nvrow, int& maxnp) {
      M.clear();
      npair = nblk = nvrow = 0;
      maxnp = 0;
      for (int i : ids) {
        JacMat m{};
        m.off = offs[i];
        m.n = sizes[i];
        m.np = m.n + (m.n & 1);
        m.pair_base = (int)npair;
        m.blk_base = nblk;
        m.vrow_base = nvrow;
        const long long h = m.np / 2;
        npair += h;
        nblk += h * h;
        nvrow += (long long)m.n * h;
        maxnp = std::max(maxnp, m.np);
        M.push_back(m);
      }
    };
    std::vector<int> all(nall);
    for (int i = 0; i < nall; ++i) all[i] = i;
    std::vector<JacMat> M;
    long long npair, nblk, nvrow;
    int maxnp;
    describe(all, M, npair, nblk, nvrow, maxnp);
    JacMat* dM = (JacMat*)alloc(M.size() * sizeof(JacMat));
    double* dnorm = (double*)alloc(2 * (size_t)nall * sizeof(double));
    double* dcs = (double*)alloc((size_t)npair * sizeof(double));
    double* dsn = (double*)alloc((size_t)npair * sizeof(double));
    int* dpp = (int*)alloc((size_t)npair * sizeof(int));
    int* dqq = (int*)alloc((size_t)npair * sizeof(int));
    upload(dM, M.data(), M.size() * sizeof(JacMat));
    hipLaunchKernelGGL(jac_identity, dim3(nall), dim3(256), 0, stream_, V, dM);
    hipLaunchKernelGGL(jac_norms, dim3(nall), dim3(256), 0, stream_, A, dM, dnorm);
    HIP_OK(hipGetLastError());
    std::vector<double> nrm(2 * (size_t)nall);
    download(nrm.data(), dnorm, nrm.size() * sizeof(double));
    std::vector<double> fro2(nall);
    std::vector<int> active;
    for (int i = 0; i < nall; ++i) {
      fro2[i] = nrm[2 * i + 1];
      if (sizes[i] > 1 && nrm[2 * i] > thr2(i) * fro2[i]) active.push_back(i);
    }
    for (int sweep = 0; sweep < max_sweeps && !active.empty(); ++sweep) {
      describe(active, M, npair, nblk, nvrow, maxnp);
      const int nm = (int)M.size();
      upload(dM, M.data(), M.size() * sizeof(JacMat));
      const unsigned ga = (unsigned)((npair + 255) / 256);
      const unsigned gb = (unsigned)((nblk + nvrow + 255) / 256);
      for (int r = 0; r < maxnp - 1; ++r) {
        hipLaunchKernelGGL(jac_angles, dim3(ga), dim3(256), 0, stream_, A, dM, nm, (int)npair, r, dcs, dsn, dpp, dqq);
        hipLaunchKernelGGL(jac_apply, dim3(gb), dim3(256), 0, stream_, A, V, dM, nm, nblk, nvrow, dcs, dsn, dpp,
                           dqq);
      }
      HIP_OK(hipGetLastError());
      hipLaunchKernelGGL(jac_norms, dim3(nm), dim3(256), 0, stream_, A, dM, dnorm);
      HIP_OK(hipGetLastError());
      download(nrm.data(), dnorm, 2 * (size_t)nm * sizeof(double));
      std::vector<int> still;
      std::vector<double> ratio;
      for (int j = 0; j < nm; ++j)
        if (nrm[2 * j] > thr2(active[j]) * fro2[active[j]]) {
          still.push_back(active[j]);
          ratio.push_back(std::sqrt(nrm[2 * j] / std::max(fro2[active[j]], 1e-300)));
        }
      active.swap(still);
      if (worst) *worst = ratio.empty() ? 0.0 : *std::max_element(ratio.begin(), ratio.end());
    }
    release(dM);
    release(dnorm);
    release(dcs);
    release(dsn);
    release(dpp);
    release(dqq);
    return (int)active.size();
  }
  hipStream_t stream() const { return stream_; }

 private:
  // ---- tile autotuner state (prepare_tuned), shared by every executor of
  // the process so that contexts with the same launches make the same choice
  static std::mutex& tune_mu() {
    static std::mutex m;
    return m;
  }
  static std::map<std::string, int>& tune_map() {  // launch class -> configuration
    static std::map<std::string, int> m;
    return m;
  }
  static int& tuned_count() {  // classes timed in this process
    static int n = 0;
    return n;
  }
  static std::string tune_key(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db,
                              int dc) {
    double work = 0.0, sm = 0.0, sn = 0.0, sk = 0.0, nk = 0.0;
    for (const RawJob& J : jobs) {
      sm += J.m;
      sn += J.n;
      double kp = 0.0;
      for (int64_t t = J.tbeg; t < J.tend; ++t)
        if (!(terms[t].flags & (TF_IDENT_A | TF_IDENT_B))) {
          kp += (double)((terms[t].k + 31) / 32 * 32);
          sk += terms[t].k;
          nk += 1.0;
        }
      work += (double)((J.m + 63) / 64) * (double)((J.n + 63) / 64) * 4096.0 * kp;
    }
    const double nj = (double)jobs.size();
    auto b2 = [](double x) { return (int)std::lround(std::log2(std::max(x, 1.0))); };
    char buf[128];
    std::snprintf(buf, sizeof buf, "a%d_b%d_c%d_w%d_j%d_m%d_n%d_k%d", da, db, dc, b2(work), b2(nj), b2(sm / nj),
                  b2(sn / nj),
                  b2(nk > 0 ? sk / nk : 1.0));
    return buf;
  }
  static void load_tune_file() {
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char* f = std::getenv("DMRG_TUNE_FILE");
    if (!f) return;
    FILE* fp = std::fopen(f, "r");
    if (!fp) return;
    char key[128];
    int cfg = 0;
    while (std::fscanf(fp, "%127s %d", key, &cfg) == 2)
      if (cfg >= 0 && cfg <= 23) tune_map()[key] = cfg;
    std::fclose(fp);
  }
  static void save_tune_file(const std::string& key, int cfg) {
    const char* f = std::getenv("DMRG_TUNE_FILE");
    if (!f) return;
    FILE* fp = std::fopen(f, "a");
    if (!fp) return;
    std::fprintf(fp, "%s %d\n", key.c_str(), cfg);
    std::fclose(fp);
  }
  // Offsets of a fixed-scratch launch's task lists from base (256-byte
  // aligned pieces); sets the device pointers if base is given.  Returns the
  // bytes they span.
  static size_t fixed_layout(Prepared* P, char* base) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t off = 0;
    const size_t oj = off;
    off = al(off + P->h_jobs.size() * sizeof(RawJob));
    const size_t ot = off;
    off = al(off + std::max<size_t>(P->h_terms.size(), 1) * sizeof(RawTerm));
    const size_t oi = off;
    off = al(off + P->h_items.size() * sizeof(WorkItem));
    const size_t orr = off;
    off = al(off + P->h_reds.size() * sizeof(RedItem));
    if (base) {
      P->d_jobs = (RawJob*)(base + oj);
      P->d_terms = (RawTerm*)(base + ot);
      P->d_items = (WorkItem*)(base + oi);
      P->d_reds = P->h_reds.empty() ? nullptr : (RedItem*)(base + orr);
    }
    return off;
  }
  void* fixed_ = nullptr;  // this device's fixed scratch (fixed_scratch_address)
  static unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }
  static size_t round_size(size_t b) {
    if (b == 0) b = 1;
    const size_t g = b <= ((size_t)1 << 20) ? 512 : ((size_t)2 << 20);
    return (b + g - 1) / g * g;
  }
  std::multimap<size_t, void*> free_;          // cached blocks by size
  std::unordered_map<void*, size_t> size_of_;  // every block obtained from hipMalloc
  size_t cached_ = 0;
  static constexpr size_t kCacheCap = (size_t)24 << 30;
  HostTimer t_alloc_, t_free_, t_up_, t_down_, t_prep_, t_sync_;
  void* part_ = nullptr;  // partial tiles of split items, shared by all launches
  size_t part_bytes_ = 0;
  double* dot_part_ = nullptr;
  double* fp8_part_ = nullptr;  // partial maxima of pack_fp8
  double* dot_out_ = nullptr;
  hipStream_t stream_ = nullptr;
  bool timing_ = false;
  hipEvent_t order_ev_[2] = {nullptr, nullptr};  // wait_for / signal
  hipEvent_t order_event(int i) {
    if (!order_ev_[i]) HIP_OK(hipEventCreateWithFlags(&order_ev_[i], hipEventDisableTiming));
    return order_ev_[i];
  }
  bool capturing_ = false;  // between capture_begin and capture_end
  long long part_gen_ = 0;  // bumped when part_ is reallocated
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events_;
};

}  // namespace

Executor* make_hip_executor() { return new HipExec(); }

}  // namespace dmrg
