// Device-side work description shared by the planner and the HIP executor.
//
// All block-sparse contractions on the hot path (renormalisation of the
// operator blocks, the two stages of H*psi, and linear combinations of
// operators) are expressed as one primitive: a list of output matrices
// ("jobs"), each accumulating a list of scaled products
//     C  (+)=  sum_t alpha_t * op(A_t) @ op(B_t)
// where op() is identity or transpose and either factor may be the identity
// matrix.  Every output region is owned by exactly one job, so the executor
// needs no atomics and sums in a fixed order (bitwise reproducible).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <stdexcept>
#include <vector>

namespace dmrg {

enum DType : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_FP8 = 3 };
inline size_t dtype_size(int dt) { return dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : dt == DT_BF16 ? 2 : 1; }

// TF_PAD_A / TF_PAD_B: the operand's rows are padded to a multiple of 8
// elements (readable up to the padded length) and start 16-byte aligned.
enum TermFlags : int { TF_TRANS_A = 1, TF_TRANS_B = 2, TF_IDENT_A = 4, TF_IDENT_B = 8, TF_PAD_A = 16, TF_PAD_B = 32 };

// Pointers are element offsets into named buffers, resolved per precision.
struct BufRef {
  int buf = -1;
  int64_t off = 0;
};

struct GemmTerm {
  BufRef A, B;
  int64_t lda = 0, ldb = 0;
  int k = 0, flags = 0;
  double alpha = 1.0;
};

struct GemmJob {
  BufRef C;
  int m = 0, n = 0;
  int64_t ldc = 0;
  int accumulate = 0;
  int64_t tbeg = 0, tend = 0;
};

struct GemmBatch {
  std::vector<GemmJob> jobs;
  std::vector<GemmTerm> terms;
  double flops = 0.0;  // algorithmic 2mnk over non-identity products
  void clear() {
    jobs.clear();
    terms.clear();
    flops = 0.0;
  }
};

// Resolved (raw pointer) forms uploaded to the device.
struct RawTerm {
  const void* A;
  const void* B;
  int64_t lda, ldb;
  int k, flags;
  double alpha;
};
struct RawJob {
  void* C;
  int m, n;
  int64_t ldc;
  int accumulate, pad;
  int64_t tbeg, tend;
};

class Executor {
 public:
  virtual ~Executor() {}
  virtual void* alloc(size_t bytes) = 0;
  virtual void release(void* p) = 0;
  virtual void upload(void* dst, const void* src, size_t bytes) = 0;
  virtual void download(void* dst, const void* src, size_t bytes) = 0;
  virtual void zero(void* p, size_t bytes) = 0;
  virtual void copy_d2d(void* dst, const void* src, size_t bytes) = 0;
  // Prepare a batch whose A/B operands have dtype tin and whose outputs have
  // dtype tout (both F64 for the exact path).  Returns an opaque handle.
  virtual void* prepare(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int tin_a,
                        int tin_b, int tout) = 0;
  // Like prepare(), choosing the kernel configuration of the launch by timing
  // the candidates on it (the outputs it writes while doing so are scratch);
  // executors without a tuner prepare with their static rule.
  virtual void* prepare_tuned(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int tin_a,
                              int tin_b, int tout) {
    return prepare(jobs, terms, tin_a, tin_b, tout);
  }
  // The tuner's choices so far (JSON object text; empty if there is no tuner).
  virtual std::string tuner_report() const { return std::string(); }
  virtual void run(void* handle) = 0;
  virtual void drop(void* handle) = 0;
  virtual void sync() = 0;
  // ---- FP64 vector primitives for the Davidson iteration (device arrays)
  // out_host[i] = <V_i, w>, V_i = V + i*ldv, i < m (m <= 64); fixed summation order
  virtual void multidot(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out_host) = 0;
  // y = beta*y + sum_i c_host[i] * V_i   (m <= 64)
  virtual void combine(double* y, const double* V, int64_t ldv, int m, const double* c_host, int64_t n,
                       double beta) = 0;
  // z = a*x + b*y
  virtual void axpby(double* z, double a, const double* x, double b, const double* y, int64_t n) = 0;
  // t_i = r_i / (theta - d_i), with |theta - d_i| floored at eps
  virtual void precond(double* t, const double* r, const double* d, double theta, double eps, int64_t n) = 0;
  // ---- the same primitives with scalars read from device memory, so that a
  // Davidson iteration can be recorded as a graph and replayed with new
  // scalars.  They launch the kernels of the host-scalar forms above (same
  // arithmetic, same summation order, so the same results bit for bit).
  // out_dev[i] = <V_i, w>, i < m (m <= 64)
  virtual void multidot_dev(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* out_dev) {
    (void)V; (void)ldv; (void)m; (void)w; (void)n; (void)out_dev;
    throw std::runtime_error("executor: no device-scalar vector primitives");
  }
  // y = beta*y + sum_i (sgn * c_dev[i]) * V_i   (m <= 64)
  virtual void combine_dev(double* y, const double* V, int64_t ldv, int m, const double* c_dev, double sgn, int64_t n,
                           double beta) {
    (void)y; (void)V; (void)ldv; (void)m; (void)c_dev; (void)sgn; (void)n; (void)beta;
    throw std::runtime_error("executor: no device-scalar vector primitives");
  }
  // z = a'*x + b'*y with a' = a * a_dev[0] (a if a_dev is null), b' likewise
  virtual void axpby_dev(double* z, double a, const double* a_dev, const double* x, double b, const double* b_dev,
                         const double* y, int64_t n) {
    (void)z; (void)a; (void)a_dev; (void)x; (void)b; (void)b_dev; (void)y; (void)n;
    throw std::runtime_error("executor: no device-scalar vector primitives");
  }
  // precond with theta = theta_dev[0]
  virtual void precond_dev(double* t, const double* r, const double* d, const double* theta_dev, double eps,
                           int64_t n) {
    (void)t; (void)r; (void)d; (void)theta_dev; (void)eps; (void)n;
    throw std::runtime_error("executor: no device-scalar vector primitives");
  }
  // Batched symmetric eigensolver (FP64): matrix i is sizes[i] x sizes[i],
  // row-major at A + offs[i]; on return its diagonal holds the eigenvalues
  // (unordered) and V + offs[i] the eigenvectors as columns.  Two-sided Jacobi
  // with parallel (round-robin) ordering; a matrix is done when its
  // off-diagonal Frobenius norm falls below max(tol, 4 n eps) * ||A||_F
  // (n its size, eps the FP64 unit roundoff: the rounding floor of the
  // rotations grows with n).  Returns the number of matrices still above
  // their threshold after max_sweeps sweeps; *worst (nullable) receives the
  // largest off-norm / ||A||_F among them (0 if none).
  virtual int sym_eig(double* A, double* V, const std::vector<int64_t>& offs, const std::vector<int>& sizes,
                      int max_sweeps, double tol, double* worst) = 0;
  // Per-launch timing of run() with device events on the executor's stream.
  // kernel_time() synchronises and returns (total ms, launches) since the
  // last call to timing(true).
  virtual void timing(bool on) { (void)on; }
  virtual std::pair<double, long long> kernel_time() { return {0.0, 0}; }
  // Host-side time spent in the executor's calls (diagnostics), one line.
  virtual std::string host_profile() const { return std::string(); }
  // dst[i] = idx[i] >= 0 ? src[idx[i]] : 0 for i < n, converted to dt_dst
  virtual void pack(void* dst, int dt_dst, const double* src, const int* idx, size_t n) = 0;
  // dst[i] = src[idx[i]] + a * x[i] (src of dtype dt_src; x FP64, or null
  // for no term) for i < n, in FP64
  virtual void gather(double* dst, const void* src, int dt_src, const int* idx, size_t n, double a = 0.0,
                      const double* x = nullptr, const double* mul = nullptr) = 0;
  // ---- FP8 (OCP E4M3) copies with power-of-two scales
  // d_scale[2y], d_scale[2y+1] = (s, 1/s) of segment y of src (nseg segments
  // of seg values): s = 2^e, the smallest with max|x| / s <= 448 (1 for zeros)
  virtual void fp8_scales(const double* src, int64_t nseg, int64_t seg, double* d_scale) {
    (void)src; (void)nseg; (void)seg; (void)d_scale;
    throw std::runtime_error("executor: no FP8 support");
  }
  // dst[i] = E4M3(src[i] / s of segment i / seg), round to nearest even, saturating
  virtual void to_fp8(void* dst, const double* src, int64_t n, int64_t seg, const double* d_scale) {
    (void)dst; (void)src; (void)n; (void)seg; (void)d_scale;
    throw std::runtime_error("executor: no FP8 support");
  }
  // d_scale[0..1] = (s, 1/s) of the n_all values at src_all, then
  // dst[i] = idx[i] >= 0 ? E4M3(src[idx[i]] / s) : 0 for i < n
  virtual void pack_fp8(void* dst, const double* src, const int* idx, size_t n, double* d_scale,
                        const double* src_all, size_t n_all) {
    (void)dst; (void)src; (void)idx; (void)n; (void)d_scale; (void)src_all; (void)n_all;
    throw std::runtime_error("executor: no FP8 support");
  }
  // dst[idx[i]] = src[idx[i]] + a rounded to dt_dst, for i < n (src FP64)
  virtual void shifted_copy_at(void* dst, int dt_dst, const double* src, const int* idx, size_t n, double a) = 0;
  // element-wise precision conversion of n values
  virtual void convert(void* dst, int dt_dst, const void* src, int dt_src, size_t n) = 0;
  // ---- optional: record the calls made between capture_begin and
  // capture_end (no allocation, synchronisation or prepare in between) into a
  // graph that replay() re-issues on the stream.  A graph refers to the
  // executor's shared scratch, so it is valid only while scratch_generation()
  // is unchanged.  Timing (timing(true)) is not recorded.
  virtual bool graphs() const { return false; }
  virtual void capture_begin() { throw std::runtime_error("executor: no graph capture"); }
  virtual void* capture_end() { throw std::runtime_error("executor: no graph capture"); }
  virtual void capture_abort() {}
  virtual void replay(void* graph) { (void)graph; throw std::runtime_error("executor: no graph capture"); }
  virtual void drop_graph(void* graph) { (void)graph; }
  virtual long long scratch_generation() const { return 0; }
  virtual bool timing_on() const { return false; }
  // ---- orbital-rotation energy and gradient (orb_grad); all FP64, device arrays
  // For each of naux symmetric n x n matrices B_L (B + L*n*n), with the
  // orbitals ordered core (nc), active (na), virtual: scal[4L..4L+3] =
  // (J, t, q, r) with J = sum_i B_ii (core), t = sum_tu gam_tu B_tu (active),
  // q = sum_ij B_ij B_ji (core-core), r = sum_{t,u,i} gam_tu B_ti B_iu; and
  // bact[L*na*na ..] = the active block of B_L, row-major.
  virtual void orb_scalars(const double* B, int naux, int n, int nc, int na, const double* gam, double* bact,
                           double* scal) {
    (void)B; (void)naux; (void)n; (void)nc; (void)na; (void)gam; (void)bact; (void)scal;
    throw std::runtime_error("executor: no orbital kernels");
  }
  // G_L = gradient of the L-sum of 2J^2 - q + 2Jt - r + e2_L with respect to
  // the n x n entries of B_L, where e2_L = 1/2 bact_L . Y_L, given
  // Y_L = D bact_L and Z_L = D^T bact_L (naux x na*na each); e2[L] receives e2_L.
  virtual void orb_assemble(const double* B, int naux, int n, int nc, int na, const double* gam, const double* scal,
                            const double* bact, const double* Y, const double* Z, double* G, double* e2) {
    (void)B; (void)naux; (void)n; (void)nc; (void)na; (void)gam; (void)scal; (void)bact; (void)Y; (void)Z;
    (void)G; (void)e2;
    throw std::runtime_error("executor: no orbital kernels");
  }
  // ---- fixed scratch of the allocation-free H*psi entry point
  // Device address and size of this device's fixed scratch array.
  virtual void* fixed_scratch(size_t* bytes) {
    *bytes = 0;
    return nullptr;
  }
  // Plan a launch like prepare() without touching device memory: the handle
  // holds the task lists on the host; *list_bytes / *part_bytes receive the
  // device bytes its lists and its split-K partial tiles need.
  virtual void* plan_fixed(const std::vector<RawJob>& jobs, const std::vector<RawTerm>& terms, int da, int db,
                           int dc, size_t* list_bytes, size_t* part_bytes) {
    (void)jobs; (void)terms; (void)da; (void)db; (void)dc; (void)list_bytes; (void)part_bytes;
    throw std::runtime_error("executor: no fixed scratch");
  }
  // Copy a plan_fixed handle's task lists to dev (list_bytes of it) and let
  // its launches write partial tiles to part; run() then launches it.
  virtual void place_fixed(void* handle, void* dev, void* part) {
    (void)handle; (void)dev; (void)part;
    throw std::runtime_error("executor: no fixed scratch");
  }
  // Release a plan_fixed handle (host memory only).
  virtual void drop_fixed(void* handle) { (void)handle; }
  // ---- ordering with a caller's stream (a hipStream_t; nullptr = the null
  // stream).  wait_for(s): later work of the executor waits for everything
  // queued on s so far.  signal(s): later work on s waits for everything
  // queued on the executor's stream so far.  Neither blocks the host.
  virtual void wait_for(void* stream) { (void)stream; }
  virtual void signal(void* stream) { (void)stream; }
};

// The product executor (HIP, gfx950).
Executor* make_hip_executor();

}  // namespace dmrg
