// Host planner for spin-adapted two-site DMRG: symmetry sectors, operator
// blocks ("environments"), their growth by one site, and the task lists of the
// Davidson matrix-vector product H*psi.
//
// Hamiltonian (Sec. "Complete active space SCF", with the standard pairing and
// factor 1/2 on the two-electron term):
//   H = sum h_pq E_pq + 1/2 sum (pq|rs) sum_st a+_ps a+_rt a_st a_qs.
// Orbitals are split at a cut into a left part X and a right part Y.  The
// cross terms are written with normal operators on X and complementary
// operators (integrals already summed in) on Y, or the reverse for the 3+1
// split, so that their number grows like |X|^2:
//   pair     sum_{i<=j in X} ap_S [A^S_ij (x) P^S_ij]^0 + h.c.
//   B-Q      sum_{i,j in X}  [B^k_ij (x) Q^k_ij]^0,  Q = ee J - ex K
//   1+3      sum_{p in X}    cs [C_p (x) SR_p]^0 + h.c.
//   3+1      sum_{r in Y}    sc [SL_r (x) C_r]^0 + h.c.
// with A^S_ij = [c_i c_j]^S, B^k_ij = [c_i d_j]^k, P^S_ij = 1/2 sum g_iqjs [d_s d_q]^S,
// J_ij = sum g_ijrs [c_r d_s]^0, K^k_ij = sum g_iqrj [c_r d_q]^k,
// SR_p = sum h_pq d_q + sum g_pqrs U(r,s,q), SL_r = sum g_pqrs T(p,q,s).
//
// Left blocks (sites 0..b-1) store H, C, D, A^S, Abar^S = [d d]^S, B^k and SL_r
// (r >= b); right blocks (sites b..n-1) store H, C, D, P^S, J, K^k and SR_p
// (p < b).  All operators are reduced (Wigner-Eckart) block-sparse matrices
// over the bond's (N, 2S) sectors, in the convention
//   <j m| T^k_q |j' m'> = <j' m'; k q | j m> <j||T||j'>.
#pragma once
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "exec.hpp"
#include "spin.hpp"

namespace dmrg {

// An allocation that would pass the context's device-memory budget.
struct BudgetExceeded : std::bad_alloc {
  std::string msg;
  explicit BudgetExceeded(std::string m) : msg(std::move(m)) {}
  const char* what() const noexcept override { return msg.c_str(); }
};

struct Sector {
  int n = 0, s2 = 0, dim = 0;
};

struct Bond {
  std::vector<Sector> secs;
  int find(int n, int s2) const;
};

// Operator blocks are stored row-major with the row stride padded to a
// multiple of 8 elements and 8-element aligned offsets, so that every row of
// every block starts on a 16-byte boundary in all precisions (vector loads in
// the H*psi kernels).  Padding elements are never read as data.
constexpr int kPad = 8;
inline int pad_up(int d) { return (d + kPad - 1) / kPad * kPad; }
struct OpBlock {
  int bra = 0, ket = 0;
  int64_t off = 0;
  int ld = 0;  // row stride (>= ket dimension)
};

struct OpLayout {
  int k2 = 0, dn = 0, nsec = 0;
  std::vector<OpBlock> blocks;
  std::vector<int> lookup;  // bra * nsec + ket -> block index, -1 if absent
  int64_t size = 0;
  int find(int bra, int ket) const {
    if (bra < 0 || ket < 0) return -1;
    return lookup[(size_t)bra * nsec + ket];
  }
};

enum Fam : int {
  F_H = 0, F_C, F_D, F_A0, F_A1, F_AB0, F_AB1, F_B0, F_B1, F_SL,
  F_P0, F_P1, F_J, F_K0, F_K1, F_SR, kNumFam,
  F_ID = 1000,      // identity operator
  F_TMP0 = 2000     // F_TMP0 + t : temporary (linear-combination) family t
};
int fam_k2(int f);
int fam_dn(int f);
const char* fam_name(int f);

struct Ref {
  int fam = F_ID;
  int idx = 0;
  bool operator<(const Ref& o) const { return fam != o.fam ? fam < o.fam : idx < o.idx; }
  bool operator==(const Ref& o) const { return fam == o.fam && idx == o.idx; }
  bool is_id() const { return fam == F_ID; }
};

struct Family {
  int k2 = 0, dn = 0;
  const OpLayout* lay = nullptr;
  int nops = 0;
  int buf = -1;              // device buffer holding nops * lay->size values
  std::vector<int> index;    // key -> op index (-1 absent); key = i or i*n + j
};

struct DevBuf {
  int64_t n = 0;       // elements
  void* p[4] = {nullptr, nullptr, nullptr, nullptr};  // per dtype copy
  bool view = false;   // points into memory the buffer does not own
  // FP8 copy: one power-of-two scale per segment of fp8_seg elements (one
  // operator of a family); the stored values are x / scale
  int64_t fp8_seg = 0;
  std::vector<double> fp8_scale;
};

class Context;

struct Block {
  bool left = true;
  // Right blocks only: true while the block stores normal pair operators
  // (A, Abar, B for pairs inside it, like a left block) instead of the
  // complementary P, J, K for pairs to its left.  Normal pairs are cheaper
  // while the block is the smaller side of the chain; to_complementary()
  // converts before the block meets a left block in H*psi.
  bool normal = false;
  int b = 0, n = 0;
  // Low-precision copies of the block Hamiltonian (family F_H) hold
  // H - h_shift * 1: the mean of its diagonal taken out, so that its entries
  // and the products they feed are rounded relative to the spread of the
  // block energies rather than their size; H*psi adds the shift back in FP64.
  double h_shift = 0.0;
  bool h_shift_set = false;
  Bond bond;
  std::map<std::pair<int, int>, std::unique_ptr<OpLayout>> layouts;
  Family fam[kNumFam];
  std::vector<Family> tmp;
  const OpLayout& layout(int k2, int dn);
  const Family& family(int f) const { return f >= F_TMP0 ? tmp[f - F_TMP0] : fam[f]; }
  int op(int f, int i, int j = -1) const;  // op index or -1
  int64_t bytes_f64() const;
};

// One term of an operator on (block (x) site): coef * [L (x) s]^k (left growth)
struct LAtom {
  double c = 1.0;
  Ref L;
  int sop = S_I;
  int kL2 = 0, ks2 = 0;
  bool hc = false;  // apply the transpose (scalar targets only)
};
// One term of an operator on (site (x) block): coef * [s (x) R]^k (right growth)
struct RAtom {
  double c = 1.0;
  int sop = S_I;
  Ref R;
  int ks2 = 0, kR2 = 0;
  bool hc = false;
};
// One term of the two-site Hamiltonian: coef * [[L (x) s1]^kX (x) [s2 (x) R]^kX]^0
struct Term4 {
  double c = 1.0;
  Ref L;
  int s1 = S_I, kL2 = 0, k12 = 0, kX2 = 0;
  int s2 = S_I, k22 = 0, kR2 = 0;
  Ref R;
  bool hc = false;
};

struct Integrals {
  int n = 0;
  std::vector<double> h, g;
  double e_core = 0.0;
  double H(int p, int q) const { return h[(size_t)p * n + q]; }
  double G(int p, int q, int r, int s) const { return g[(((size_t)p * n + q) * n + r) * n + s]; }
};

// Site tensor of the MPS held on the device (FP64), with block offsets.
struct SiteTensor {
  bool left = true;  // A: (l, sigma, a) ; B: (c, sigma, r)
  int j = 0;
  struct Blk {
    int s0, sig, s1;
    int64_t off;
    int rows, cols;
  };
  std::vector<Blk> blocks;
  std::map<std::tuple<int, int, int>, int> find;
  int buf = -1;
};

// Two-site wavefunction layout (super-blocks, see the ABI header).
// psi in the caller's layout (dense super-blocks) and, for the contraction
// kernels, a padded copy in which every column sub-block starts on a multiple
// of 8 elements (pc0), rows have stride pncols (a multiple of 8) and
// super-blocks start at 8-aligned offsets poff; padding holds zeros.
struct PsiLayout {
  // r0: first row in the caller's layout ((l, sigma1) order); ir0: first row
  // in the internal order of the contraction buffers ((sigma1, l) order), in
  // which the row bands a site operator cannot reach are contiguous.
  struct Row {
    int il, s1, r0, dl, ir0;
  };
  struct Col {
    int s2, ir, c0, dr, pc0;
  };
  struct SB {
    int an, as2, cn, cs2, nrows, ncols, pncols;
    int64_t off, poff;
    std::vector<Row> rows;
    std::vector<Col> cols;
  };
  std::vector<SB> sbs;
  int64_t size = 0, psize = 0;
  // padded index (internal row order) -> caller index (-1 for padding)
  std::vector<int> pack_map() const;
  // caller index -> index of the same element in an unpadded copy with rows
  // in internal order (the layout stage R accumulates psi' in)
  std::vector<int> unpack_map() const;
  void build(const Bond& lb, const Bond& rb, int n_elec, int two_s);
};

// Everything H*psi needs at one two-site position, prepared once per position.
struct HpsiPlan {
  int k = -1;
  PsiLayout lay;
  std::vector<Term4> terms;
  // chunks of terms: stage L then stage R batches (symbolic)
  struct Chunk {
    GemmBatch stageL, stageR;
    int64_t xsize = 0;
  };
  std::vector<Chunk> chunks;
  GemmBatch diag;   // diagonal of H_eff, accumulated into the diag buffer
  double flops = 0.0;       // algorithmic: 2mnk over the rows and columns of structurally non-zero products
  double flops_exec = 0.0;  // executed by the launches (merged row segments include some zero bands)
  double flops_dense = 0.0; // 2mnk over whole X regions (every row band and column of a touched region)
  int64_t xmax = 0;
  size_t n_stage_terms = 0;
};

class Context {
 public:
  Context(Executor* ex, const Integrals& ints, int n_elec, int two_s);
  ~Context();
  Executor* ex;
  Integrals I;
  int n_elec, two_s;
  std::vector<SiteOp> sops;        // fixed site ops followed by per-orbital site Hamiltonians
  int site_h(int o) const { return kNumFixedSite + o; }

  // device buffer registry
  std::vector<DevBuf> bufs;
  int new_buf(int64_t n);           // FP64 buffer, zeroed
  void free_buf(int id);
  void* ptr(int buf, int dt = DT_F64) const { return bufs[buf].p[dt]; }
  void ensure_dtype(int buf, int dt);  // create converted copy from the F64 master
  void alloc_dtype(int buf, int dt);   // storage in dtype dt, contents undefined
  // FP8 copy of buf with one scale per segment of seg elements, converted
  // from src (default: the buffer's FP64 master)
  void ensure_fp8(int buf, int64_t seg, const double* src = nullptr);
  int view_buf();                      // entry that points into memory it does not own
  void set_view(int buf, int dt, void* p, int64_t n);
  int ph[8] = {-1, -1, -1, -1, -1, -1, -1, -1};  // placeholder buffers (-1..-7) of the current plan

  // MPS
  int n = 0, k = -1;
  std::vector<Bond> bonds;                 // bonds 0..n (left QNs up to k, right QNs from k+2)
  std::vector<SiteTensor> sites;           // size n (entries k, k+1 unused)
  std::unique_ptr<Block> Lblk, Rblk;       // blocks at bonds k and k+2
  std::vector<std::unique_ptr<Block>> Lhist, Rhist;  // blocks kept per bond (optional, indexed by bond)

  // building
  std::unique_ptr<Block> vacuum_left();
  std::unique_ptr<Block> vacuum_right();
  std::unique_ptr<Block> grow_left(Block& L, const SiteTensor& A, const Bond& newbond);
  std::unique_ptr<Block> grow_right(Block& R, const SiteTensor& B, const Bond& newbond);
  void to_complementary(Block& R);  // right block: normal pairs -> P, J, K over pairs to its left
  void free_block(Block& blk);

  // operator expressions
  std::vector<LAtom> lgrow(const Block& L, int f, int i, int j) const;
  std::vector<RAtom> rgrow(const Block& R, int f, int i, int j) const;
  std::vector<LAtom> lgrow_h(const Block& L) const;
  std::vector<RAtom> rgrow_h(const Block& R) const;

  // H*psi
  std::unique_ptr<HpsiPlan> plan_hpsi(int64_t x_budget_elems);
  std::vector<Term4> hpsi_terms(Block& L, Block& R);

  // linear combinations -> temporary families on a block
  Ref make_lincomb(Block& blk, int k2, int dn, const std::vector<std::pair<Ref, double>>& parts,
                   std::vector<std::vector<std::pair<Ref, double>>>* pending, std::vector<int>* pending_fam);
  void materialise_lincombs(Block& blk, const std::vector<std::vector<std::pair<Ref, double>>>& pending,
                            const std::vector<int>& pending_fam);

  // resolve a symbolic batch to raw pointers (A/B/C dtypes per buffer role)
  void resolve(const GemmBatch& b, std::vector<RawJob>& jobs, std::vector<RawTerm>& terms, int dta, int dtb,
               int dtc) const;
  void run_batch(const GemmBatch& b, int dta = DT_F64, int dtb = DT_F64, int dtc = DT_F64);

  double last_flops = 0.0;
  int64_t bytes_in_use = 0, peak_bytes = 0;
  int64_t budget_bytes = 0;  // 0: no cap
  // Account for `bytes` more device memory; throws BudgetExceeded (checked
  // before the allocation is made) if that would pass budget_bytes.
  void charge(int64_t bytes);
};

}  // namespace dmrg
