/* dmrg.h -- C ABI of the spin-adapted two-site DMRG hot path on MI355X (gfx950).
 *
 * The operation is the Davidson matrix-vector product of the two-site DMRG
 * step, H_eff psi = V^T H V psi, for the ab-initio Hamiltonian of the paper's
 * Sec. "Complete active space SCF" (integrals h_pq and (pq|rs), read with the
 * standard pairing and the factor 1/2 on the two-electron term) restricted to
 * the variational space of a spin-adapted matrix product state (Sec. "Tensor
 * network states and density matrix renormalization group"; bond dimension D
 * counts SU(2) multiplets as in Sec. "Conservation of the total spin").  The
 * loop around it -- Davidson with residual norm 1e-7 (Sec. "Numerical
 * procedure"), truncation to D multiplets and the renormalisation of the
 * operator blocks -- is exposed as well.
 *
 * Conventions
 *   - Every call returns int: 0 = DMRG_OK, < 0 = error; dmrg_last_error()
 *     gives a thread-local message.  Arguments are validated on the host
 *     before any GPU work is queued.
 *   - Host arrays are C row-major FP64, owned by the caller, copied before
 *     return and never retained.  *_dev pointers are device pointers borrowed
 *     for the duration of the call.
 *   - Orbitals are 0-based in chain order.  h is n*n, g is n^4 with
 *     g[p][q][r][s] = (pq|rs) (chemists' notation, 8-fold symmetric).
 *   - Local multiplets per site: sigma = 0 (empty), 1 (doublet), 2 (doubly
 *     occupied).  Creation-operator order is orbital-major, up before down.
 *   - The two-site block is (k, k+1).  Bonds 0..k carry the (N, 2S) of the
 *     block of sites to their left, bonds k+2..n the (N, 2S) of the block of
 *     sites to their right; bond k+1 is inside the two-site block and is
 *     passed with zero sectors.  Bonds 0 and n hold the single sector (0,0,1).
 *   - Site tensors: sites j < k are left-canonical, blocks (l, sigma, a) of
 *     shape D_l x D_a with N_a = N_l + N_sigma and triangle(S_l, s_sigma, S_a),
 *     coupling the block state l and the site (in that order) to a.  Sites
 *     j >= k+2 are right-canonical, blocks (c, sigma, r) of shape D_c x D_r with
 *     N_c = N_sigma + N_r, coupling the site and the block state r (in that
 *     order) to c.  Blocks are ordered by (first sector, sigma, second sector),
 *     sector indices in bond order; each block is row-major.  The concatenation
 *     over sites 0..k-1 then k+2..n-1 is the `blocks` argument.
 *   - psi is coupled as ((l sigma1) S_a, (sigma2 r) S_c) S and stored as dense
 *     super-blocks (a, c) with N_a + N_c = N and triangle(S_a, S_c, S), sorted by
 *     (N_a, 2S_a, 2S_c); rows are the (l, sigma1) sub-blocks sorted by
 *     (l, sigma1), columns the (sigma2, r) sub-blocks sorted by (sigma2, r).
 */
#ifndef DMRG_MI355X_H
#define DMRG_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DMRG_OK = 0,
  DMRG_ERR_ARG = -1,       /* null pointer, bad enum, k out of range           */
  DMRG_ERR_SHAPE = -2,     /* inconsistent sizes, wrong block counts            */
  DMRG_ERR_SYMMETRY = -3,  /* N and 2S parity mismatch, impossible sector       */
  DMRG_ERR_BUDGET = -4,    /* device allocation failed / over hbm budget        */
  DMRG_ERR_HIP = -5,       /* HIP runtime error                                  */
  DMRG_ERR_NOCONV = -6,    /* Davidson not converged; outputs hold best iterate */
  DMRG_ERR_NONFINITE = -7  /* NaN or Inf in an input                             */
};

/* Arithmetic of the H*psi contraction.  FP64: exact path.  FP32 / BF16:
 * operator blocks, psi and the intermediates stored in that type, FP32
 * accumulation.  FP8: operator blocks and psi stored as OCP E4M3 with a
 * power-of-two scale per operator (psi: per call), widened exactly to BF16
 * for the BF16 MFMA, intermediates in BF16, FP32 accumulation.  The low-
 * precision copies of the block Hamiltonians hold H minus the mean of their
 * diagonal, which the product adds back in FP64. */
typedef enum { DMRG_FP64 = 0, DMRG_FP32 = 1, DMRG_BF16 = 2, DMRG_FP8 = 3 } dmrg_prec;

typedef struct dmrg_ctx dmrg_ctx;

typedef struct {
  int n_orb;                   /* active orbitals n                                  */
  int n_elec;                  /* active electrons N                                 */
  int two_s;                   /* twice the total spin                               */
  double e_core;               /* constant added to every energy                     */
  double davidson_tol;         /* residual 2-norm threshold (paper: 1e-7)            */
  int davidson_max_iter;       /* outer iterations per davidson_step                 */
  int davidson_max_subspace;   /* basis size before restart                          */
  int hpsi_prec;               /* dmrg_prec used for the bulk matvecs in Davidson    */
  long long work_budget_elems; /* cap on intermediate buffers (elements) per H*psi
                                  chunk; 0: default 2^32                           */
  int keep_blocks;             /* 1: keep the operator blocks of every bond that
                                  dmrg_set_mps builds, so dmrg_truncate can move
                                  the two-site block (memory grows with n);
                                  m >= 2: keep only the m bonds nearest the block
                                  on each side (m moves); -m <= -2: only the m
                                  nearest on the right side (m moves to the
                                  right, nothing kept for a move back); 0: none */
  int davidson_refine_iter;    /* iterations of the FP64 refinement phase when
                                  hpsi_prec is not FP64; 0: davidson_max_iter     */
  int davidson_jd_inner;       /* refinement with hpsi_prec not FP64: 0 expands the
                                  basis with the diagonally preconditioned residual;
                                  k > 0 with the Jacobi-Davidson correction from k
                                  conjugate-gradient steps whose matvecs use
                                  hpsi_prec                                        */
  int davidson_lowprec_iter;   /* iterations of the low-precision Davidson phase
                                  before refinement; -1: davidson_max_iter, 0: none */
  int hpsi_graph;              /* 1: record each precision's H*psi launch sequence
                                  as a HIP graph on first use and replay it (less
                                  host overhead for small blocks); re-recorded when
                                  the library's scratch moves; not used while
                                  dmrg_kernel_timing records                       */
  int next_guess;              /* 1: dmrg_truncate (either direction) also forms
                                  the start vector of the block it moves to (read
                                  it with dmrg_next_guess)                         */
  long long hbm_budget_bytes;  /* cap on the device memory the context's buffers
                                  hold (operator blocks and their low-precision
                                  copies, H*psi intermediates, Davidson vectors);
                                  checked on the host before each allocation, which
                                  fails with DMRG_ERR_BUDGET instead of exceeding it
                                  (the executor's task lists and split-K partial
                                  tiles come on top); 0: no cap                     */
  int davidson_mid_fp32;       /* 1 (hpsi_prec BF16 or FP8): between the low-
                                  precision phase and the FP64 refinement, a phase
                                  with FP32 matvecs from the low-precision phase's
                                  lowest Ritz vectors, until the residual is 1e-6
                                  of the spectrum scale or stalls; its matvecs
                                  count as low-precision ones                      */
  int davidson_graph;          /* 1: record the device work of a Davidson
                                  iteration (Ritz vector, residual, new basis
                                  vector, its H*psi and projections) as two HIP
                                  graphs per precision and basis size, replayed
                                  with the host's Rayleigh-Ritz coefficients in
                                  between; same results bit for bit as 0.  Not
                                  used with davidson_jd_inner > 0 in the
                                  refinement, in dmrg_batch_davidson, or while
                                  dmrg_kernel_timing records                       */
} dmrg_opts;

/* Create a context; copies h (n*n) and g (n^4).  h must be symmetric and g
 * 8-fold symmetric ((pq|rs) = (qp|rs) = (pq|sr) = (rs|pq), real orbitals),
 * to 1e-12 of their largest element.  Errors: ARG (null, sizes, an integral
 * without these symmetries, hbm_budget_bytes < 0), SYMMETRY (N odd with 2S
 * even, N > 2n, ...), NONFINITE. */
int dmrg_create(dmrg_ctx **out, const dmrg_opts *opts, const double *h, const double *g);

/* Replace the context's options between calls (e.g. Davidson tolerances and
 * precisions that change from sweep to sweep).  Only davidson_*, hpsi_prec,
 * hpsi_graph and next_guess may differ from the current options; the other
 * fields must be passed unchanged.  Errors: ARG. */
int dmrg_update_opts(dmrg_ctx *c, const dmrg_opts *opts);

/* Load a mixed-canonical MPS around the two-site block (k, k+1) and build the
 * left operator block at bond k and the right operator block at bond k+2 on
 * the GPU.  bond_sectors: sum(sectors_per_bond) rows of (N, 2S, dim) int32;
 * sectors_per_bond: n+1 counts.  Errors: ARG, SHAPE, SYMMETRY, NONFINITE,
 * BUDGET, HIP. */
int dmrg_set_mps(dmrg_ctx *c, int k, const int *bond_sectors, const int *sectors_per_bond,
                 const double *blocks, long long n_values);

/* psi layout at the current two-site block: number of super-blocks, total
 * length, and (if desc != NULL) 7 values per super-block:
 * (N_a, 2S_a, N_c, 2S_c, rows, cols, offset). */
int dmrg_psi_layout(dmrg_ctx *c, int k, long long *n_superblocks, long long *desc, long long *n_elems);

/* psi_out = H_eff psi_in at block (k, k+1) (host buffers of n_elems FP64).
 * prec selects the arithmetic of the contraction (FP64 exact path, FP32 or
 * BF16 operands with FP32 accumulation).  flops_out (nullable) receives the
 * algorithmic flop count (sum of 2mnk over structurally non-zero block
 * products, identities excluded). */
int dmrg_hpsi(dmrg_ctx *c, int k, const double *psi_in, double *psi_out, int prec, double *flops_out);

/* Same on device buffers (FP64, n_elems each), on the library's stream; the
 * copy into d_out may still be queued on return (synchronise the device
 * before reading it). */
int dmrg_hpsi_dev(dmrg_ctx *c, int k, const void *d_in, void *d_out, int prec);

/* Same, ordered with the caller's HIP stream hip_stream (a hipStream_t;
 * NULL = the null stream): the product starts after all work queued on
 * hip_stream before the call (which may still be producing d_in), and work
 * queued on hip_stream after the call runs after d_out is written.  Neither
 * side is host-synchronised for this ordering: the call returns once the
 * work is queued (the first call of a precision on a new block also prepares
 * its task lists, which waits for the device).  Errors as dmrg_hpsi_dev. */
int dmrg_hpsi_dev_stream(dmrg_ctx *c, int k, const void *d_in, void *d_out, int prec, void *hip_stream);

/* Allocation-free variant of dmrg_hpsi_dev, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same product, inputs and outputs (device FP64,
 * n_elems each, caller layout).  Every intermediate of the call -- task
 * lists, the padded copy of psi, the psi' accumulator, the X intermediates
 * and split-K partial tiles -- lives in a fixed device array of the library
 * (128 MiB, one per GPU, held until the process ends, shared by all contexts)
 * instead of buffers the library allocates; the call allocates no device
 * memory.  Preconditions: the block's H*psi plan exists (dmrg_psi_layout or
 * any H*psi call at this block made it) and, for prec != DMRG_FP64, the
 * operator blocks have their copies in that precision (any earlier H*psi or
 * Davidson call with it made them).  Returns once d_out is written.  Calls
 * that overlap on one GPU (other threads or contexts) race on the shared
 * array.  Errors: ARG (null pointer, bad precision, the preconditions),
 * BUDGET (the block needs more scratch than the array holds; nothing is
 * launched), HIP. */
int dmrg_hpsi_dev_noalloc(dmrg_ctx *c, int k, const void *d_in, void *d_out, int prec);

/* Diagonal of H_eff at the current block (host, n_elems). */
int dmrg_heff_diag(dmrg_ctx *c, int k, double *diag);

/* Davidson for the lowest eigenpair of H_eff at block (k, k+1), starting from
 * psi_inout (host, n_elems; a zero vector selects a random start).  Bulk
 * matvecs in opts.hpsi_prec, residuals and Rayleigh-Ritz in FP64 with FP64
 * correction matvecs (with opts.davidson_jd_inner > 0, Jacobi-Davidson
 * refinement whose correction equations are solved with hpsi_prec matvecs).
 * On return psi_inout holds the normalised eigenvector, energy the
 * eigenvalue plus e_core, resid_norm ||H x - E x||_2; n_matvec_lowprec counts
 * every hpsi_prec matvec (inner solves included), n_matvec_fp64 the FP64 ones.
 * Returns NOCONV (outputs still written) if tol is not reached.
 *
 * Step log: if the environment variable DMRG_LOG names a file, every
 * dmrg_davidson_step and dmrg_truncate(_dbss) that returns OK (or NOCONV for
 * Davidson) appends one JSON object per line to it -- for Davidson the block,
 * length, precision, energy, residual, matvec counts, H*psi flops, wall
 * seconds and the host seconds spent planning and preparing task lists; for
 * a truncation the block, direction, multiplets D and U(1) states D~ of the
 * new bond, discarded weight, wall seconds and the next block. */
int dmrg_davidson_step(dmrg_ctx *c, int k, double *psi_inout, double *energy, double *resid_norm,
                       int *n_matvec_lowprec, int *n_matvec_fp64);

/* Truncate psi at the middle cut (Sec. "Numerical procedure": fixed D, or a
 * truncation-error threshold).  Multiplet weights are the eigenvalues of the
 * reduced density matrix of the enlarged left block (direction +1) or the
 * enlarged right block (direction -1), rho_a = sum_c psi_ac psi_ac^T, summed
 * over spin projections; the d_max largest are kept (ties broken by 2S, N,
 * index); eps_tr > 0 keeps fewer when the discarded weight stays <= eps_tr.
 * The kept eigenvectors form a new left-canonical tensor at site k (+1) or a
 * right-canonical tensor at site k+1 (-1), and the operator block is grown to
 * bond k+1 on the GPU.  If keep_blocks was set, the two-site block then moves
 * to (k+1, k+2) or (k-1, k).  trunc_err = discarded weight / total weight.
 * Returns NOCONV (all outputs still written) if the batched eigensolver left
 * a sector's density matrix unconverged to its rounding floor. */
int dmrg_truncate(dmrg_ctx *c, int k, const double *psi, int direction, int d_max, double eps_tr,
                  double *trunc_err, int *d_kept);

/* Dynamic block state selection (Sec. "Numerical procedure": bond dimension
 * chosen per bond at a fixed truncation error eps_tr instead of a fixed D):
 * as dmrg_truncate, keeping the fewest multiplets whose discarded weight
 * stays <= eps_tr of the total, clamped to [d_min, d_max] (and to the number
 * of multiplets the cut has).  With eps_tr = 0, d_max multiplets are kept.
 * dmrg_truncate is this call with d_min = 0.  Errors as dmrg_truncate, and
 * ARG unless 0 <= d_min <= d_max. */
int dmrg_truncate_dbss(dmrg_ctx *c, int k, const double *psi, int direction, int d_min, int d_max,
                       double eps_tr, double *trunc_err, int *d_kept);

/* Start vector for the current block (k, k+1) carried over by the last
 * dmrg_truncate with opts.next_guess set (Sec. "Numerical procedure": each
 * sweep step starts from the previous step's wavefunction): the kept part of
 * the previous psi, contracted with the right-canonical tensor of site k+1
 * (after a move to the right) or the left-canonical tensor of site k (after
 * a move to the left) and recoupled to this block's middle-cut basis (one 6j
 * per block).  Without truncation it is the same state; its norm squared is
 * 1 - trunc_err for a normalised psi.  psi: n_elems host values (the layout of
 * dmrg_psi_layout).  Errors: ARG if no vector was carried to this block,
 * SHAPE for a wrong length. */
int dmrg_next_guess(dmrg_ctx *c, int k, double *psi, long long n_elems);

/* Read back bond b's sectors ((N, 2S, dim) rows, *n sectors) and site j's
 * tensor (blocks in the canonical order of dmrg_set_mps, *n values); with a
 * NULL output only the count is returned. */
int dmrg_get_bond(dmrg_ctx *c, int b, int *sectors, int *n);
int dmrg_get_site(dmrg_ctx *c, int j, double *values, long long *n);

/* Left site index k of the current two-site block (-1 if the block could not
 * move after a truncation because the needed operator block was not kept). */
int dmrg_current_block(dmrg_ctx *c, int *k);

/* Reduced singular values of the last truncation (all sectors, descending),
 * with their sector spins 2S; returns the count in *n. */
int dmrg_cut_spectrum(dmrg_ctx *c, double *values, int *two_s, int *n, int capacity);

/* Counters: out[0] = algorithmic flops of one H*psi (2mnk over the rows and
 * columns of structurally non-zero block products), out[1] = bytes of operator
 * blocks (left + right, FP64), out[2] = peak device bytes, out[3] = number of
 * terms, out[4] = number of block-product tasks per H*psi, out[5] = flops the
 * launches execute (row segments merged for fuller tiles include some zero
 * rows), out[6] = 2mnk over every row and column of each intermediate a term
 * touches (an upper bound that also counts structurally zero rows and unread
 * columns).  n: number of entries wanted (at most 7). */
int dmrg_stats(dmrg_ctx *c, double *out, int n);

/* The H*psi tile autotuner's choices in this process, as JSON text in buf
 * (capacity bytes, NUL-terminated): the number of launch classes, how many
 * were timed here (the rest came from the file DMRG_TUNE_FILE names), and how
 * many chose each kernel configuration.  The tuner times every candidate
 * configuration of a padded BF16 H*psi launch (tiles 64x64, 64x128, 128x64
 * and the one-wave 32x32 kernel) on the launch itself when the plan is first
 * prepared and keeps the fastest; DMRG_TUNE=0 uses the static rule instead.
 * Errors: ARG (null, buffer too small). */
int dmrg_tuner_report(dmrg_ctx *c, char *buf, int capacity);

/* Device-event timing of the library's GEMM launches on its own stream.
 * mode 1: clear and start recording; 0: report and stop; -1: report only.
 * ms / launches (nullable) receive the summed kernel time and launch count. */
int dmrg_kernel_timing(dmrg_ctx *c, int mode, double *ms, long long *launches);

/* Kernel self-test: C (m x n) = beta*C + alpha * op(A) op(B) through the same
 * grouped MFMA kernel the hot path uses (host FP64 buffers; A is m x k or,
 * with trans_a, k x m row-major; B is k x n or n x k).  ident_a / ident_b
 * replace the operand by the identity (k must then equal m / n).  prec as in
 * dmrg_hpsi: operands are rounded to it, accumulation is FP64 (FP64) or FP32.
 * Bit 1 of trans_a / trans_b (value 2) stores that operand with its rows
 * padded to a multiple of 8 elements (padding filled with NaN) and marks it
 * padded, which selects the kernel's 16-byte vector staging path. */
int dmrg_gemm_selftest(int m, int n, int k, const double *A, int trans_a, int ident_a, const double *B,
                       int trans_b, int ident_b, double alpha, double beta, double *C, int prec);

/* Batched H*psi over independent contexts (Sec. "Numerical procedure" runs
 * the same H_eff psi product in every Davidson iteration of every instance;
 * many small instances -- different molecules, geometries or spin states --
 * fill the GPU together where one alone cannot).  dmrg_batch_create takes
 * `count` distinct contexts, each with an MPS loaded (dmrg_set_mps), builds
 * each one's H*psi plan at its current two-site block if needed, and merges
 * the block-product tasks of all of them into one grouped launch per stage
 * and chunk, run on the first context's stream.  prec as in dmrg_hpsi.
 * The contexts must outlive the batch; a context whose block changes after
 * the batch was made (dmrg_set_mps, dmrg_truncate) makes dmrg_batch_hpsi fail
 * with ARG.  dmrg_batch_hpsi: d_in[i] / d_out[i] are device FP64 buffers of
 * context i's n_elems (dmrg_psi_layout); the result equals dmrg_hpsi_dev on
 * each context with the same prec (FP64: up to summation order within a
 * split-K reduction, which is fixed by the merged plan).  Errors: ARG, BUDGET,
 * HIP. */
typedef struct dmrg_batch dmrg_batch;
int dmrg_batch_create(dmrg_ctx *const *ctxs, int count, int prec, dmrg_batch **out);
int dmrg_batch_hpsi(dmrg_batch *b, const void *const *d_in, void *const *d_out);
void dmrg_batch_destroy(dmrg_batch *b);

/* Batched Davidson: dmrg_davidson_step on every context of the batch at once
 * (each with its own opts: precision, tolerance, refinement), with the
 * matvecs of all instances gathered into the batch's merged launches.  Each
 * context's solver runs on a host thread of its own; whenever every
 * unfinished solver waits for a matvec, one merged H*psi per requested
 * precision serves them all (instances that already finished are computed
 * on stale inputs and ignored).  psi[i]: host start vector / result of
 * context i (n_elems, as dmrg_davidson_step); energy, resid, status and the
 * (nullable) matvec counts are arrays of batch size.  status[i] is the code
 * dmrg_davidson_step would return for instance i; the call returns OK if all
 * are OK, else the first non-NOCONV error, else NOCONV.  The contexts must
 * not be used by other threads during the call.  Errors: ARG (as
 * dmrg_batch_hpsi), HIP, NOCONV, NONFINITE. */
int dmrg_batch_davidson(dmrg_batch *b, double *const *psi, double *energy, double *resid, int *n_matvec_lowprec,
                        int *n_matvec_fp64, int *status);

/* CAS-SCF orbital step (Sec. "Complete active space SCF": the orbitals are
 * optimised at fixed RDMs between DMRG solves, through the rotated integrals
 * h(kappa) and (pq|rs)(kappa)): the energy after the rotation kappa and its
 * gradient, forward and backward on the GPU, all FP64.
 *   orbitals: n = n_core + n_act + n_virt, ordered core, active, virtual;
 *   h_full: n*n symmetric; B: naux*n*n, symmetric matrices B^L with
 *     (pq|rs) = sum_L B^L_pq B^L_rs;
 *   kappa: n*n, strict lower triangle read: K_pq = kappa_pq (p > q),
 *     K_qp = -kappa_pq, U = exp(-K), h(kappa) = U^T h U, B^L(kappa) = U^T B^L U;
 *   gamma: n_act^2 spin-summed 1-RDM gamma~_tu = <sum_s a+_ts a_us>;
 *   Gamma: n_act^4, Gamma~_tuvw = <sum_st a+_ts a+_ut a_vt a_ws>;
 *   energy: 2 sum_i h_ii + sum_ij [2(ii|jj) - (ij|ji)] + sum_tu F^c_tu gamma~_tu
 *     + 1/2 sum_tuvw (tu|vw) Gamma~_tvwu, F^c_pq = h_pq + sum_i [2(pq|ii) - (pi|iq)],
 *     integrals at kappa;
 *   grad: n*n antisymmetric, grad[p*n+q] = dE/dkappa_pq for p > q.
 * Host buffers, copied; nothing retained.  Errors: ARG (null, h or a B^L not
 * symmetric), SHAPE (counts), NONFINITE, BUDGET, HIP. */
int orb_grad(int n_core, int n_act, int n_virt, const double *h_full, const double *B, int naux,
             const double *kappa, const double *gamma, const double *Gamma, double *energy, double *grad);

/* The SU(2) coupling coefficients the planner weights every term with (Sec.
 * "Conservation of the total spin": the Clebsch-Gordan layer kept apart from
 * the tensor layer), exposed for checking against independent tables.  All
 * arguments are doubled spins 2j (and doubled projections 2m).  kind 0:
 * <j1 m1; j2 m2 | J M> from two_j = (2j1, 2m1, 2j2, 2m2, 2J, 2M); kind 1: the
 * 6j symbol {j1 j2 j3; j4 j5 j6} from six values; kind 2: the 9j symbol
 * {j1 j2 j3; j4 j5 j6; j7 j8 j9} from nine values, row by row.  Host only.
 * Errors: ARG (null pointer, bad kind, negative spin). */
int dmrg_su2_coefficient(int kind, const int *two_j, double *value);

const char *dmrg_last_error(void);
void dmrg_destroy(dmrg_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
