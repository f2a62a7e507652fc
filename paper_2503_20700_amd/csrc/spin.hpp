// Spin-coupling engine and site operators.
//
// Every operator on the hot path is an SU(2) tensor operator written with the
// spin-1/2 creation tensor c = f+ = (a+_up, a+_dn) and annihilation tensor
// d = f = (a_dn, -a_up) (Sec. "Conservation of the total spin", the f, f+
// definitions).  Products of several such operators, e.g. the two-electron
// spin sum sum_{st} a+_ps a+_rt a_st a_qs, are vectors in a 2^L dimensional
// "component space" (one m = +-1/2 per factor).  Rewriting such a product as
// a sum of coupled forms [[X]^kx (x) [Y]^ky]^k, after moving the factors that
// live on the left sub-block in front of those on the right sub-block, is an
// orthogonal projection in that space.  This file computes those projection
// coefficients numerically (with residual checks), so no recoupling constant
// is typed by hand.
#pragma once
#include <array>
#include <map>
#include <string>
#include <vector>

namespace dmrg {

// ---------------------------------------------------------------- component space
// Index bit i = 0 -> m_i = +1/2, 1 -> m_i = -1/2.
struct CForm {
  int L = 0;
  std::map<int, std::vector<double>> comp;  // total doubled projection q -> 2^L vector
};

CForm cf_leaf(int L, int pos);                                   // rank-1/2 leaf at position pos
CForm cf_couple(const CForm& a, int ka2, const CForm& b, int kb2, int k2);  // [a (x) b]^k (disjoint)
double cf_dot(const std::vector<double>& x, const std::vector<double>& y);
// Reorder factors: new position p takes old factor perm[p]; multiplies by the
// permutation's fermionic sign (all factors odd, all on distinct orbitals).
std::vector<double> cf_permute(const std::vector<double>& v, int L, const std::vector<int>& perm);

// Physical spin sums, as component vectors of total rank k (component q = k).
// a_{x,s} = phi(s) d_{x,-s} with phi(+1/2) = -1, phi(-1/2) = +1.
std::vector<double> phys_e4_pair(int L);      // sum_st a+_p,s a+_r,t a_s,t a_q,s   factors (c_p c_r d_s d_q)
std::vector<double> phys_ee(int L);           // sum_st a+_p,s a_q,s a+_r,t a_s,t   factors (c_p d_q c_r d_s)
std::vector<double> phys_exch(int L);         // sum_st a+_p,s a_s,t a+_r,t a_q,s   factors (c_p d_s c_r d_q)
std::vector<double> phys_cz(int L);           // sum_s a+_p,s Z_s, Z rank-1/2 tilde  factors (c_p Z)
std::vector<double> phys_xc(int L);           // sum_t X_t a+_r,t, X rank-1/2 tilde factors (X c_r)
std::vector<double> phys_t3(int L);           // tilde(+1/2) of t -> sum_s a+_p,s a_s',t a_q,s  factors (c_p d_s' d_q)
std::vector<double> phys_u3(int L);           // tilde(+1/2) of s -> sum_t a+_r,t a_s,t a_q,s   factors (c_r d_s d_q)

// Coefficients of the coupled expansion of a target (rank k2, component
// q = k2) over a split: factors xs (in order) go to X, ys to Y; X coupled
// with tree tx, Y with tree ty.  A tree over 1 factor is a leaf; over 2
// factors it is [f0 f1]^kx; over 3 it is [[f0 f1]^k12 f2]^kx with k12 given.
// Returns coefficient for each (kx2, ky2) that appears; throws if the target
// is not fully reproduced.
struct SplitSpec {
  std::vector<int> xs, ys;  // positions in the target's factor list
  int x_k12 = -1, y_k12 = -1;  // intermediate rank for 3-factor sides
};
std::map<std::pair<int, int>, double> split_coeffs(const std::vector<double>& target, int L, int k2,
                                                   const SplitSpec& s);

// ---------------------------------------------------------------- site operators
// Local multiplets: 0 = |0> (N=0,S=0), 1 = doublet (N=1,S=1/2), 2 = |up dn> (N=2,S=0).
constexpr int kLocN[3] = {0, 1, 2};
constexpr int kLocS2[3] = {0, 1, 0};

struct SiteOp {
  std::string name;
  int k2 = 0, dn = 0, parity = 0;
  double r[3][3] = {{0}};  // reduced elements <s'||T||s>, bra first
};

// Site-operator registry: fixed ops are created on first use.
enum SiteId {
  S_I = 0, S_C, S_D, S_CC0, S_DD0, S_CD0, S_CD1, S_T3, S_U3, S_NUP_NDN, S_N, kNumFixedSite
};
const SiteOp& site_op(int id);
// Scalar site Hamiltonian h n + (1/2) g sum_st a+_s a+_t a_t a_s
SiteOp site_hamiltonian(double h_oo, double g_oooo);

// ---------------------------------------------------------------- derived constants
struct SpinConstants {
  double ap[2];        // sum_st a+p a+r a_s a_q = sum_S ap[S] [[c_p c_r]^S (x) [d_s d_q]^S]^0
  double ee[2];        // E_pq E_rs               = sum_k ee[k] [[c_p d_q]^k (x) [c_r d_s]^k]^0
  double ex[2];        // exchange spin sum       = sum_k ex[k] [[c_p d_s]^k (x) [c_r d_q]^k]^0
  double cs;           // sum_s a+_p,s Z_s        = cs [c_p (x) Z]^0
  double sc;           // sum_t X_t a+_r,t        = sc [X (x) c_r]^0
  // left growth parts, X = block L, Y = site o
  double b_swap[2];    // [c_o d_j]^k = b_swap[k] [d_j (x) c_o]^k
  double t_p1[2];      // T(p,q=o,s) with p,s in L: sum_k t_p1[k] [B^k_ps (x) d_o]
  double t_p2[2];      // T(p,q,s=o), p,q in L:      sum_k t_p2[k] [B^k_pq (x) d_o]
  double t_p3[2];      // T(p=o,q,s), q,s in L:      sum_S t_p3[S] [[d_s d_q]^S (x) c_o]
  double t_p4[2];      // T(p,q=o,s=o), p in L:      sum_S t_p4[S] [c_p (x) [d_o d_o]^S]
  double t_p5[2];      // T(p=o,q=o,s), s in L:      sum_k t_p5[k] [d_s (x) [c_o d_o]^k]
  double t_p6[2];      // T(p=o,q,s=o), q in L:      sum_k t_p6[k] [d_q (x) [c_o d_o]^k]
  // right growth parts, X = site o, Y = block R
  double dd_swap[2];   // [d_s d_o]^S = dd_swap[S] [d_o (x) d_s]^S
  double cd_swap[2];   // [c_r d_o]^k = cd_swap[k] [d_o (x) c_r]^k
  double u_q1[2];      // U(r=o,s,q), s,q in R: sum_S u_q1[S] [c_o (x) [d_s d_q]^S]
  double u_q2[2];      // U(r,s=o,q):           sum_k u_q2[k] [d_o (x) [c_r d_q]^k]
  double u_q3[2];      // U(r,s,q=o):           sum_k u_q3[k] [d_o (x) [c_r d_s]^k]
  double u_q4[2];      // U(r=o,s=o,q):         sum_k u_q4[k] [[c_o d_o]^k (x) d_q]
  double u_q5[2];      // U(r=o,s,q=o):         sum_k u_q5[k] [[c_o d_o]^k (x) d_s]
  double u_q6[2];      // U(r,s=o,q=o):         sum_S u_q6[S] [[d_o d_o]^S (x) c_r]
};
const SpinConstants& spin_constants();

}  // namespace dmrg
