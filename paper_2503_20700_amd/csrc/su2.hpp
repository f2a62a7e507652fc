// SU(2) coupling coefficients: Clebsch-Gordan, Wigner 6j and 9j symbols.
//
// The spin layer is kept apart from the tensor layer (the paper decouples its
// Clebsch-Gordan layer from the MPS layer, Sec. "Conservation of the total
// spin"): every routine here takes doubled spins (2j) as ints and returns a
// double; results are cached.  Closed forms: Racah's formulas for CG and 6j,
// and the 9j as a single sum over products of three 6j symbols.
#pragma once
#include <cstdint>

namespace dmrg {

inline bool tri2(int a, int b, int c) {
  return c >= (a > b ? a - b : b - a) && c <= a + b && ((a + b + c) & 1) == 0;
}

double cg2(int j1, int m1, int j2, int m2, int J, int M);        // <j1 m1; j2 m2 | J M>
double sixj2(int a, int b, int c, int d, int e, int f);            // {a b c; d e f}
double ninej2(int a, int b, int c, int d, int e, int f, int g, int h, int i);

// Reduced matrix element of a coupled product acting on a coupled state,
// in the convention <j m| T^k_q |j' m'> = <j' m'; k q | j m> <j||T||j'>:
//   <(j1 j2) J || [T^k1 (x) U^k2]^k || (j1' j2') J'> =
//     sqrt((2J'+1)(2k+1)(2j1+1)(2j2+1)) {j1 j1' k1; j2 j2' k2; J J' k} <j1||T||j1'><j2||U||j2'>
// (Edmonds' tensor-product rule rewritten for this normalisation; bra labels
// unprimed).  Fermion signs are applied by the caller.
double coupled_factor(int j1b, int j1k, int k1, int j2b, int j2k, int k2, int Jb, int Jk, int k);

}  // namespace dmrg
