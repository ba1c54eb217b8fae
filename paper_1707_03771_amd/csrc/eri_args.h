// Arguments of the Rys integral kernels (shared by the kernels and the host code).
#pragma once
#include "common.h"

namespace dfx {

// STORE_CLASS: out[P][cbase + p na nb + ma nb + mb] for pair p of the class
// list, ma over the na functions of its first shell (pf, the larger l), mb over
// the nb of its second: the raw columns of a class, pair by pair, each pair's
// block row-major.  STORE_DENSE: out[mu][P].
enum { STORE_CLASS = 0, STORE_DENSE = 1 };

struct Eri3Args {
  DevShells F, S, K;         // shells of the first and second bra index and of the ket
  const int* pf;             // [npairs] first bra shell (angular momentum LA)
  const int* ps;             // [npairs] second bra shell (LB); unused with UNITB
  const double* pq;          // [npairs] Schwarz factor of the pair, or null
  int64_t cbase;             // first raw column of the class (STORE_CLASS)
  int npairs;
  const int* kl;             // [nk] ket shells of angular momentum LC
  const double* kq;          // [nk] their Schwarz factors
  int nk;
  int kchunk;                // ket shells per workgroup
  double tau;                // screening threshold: evaluate iff Q_ab Q_C >= tau
  double* out;
  int64_t ld;                // row stride of out (elements)
  const double* rys;         // device Rys table
};

}  // namespace dfx
