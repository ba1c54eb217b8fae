// Arguments of the Rys integral kernels (shared by the kernels and the host code).
#pragma once
#include "common.h"

namespace dfx {

// STORE_PACKED: out[P][pcol[pair] + i nb + j], i over the functions of the pair's
// first (higher-index) shell, j over the nb of its second; STORE_DENSE: out[mu][P]
enum { STORE_PACKED = 0, STORE_DENSE = 1 };

struct Eri3Args {
  DevShells F, S, K;         // shells of the first and second bra index and of the ket
  const int* pf;             // [npairs] first bra shell (angular momentum LA)
  const int* ps;             // [npairs] second bra shell (LB); unused with UNITB
  const unsigned char* rowfirst;  // [npairs] 1: first shell indexes rows of B
  const double* pq;          // [npairs] Schwarz factor of the pair, or null
  const int64_t* pcol;       // [npairs] first packed column of the pair (STORE_PACKED)
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
