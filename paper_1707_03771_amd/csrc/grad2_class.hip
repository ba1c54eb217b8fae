// Derivatives of the metric (P|Q) along axis GRAD_AX for every class (LA | LC),
// LA, LC = 0..4: the derivative kernels with the second bra function the
// constant 1, moving the first auxiliary shell (see grad_kernel.h).  The build
// compiles this file once per axis.
#include "grad_kernel.h"

namespace dfx {

template <>
void grad2_class<GRAD_AX>(int LA, int LC, GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride, hipStream_t st) {
  constexpr int AX = GRAD_AX;
#define G2(A_, C_)                                                                   \
  case A_ * 8 + C_:                                                                  \
    grad_launch_groups<A_, 0, C_, true, 0, AX>(ga, grid, pstride, kstride, st);      \
    break;
  switch (LA * 8 + LC) {
    G2(0, 0) G2(0, 1) G2(0, 2) G2(0, 3) G2(0, 4)
    G2(1, 0) G2(1, 1) G2(1, 2) G2(1, 3) G2(1, 4)
    G2(2, 0) G2(2, 1) G2(2, 2) G2(2, 3) G2(2, 4)
    G2(3, 0) G2(3, 1) G2(3, 2) G2(3, 3) G2(3, 4)
    G2(4, 0) G2(4, 1) G2(4, 2) G2(4, 3) G2(4, 4)
    default: throw Error(DFX_EUNSUPPORTED, "metric gradient: unsupported angular momentum");
  }
#undef G2
}

}  // namespace dfx
