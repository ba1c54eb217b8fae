// Derivative integrals of one orbital class (GRAD_LA, GRAD_LB | LC), LC = 0..4,
// for the moved centre GRAD_W and axis GRAD_AX (see grad_kernel.h).  The build
// compiles this file once per combination of the four, so that the heavy
// instantiations build in parallel.
#include "grad_kernel.h"

namespace dfx {

template <>
void grad3_class<GRAD_LA, GRAD_LB, GRAD_W, GRAD_AX>(int LC, GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride,
                                                    hipStream_t st) {
  constexpr int LA = GRAD_LA, LB = GRAD_LB, W = GRAD_W, AX = GRAD_AX;
  switch (LC) {
    case 0: grad_launch_groups<LA, LB, 0, false, W, AX>(ga, grid, pstride, kstride, st); break;
    case 1: grad_launch_groups<LA, LB, 1, false, W, AX>(ga, grid, pstride, kstride, st); break;
    case 2: grad_launch_groups<LA, LB, 2, false, W, AX>(ga, grid, pstride, kstride, st); break;
    case 3: grad_launch_groups<LA, LB, 3, false, W, AX>(ga, grid, pstride, kstride, st); break;
    case 4: grad_launch_groups<LA, LB, 4, false, W, AX>(ga, grid, pstride, kstride, st); break;
    default: throw Error(DFX_EUNSUPPORTED, "gradient: unsupported auxiliary angular momentum");
  }
}

}  // namespace dfx
