// Two-centre Coulomb metric (P|Q): the three-index kernel with the second bra
// function replaced by the constant 1 (see eri3_kernel.h).
#include "eri3_kernel.h"

namespace dfx {

#define MCASE(LA, LC)                                                          \
  case (LA)*8 + (LC):                                                          \
    eri3_launch_groups<(LA), 0, (LC), true, STORE_DENSE>(a, g, st);            \
    break;

void metric_dispatch(int LA, int LC, Eri3Args a, hipStream_t st) {
  const dim3 g = eri3_grid(a);
  switch (LA * 8 + LC) {
    MCASE(0, 0) MCASE(0, 1) MCASE(0, 2) MCASE(0, 3) MCASE(0, 4)
    MCASE(1, 0) MCASE(1, 1) MCASE(1, 2) MCASE(1, 3) MCASE(1, 4)
    MCASE(2, 0) MCASE(2, 1) MCASE(2, 2) MCASE(2, 3) MCASE(2, 4)
    MCASE(3, 0) MCASE(3, 1) MCASE(3, 2) MCASE(3, 3) MCASE(3, 4)
    MCASE(4, 0) MCASE(4, 1) MCASE(4, 2) MCASE(4, 3) MCASE(4, 4)
    default:
      throw Error(-6, "metric: unsupported angular momentum class");
  }
}

}  // namespace dfx
