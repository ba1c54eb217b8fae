// Three-index ERI classes (3 1 | LC), LC = 0..4 (see eri3_kernel.h).
#include "eri3_kernel.h"

namespace dfx {

template <>
void eri3_dispatch_pair<3, 1>(int LC, Eri3Args a, hipStream_t st) {
  const dim3 g = eri3_grid(a);
  switch (LC) {
    case 0: eri3_launch_groups<3, 1, 0, false, STORE_CLASS>(a, g, st); break;
    case 1: eri3_launch_groups<3, 1, 1, false, STORE_CLASS>(a, g, st); break;
    case 2: eri3_launch_groups<3, 1, 2, false, STORE_CLASS>(a, g, st); break;
    case 3: eri3_launch_groups<3, 1, 3, false, STORE_CLASS>(a, g, st); break;
    case 4: eri3_launch_groups<3, 1, 4, false, STORE_CLASS>(a, g, st); break;
    default: throw Error(-6, "eri3: unsupported auxiliary angular momentum");
  }
}

}  // namespace dfx
