// Three-index ERI classes (2 2 | LC), LC = 0..4 (see eri3_kernel.h).
#include "eri3_kernel.h"

namespace dfx {

template <>
void eri3_dispatch_pair<2, 2>(int LC, Eri3Args a, hipStream_t st) {
  const dim3 g = eri3_grid(a);
  switch (LC) {
    case 0: eri3_launch_groups<2, 2, 0, false, STORE_CLASS>(a, g, st); break;
    case 1: eri3_launch_groups<2, 2, 1, false, STORE_CLASS>(a, g, st); break;
    case 2: eri3_launch_groups<2, 2, 2, false, STORE_CLASS>(a, g, st); break;
    case 3: eri3_launch_groups<2, 2, 3, false, STORE_CLASS>(a, g, st); break;
    case 4: eri3_launch_groups<2, 2, 4, false, STORE_CLASS>(a, g, st); break;
    default: throw Error(-6, "eri3: unsupported auxiliary angular momentum");
  }
}

}  // namespace dfx
