// Class dispatch for the three-index ERI kernels.
#include "eri3_kernel.h"
#include "kernels.h"

namespace dfx {

void eri3_dispatch(int LA, int LB, int LC, bool unitb, int mode, Eri3Args a, hipStream_t st) {
  if (unitb || mode != STORE_CLASS) throw Error(-6, "eri3: unsupported mode");
  switch (LA * 8 + LB) {
    case 0: eri3_dispatch_pair<0, 0>(LC, a, st); break;
    case 8: eri3_dispatch_pair<1, 0>(LC, a, st); break;
    case 9: eri3_dispatch_pair<1, 1>(LC, a, st); break;
    case 16: eri3_dispatch_pair<2, 0>(LC, a, st); break;
    case 17: eri3_dispatch_pair<2, 1>(LC, a, st); break;
    case 18: eri3_dispatch_pair<2, 2>(LC, a, st); break;
    case 24: eri3_dispatch_pair<3, 0>(LC, a, st); break;
    case 25: eri3_dispatch_pair<3, 1>(LC, a, st); break;
    case 26: eri3_dispatch_pair<3, 2>(LC, a, st); break;
    case 27: eri3_dispatch_pair<3, 3>(LC, a, st); break;
    default: throw Error(-6, "eri3: unsupported orbital angular momentum");
  }
}

}  // namespace dfx
