// dfx_jk_noalloc: the Coulomb and exchange builds of dfx_jk for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  Same kernels as dfx_jk; their
// scratch (the density, the packed density and the Coulomb vectors for J; the
// padded C, the half-transformed chunk X and the SYRK's partial sums for K)
// lives in one file-scope device array instead of the B handle's workspace.
//
// The array is the same for every call on a GPU and keeps the last call's
// contents.  Nothing in it needs to start at zero: every kernel here writes
// what it later reads.  Calls that overlap on one GPU (two streams, two host
// threads) race on it.
#include <map>
#include <mutex>
#include <string>

#include "host.h"

namespace dfx {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)DFX_NOALLOC_SCRATCH_MIB << 20;

// one copy per GPU the library runs on, held until the process ends
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// The array's device address on the current device, taken once per device
// with that device current.  In host code the name `scratch` is only a host
// stand-in: kernels receive this pointer.
static void* scratch_ptr() {
  static std::mutex mu;
  static std::map<int, void*> ptrs;
  int dev = 0;
  DFX_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw Error(DFX_EHIP, std::string("dfx_jk_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                              hipGetErrorString(e));
  ptrs[dev] = p;
  return p;
}

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace dfx

using namespace dfx;

extern "C" {

int dfx_jk_noalloc(const dfx_B* b, const double* dev_C, int nocc, int precision, double* dev_J, double* dev_K,
                   void* stream) {
  return guard([&] {
    if (!b || !dev_C) throw Error(DFX_EINVAL, "dfx_jk_noalloc: NULL argument");
    if (precision < DFX_FP64 || precision > DFX_BF16) throw Error(DFX_EINVAL, "dfx_jk_noalloc: bad precision");
    if (nocc <= 0 || nocc > b->nbf) throw Error(DFX_EINVAL, "dfx_jk_noalloc: bad nocc");
    if (nocc > 512) throw Error(DFX_EUNSUPPORTED, "dfx_jk_noalloc: more than 512 occupied orbitals");
    hipStream_t st = (hipStream_t)stream;
    const int nbf = b->nbf;
    JKArgs a{b->hi.as<float>(), b->lo.as<float>(), b->naux, nbf, b->ncols_t, precision};
    a.ws_cap = NOALLOC_SCRATCH_BYTES;
    // sizes first: nothing is launched unless both builds fit
    const size_t dbytes = up256(sizeof(double) * (size_t)nbf * nbf);
    const size_t jbytes = dev_J ? dbytes + sizeof(double) * (2 * (size_t)b->ncols_t + b->naux + 8) : 0;
    const size_t kbytes = dev_K ? k_work_bytes(a, nocc) : 0;  // DFX_ENOMEM if no chunk fits
    if (jbytes > NOALLOC_SCRATCH_BYTES || kbytes > NOALLOC_SCRATCH_BYTES)
      throw Error(DFX_ENOMEM, "dfx_jk_noalloc: needs " + std::to_string(std::max(jbytes, kbytes)) +
                                  " bytes of scratch, " + std::to_string(NOALLOC_SCRATCH_BYTES) + " available");
    char* w = static_cast<char*>(scratch_ptr());
    if (dev_J) {
      // D = C_occ C_occ^T, then J (Eqs. 3a, 3b) with the Coulomb vectors after it
      double* D = reinterpret_cast<double*>(w);
      GemmF64 g{};
      g.M = nbf; g.N = nbf; g.K = nocc;
      g.A = dev_C; g.lda = nocc;
      g.B = dev_C; g.ldb = nocc; g.tb = true;
      g.C = D; g.ldc = nbf;
      g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
      dgemm(g, st);
      j_build(a, D, dev_J, reinterpret_cast<double*>(w + dbytes), st);
    }
    // K (Eqs. 1a, 2a) reuses the whole array: the stream orders it after J
    if (dev_K) k_build(a, dev_C, nocc, dev_K, w, st);
    DFX_HIP(hipGetLastError());
  });
}

}  // extern "C"
