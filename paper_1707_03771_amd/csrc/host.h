// Host-side runtime of the dfx library: shells, device buffers, screening lists.
#pragma once
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/dfx.h"
#include "kernels.h"

namespace dfx {

// ---- device memory ---------------------------------------------------------
// Sub-allocator over one range of caller-owned device memory: first fit over
// the free blocks, 256-byte aligned, neighbouring free blocks merged.  Pure host
// bookkeeping, no HIP calls.  take() throws DFX_ENOMEM when no free block fits.
class Arena {
 public:
  Arena(void* base, size_t bytes);
  void* take(size_t bytes);
  void give(void* p);
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }
  char* base() const { return base_; }

 private:
  char* base_;
  size_t size_;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
  size_t in_use_ = 0, peak_ = 0;
  std::mutex mu_;
};

// The arena that DevMem::alloc draws from on this thread (null: hipMalloc).
// ArenaScope makes one current for its lifetime and restores the previous.
Arena*& current_arena();
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(current_arena()) { current_arena() = a; }
  ~ArenaScope() { current_arena() = prev; }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
};

struct DevMem {
  void* p = nullptr;
  size_t n = 0;
  Arena* ar = nullptr;  // the arena p came from, if any
  DevMem() = default;
  explicit DevMem(size_t bytes) { alloc(bytes); }
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), n(o.n), ar(o.ar) { o.p = nullptr; o.n = 0; o.ar = nullptr; }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; ar = o.ar; o.p = nullptr; o.n = 0; o.ar = nullptr; }
    return *this;
  }
  ~DevMem() { release(); }
  void alloc(size_t bytes);
  void release();
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

template <class T>
DevMem upload(const std::vector<T>& v, hipStream_t st) {
  DevMem m(std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) DFX_HIP(hipMemcpyAsync(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return m;
}

// ---- shells ------------------------------------------------------------------
struct HostShells {
  int nsh = 0, nbf = 0, lmax = 0;
  std::vector<double> ctr;
  std::vector<int> l, nprim, poff, foff;
  std::vector<double> exps, coef;  // coef multiplies x^i y^j z^k exp(-a r^2)
};
HostShells make_shells(const dfx_shell* s, int n, int lmax_allowed, const char* what);

struct DevShellSet {
  DevMem ctr, l, nprim, poff, foff, exps, coef;
  int nsh = 0;
  void upload(const HostShells& h, hipStream_t st);
  DevShells view() const {
    return DevShells{ctr.as<double>(), l.as<int>(), nprim.as<int>(), poff.as<int>(), foff.as<int>(),
                     exps.as<double>(), coef.as<double>(), nsh};
  }
};

const double* rys_table_device();  // per current device, built on first use

// The calling thread's stream and rocBLAS handle on the current device (scf.hip),
// made on first use and kept until the process ends.
struct DevCtx {
  hipStream_t st = nullptr;
};
DevCtx& thread_ctx();

// K from a symmetric density by signed eigen-factorisation (scf.hip); synchronous
void k_from_density(const JKArgs& a, const double* D, double* K, hipStream_t st);

// learned starting guess (guess.cpp): predicted density, host [nbf][nbf]
void guess_predict_density(const dfx_guess* g, const dfx_geom* geom, double* D, hipStream_t st);
// throws unless the orbital shells are listed atom by atom with the model's shells per element
void guess_check_basis(const dfx_guess* g, const dfx_geom* geom, const dfx_shell* shells, int nsh);

// ---- timing ---------------------------------------------------------------------
struct GpuTimer {
  hipEvent_t a{}, b{};
  hipStream_t st;
  explicit GpuTimer(hipStream_t s) : st(s) {
    DFX_HIP(hipEventCreate(&a));
    DFX_HIP(hipEventCreate(&b));
  }
  ~GpuTimer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  void start() { DFX_HIP(hipEventRecord(a, st)); }
  void stop() { DFX_HIP(hipEventRecord(b, st)); }
  double seconds() {
    DFX_HIP(hipEventSynchronize(b));
    float ms = 0;
    DFX_HIP(hipEventElapsedTime(&ms, a, b));
    return ms * 1e-3;
  }
};

// Accumulates GPU time of repeated intervals: events are recorded on the
// stream and only read once, after the final synchronisation.
struct EventSpans {
  hipStream_t st{};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> spans;
  bool open = false;
  void begin() {
    hipEvent_t a, b;
    DFX_HIP(hipEventCreate(&a));
    DFX_HIP(hipEventCreate(&b));
    DFX_HIP(hipEventRecord(a, st));
    spans.emplace_back(a, b);
    open = true;
  }
  void end() {
    DFX_HIP(hipEventRecord(spans.back().second, st));
    open = false;
  }
  double seconds() {
    double t = 0.0;
    for (auto& p : spans) {
      float ms = 0.0f;
      DFX_HIP(hipEventSynchronize(p.second));
      DFX_HIP(hipEventElapsedTime(&ms, p.first, p.second));
      t += ms * 1e-3;
    }
    return t;
  }
  int count() const { return (int)spans.size(); }
  ~EventSpans() {
    for (auto& p : spans) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  }
};

}  // namespace dfx

// ---- the fitted tensor handle -------------------------------------------------------
struct dfx_B {
  // declared first, destroyed last: every DevMem below may live in it
  std::unique_ptr<dfx::Arena> arena;  // over the caller's workspace (dfx_eri3)
  int device = 0;
  dfx::HostShells bas, aux;
  dfx::DevShellSet dbas, daux;
  int nbf = 0, naux = 0;
  int64_t ncols_t = 0, ncols_p = 0;
  double tau = 1e-12;
  std::vector<int> pa, pb;          // kept pairs (canonical)
  std::vector<int64_t> col_off;     // [npairs + 1]
  std::vector<double> Qab, QC;      // host copies
  dfx::DevMem hi, lo, raw, J2, L;   // device tensors
  dfx::DevMem work;                 // grow-only scratch for dfx_jk
  dfx::DevMem toff;                 // packed column -> tile offset (built on demand)
  // raw's column layout: class cls = 4 max(la, lb) + min(la, lb) holds its pairs
  // (first shell cls_f, the larger l; second cls_s) from column cls_base[cls],
  // component-major: column cls_base + (ma nb + mb) npairs_cls + p
  std::vector<std::vector<int>> cls_f, cls_s;
  std::vector<int64_t> cls_base;    // [17]
  std::vector<int64_t> rawcol;      // canonical packed column -> raw column
  dfx::DevMem rawcol_d;             // (built on demand, for the raw export)
  dfx_B_info info{};
  void* ensure_work(size_t bytes);
};

namespace dfx {
// device bytes of dfx_eri3 inside a caller's workspace (upper bounds)
struct Eri3Need {
  int64_t bytes_B, bytes_raw, bytes_metric;
  int64_t bottom;  // outlives the call: shells, B (hi, lo), J_PQ slot, kept metric / raw
  int64_t setup;   // released before the call returns
  int64_t jk;      // largest dfx_jk work on the result
  int64_t total;   // bottom + max(setup, jk + export map) + fragmentation slack
};
Eri3Need eri3_need(const HostShells& b, const HostShells& a, int flags);
int64_t jk_need(int nbf, int naux, int64_t ncols_t);
// device bytes of dfx_scf / dfx_uhf / dfx_rohf inside a caller's workspace
int64_t scf_need(const HostShells& b, const HostShells& a, int natom, int diis_size);

// internal builders shared by the C-ABI entry points and the SCF driver
std::unique_ptr<dfx_B> build_B(HostShells bas, HostShells aux, double tau, int flags, hipStream_t st);
void int1e_build(const HostShells& h, const dfx_geom* geom, double* S, double* T, double* V,
                 hipStream_t st);

// run f, turning exceptions into a status code and a thread-local message
template <class F>
int guard(F&& f) {
  try {
    f();
    return DFX_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return DFX_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return DFX_EINVAL;
  } catch (...) {
    set_last_error("unknown error");
    return DFX_EINVAL;
  }
}
}  // namespace dfx
