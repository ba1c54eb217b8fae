// C-ABI entry points of libdfx.so (include/dfx.h) and the host runtime behind them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "host.h"
#include "rys.h"

namespace dfx {

static thread_local std::string g_err;
void set_last_error(const std::string& m) { g_err = m; }

// ---- device memory ------------------------------------------------------------------
static constexpr size_t ARENA_ALIGN = 256;

Arena::Arena(void* base, size_t bytes) : base_(static_cast<char*>(base)), size_(0) {
  // start and length trimmed to the alignment
  const uintptr_t b = reinterpret_cast<uintptr_t>(base_);
  const size_t skip = (ARENA_ALIGN - b % ARENA_ALIGN) % ARENA_ALIGN;
  if (bytes > skip) {
    base_ += skip;
    size_ = (bytes - skip) / ARENA_ALIGN * ARENA_ALIGN;
  }
  if (size_) free_[0] = size_;
}

void* Arena::take(size_t bytes) {
  const size_t need = std::max<size_t>(ARENA_ALIGN, (bytes + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN);
  std::lock_guard<std::mutex> g(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > need) free_[off + need] = len - need;
    used_[off] = need;
    in_use_ += need;
    peak_ = std::max(peak_, in_use_);
    return base_ + off;
  }
  throw Error(DFX_ENOMEM, "workspace too small: no free block of " + std::to_string(need) + " bytes (" +
                              std::to_string(in_use_) + " of " + std::to_string(size_) + " bytes in use)");
}

void Arena::give(void* p) {
  std::lock_guard<std::mutex> g(mu_);
  const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t start = off, len = u->second;
  in_use_ -= len;
  used_.erase(u);
  auto nx = free_.lower_bound(start);
  if (nx != free_.end() && nx->first == start + len) {  // merge with the next free block
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // and with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == start) {
      start = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = len;
}

Arena*& current_arena() {
  static thread_local Arena* a = nullptr;
  return a;
}

void DevMem::alloc(size_t bytes) {
  release();
  if (bytes == 0) return;
  if (Arena* a = current_arena()) {
    p = a->take(bytes);
    ar = a;
    n = bytes;
    return;
  }
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error(DFX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  n = bytes;
}
void DevMem::release() {
  if (p) {
    if (ar)
      ar->give(p);
    else
      (void)hipFree(p);
  }
  p = nullptr;
  n = 0;
  ar = nullptr;
}

// ---- shells ---------------------------------------------------------------------------
// Primitive normalisation for r^l Y_lm exp(-a r^2) with Y_lm orthonormal:
// N^2 Gamma(l + 3/2) / (2 (2a)^(l + 3/2)) = 1.  The contraction is renormalised
// with the overlap of normalised primitives, (2 sqrt(a b) / (a + b))^(l + 3/2).
HostShells make_shells(const dfx_shell* s, int n, int lmax_allowed, const char* what) {
  if (n < 0 || (n > 0 && !s)) throw Error(DFX_EINVAL, std::string(what) + ": bad shell array");
  HostShells h;
  h.nsh = n;
  int f = 0, pcount = 0;
  for (int i = 0; i < n; ++i) {
    const dfx_shell& sh = s[i];
    if (sh.l < 0 || sh.nprim < 1 || !sh.exps || !sh.coefs)
      throw Error(DFX_EINVAL, std::string(what) + ": shell " + std::to_string(i) + " malformed");
    if (sh.l > lmax_allowed)
      throw Error(DFX_EUNSUPPORTED, std::string(what) + ": shell " + std::to_string(i) + " has l = " +
                                        std::to_string(sh.l) + " > " + std::to_string(lmax_allowed));
    const int l = sh.l;
    for (int k = 0; k < 3; ++k) h.ctr.push_back(sh.xyz[k]);
    h.l.push_back(l);
    h.nprim.push_back(sh.nprim);
    h.poff.push_back(pcount);
    h.foff.push_back(f);
    double norm2 = 0.0;
    for (int a = 0; a < sh.nprim; ++a)
      for (int b = 0; b < sh.nprim; ++b) {
        const double ea = sh.exps[a], eb = sh.exps[b];
        norm2 += sh.coefs[a] * sh.coefs[b] * std::pow(2.0 * std::sqrt(ea * eb) / (ea + eb), l + 1.5);
      }
    if (!(norm2 > 0.0)) throw Error(DFX_EINVAL, std::string(what) + ": zero-norm contraction");
    for (int a = 0; a < sh.nprim; ++a) {
      const double ea = sh.exps[a];
      if (!(ea > 0.0)) throw Error(DFX_EINVAL, std::string(what) + ": non-positive exponent");
      const double N = std::sqrt(2.0 * std::pow(2.0 * ea, l + 1.5) / std::tgamma(l + 1.5));
      h.exps.push_back(ea);
      h.coef.push_back(sh.coefs[a] * N / std::sqrt(norm2));
    }
    pcount += sh.nprim;
    f += 2 * l + 1;
    h.lmax = std::max(h.lmax, l);
  }
  h.nbf = f;
  return h;
}

void DevShellSet::upload(const HostShells& h, hipStream_t st) {
  nsh = h.nsh;
  ctr = dfx::upload(h.ctr, st);
  l = dfx::upload(h.l, st);
  nprim = dfx::upload(h.nprim, st);
  poff = dfx::upload(h.poff, st);
  foff = dfx::upload(h.foff, st);
  exps = dfx::upload(h.exps, st);
  coef = dfx::upload(h.coef, st);
}

// ---- Rys table image -----------------------------------------------------------------------
static const double RYS_COEFS[RYS_TABLE_SIZE] = RYS_TABLE_INIT;

void rys_host_image(double* out) {
  int src = 0;
  for (int n = 1; n <= RYS_NMAX; ++n) {
    const int nc = 2 * n * (RYS_DEG + 1);  // coefficients of one interval
    double* dst = out + rys_dev_off(n);
    for (int k = 0; k < RYS_NINT[n]; ++k) {
      std::memcpy(dst + (size_t)k * rys_blk(n), RYS_COEFS + src, sizeof(double) * nc);
      for (int j = nc; j < rys_blk(n); ++j) dst[(size_t)k * rys_blk(n) + j] = 0.0;
      src += nc;
    }
    double* lim = dst + (size_t)RYS_NINT[n] * rys_blk(n);
    for (int i = 0; i < n; ++i) {
      lim[i] = RYS_X2[n][i];
      lim[n + i] = RYS_W[n][i];
    }
  }
}

const double* rys_table_device() {
  static std::mutex mu;
  static std::map<int, double*> tabs;
  int dev = 0;
  DFX_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = tabs.find(dev);
  if (it != tabs.end()) return it->second;
  std::vector<double> img(RYS_DEV_TOTAL);
  rys_host_image(img.data());
  double* d = nullptr;
  DFX_HIP(hipMalloc(&d, sizeof(double) * img.size()));
  DFX_HIP(hipMemcpy(d, img.data(), sizeof(double) * img.size(), hipMemcpyHostToDevice));
  tabs[dev] = d;
  return d;
}

// ---- screening lists ---------------------------------------------------------------------------
static int64_t count_kept(double qab, const std::vector<double>& qc_sorted, double tau) {
  // qc_sorted ascending; fl(qab * x) is monotone in x for qab > 0
  if (!(qab > 0.0)) return tau <= 0.0 ? (int64_t)qc_sorted.size() : 0;
  auto it = std::partition_point(qc_sorted.begin(), qc_sorted.end(),
                                 [&](double x) { return !(qab * x >= tau); });
  return (int64_t)(qc_sorted.end() - it);
}

// (P|Q) for every (P, Q) auxiliary shell combination, both orders, dense.
static void compute_metric(const DevShellSet& daux, const std::vector<std::vector<int>>& auxby,
                           const std::vector<DevMem>& auxby_d, double* out, int naux, const double* rys,
                           hipStream_t st) {
  for (int la = 0; la <= 4; ++la)
    for (int lc = 0; lc <= 4; ++lc) {
      if (auxby[la].empty() || auxby[lc].empty()) continue;
      Eri3Args a{};
      a.F = daux.view();
      a.S = daux.view();
      a.K = daux.view();
      a.pf = auxby_d[la].as<int>();
      a.npairs = (int)auxby[la].size();
      a.kl = auxby_d[lc].as<int>();
      a.nk = (int)auxby[lc].size();
      a.tau = -1.0;
      a.out = out;
      a.ld = naux;
      a.rys = rys;
      metric_dispatch(la, lc, a, st);
    }
  DFX_HIP(hipGetLastError());
}

}  // namespace dfx

using namespace dfx;

// ---- workspace sizes (upper bounds; host arithmetic only) ---------------------------
static int64_t pad256(int64_t b) { return (b + 255) / 256 * 256; }

static int64_t shells_bytes(const HostShells& h) {
  return 7 * 256 + pad256(24 * (int64_t)h.nsh) + 4 * pad256(4 * (int64_t)h.nsh) +
         2 * pad256(8 * (int64_t)h.exps.size());
}

// columns of raw if no pair were screened: sum over a >= b of n_a n_b
static int64_t cols_bound(const HostShells& b) {
  int64_t s = 0, d = 0;
  for (int a = 0; a < b.nsh; ++a) {
    const int64_t na = 2 * b.l[a] + 1;
    s += na;
    d += na * na;
  }
  return (s * s + d) / 2;
}

// largest dfx_jk work on a B of these sizes: any kind and precision, nocc <= 512
int64_t dfx::jk_need(int nbf, int naux, int64_t ncols_t) {
  const int64_t n2 = (int64_t)nbf * nbf;
  int64_t kmax = 0;
  for (int p = PREC_FP64; p <= PREC_BF16; ++p) {
    const JKArgs a{nullptr, nullptr, naux, nbf, ncols_t, p};
    for (int nocc = 1; nocc <= std::min(nbf, 512); ++nocc) kmax = std::max<int64_t>(kmax, k_work_bytes(a, nocc));
  }
  const int64_t jw = pad256(8 * (2 * ncols_t + naux + 8)) + pad256(8 * n2);
  // the density route adds its eigen-decomposition (and eigenvectors), one K
  // and a chunk of 512 columns
  const int64_t dens = pad256(8 * n2) * 2 + pad256(8 * (int64_t)nbf) + pad256(8 * (int64_t)nbf * 512) +
                       pad256(512 * 4) + pad256(512 * 8) + pad256(kmax) + pad256(sym_eig_work_bytes(nbf));
  return pad256(std::max(jw, kmax)) + dens;
}

dfx::Eri3Need dfx::eri3_need(const HostShells& b, const HostShells& a, int flags) {
  Eri3Need z{};
  const int64_t nbf = b.nbf, naux = a.nbf, nsh = b.nsh, nauxsh = a.nsh;
  const int64_t nct = tiled_cols((int)nbf), ncb = cols_bound(b);
  const int64_t m2 = pad256(8 * naux * naux), raw = pad256(8 * naux * ncb);
  const int64_t npall = nsh * (nsh + 1) / 2;
  z.bytes_B = 2 * pad256(4 * naux * nct);
  z.bytes_raw = raw;
  z.bytes_metric = 2 * m2;
  z.bottom = shells_bytes(b) + shells_bytes(a) + z.bytes_B + m2 + ((flags & DFX_KEEP_METRIC) ? m2 : 0) +
             ((flags & DFX_KEEP_RAW) ? raw : 0);
  const int64_t lists = 16 * npall + 25 * npall + 20 * nauxsh + 256 * 256;
  // raw itself, or its working copy when raw is kept; L when not kept; the
  // Cholesky work (also the solve's packed diagonal blocks) and the tile map
  z.setup = lists + raw + ((flags & DFX_KEEP_METRIC) ? 0 : m2) +
            pad256(8 * (int64_t)cholesky_work_elems((int)naux)) + 256 + std::max(2 * pad256(8 * ncb), pad256(8 * nct));
  z.jk = jk_need((int)nbf, (int)naux, nct);
  const int64_t top = std::max(z.setup, z.jk + pad256(8 * ncb));
  z.total = z.bottom + top + top / 64 + ((int64_t)16 << 20);
  return z;
}

int64_t dfx::scf_need(const HostShells& b, const HostShells& a, int natom, int diis_size) {
  const Eri3Need e = eri3_need(b, a, 0);
  const int64_t n = b.nbf, n2 = pad256(8 * n * n);
  // the SCF's dense matrices (open shell: both spins, 2 x diis_size entries each
  // for the Fock matrices and errors), their thin companions and small buffers
  const int64_t mats = (26 + 4 * (int64_t)diis_size) * n2 + 8 * pad256(8 * n * 512) + 512 * 256 +
                       pad256(sym_eig_work_bytes((int)n));  // eigen-decompositions (eig.hip)
  // learned guess: per pair-type inputs, outputs and network work, FP32
  const int64_t guess = (int64_t)natom * natom * 4 * 9842 + ((int64_t)1 << 20);
  const int64_t pre = 4 * n2 + 3 * 256;  // split-K partials and small buffers made before B
  const int64_t top = std::max(e.setup + pre, mats + guess + e.jk);
  return e.bottom + top + top / 64 + ((int64_t)16 << 20);
}

void* dfx_B::ensure_work(size_t bytes) {
  if (work.n < bytes) work.alloc(bytes);
  return work.p;
}

// ===========================================================================
extern "C" {

const char* dfx_last_error(void) { return g_err.c_str(); }

}  // extern "C"

std::unique_ptr<dfx_B> dfx::build_B(HostShells bas, HostShells auxs, double tau_, int flags,
                                     hipStream_t st) {
    std::unique_ptr<dfx_B> B(new dfx_B());
    B->tau = tau_;
    B->bas = std::move(bas);
    B->aux = std::move(auxs);
    const int nsh = B->bas.nsh, nauxsh = B->aux.nsh;
    DFX_HIP(hipGetDevice(&B->device));
    B->nbf = B->bas.nbf;
    B->naux = B->aux.nbf;
    B->dbas.upload(B->bas, st);
    B->daux.upload(B->aux, st);
    const double* rys = rys_table_device();
    const int nbf = B->nbf, naux = B->naux;
    B->ncols_t = tiled_cols(nbf);
    // What outlives this call first, at the bottom of a caller's workspace: B's
    // two words (every element written by the split below), then the metric and
    // its factor when kept.  Everything allocated after them is released before
    // returning, into one contiguous free block.
    B->hi.alloc(sizeof(float) * (size_t)naux * B->ncols_t);
    B->lo.alloc(sizeof(float) * (size_t)naux * B->ncols_t);
    B->J2.alloc(sizeof(double) * naux * (size_t)naux);
    if (flags & DFX_KEEP_METRIC) B->L.alloc(sizeof(double) * naux * (size_t)naux);
    GpuTimer tm(st);

    // -- metric J_PQ = (P|Q)
    tm.start();
    std::vector<std::vector<int>> auxby(5);
    for (int c = 0; c < nauxsh; ++c) auxby[B->aux.l[c]].push_back(c);
    std::vector<DevMem> auxby_d(5);
    for (int l = 0; l <= 4; ++l) auxby_d[l] = upload(auxby[l], st);
    compute_metric(B->daux, auxby, auxby_d, B->J2.as<double>(), naux, rys, st);
    DevMem qc_d(sizeof(double) * nauxsh);
    aux_schwarz(B->J2.as<double>(), naux, B->daux.view(), qc_d.as<double>(), st);

    // -- Schwarz factors of all orbital shell pairs a >= b
    std::vector<std::vector<int>> sp_f(16), sp_s(16), sp_a(16), sp_b(16);
    for (int a = 0; a < nsh; ++a)
      for (int b = 0; b <= a; ++b) {
        const int la = B->bas.l[a], lb = B->bas.l[b];
        const int f = la >= lb ? a : b, s = la >= lb ? b : a;
        const int cls = std::max(la, lb) * 4 + std::min(la, lb);
        sp_f[cls].push_back(f);
        sp_s[cls].push_back(s);
        sp_a[cls].push_back(a);
        sp_b[cls].push_back(b);
      }
    std::vector<DevMem> sq(16), sf(16), ss(16);
    for (int cls = 0; cls < 16; ++cls) {
      if (sp_f[cls].empty()) continue;
      sf[cls] = upload(sp_f[cls], st);
      ss[cls] = upload(sp_s[cls], st);
      sq[cls].alloc(sizeof(double) * sp_f[cls].size());
      SchwarzArgs a{};
      a.sh = B->dbas.view();
      a.pf = sf[cls].as<int>();
      a.ps = ss[cls].as<int>();
      a.npairs = (int)sp_f[cls].size();
      a.q = sq[cls].as<double>();
      a.rys = rys;
      schwarz_dispatch(cls / 4, cls % 4, a, st);
    }
    DFX_HIP(hipGetLastError());
    B->Qab.assign((size_t)nsh * nsh, 0.0);
    B->QC.assign(nauxsh, 0.0);
    DFX_HIP(hipMemcpyAsync(B->QC.data(), qc_d.p, sizeof(double) * nauxsh, hipMemcpyDeviceToHost, st));
    std::vector<std::vector<double>> qhost(16);
    for (int cls = 0; cls < 16; ++cls) {
      if (sp_f[cls].empty()) continue;
      qhost[cls].resize(sp_f[cls].size());
      DFX_HIP(hipMemcpyAsync(qhost[cls].data(), sq[cls].p, sizeof(double) * qhost[cls].size(),
                             hipMemcpyDeviceToHost, st));
    }
    DFX_HIP(hipStreamSynchronize(st));
    for (int cls = 0; cls < 16; ++cls)
      for (size_t k = 0; k < sp_a[cls].size(); ++k) {
        const int a = sp_a[cls][k], b = sp_b[cls][k];
        B->Qab[(size_t)a * nsh + b] = B->Qab[(size_t)b * nsh + a] = qhost[cls][k];
      }

    // -- kept pairs (canonical order) and per-class work lists
    const double tau = B->tau;
    const double qcmax = *std::max_element(B->QC.begin(), B->QC.end());
    B->col_off.assign(1, 0);
    std::vector<double> qc_sorted = B->QC;
    std::vector<std::vector<double>> qc_by_l(5);
    for (int c = 0; c < nauxsh; ++c) qc_by_l[B->aux.l[c]].push_back(B->QC[c]);
    for (auto& v : qc_by_l) std::sort(v.begin(), v.end());
    std::vector<std::vector<int>>& cf = B->cls_f;
    std::vector<std::vector<int>>& cs = B->cls_s;
    cf.assign(16, {});
    cs.assign(16, {});
    std::vector<std::vector<double>> cq(16);
    std::vector<int> kcls, kidx;  // class and position in it of every kept pair
    int64_t ntrip = 0, nint = 0;
    for (int a = 0; a < nsh; ++a)
      for (int b = 0; b <= a; ++b) {
        const double q = B->Qab[(size_t)a * nsh + b];
        if (!(q * qcmax >= tau)) continue;
        B->pa.push_back(a);
        B->pb.push_back(b);
        const int na = 2 * B->bas.l[a] + 1, nb = 2 * B->bas.l[b] + 1;
        const int64_t first_col = B->col_off.back();
        B->col_off.push_back(first_col + (int64_t)na * nb);
        const int la = B->bas.l[a], lb = B->bas.l[b];
        const int cls = std::max(la, lb) * 4 + std::min(la, lb);
        kcls.push_back(cls);
        kidx.push_back((int)cf[cls].size());
        cf[cls].push_back(la >= lb ? a : b);
        cs[cls].push_back(la >= lb ? b : a);
        cq[cls].push_back(q);
        const int64_t uniq = (a == b) ? (int64_t)na * (na + 1) / 2 : (int64_t)na * nb;
        for (int lc = 0; lc <= 4; ++lc) {
          const int64_t k = count_kept(q, qc_by_l[lc], tau);
          ntrip += k;
          nint += k * uniq * (2 * lc + 1);
        }
      }
    B->ncols_p = B->col_off.back();
    // raw's columns class by class, pair by pair, each pair's block row-major in
    // (first shell, second shell) (the ERI stores of a wave fill one contiguous
    // block); canonical column -> raw column for export
    B->cls_base.assign(17, 0);
    for (int cls = 0; cls < 16; ++cls)
      B->cls_base[cls + 1] = B->cls_base[cls] + (int64_t)cf[cls].size() * (2 * (cls / 4) + 1) * (2 * (cls % 4) + 1);
    B->rawcol.resize(B->ncols_p);
    for (size_t k = 0; k < B->pa.size(); ++k) {
      const int a = B->pa[k], b = B->pb[k], cls = kcls[k], pos = kidx[k];
      const int na = 2 * B->bas.l[a] + 1, nb = 2 * B->bas.l[b] + 1;
      const bool afirst = B->bas.l[a] >= B->bas.l[b];
      const int SB = 2 * (cls % 4) + 1, SASB = (2 * (cls / 4) + 1) * SB;
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          const int ma = afirst ? i : j, mb = afirst ? j : i;
          B->rawcol[B->col_off[k] + (int64_t)i * nb + j] = B->cls_base[cls] + (int64_t)pos * SASB + (ma * SB + mb);
        }
    }

    // -- raw (mu nu|P), aux-major, packed pair columns; every element is written
    // by the class launches below (screened triplets as zeros), so no clearing
    B->raw.alloc(sizeof(double) * (size_t)naux * B->ncols_p);
    std::vector<DevMem> qcl_d(5);
    for (int l = 0; l <= 4; ++l) {
      std::vector<double> q;
      for (int c : auxby[l]) q.push_back(B->QC[c]);
      qcl_d[l] = upload(q, st);
    }
    std::vector<DevMem> cf_d(16), cs_d(16), cq_d(16);
    for (int cls = 0; cls < 16; ++cls) {
      if (cf[cls].empty()) continue;
      cf_d[cls] = upload(cf[cls], st);
      cs_d[cls] = upload(cs[cls], st);
      cq_d[cls] = upload(cq[cls], st);
    }
    tm.stop();
    const double t_metric0 = tm.seconds();
    GpuTimer te(st);
    te.start();
    // The (class, l_C) launches write disjoint blocks of raw: they run on NSTR
    // streams forked from and joined back to st, most expensive first, each on
    // the least loaded stream, so that short launches fill the others' tails.
    // Three: HIP's default of four hardware queues per process, with the
    // caller's stream on one, leaves three; a fourth side stream shared a queue
    // with another and ran serialised behind it.
    // The side streams and events belong to the calling thread on this device,
    // made on first use and kept until the process ends.
    constexpr int NSTR = 3;
    struct ForkRes {
      hipStream_t s[NSTR] = {};
      hipEvent_t ev[NSTR + 1] = {};
    };
    struct Fork {
      ForkRes& r;
      hipStream_t main;
      hipStream_t* s;
      static ForkRes& res() {
        static thread_local std::map<int, ForkRes> all;
        int dev = 0;
        DFX_HIP(hipGetDevice(&dev));
        ForkRes& x = all[dev];
        if (!x.s[0]) {
          for (int i = 0; i < NSTR; ++i) DFX_HIP(hipStreamCreateWithFlags(&x.s[i], hipStreamNonBlocking));
          for (int i = 0; i <= NSTR; ++i) DFX_HIP(hipEventCreateWithFlags(&x.ev[i], hipEventDisableTiming));
        }
        return x;
      }
      explicit Fork(hipStream_t m) : r(res()), main(m), s(r.s) {
        DFX_HIP(hipEventRecord(r.ev[NSTR], main));
        for (int i = 0; i < NSTR; ++i) DFX_HIP(hipStreamWaitEvent(s[i], r.ev[NSTR], 0));
      }
      void join() {
        for (int i = 0; i < NSTR; ++i) {
          DFX_HIP(hipEventRecord(r.ev[i], s[i]));
          DFX_HIP(hipStreamWaitEvent(main, r.ev[i], 0));
        }
      }
      ~Fork() { (void)hipStreamSynchronize(main); }
    } fork(st);
    struct Launch {
      double cost;
      int cls, lc;
    };
    std::vector<Launch> launches;
    for (int cls = 0; cls < 16; ++cls) {
      if (cf[cls].empty()) continue;
      const int la = cls / 4, lb = cls % 4;
      for (int lc = 0; lc <= 4; ++lc) {
        if (auxby[lc].empty()) continue;
        const double roots = (la + lb + lc) / 2 + 1;
        launches.push_back({(double)cf[cls].size() * auxby[lc].size() * ncart(la) * ncart(lb) * ncart(lc) * roots,
                            cls, lc});
      }
    }
    std::sort(launches.begin(), launches.end(), [](const Launch& x, const Launch& y) { return x.cost > y.cost; });
    double load[NSTR] = {};
    for (const Launch& L : launches) {
      const int cls = L.cls, lc = L.lc;
      const int k = (int)(std::min_element(load, load + NSTR) - load);
      load[k] += L.cost;
      {
        Eri3Args a{};
        a.F = B->dbas.view();
        a.S = B->dbas.view();
        a.K = B->daux.view();
        a.pf = cf_d[cls].as<int>();
        a.ps = cs_d[cls].as<int>();
        a.pq = cq_d[cls].as<double>();
        a.cbase = B->cls_base[cls];
        a.npairs = (int)cf[cls].size();
        a.kl = auxby_d[lc].as<int>();
        a.kq = qcl_d[lc].as<double>();
        a.nk = (int)auxby[lc].size();
        a.tau = tau;
        a.out = B->raw.as<double>();
        a.ld = B->ncols_p;
        a.rys = rys;
        eri3_dispatch(cls / 4, cls % 4, lc, false, STORE_CLASS, a, fork.s[k]);
      }
    }
    DFX_HIP(hipGetLastError());
    fork.join();
    te.stop();
    B->info.eri_seconds = te.seconds();

    // -- Cholesky of the metric and L^-1
    DevMem Lw;  // L, factored in place (in B->L when kept)
    if (!(flags & DFX_KEEP_METRIC)) Lw.alloc(sizeof(double) * (size_t)naux * naux);
    double* Lp = (flags & DFX_KEEP_METRIC) ? B->L.as<double>() : Lw.as<double>();
    DevMem cw(sizeof(double) * cholesky_work_elems(naux));
    DevMem info_d(sizeof(int));
    GpuTimer tc(st);
    tc.start();
    DFX_HIP(hipMemcpyAsync(Lp, B->J2.p, sizeof(double) * (size_t)naux * naux, hipMemcpyDeviceToDevice, st));
    cholesky_factor(Lp, naux, cw.as<double>(), info_d.as<int>(), st);
    int info = 0;
    DFX_HIP(hipMemcpyAsync(&info, info_d.p, sizeof(int), hipMemcpyDeviceToHost, st));
    tc.stop();
    B->info.metric_seconds = t_metric0 + tc.seconds();
    if (info != 0)
      throw Error(DFX_ENOTPOSDEF, "fitting metric is not positive definite (pivot " + std::to_string(info - 1) + ")");
    {
      std::vector<double> diag(naux);
      DFX_HIP(hipMemcpy2DAsync(diag.data(), sizeof(double), Lp, sizeof(double) * (naux + 1),
                               sizeof(double), naux, hipMemcpyDeviceToHost, st));
      DFX_HIP(hipStreamSynchronize(st));
      const auto mm = std::minmax_element(diag.begin(), diag.end());
      B->info.kappa_lb = (*mm.second / *mm.first) * (*mm.second / *mm.first);
    }

    // -- B = L^-1 raw over raw's columns, split into FP32 hi / lo in the tiled
    // layout.  src[t] is the raw column that tile element t takes: a pair block's
    // element (mu, nu) goes to row max, column min of its lower tile, and inside
    // a diagonal tile also to the mirror position; of the duplicate columns (i, j)
    // and (j, i) of a diagonal shell pair only i >= j is used.  Elements of
    // screened pairs and of the padding take none (zero).
    std::vector<int64_t> src(B->ncols_t, -1);
    auto take = [&](int64_t t, int64_t col) {
      if (src[t] >= 0) throw Error(DFX_EINVAL, "eri3: two pair columns map to one tile element");
      src[t] = col;
    };
    for (int cls = 0; cls < 16; ++cls) {
      const int SA = 2 * (cls / 4) + 1, SB = 2 * (cls % 4) + 1;
      const int64_t npc = (int64_t)cf[cls].size();
      for (int64_t p = 0; p < npc; ++p) {
        const int f = cf[cls][p], sh = cs[cls][p];
        for (int ma = 0; ma < SA; ++ma)
          for (int mb = 0; mb < SB; ++mb) {
            const int64_t col = B->cls_base[cls] + p * (SA * SB) + (ma * SB + mb);
            const int mu = B->bas.foff[f] + ma, nu = B->bas.foff[sh] + mb;
            if (f == sh && mu < nu) continue;  // the other triangle of a diagonal block: a duplicate
            const int r = std::max(mu, nu), c = std::min(mu, nu);
            const int I = r >> 5, J = c >> 5;
            take(tile_base(I, J) + ((r & 31) << 5) + (c & 31), col);
            if (I == J && r != c) take(tile_base(I, J) + ((c & 31) << 5) + (r & 31), col);
          }
      }
    }
    DevMem src_d = upload(src, st);
    // B = L^-1 raw by blocked forward substitution, in place (on a copy when the
    // raw integrals are kept), then split into the two FP32 words.  The timed
    // span holds these launches and nothing else; the update products are also
    // timed on their own.
    DevMem rawcopy;
    double* Bw = B->raw.as<double>();
    if (flags & DFX_KEEP_RAW) {
      rawcopy.alloc(B->raw.n);
      DFX_HIP(hipMemcpyAsync(rawcopy.p, B->raw.p, B->raw.n, hipMemcpyDeviceToDevice, st));
      Bw = rawcopy.as<double>();
    }
    struct UpdTimer : TrsmTimer {
      EventSpans sp;
      void begin() override { sp.begin(); }
      void end() override { sp.end(); }
    } ut;
    ut.sp.st = st;
    GpuTimer tt(st);
    tt.start();
    // the Cholesky work (at least 65 naux doubles) holds the packed diagonal blocks
    if (cw.n < sizeof(double) * trsm_work_elems(naux)) throw Error(-1, "eri3: Cholesky work too small for the solve");
    const TrsmStats ts = trsm_solve(Lp, naux, Bw, B->ncols_p, cw.as<double>(), st, &ut);
    tile_split(Bw, naux, B->ncols_p, src_d.as<int64_t>(), B->hi.as<float>(), B->lo.as<float>(), B->ncols_t, st);
    DFX_HIP(hipGetLastError());
    tt.stop();
    B->info.trsm_seconds = tt.seconds();
    B->info.trsm_update_seconds = ut.sp.seconds();
    B->info.trsm_update_flops = ts.update_flops;
    B->info.trsm_update_launches = ts.update_launches;
    cw.release();
    if (!(flags & DFX_KEEP_METRIC)) B->J2.release();
    if (!(flags & DFX_KEEP_RAW)) B->raw.release();
    DFX_HIP(hipStreamSynchronize(st));

    dfx_B_info& I = B->info;
    I.nbf = nbf;
    I.naux = naux;
    I.nsh = nsh;
    I.nauxsh = nauxsh;
    I.npairs = (int)B->pa.size();
    I.ncols = B->ncols_p;
    I.ncols_tiled = B->ncols_t;
    I.ntriplets = ntrip;
    I.nintegrals = nint;
    return B;
}

extern "C" {

int dfx_eri3(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, const dfx_eri3_opts* opts,
             void* dev_workspace, size_t ws_bytes, void* stream, dfx_B** out) {
  return guard([&] {
    if (!out) throw Error(DFX_EINVAL, "dfx_eri3: out is NULL");
    *out = nullptr;
    if (nsh <= 0 || nauxsh <= 0) throw Error(DFX_EINVAL, "dfx_eri3: empty basis");
    HostShells b = make_shells(shells, nsh, 3, "orbital basis");
    HostShells a = make_shells(aux, nauxsh, 4, "auxiliary basis");
    if (!dev_workspace) throw Error(DFX_EINVAL, "dfx_eri3: no workspace (size it with dfx_eri3_plan)");
    const int flags = opts ? opts->flags : 0;
    const Eri3Need need = eri3_need(b, a, flags);
    if ((int64_t)ws_bytes < need.total)
      throw Error(DFX_ENOMEM, "dfx_eri3: workspace of " + std::to_string(ws_bytes) + " bytes, " +
                                  std::to_string(need.total) + " needed (dfx_eri3_plan)");
    auto arena = std::make_unique<Arena>(dev_workspace, ws_bytes);
    std::unique_ptr<dfx_B> B;
    {
      ArenaScope scope(arena.get());
      B = build_B(std::move(b), std::move(a), opts ? opts->tau : 1e-12, flags, (hipStream_t)stream);
    }
    B->arena = std::move(arena);
    *out = B.release();
  });
}

int dfx_metric(const dfx_shell* aux, int nauxsh, double* dev_J, void* stream) {
  return guard([&] {
    if (!dev_J || nauxsh <= 0) throw Error(DFX_EINVAL, "dfx_metric: bad argument");
    hipStream_t st = (hipStream_t)stream;
    HostShells h = make_shells(aux, nauxsh, 4, "auxiliary basis");
    DevShellSet d;
    d.upload(h, st);
    std::vector<std::vector<int>> auxby(5);
    for (int c = 0; c < nauxsh; ++c) auxby[h.l[c]].push_back(c);
    std::vector<DevMem> auxby_d(5);
    for (int l = 0; l <= 4; ++l) auxby_d[l] = upload(auxby[l], st);
    compute_metric(d, auxby, auxby_d, dev_J, h.nbf, rys_table_device(), st);
    DFX_HIP(hipStreamSynchronize(st));
  });
}

int dfx_cholesky(double* dev_A, int n, double* dev_Linv, void* stream) {
  return guard([&] {
    if (!dev_A || !dev_Linv || n <= 0) throw Error(DFX_EINVAL, "dfx_cholesky: bad argument");
    hipStream_t st = (hipStream_t)stream;
    DevMem cw(sizeof(double) * cholesky_work_elems(n));
    DevMem info_d(sizeof(int));
    cholesky_inverse(dev_A, n, dev_Linv, cw.as<double>(), info_d.as<int>(), st);
    int info = 0;
    DFX_HIP(hipMemcpyAsync(&info, info_d.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    if (info != 0) throw Error(DFX_ENOTPOSDEF, "matrix is not positive definite (pivot " + std::to_string(info - 1) + ")");
  });
}

int dfx_eigh(double* dev_A, int n, double* dev_w, int* sweeps, void* stream) {
  return guard([&] {
    if (!dev_A || !dev_w || n <= 0) throw Error(DFX_EINVAL, "dfx_eigh: bad argument");
    const int s = sym_eig(dev_A, n, dev_w, (hipStream_t)stream);
    if (sweeps) *sweeps = s;
  });
}

int dfx_eri3_plan(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, const dfx_eri3_opts* opts,
                  dfx_eri3_sizes* out) {
  return guard([&] {
    if (!out) throw Error(DFX_EINVAL, "dfx_eri3_plan: out is NULL");
    if (nsh <= 0 || nauxsh <= 0) throw Error(DFX_EINVAL, "dfx_eri3_plan: empty basis");
    const HostShells b = make_shells(shells, nsh, 3, "orbital basis");
    const HostShells a = make_shells(aux, nauxsh, 4, "auxiliary basis");
    const Eri3Need n = eri3_need(b, a, opts ? opts->flags : 0);
    dfx_eri3_sizes z{};
    z.nbf = b.nbf;
    z.naux = a.nbf;
    z.ncols_tiled = tiled_cols(b.nbf);
    z.bytes_B = n.bytes_B;
    z.bytes_raw = n.bytes_raw;
    z.bytes_metric = n.bytes_metric;
    z.bytes_persistent = n.bottom;
    z.bytes_jk = n.jk;
    z.bytes_workspace = n.total;
    *out = z;
  });
}

int dfx_B_unpack(const dfx_B* b, int q0, int q1, double* dev_out, void* stream) {
  return guard([&] {
    if (!b || !dev_out) throw Error(DFX_EINVAL, "dfx_B_unpack: NULL argument");
    if (q0 < 0 || q1 > b->naux || q1 < q0) throw Error(DFX_EINVAL, "dfx_B_unpack: bad row range");
    unpack_rows(b->hi.as<float>(), b->lo.as<float>(), b->ncols_t, b->nbf, q0, q1, dev_out, (hipStream_t)stream);
    DFX_HIP(hipGetLastError());
  });
}

int dfx_B_info_get(const dfx_B* b, dfx_B_info* info) {
  return guard([&] {
    if (!b || !info) throw Error(DFX_EINVAL, "dfx_B_info_get: NULL argument");
    *info = b->info;
  });
}

int dfx_B_lists(const dfx_B* b, int32_t* pairs, int64_t* col_off, uint8_t* keep, double* Qab,
                double* QC) {
  return guard([&] {
    if (!b) throw Error(DFX_EINVAL, "dfx_B_lists: NULL handle");
    const size_t np = b->pa.size();
    if (pairs)
      for (size_t k = 0; k < np; ++k) {
        pairs[2 * k] = b->pa[k];
        pairs[2 * k + 1] = b->pb[k];
      }
    if (col_off) std::copy(b->col_off.begin(), b->col_off.end(), col_off);
    const int nsh = b->bas.nsh, nc = b->aux.nsh;
    if (keep)
      for (size_t k = 0; k < np; ++k) {
        const double q = b->Qab[(size_t)b->pa[k] * nsh + b->pb[k]];
        for (int c = 0; c < nc; ++c) keep[k * nc + c] = (q * b->QC[c] >= b->tau) ? 1 : 0;
      }
    if (Qab) std::copy(b->Qab.begin(), b->Qab.end(), Qab);
    if (QC) std::copy(b->QC.begin(), b->QC.end(), QC);
  });
}

int dfx_B_export(const dfx_B* bc, int what, int q0, int q1, double* dev_out, void* stream) {
  return guard([&] {
    dfx_B* b = const_cast<dfx_B*>(bc);
    if (!b || !dev_out) throw Error(DFX_EINVAL, "dfx_B_export: NULL argument");
    if (q0 < 0 || q1 > b->naux || q1 < q0) throw Error(DFX_EINVAL, "dfx_B_export: bad row range");
    if (what == DFX_EXPORT_RAW && !b->raw.p) throw Error(DFX_EINVAL, "dfx_B_export: raw not kept");
    hipStream_t st = (hipStream_t)stream;
    ArenaScope scope(b->arena.get());
    if (!b->toff.p) {
      std::vector<int64_t> toff(b->ncols_p);
      for (size_t k = 0; k < b->pa.size(); ++k) {
        const int a = b->pa[k], bb = b->pb[k];
        const int na = 2 * b->bas.l[a] + 1, nb = 2 * b->bas.l[bb] + 1;
        for (int i = 0; i < na; ++i)
          for (int j = 0; j < nb; ++j) {
            int r = b->bas.foff[a] + i, c = b->bas.foff[bb] + j;
            if (r < c) std::swap(r, c);
            toff[b->col_off[k] + i * nb + j] = tile_base(r >> 5, c >> 5) + ((r & 31) << 5) + (c & 31);
          }
      }
      b->toff = upload(toff, st);
    }
    if (what == DFX_EXPORT_RAW && !b->rawcol_d.p) b->rawcol_d = upload(b->rawcol, st);
    export_rows(what == DFX_EXPORT_RAW ? nullptr : b->hi.as<float>(),
                what == DFX_EXPORT_B ? b->lo.as<float>() : nullptr,
                what == DFX_EXPORT_RAW ? b->raw.as<double>() : nullptr, b->ncols_t, q0, q1,
                what == DFX_EXPORT_RAW ? b->rawcol_d.as<int64_t>() : b->toff.as<int64_t>(), b->ncols_p, dev_out, st);
    DFX_HIP(hipGetLastError());
  });
}

int dfx_B_metric(const dfx_B* b, int what, double* dev_out, void* stream) {
  return guard([&] {
    if (!b || !dev_out) throw Error(DFX_EINVAL, "dfx_B_metric: NULL argument");
    const DevMem& m = what == 0 ? b->J2 : b->L;
    if (!m.p) throw Error(DFX_EINVAL, "dfx_B_metric: metric not kept (DFX_KEEP_METRIC)");
    DFX_HIP(hipMemcpyAsync(dev_out, m.p, sizeof(double) * (size_t)b->naux * b->naux,
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
  });
}

int dfx_B_free(dfx_B* b) {
  return guard([&] { delete b; });
}

int dfx_jk(const dfx_B* bc, const double* dev_in, int kind, int nocc, int precision, double* dev_J,
           double* dev_K, void* stream) {
  return guard([&] {
    dfx_B* b = const_cast<dfx_B*>(bc);
    if (!b || !dev_in) throw Error(DFX_EINVAL, "dfx_jk: NULL argument");
    if (kind != DFX_DENSITY && kind != DFX_COCC) throw Error(DFX_EINVAL, "dfx_jk: bad kind");
    if (precision < DFX_FP64 || precision > DFX_BF16) throw Error(DFX_EINVAL, "dfx_jk: bad precision");
    if (kind == DFX_COCC && (nocc <= 0 || nocc > b->nbf)) throw Error(DFX_EINVAL, "dfx_jk: bad nocc");
    hipStream_t st = (hipStream_t)stream;
    ArenaScope scope(b->arena.get());
    JKArgs a{b->hi.as<float>(), b->lo.as<float>(), b->naux, b->nbf, b->ncols_t, precision};
    const int nbf = b->nbf;
    size_t need = 0;
    const size_t jw = sizeof(double) * (2 * (size_t)b->ncols_t + b->naux + 8);
    const size_t dbytes = (kind == DFX_COCC) ? sizeof(double) * (size_t)nbf * nbf : 0;
    if (dev_J) need = std::max(need, jw + dbytes);
    if (dev_K && kind == DFX_COCC) need = std::max(need, k_work_bytes(a, nocc));
    char* w = static_cast<char*>(b->ensure_work(need));
    if (dev_J) {
      const double* D = dev_in;
      if (kind == DFX_COCC) {
        double* Dd = reinterpret_cast<double*>(w + jw);
        GemmF64 g{};
        g.M = nbf; g.N = nbf; g.K = nocc;
        g.A = dev_in; g.lda = nocc;
        g.B = dev_in; g.ldb = nocc; g.tb = true;
        g.C = Dd; g.ldc = nbf;
        g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
        dgemm(g, st);
        D = Dd;
      }
      j_build(a, D, dev_J, reinterpret_cast<double*>(w), st);
    }
    if (dev_K && kind == DFX_COCC) k_build(a, dev_in, nocc, dev_K, w, st);
    if (dev_K && kind == DFX_DENSITY) k_from_density(a, dev_in, dev_K, st);
    DFX_HIP(hipGetLastError());
  });
}

int dfx_mp2(const dfx_B* bc, const double* dev_C, int nmo, const double* eps, int nocc, int nfrozen, double* E2,
            void* stream) {
  return guard([&] {
    if (!bc || !dev_C || !eps || !E2) throw Error(DFX_EINVAL, "dfx_mp2: NULL argument");
    dfx_B* b = const_cast<dfx_B*>(bc);
    if (nmo <= 0 || nmo > b->nbf || nocc <= 0 || nocc >= nmo || nfrozen < 0 || nfrozen >= nocc)
      throw Error(DFX_EINVAL, "dfx_mp2: bad orbital counts");
    JKArgs a{b->hi.as<float>(), b->lo.as<float>(), b->naux, b->nbf, b->ncols_t, DFX_FP64};
    *E2 = mp2_energy(a, dev_C, nmo, eps, nocc, nfrozen, (hipStream_t)stream);
  });
}

int dfx_int1e(const dfx_shell* shells, int nsh, const dfx_geom* geom, double* dev_S, double* dev_T,
              double* dev_V, void* stream) {
  return guard([&] {
    if (!geom || !dev_S || !dev_T || !dev_V) throw Error(DFX_EINVAL, "dfx_int1e: NULL argument");
    if (geom->natom < 0 || (geom->natom > 0 && (!geom->xyz || !geom->Z)))
      throw Error(DFX_EINVAL, "dfx_int1e: bad geometry");
    HostShells h = make_shells(shells, nsh, 3, "orbital basis");
    int1e_build(h, geom, dev_S, dev_T, dev_V, (hipStream_t)stream);
  });
}

}  // extern "C"

void dfx::int1e_build(const HostShells& h, const dfx_geom* geom, double* dev_S, double* dev_T,
                      double* dev_V, hipStream_t st) {
    const int nsh = h.nsh;
    DevShellSet d;
    d.upload(h, st);
    std::vector<double> xyz(geom->xyz, geom->xyz + 3 * geom->natom);
    std::vector<double> Z(geom->natom);
    for (int i = 0; i < geom->natom; ++i) Z[i] = geom->Z[i];
    DevMem xyz_d = upload(xyz, st), Z_d = upload(Z, st);
    std::vector<std::vector<int>> pf(16), ps(16);
    for (int a = 0; a < nsh; ++a)
      for (int b = 0; b <= a; ++b) {
        const int cls = h.l[a] * 4 + h.l[b];
        pf[cls].push_back(a);
        ps[cls].push_back(b);
      }
    const double* rys = rys_table_device();
    std::vector<DevMem> keep;
    for (int cls = 0; cls < 16; ++cls) {
      if (pf[cls].empty()) continue;
      keep.push_back(upload(pf[cls], st));
      keep.push_back(upload(ps[cls], st));
      OneEArgs a{};
      a.sh = d.view();
      a.pf = keep[keep.size() - 2].as<int>();
      a.ps = keep.back().as<int>();
      a.npairs = (int)pf[cls].size();
      a.n = h.nbf;
      a.S = dev_S;
      a.T = dev_T;
      a.V = dev_V;
      a.xyz = xyz_d.as<double>();
      a.Z = Z_d.as<double>();
      a.natom = geom->natom;
      a.rys = rys;
      onee_dispatch(cls / 4, cls % 4, a, st);
    }
    DFX_HIP(hipGetLastError());
    DFX_HIP(hipStreamSynchronize(st));
}
