// Learned SCF starting guess: one multilayer perceptron per atom-pair type maps
// invariant descriptors of the pair's local geometry to the pair's block of the
// density matrix in the symmetrically orthogonalised (Loewdin) basis, written in
// a local frame; blocks are rotated back to the laboratory frame with
// real-solid-harmonic rotation matrices and assembled.
// The networks are trained on converged densities of the method itself.  The
// MLP arithmetic runs in the FP32 kernels of mlp.hip; geometry work (local
// frames, descriptors, rotations) is host C++, spread over a few host threads,
// one sample at a time each, so the results do not depend on the thread count.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <numeric>
#include <random>
#include <atomic>
#include <cstdlib>
#include <exception>
#include <mutex>
#include <thread>

#include "host.h"
#include "mlp.h"
#include "sph_tables.inc"

namespace dfx {

static const int ELEM[3] = {1, 6, 8};  // descriptor channels: H, C, O
constexpr int NCH = 3, NRAD = 8, NPRAD = 16, NY = 9;
constexpr double RMIN = 0.5;  // first radial centre; the last sits at the cutoff

static int channel(int Z) {
  for (int i = 0; i < NCH; ++i)
    if (ELEM[i] == Z) return i;
  throw Error(DFX_EUNSUPPORTED, "learned guess: element Z = " + std::to_string(Z) + " has no descriptor channel");
}

// f(i) for i in [0, n) on up to 16 host threads (fewer if OMP_NUM_THREADS or the
// hardware says so), in chunks taken in order; each i is independent.  The first
// exception thrown is rethrown after all threads have joined.
template <class Fn>
static void parallel_for(size_t n, Fn f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(e);
    if (v >= 1) nt = std::min<unsigned>(nt, (unsigned)v);
  }
  const size_t chunk = 16;
  if (nt <= 1 || n <= chunk) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  nt = (unsigned)std::min<size_t>(nt, (n + chunk - 1) / chunk);
  std::atomic<size_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&] {
    try {
      for (;;) {
        const size_t i0 = next.fetch_add(chunk);
        if (i0 >= n) break;
        for (size_t i = i0; i < std::min(n, i0 + chunk); ++i) f(i);
      }
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!err) err = std::current_exception();
      next.store(n);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

// ---- geometry helpers -------------------------------------------------------------------
struct V3 {
  double x, y, z;
};
static V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
static V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
static double norm(V3 a) { return std::sqrt(dot(a, a)); }
static V3 unit(V3 a) { return scale(a, 1.0 / norm(a)); }

// Local frame (rows x, y, z) of pair (a, b), or of atom a when b == a.
// z: a -> b, or a -> its nearest neighbour; x: the nearest further neighbour of a
// at least 0.1 rad away from the z axis, projected off z (else the lab axis least
// aligned with z).  Neighbours are ranked by distance rounded to 1e-8 bohr, then
// by index, so that equal bond lengths keep their order under rotation.
static void local_frame(const std::vector<V3>& r, int a, int b, double F[3][3]) {
  std::vector<std::pair<long long, int>> key;
  for (int k = 0; k < (int)r.size(); ++k)
    if (k != a) key.push_back({(long long)std::floor(norm(sub(r[k], r[a])) * 1e8 + 0.5), k});
  std::sort(key.begin(), key.end());
  std::vector<int> order;
  for (auto& kv : key) order.push_back(kv.second);
  V3 z;
  std::vector<int> cand;
  if (b != a) {
    z = unit(sub(r[b], r[a]));
    for (int k : order)
      if (k != b) cand.push_back(k);
  } else {
    if (order.empty()) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i][j] = i == j;
      return;
    }
    z = unit(sub(r[order[0]], r[a]));
    cand.assign(order.begin() + 1, order.end());
  }
  bool found = false;
  V3 xv{0, 0, 0};
  for (int k : cand) {
    const V3 v = sub(r[k], r[a]);
    if (norm(cross(unit(v), z)) > std::sin(0.1)) {
      xv = sub(v, scale(z, dot(v, z)));
      found = true;
      break;
    }
  }
  if (!found) {
    const double az[3] = {std::fabs(z.x), std::fabs(z.y), std::fabs(z.z)};
    const int ax = (int)(std::min_element(az, az + 3) - az);
    const V3 e{ax == 0 ? 1.0 : 0.0, ax == 1 ? 1.0 : 0.0, ax == 2 ? 1.0 : 0.0};
    xv = sub(e, scale(z, dot(e, z)));
  }
  const V3 x = unit(xv), y = cross(z, x);
  const V3 rows[3] = {x, y, z};
  for (int i = 0; i < 3; ++i) {
    F[i][0] = rows[i].x;
    F[i][1] = rows[i].y;
    F[i][2] = rows[i].z;
  }
}

// real solid harmonics of degree <= 2 of a unit vector, m = -l..l per l (9 values)
static void ylm2(V3 u, double* out) {
  const double p[3] = {u.x, u.y, u.z};
  int o = 0;
  auto eval = [&](int l, const double* T, int nc) {
    for (int m = 0; m < 2 * l + 1; ++m) {
      double s = 0.0;
      for (int c = 0; c < nc; ++c) {
        double mono = 1.0;
        for (int ax = 0; ax < 3; ++ax)
          for (int e = 0; e < cpow(l, c, ax); ++e) mono *= p[ax];
        s += T[m * nc + c] * mono;
      }
      out[o++] = s;
    }
  };
  eval(0, &SPH_L0[0][0], 1);
  eval(1, &SPH_L1[0][0], 3);
  eval(2, &SPH_L2[0][0], 6);
}

// k-th of n Gaussians with centres evenly spaced on [RMIN, rmax], width = spacing
static double radial(double r, int k, int n, double rmax) {
  const double w = (rmax - RMIN) / (n - 1), mu = RMIN + k * w;
  const double t = (r - mu) / w;
  return std::exp(-t * t);
}
static double fcut(double r, double rc) { return r < rc ? 0.5 * (std::cos(M_PI * r / rc) + 1.0) : 0.0; }

// sum_k radial_n(r) f_c(r) Y(F (r_k - r_a) / r) per element channel, k not a, not excluded
static void env_features(const std::vector<V3>& r, const std::vector<int>& Z, int a, int excl, const double F[3][3],
                         double rc, double* out) {
  std::fill(out, out + NCH * NRAD * NY, 0.0);
  for (int k = 0; k < (int)r.size(); ++k) {
    if (k == a || k == excl) continue;
    const V3 v = sub(r[k], r[a]);
    const double d = norm(v);
    if (d >= rc) continue;
    const V3 u{(F[0][0] * v.x + F[0][1] * v.y + F[0][2] * v.z) / d, (F[1][0] * v.x + F[1][1] * v.y + F[1][2] * v.z) / d,
               (F[2][0] * v.x + F[2][1] * v.y + F[2][2] * v.z) / d};
    double y[NY];
    ylm2(u, y);
    const int ch = channel(Z[k]);
    const double fc = fcut(d, rc);
    for (int n = 0; n < NRAD; ++n) {
      const double g = radial(d, n, NRAD, rc) * fc;
      for (int m = 0; m < NY; ++m) out[(ch * NRAD + n) * NY + m] += g * y[m];
    }
  }
}

static int nfeat_pair() { return 2 * NCH + NPRAD + 2 * NCH * NRAD * NY; }
static int nfeat_diag() { return NCH + NCH * NRAD * NY; }

// descriptors of sample (a, b) (atom a when b == a) and its local frame; rc is the
// pair cutoff (range of the pair-distance Gaussians), rce the environment cutoff
static void pair_features(const std::vector<V3>& r, const std::vector<int>& Z, int a, int b, double rc, double rce,
                          double* f, double F[3][3]) {
  local_frame(r, a, b, F);
  if (a == b) {
    for (int i = 0; i < NCH; ++i) f[i] = (Z[a] == ELEM[i]);
    env_features(r, Z, a, -1, F, rce, f + NCH);
    return;
  }
  for (int i = 0; i < NCH; ++i) {
    f[i] = (Z[a] == ELEM[i]);
    f[NCH + i] = (Z[b] == ELEM[i]);
  }
  const double d = norm(sub(r[b], r[a]));
  for (int n = 0; n < NPRAD; ++n) f[2 * NCH + n] = radial(d, n, NPRAD, rc);
  env_features(r, Z, a, b, F, rce, f + 2 * NCH + NPRAD);
  env_features(r, Z, b, a, F, rce, f + 2 * NCH + NPRAD + NCH * NRAD * NY);
}

// ---- rotation of real solid harmonics by polynomial substitution --------------------
// U with f_m(F^T x) = sum_m' U[m][m'] f_m'(x) for degree l (row-major (2l+1)^2).
static const double* sph_table(int l) {
  static const double* t[4] = {&SPH_L0[0][0], &SPH_L1[0][0], &SPH_L2[0][0], &SPH_L3[0][0]};
  return t[l];
}
static std::vector<double> sh_rotation(int l, const double F[3][3]) {
  const int nc = ncart(l), ns = 2 * l + 1;
  std::vector<double> U((size_t)ns * ns, 0.0);
  if (l == 0) {
    U[0] = 1.0;
    return U;
  }
  auto cidx = [&](int i, int j) {  // Cartesian index of x^i y^j z^(l-i-j)
    int n = 0;
    for (int a = l; a >= 0; --a)
      for (int b = l - a; b >= 0; --b) {
        if (a == i && b == j) return n;
        ++n;
      }
    return -1;
  };
  // lab monomial c -> polynomial in the local coordinates
  std::vector<std::vector<double>> sub_c(nc, std::vector<double>(nc, 0.0));
  for (int c = 0; c < nc; ++c) {
    // product of linear forms lab_ax = sum_j F[j][ax] x_j, as a map (i, j) -> coef at the running degree
    std::map<std::pair<int, int>, double> poly{{{0, 0}, 1.0}};
    int deg = 0;
    for (int ax = 0; ax < 3; ++ax)
      for (int e = 0; e < cpow(l, c, ax); ++e) {
        std::map<std::pair<int, int>, double> nxt;
        for (auto& kv : poly) {
          const int i = kv.first.first, j = kv.first.second;
          nxt[{i + 1, j}] += kv.second * F[0][ax];
          nxt[{i, j + 1}] += kv.second * F[1][ax];
          nxt[{i, j}] += kv.second * F[2][ax];  // z power rises implicitly with the degree
        }
        poly.swap(nxt);
        ++deg;
      }
    for (auto& kv : poly) sub_c[c][cidx(kv.first.first, kv.first.second)] += kv.second;
  }
  const double* T = sph_table(l);
  // coefficient vectors of f_m(F^T x) over local monomials
  std::vector<double> cm((size_t)ns * nc, 0.0);
  for (int m = 0; m < ns; ++m)
    for (int c = 0; c < nc; ++c)
      if (T[m * nc + c] != 0.0)
        for (int c2 = 0; c2 < nc; ++c2) cm[m * nc + c2] += T[m * nc + c] * sub_c[c][c2];
  // U = cm T^T (T T^T)^-1  (cm lies in the row space of T)
  std::vector<double> G((size_t)ns * ns, 0.0), R((size_t)ns * ns, 0.0);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) {
      double g = 0.0, rr = 0.0;
      for (int c = 0; c < nc; ++c) {
        g += T[i * nc + c] * T[j * nc + c];
        rr += cm[i * nc + c] * T[j * nc + c];
      }
      G[i * ns + j] = g;
      R[i * ns + j] = rr;
    }
  // solve U G = R by Gauss-Jordan on G (symmetric positive definite)
  std::vector<double> Gi((size_t)ns * ns, 0.0);
  for (int i = 0; i < ns; ++i) Gi[i * ns + i] = 1.0;
  std::vector<double> A = G;
  for (int k = 0; k < ns; ++k) {
    int p = k;
    for (int i = k + 1; i < ns; ++i)
      if (std::fabs(A[i * ns + k]) > std::fabs(A[p * ns + k])) p = i;
    for (int j = 0; j < ns; ++j) {
      std::swap(A[k * ns + j], A[p * ns + j]);
      std::swap(Gi[k * ns + j], Gi[p * ns + j]);
    }
    const double piv = A[k * ns + k];
    for (int j = 0; j < ns; ++j) {
      A[k * ns + j] /= piv;
      Gi[k * ns + j] /= piv;
    }
    for (int i = 0; i < ns; ++i)
      if (i != k) {
        const double f = A[i * ns + k];
        for (int j = 0; j < ns; ++j) {
          A[i * ns + j] -= f * A[k * ns + j];
          Gi[i * ns + j] -= f * Gi[k * ns + j];
        }
      }
  }
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) {
      double s = 0.0;
      for (int k = 0; k < ns; ++k) s += R[i * ns + k] * Gi[k * ns + j];
      U[i * ns + j] = s;
    }
  return U;
}

}  // namespace dfx

using namespace dfx;

// ---- the model ---------------------------------------------------------------------------------
struct GuessType {
  bool diag = false;
  int za = 0, zb = 0;  // za >= zb
  int nin = 0, nout = 0;
  std::vector<int> widths;
  std::vector<double> fmean, fstd, tmean, tstd;
  bool normalised = false;
  std::vector<float> theta_h;  // host copy (authoritative between calls)
  DevMem theta, m, v;
  int adam_step = 0;
  std::vector<double> X, T;    // training samples (raw)
  int nsamp = 0;
};

struct dfx_guess {
  double rc = 8.0, rc_env = 6.0;
  int hidden = 256, depth = 3;
  uint64_t seed = 0;
  std::map<int, std::vector<int>> shells;  // Z -> shell l list
  std::vector<GuessType> types;
  int find(bool diag, int za, int zb) const {
    for (size_t i = 0; i < types.size(); ++i)
      if (types[i].diag == diag && types[i].za == za && types[i].zb == zb) return (int)i;
    return -1;
  }
};

namespace dfx {

static int atom_nbf(const dfx_guess* g, int Z) {
  auto it = g->shells.find(Z);
  if (it == g->shells.end()) throw Error(DFX_EUNSUPPORTED, "learned guess: element Z = " + std::to_string(Z) + " not in the model");
  int n = 0;
  for (int l : it->second) n += 2 * l + 1;
  return n;
}

// block-diagonal rotation over an atom's shells (row-major n x n)
static std::vector<double> atom_rotation(const dfx_guess* g, int Z, const double F[3][3]) {
  const auto& ls = g->shells.at(Z);
  const int n = atom_nbf(g, Z);
  std::vector<double> U((size_t)n * n, 0.0);
  int o = 0;
  std::map<int, std::vector<double>> cache;
  for (int l : ls) {
    if (!cache.count(l)) cache[l] = sh_rotation(l, F);
    const auto& u = cache[l];
    const int s = 2 * l + 1;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) U[(size_t)(o + i) * n + o + j] = u[i * s + j];
    o += s;
  }
  return U;
}

struct GeomView {
  std::vector<V3> r;
  std::vector<int> Z, off;
  int nbf = 0;
};
static GeomView view(const dfx_guess* g, const dfx_geom* geom) {
  if (!geom || geom->natom <= 0 || !geom->xyz || !geom->Z) throw Error(DFX_EINVAL, "learned guess: bad geometry");
  GeomView v;
  for (int a = 0; a < geom->natom; ++a) {
    v.r.push_back({geom->xyz[3 * a], geom->xyz[3 * a + 1], geom->xyz[3 * a + 2]});
    v.Z.push_back(geom->Z[a]);
    v.off.push_back(v.nbf);
    v.nbf += atom_nbf(g, geom->Z[a]);
  }
  return v;
}

// the samples (a -> b) of a geometry, with the ordering rules for the pair direction
struct Sample {
  int a, b, type;
};
static std::vector<Sample> samples_of(dfx_guess* g, const GeomView& v, bool create_types) {
  std::vector<Sample> out;
  const int na = (int)v.r.size();
  auto type_of = [&](bool diag, int za, int zb) {
    int t = g->find(diag, za, zb);
    if (t < 0) {
      if (!create_types) return -1;
      GuessType T;
      T.diag = diag;
      T.za = za;
      T.zb = zb;
      T.nin = diag ? nfeat_diag() : nfeat_pair();
      T.nout = atom_nbf(g, za) * atom_nbf(g, zb);
      T.widths.push_back(T.nin);
      for (int i = 0; i < g->depth; ++i) T.widths.push_back(g->hidden);
      T.widths.push_back(T.nout);
      g->types.push_back(std::move(T));
      t = (int)g->types.size() - 1;
    }
    return t;
  };
  for (int a = 0; a < na; ++a) {
    out.push_back({a, a, type_of(true, v.Z[a], v.Z[a])});
    for (int b = a + 1; b < na; ++b) {
      if (norm(sub(v.r[b], v.r[a])) >= g->rc) continue;
      if (v.Z[a] > v.Z[b]) {
        out.push_back({a, b, type_of(false, v.Z[a], v.Z[b])});
      } else if (v.Z[a] < v.Z[b]) {
        out.push_back({b, a, type_of(false, v.Z[b], v.Z[a])});
      } else {
        const int t = type_of(false, v.Z[a], v.Z[b]);
        out.push_back({a, b, t});
        out.push_back({b, a, t});
      }
    }
  }
  return out;
}

// initial weights: N(0, 1/fan_in), zero biases (mt19937_64 + Box-Muller)
static void init_theta(GuessType& T, uint64_t seed) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  T.theta_h.assign(mlp_nparams(T.widths), 0.0f);
  size_t o = 0;
  for (size_t l = 0; l + 1 < T.widths.size(); ++l) {
    const int ni = T.widths[l], no = T.widths[l + 1];
    const double s = 1.0 / std::sqrt((double)ni);
    for (int i = 0; i < ni * no; ++i) T.theta_h[o + i] = (float)(nd(rng) * s);
    o += (size_t)ni * no + no;
  }
}

// Device copy of the weights with Adam moments; once allocated it is current
// (training updates it and copies back, import and load start without one).
static void ensure_device(GuessType& T) {
  const size_t n = T.theta_h.size();
  if (T.theta.n == n * sizeof(float)) return;
  // the model outlives any call's workspace: its weights never come from one
  ArenaScope own(nullptr);
  T.theta.alloc(n * sizeof(float));
  T.m.alloc(n * sizeof(float));
  T.v.alloc(n * sizeof(float));
  T.adam_step = 0;
  DFX_HIP(hipMemset(T.m.p, 0, T.m.n));
  DFX_HIP(hipMemset(T.v.p, 0, T.v.n));
  DFX_HIP(hipMemcpy(T.theta.p, T.theta_h.data(), n * sizeof(float), hipMemcpyHostToDevice));
}

// predicted local-frame blocks (raw units) for the given samples
static std::vector<std::vector<double>> predict_blocks(dfx_guess* g, const GeomView& v, const std::vector<Sample>& S,
                                                       std::vector<std::array<double, 9>>& frames, hipStream_t st) {
  std::vector<std::vector<double>> out(S.size());
  frames.resize(S.size());
  std::map<int, std::vector<size_t>> by_type;
  for (size_t i = 0; i < S.size(); ++i) by_type[S[i].type].push_back(i);
  for (auto& kv : by_type) {
    GuessType& T = g->types[kv.first];
    if (!T.normalised) throw Error(DFX_EINVAL, "learned guess: model is not trained");
    const int n = (int)kv.second.size();
    std::vector<float> X((size_t)n * T.nin);
    parallel_for((size_t)n, [&](size_t k) {
      const Sample& s = S[kv.second[k]];
      std::vector<double> f(T.nin);
      double F[3][3];
      pair_features(v.r, v.Z, s.a, s.b, g->rc, g->rc_env, f.data(), F);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) frames[kv.second[k]][i * 3 + j] = F[i][j];
      for (int i = 0; i < T.nin; ++i) X[k * T.nin + i] = (float)((f[i] - T.fmean[i]) / T.fstd[i]);
    });
    ensure_device(T);
    DevMem Xd(sizeof(float) * X.size()), Yd(sizeof(float) * (size_t)n * T.nout);
    DevMem work(sizeof(float) * mlp_work_floats(T.widths, n));
    DFX_HIP(hipMemcpyAsync(Xd.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, st));
    mlp_forward(T.widths, T.theta.as<float>(), Xd.as<float>(), n, Yd.as<float>(), work.as<float>(), st);
    std::vector<float> Y((size_t)n * T.nout);
    DFX_HIP(hipMemcpyAsync(Y.data(), Yd.p, sizeof(float) * Y.size(), hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < n; ++k) {
      auto& o = out[kv.second[k]];
      o.resize(T.nout);
      for (int i = 0; i < T.nout; ++i) o[i] = Y[(size_t)k * T.nout + i] * T.tstd[i] + T.tmean[i];
    }
  }
  return out;
}

// D_lab^{ab} = U_a P U_b^T
static void rotate_out(const std::vector<double>& Ua, int na, const std::vector<double>& P, const std::vector<double>& Ub,
                       int nb, std::vector<double>& M) {
  std::vector<double> t((size_t)na * nb, 0.0);
  for (int i = 0; i < na; ++i)
    for (int k = 0; k < na; ++k) {
      const double u = Ua[(size_t)i * na + k];
      if (u == 0.0) continue;
      for (int j = 0; j < nb; ++j) t[(size_t)i * nb + j] += u * P[(size_t)k * nb + j];
    }
  M.assign((size_t)na * nb, 0.0);
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += t[(size_t)i * nb + k] * Ub[(size_t)j * nb + k];
      M[(size_t)i * nb + j] = s;
    }
}

void guess_check_basis(const dfx_guess* g, const dfx_geom* geom, const dfx_shell* shells, int nsh) {
  if (!g || !geom || !shells) throw Error(DFX_EINVAL, "learned guess: NULL argument");
  int s = 0;
  for (int a = 0; a < geom->natom; ++a) {
    auto it = g->shells.find(geom->Z[a]);
    if (it == g->shells.end())
      throw Error(DFX_EUNSUPPORTED, "learned guess: element Z = " + std::to_string(geom->Z[a]) + " not in the model");
    for (int l : it->second) {
      bool ok = s < nsh && shells[s].l == l;
      for (int k = 0; ok && k < 3; ++k) ok = std::fabs(shells[s].xyz[k] - geom->xyz[3 * a + k]) <= 1e-8;
      if (!ok)
        throw Error(DFX_EINVAL, "learned guess: orbital shell " + std::to_string(s) +
                                    " does not match the model's basis for atom " + std::to_string(a));
      ++s;
    }
  }
  if (s != nsh) throw Error(DFX_EINVAL, "learned guess: more orbital shells than the model's basis");
}

void guess_predict_density(const dfx_guess* gc, const dfx_geom* geom, double* D, hipStream_t st) {
  dfx_guess* g = const_cast<dfx_guess*>(gc);  // only the device copies of the weights are touched
  const GeomView v = view(g, geom);
  std::vector<Sample> S = samples_of(g, v, false);
  for (const auto& s : S)
    if (s.type < 0) throw Error(DFX_EINVAL, "learned guess: pair type not in the model");
  std::vector<std::array<double, 9>> frames;
  const auto blocks = predict_blocks(g, v, S, frames, st);
  const int n = v.nbf;
  std::fill(D, D + (size_t)n * n, 0.0);
  // lab-frame blocks in parallel, then assembled in sample order
  std::vector<std::vector<double>> Ms(S.size());
  parallel_for(S.size(), [&](size_t i) {
    const int a = S[i].a, b = S[i].b;
    double F[3][3];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) F[p][q] = frames[i][p * 3 + q];
    const int na = atom_nbf(g, v.Z[a]), nb = atom_nbf(g, v.Z[b]);
    rotate_out(atom_rotation(g, v.Z[a], F), na, blocks[i], atom_rotation(g, v.Z[b], F), nb, Ms[i]);
  });
  for (size_t i = 0; i < S.size(); ++i) {
    const int a = S[i].a, b = S[i].b;
    const int na = atom_nbf(g, v.Z[a]), nb = atom_nbf(g, v.Z[b]);
    const std::vector<double>& M = Ms[i];
    // homonuclear pairs appear in both directions: each contributes half
    const double w = (a != b && v.Z[a] == v.Z[b]) ? 0.5 : 1.0;
    for (int p = 0; p < na; ++p)
      for (int q = 0; q < nb; ++q) {
        const double x = w * M[(size_t)p * nb + q];
        if (a == b) {
          D[(size_t)(v.off[a] + p) * n + v.off[b] + q] += 0.5 * x;
          D[(size_t)(v.off[b] + q) * n + v.off[a] + p] += 0.5 * x;
        } else {
          D[(size_t)(v.off[a] + p) * n + v.off[b] + q] += x;
          D[(size_t)(v.off[b] + q) * n + v.off[a] + p] += x;
        }
      }
  }
}

}  // namespace dfx

extern "C" {

int dfx_guess_create(const dfx_guess_spec* spec, dfx_guess** out) {
  return guard([&] {
    if (!spec || !out || spec->nelem <= 0 || !spec->Z || !spec->nshell || !spec->shell_l)
      throw Error(DFX_EINVAL, "dfx_guess_create: bad spec");
    std::unique_ptr<dfx_guess> g(new dfx_guess());
    g->rc = spec->rc > 0 ? spec->rc : 8.0;
    g->rc_env = spec->rc_env > 0 ? spec->rc_env : 6.0;
    g->hidden = spec->hidden > 0 ? spec->hidden : 256;
    g->depth = spec->depth > 0 ? spec->depth : 3;
    g->seed = spec->seed;
    int o = 0;
    for (int e = 0; e < spec->nelem; ++e) {
      channel(spec->Z[e]);
      std::vector<int> ls(spec->shell_l + o, spec->shell_l + o + spec->nshell[e]);
      for (int l : ls)
        if (l < 0 || l > 3) throw Error(DFX_EUNSUPPORTED, "dfx_guess_create: shell l > 3");
      g->shells[spec->Z[e]] = ls;
      o += spec->nshell[e];
    }
    *out = g.release();
  });
}

int dfx_guess_free(dfx_guess* g) {
  return guard([&] { delete g; });
}

int dfx_guess_add(dfx_guess* g, const dfx_geom* geom, const double* D) {
  return guard([&] {
    if (!g || !D) throw Error(DFX_EINVAL, "dfx_guess_add: NULL argument");
    // D is the Loewdin-basis density P = S^1/2 D_AO S^1/2 (dfx_lowdin)
    const GeomView v = view(g, geom);
    const std::vector<Sample> S = samples_of(g, v, true);
    const int n = v.nbf;
    for (const Sample& s : S)
      if (g->types[s.type].normalised) throw Error(DFX_EINVAL, "dfx_guess_add: model already trained");
    // descriptors and local blocks per sample in parallel, stored in sample order
    std::vector<std::vector<double>> fs(S.size()), Ps(S.size());
    parallel_for(S.size(), [&](size_t i) {
      const Sample& s = S[i];
      std::vector<double>& f = fs[i];
      f.resize(g->types[s.type].nin);
      double F[3][3];
      pair_features(v.r, v.Z, s.a, s.b, g->rc, g->rc_env, f.data(), F);
      const int na = atom_nbf(g, v.Z[s.a]), nb = atom_nbf(g, v.Z[s.b]);
      const auto Ua = atom_rotation(g, v.Z[s.a], F), Ub = atom_rotation(g, v.Z[s.b], F);
      // local block U_a^T D^{ab} U_b
      std::vector<double> t((size_t)na * nb, 0.0);
      std::vector<double>& P = Ps[i];
      P.assign((size_t)na * nb, 0.0);
      for (int k = 0; k < na; ++k)
        for (int j = 0; j < nb; ++j) {
          double x = 0.0;
          for (int q = 0; q < nb; ++q) x += D[(size_t)(v.off[s.a] + k) * n + v.off[s.b] + q] * Ub[(size_t)q * nb + j];
          t[(size_t)k * nb + j] = x;
        }
      for (int ii = 0; ii < na; ++ii)
        for (int j = 0; j < nb; ++j) {
          double x = 0.0;
          for (int k = 0; k < na; ++k) x += Ua[(size_t)k * na + ii] * t[(size_t)k * nb + j];
          P[(size_t)ii * nb + j] = x;
        }
    });
    for (size_t i = 0; i < S.size(); ++i) {
      GuessType& T = g->types[S[i].type];
      T.X.insert(T.X.end(), fs[i].begin(), fs[i].end());
      T.T.insert(T.T.end(), Ps[i].begin(), Ps[i].end());
      ++T.nsamp;
    }
  });
}

int dfx_guess_train(dfx_guess* g, int epochs, int batch, double lr, double* loss_out) {
  return guard([&] {
    if (!g || epochs < 0 || batch <= 0 || !(lr > 0)) throw Error(DFX_EINVAL, "dfx_guess_train: bad argument");
    hipStream_t st = nullptr;
    std::vector<double> eloss(epochs, 0.0);
    size_t total = 0;
    for (size_t ti = 0; ti < g->types.size(); ++ti) {
      GuessType& T = g->types[ti];
      if (T.nsamp == 0) continue;
      if (!T.normalised) {  // feature / target standardisation from the training set
        T.fmean.assign(T.nin, 0.0);
        T.fstd.assign(T.nin, 0.0);
        T.tmean.assign(T.nout, 0.0);
        T.tstd.assign(T.nout, 0.0);
        for (int s = 0; s < T.nsamp; ++s) {
          for (int i = 0; i < T.nin; ++i) T.fmean[i] += T.X[(size_t)s * T.nin + i] / T.nsamp;
          for (int i = 0; i < T.nout; ++i) T.tmean[i] += T.T[(size_t)s * T.nout + i] / T.nsamp;
        }
        for (int s = 0; s < T.nsamp; ++s) {
          for (int i = 0; i < T.nin; ++i) {
            const double d = T.X[(size_t)s * T.nin + i] - T.fmean[i];
            T.fstd[i] += d * d / T.nsamp;
          }
          for (int i = 0; i < T.nout; ++i) {
            const double d = T.T[(size_t)s * T.nout + i] - T.tmean[i];
            T.tstd[i] += d * d / T.nsamp;
          }
        }
        // Descriptors are O(0.1 - 5).  One that barely varies over the training set
        // (a rigid bond length, a one-hot) keeps a scale of at least 0.1, so that a
        // small departure at prediction time is not blown up into a huge input.
        for (auto& x : T.fstd) x = std::max(std::sqrt(x), 0.1);
        for (auto& x : T.tstd) x = std::max(std::sqrt(x), 1e-6);
        init_theta(T, g->seed * 1000003ull + ti);
        T.normalised = true;
      }
      // normalised FP32 data on the device
      std::vector<float> Xn((size_t)T.nsamp * T.nin), Tn((size_t)T.nsamp * T.nout);
      for (int s = 0; s < T.nsamp; ++s) {
        for (int i = 0; i < T.nin; ++i) Xn[(size_t)s * T.nin + i] = (float)((T.X[(size_t)s * T.nin + i] - T.fmean[i]) / T.fstd[i]);
        for (int i = 0; i < T.nout; ++i) Tn[(size_t)s * T.nout + i] = (float)((T.T[(size_t)s * T.nout + i] - T.tmean[i]) / T.tstd[i]);
      }
      DevMem Xd = upload(Xn, st), Td = upload(Tn, st);
      ensure_device(T);
      const int bs = std::min(batch, T.nsamp);
      DevMem xb(sizeof(float) * (size_t)bs * T.nin), tb(sizeof(float) * (size_t)bs * T.nout);
      DevMem grad(sizeof(float) * T.theta_h.size()), idx(sizeof(int) * (size_t)T.nsamp);
      DevMem work(sizeof(float) * mlp_work_floats(T.widths, bs));
      std::vector<int> perm(T.nsamp);
      std::iota(perm.begin(), perm.end(), 0);
      std::mt19937_64 rng(g->seed * 7919ull + ti);
      // minibatch losses accumulate on the device; the host reads them once per epoch
      DevMem lacc(sizeof(double) * (size_t)std::max(epochs, 1));
      DFX_HIP(hipMemsetAsync(lacc.p, 0, lacc.n, st));
      std::vector<int> nbatch(epochs, 0);
      for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        DFX_HIP(hipMemcpyAsync(idx.p, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice, st));
        for (int s0 = 0; s0 + bs <= T.nsamp; s0 += bs) {
          gather_rows(Xd.as<float>(), idx.as<int>() + s0, bs, T.nin, xb.as<float>(), st);
          gather_rows(Td.as<float>(), idx.as<int>() + s0, bs, T.nout, tb.as<float>(), st);
          mlp_loss_grad_acc(T.widths, T.theta.as<float>(), xb.as<float>(), tb.as<float>(), bs, grad.as<float>(),
                            work.as<float>(), lacc.as<double>() + ep, st);
          mlp_adam(T.theta.as<float>(), grad.as<float>(), T.m.as<float>(), T.v.as<float>(),
                   (int64_t)T.theta_h.size(), ++T.adam_step, (float)lr, st);
          ++nbatch[ep];
        }
        // the permutation buffer is rewritten next epoch: wait for this epoch's gathers
        DFX_HIP(hipStreamSynchronize(st));
      }
      std::vector<double> lh(std::max(epochs, 1), 0.0);
      DFX_HIP(hipMemcpy(lh.data(), lacc.p, sizeof(double) * lh.size(), hipMemcpyDeviceToHost));
      for (int ep = 0; ep < epochs; ++ep) eloss[ep] += (nbatch[ep] ? lh[ep] / nbatch[ep] : 0.0) * T.nsamp;
      DFX_HIP(hipMemcpy(T.theta_h.data(), T.theta.p, sizeof(float) * T.theta_h.size(), hipMemcpyDeviceToHost));
      total += T.nsamp;
    }
    if (loss_out)
      for (int ep = 0; ep < epochs; ++ep) loss_out[ep] = total ? eloss[ep] / total : 0.0;
  });
}

int dfx_guess_predict(const dfx_guess* gc, const dfx_geom* geom, double* D) {
  return guard([&] {
    if (!gc || !D) throw Error(DFX_EINVAL, "dfx_guess_predict: NULL argument");
    guess_predict_density(gc, geom, D, nullptr);
    const GeomView v = view(gc, geom);
    for (size_t i = 0; i < (size_t)v.nbf * v.nbf; ++i)
      if (!std::isfinite(D[i])) throw Error(DFX_EINVAL, "dfx_guess_predict: non-finite prediction");
  });
}

int dfx_guess_info(const dfx_guess* g, int* ntypes, int32_t* desc) {
  return guard([&] {
    if (!g || !ntypes) throw Error(DFX_EINVAL, "dfx_guess_info: NULL argument");
    *ntypes = (int)g->types.size();
    if (desc)
      for (size_t i = 0; i < g->types.size(); ++i) {
        const GuessType& T = g->types[i];
        desc[6 * i] = T.diag;
        desc[6 * i + 1] = T.za;
        desc[6 * i + 2] = T.zb;
        desc[6 * i + 3] = T.nin;
        desc[6 * i + 4] = T.nout;
        desc[6 * i + 5] = T.nsamp;
      }
  });
}

int dfx_guess_export(const dfx_guess* g, int type, float* theta, double* fmean, double* fstd, double* tmean,
                     double* tstd) {
  return guard([&] {
    if (!g || type < 0 || type >= (int)g->types.size()) throw Error(DFX_EINVAL, "dfx_guess_export: bad type");
    const GuessType& T = g->types[type];
    if (!T.normalised) throw Error(DFX_EINVAL, "dfx_guess_export: not trained");
    if (theta) std::copy(T.theta_h.begin(), T.theta_h.end(), theta);
    if (fmean) std::copy(T.fmean.begin(), T.fmean.end(), fmean);
    if (fstd) std::copy(T.fstd.begin(), T.fstd.end(), fstd);
    if (tmean) std::copy(T.tmean.begin(), T.tmean.end(), tmean);
    if (tstd) std::copy(T.tstd.begin(), T.tstd.end(), tstd);
  });
}

int dfx_guess_import(dfx_guess* g, int is_atom, int za, int zb, const float* theta, const double* fmean,
                     const double* fstd, const double* tmean, const double* tstd) {
  return guard([&] {
    if (!g || !theta || !fmean || !fstd || !tmean || !tstd) throw Error(DFX_EINVAL, "dfx_guess_import: NULL argument");
    if (is_atom ? za != zb : za < zb) throw Error(DFX_EINVAL, "dfx_guess_import: atom types need Z_a == Z_b, pair types Z_a >= Z_b");
    channel(za);
    channel(zb);
    int t = g->find(is_atom != 0, za, zb);
    if (t < 0) {
      GuessType T;
      T.diag = is_atom != 0;
      T.za = za;
      T.zb = zb;
      T.nin = T.diag ? nfeat_diag() : nfeat_pair();
      T.nout = atom_nbf(g, za) * atom_nbf(g, zb);
      T.widths.push_back(T.nin);
      for (int i = 0; i < g->depth; ++i) T.widths.push_back(g->hidden);
      T.widths.push_back(T.nout);
      g->types.push_back(std::move(T));
      t = (int)g->types.size() - 1;
    }
    GuessType& T = g->types[t];
    T.theta_h.assign(theta, theta + mlp_nparams(T.widths));
    T.fmean.assign(fmean, fmean + T.nin);
    T.fstd.assign(fstd, fstd + T.nin);
    T.tmean.assign(tmean, tmean + T.nout);
    T.tstd.assign(tstd, tstd + T.nout);
    T.normalised = true;
    T.theta.release();  // re-uploaded, moments cleared, on next use
  });
}

int dfx_guess_samples(const dfx_guess* g, int type, double* X, double* T) {
  return guard([&] {
    if (!g || type < 0 || type >= (int)g->types.size()) throw Error(DFX_EINVAL, "dfx_guess_samples: bad type");
    const GuessType& Ty = g->types[type];
    if (X) std::copy(Ty.X.begin(), Ty.X.end(), X);
    if (T) std::copy(Ty.T.begin(), Ty.T.end(), T);
  });
}

int dfx_guess_features(const dfx_guess* g, const dfx_geom* geom, int a, int b, double* feat, double* frame,
                       int* nfeat) {
  return guard([&] {
    if (!g) throw Error(DFX_EINVAL, "dfx_guess_features: NULL model");
    const GeomView v = view(g, geom);
    if (a < 0 || b < 0 || a >= (int)v.r.size() || b >= (int)v.r.size()) throw Error(DFX_EINVAL, "bad atom index");
    const int nf = a == b ? nfeat_diag() : nfeat_pair();
    if (nfeat) *nfeat = nf;
    std::vector<double> f(nf);
    double F[3][3];
    pair_features(v.r, v.Z, a, b, g->rc, g->rc_env, f.data(), F);
    if (feat) std::copy(f.begin(), f.end(), feat);
    if (frame)
      for (int i = 0; i < 9; ++i) frame[i] = F[i / 3][i % 3];
  });
}

int dfx_sh_rotation(int l, const double* F, double* U) {
  return guard([&] {
    if (l < 0 || l > 3 || !F || !U) throw Error(DFX_EINVAL, "dfx_sh_rotation: bad argument");
    double Fm[3][3];
    for (int i = 0; i < 9; ++i) Fm[i / 3][i % 3] = F[i];
    const auto u = sh_rotation(l, Fm);
    std::copy(u.begin(), u.end(), U);
  });
}

int dfx_guess_save(const dfx_guess* g, const char* path) {
  return guard([&] {
    if (!g || !path) throw Error(DFX_EINVAL, "dfx_guess_save: NULL argument");
    std::ofstream f(path, std::ios::binary);
    if (!f) throw Error(DFX_EINVAL, std::string("dfx_guess_save: cannot open ") + path);
    auto w = [&](const void* p, size_t n) { f.write(reinterpret_cast<const char*>(p), n); };
    const char magic[8] = {'D', 'F', 'X', 'G', 'U', 'E', 'S', '2'};
    w(magic, 8);
    w(&g->rc, 8);
    w(&g->rc_env, 8);
    w(&g->hidden, 4);
    w(&g->depth, 4);
    w(&g->seed, 8);
    const int ne = (int)g->shells.size();
    w(&ne, 4);
    for (auto& kv : g->shells) {
      const int n = (int)kv.second.size();
      w(&kv.first, 4);
      w(&n, 4);
      w(kv.second.data(), 4 * n);
    }
    const int nt = (int)g->types.size();
    w(&nt, 4);
    for (const GuessType& T : g->types) {
      const int hdr[5] = {T.diag, T.za, T.zb, T.nin, T.nout};
      w(hdr, sizeof(hdr));
      const int tr = T.normalised;
      w(&tr, 4);
      if (!tr) continue;
      w(T.fmean.data(), 8 * T.nin);
      w(T.fstd.data(), 8 * T.nin);
      w(T.tmean.data(), 8 * T.nout);
      w(T.tstd.data(), 8 * T.nout);
      const int64_t np = (int64_t)T.theta_h.size();
      w(&np, 8);
      w(T.theta_h.data(), 4 * np);
    }
  });
}

int dfx_guess_load(const char* path, dfx_guess** out) {
  return guard([&] {
    if (!path || !out) throw Error(DFX_EINVAL, "dfx_guess_load: NULL argument");
    std::ifstream f(path, std::ios::binary);
    if (!f) throw Error(DFX_EINVAL, std::string("dfx_guess_load: cannot open ") + path);
    auto r = [&](void* p, size_t n) {
      f.read(reinterpret_cast<char*>(p), n);
      if (!f) throw Error(DFX_EINVAL, "dfx_guess_load: truncated file");
    };
    char magic[8];
    r(magic, 8);
    if (std::memcmp(magic, "DFXGUES2", 8) != 0) throw Error(DFX_EINVAL, "dfx_guess_load: not a model file");
    std::unique_ptr<dfx_guess> g(new dfx_guess());
    r(&g->rc, 8);
    r(&g->rc_env, 8);
    r(&g->hidden, 4);
    r(&g->depth, 4);
    r(&g->seed, 8);
    int ne = 0;
    r(&ne, 4);
    for (int e = 0; e < ne; ++e) {
      int Z = 0, n = 0;
      r(&Z, 4);
      r(&n, 4);
      std::vector<int> ls(n);
      r(ls.data(), 4 * n);
      g->shells[Z] = ls;
    }
    int nt = 0;
    r(&nt, 4);
    for (int t = 0; t < nt; ++t) {
      GuessType T;
      int hdr[5];
      r(hdr, sizeof(hdr));
      T.diag = hdr[0];
      T.za = hdr[1];
      T.zb = hdr[2];
      T.nin = hdr[3];
      T.nout = hdr[4];
      T.widths.push_back(T.nin);
      for (int i = 0; i < g->depth; ++i) T.widths.push_back(g->hidden);
      T.widths.push_back(T.nout);
      int tr = 0;
      r(&tr, 4);
      if (tr) {
        T.fmean.resize(T.nin);
        T.fstd.resize(T.nin);
        T.tmean.resize(T.nout);
        T.tstd.resize(T.nout);
        r(T.fmean.data(), 8 * T.nin);
        r(T.fstd.data(), 8 * T.nin);
        r(T.tmean.data(), 8 * T.nout);
        r(T.tstd.data(), 8 * T.nout);
        int64_t np = 0;
        r(&np, 8);
        if (np != mlp_nparams(T.widths)) throw Error(DFX_EINVAL, "dfx_guess_load: parameter count mismatch");
        T.theta_h.resize(np);
        r(T.theta_h.data(), 4 * np);
        T.normalised = true;
      }
      g->types.push_back(std::move(T));
    }
    *out = g.release();
  });
}

}  // extern "C"
