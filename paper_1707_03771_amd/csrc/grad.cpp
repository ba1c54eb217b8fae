// dfx_rhf_grad: the analytic nuclear gradient of the DF-RHF energy on the GPU
// (section "Standard algorithms": analytic gradients of the SCF methods;
// section "Molecular integrals": the integral derivatives; the fitted integrals
// are those of Eqs. (1)-(3)).
//
// With D = C_occ C_occ^T, W = C_occ diag(eps) C_occ^T, B_Q = sum_P (L^-1)_QP (mu nu|P)
// (J_PQ = L L^T), gamma = B d, b_Q = C^T B_Q C:
//   dE/dx = 2 tr(D h^x) - 2 tr(W S^x) + dE_nn/dx
//         + sum_{mu nu P} Gam_P,mu nu (mu nu|P)^x + sum_{PQ} Gam2_PQ (P|Q)^x,
//   Gam  = L^-T Gam~,  Gam~_Q = 4 gamma_Q D - 2 C b_Q C^T = 4 gamma_Q D - 2 (D X_Q) C^T,
//   Gam2 = L^-T (-2 gamma gamma^T + sum_ij b_ij b_ij^T) L^-1,
// where X_Q = B_Q C is the exchange build's half transform and ^x
// differentiates the integrals (the basis functions move with their atoms, the
// nuclear attraction operator with its nucleus); the orbital response enters
// only through W, the energy being stationary in the orbitals.
//
// Every step runs on the GPU: B (the SCF's dfx_eri3 path, keeping L), the
// weights (MFMA DGEMMs, the blocked back substitution L^-T), the derivative
// integrals contracted with the weights (grad_kernel.h, grad_misc.hip).  The
// kernels leave per-lane and per-workgroup partial sums that the host adds
// per atom in a fixed order, so the result is deterministic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "grad_kernel.h"
#include "host.h"

namespace dfx {

// ---- the three-index class dispatch ----------------------------------------------
void grad3_dispatch(int LA, int LB, int LC, int which, int axis, GradArgs ga, dim3 grid, int64_t pstride,
                    int64_t kstride, hipStream_t st) {
  const int key = ((LA * 4 + LB) * 2 + which) * 3 + axis;
#define G3(A_, B_, W_, X_)                                                                 \
  case ((A_ * 4 + B_) * 2 + W_) * 3 + X_:                                                 \
    grad3_class<A_, B_, W_, X_>(LC, ga, grid, pstride, kstride, st);                      \
    break;
  switch (key) {
    DFX_GRAD3_ALL(G3)
    default: throw Error(DFX_EUNSUPPORTED, "gradient: unsupported orbital angular momentum");
  }
#undef G3
}

static void grad2_dispatch(int LA, int LC, int axis, GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride,
                           hipStream_t st) {
  switch (axis) {
    case 0: grad2_class<0>(LA, LC, ga, grid, pstride, kstride, st); break;
    case 1: grad2_class<1>(LA, LC, ga, grid, pstride, kstride, st); break;
    default: grad2_class<2>(LA, LC, ga, grid, pstride, kstride, st); break;
  }
}

}  // namespace dfx

namespace dfx {

// atom of every shell: the atom whose coordinates equal the shell's centre
static std::vector<int> shell_atoms(const HostShells& h, const dfx_geom* g, const char* what) {
  std::vector<int> at(h.nsh);
  for (int s = 0; s < h.nsh; ++s) {
    int best = -1;
    for (int a = 0; a < g->natom; ++a) {
      const double* x = g->xyz + 3 * a;
      if (x[0] == h.ctr[3 * s] && x[1] == h.ctr[3 * s + 1] && x[2] == h.ctr[3 * s + 2]) {
        best = a;
        break;
      }
    }
    if (best < 0)
      throw Error(DFX_EINVAL, std::string("dfx_rhf_grad: ") + what + " shell " + std::to_string(s) +
                                  " is not centred on an atom of the geometry");
    at[s] = best;
  }
  return at;
}

// Q rows per chunk of the weight assembly: X and D X (nbf x q nocc each) and the
// dense -2 (D X_Q) C^T (q nbf^2) within about 4 GiB
static int grad_qchunk(int nbf, int nocc, int naux) {
  const double per_q = 8.0 * (2.0 * nbf * (double)nocc + 8.0 + (double)nbf * nbf);
  int q = (int)std::max(1.0, std::floor((double)((size_t)4 << 30) / per_q));
  return std::min(q, std::min(naux, 4096));
}

int64_t grad_need(const HostShells& b, const HostShells& a, int natom, int nocc) {
  const Eri3Need e = eri3_need(b, a, DFX_KEEP_METRIC);
  const int64_t n = b.nbf, na = a.nbf, no = nocc;
  const int64_t nsh = b.nsh, npall = nsh * (nsh + 1) / 2, ncb = e.bytes_raw / std::max<int64_t>(1, 8 * na);
  const int q = grad_qchunk((int)n, nocc, (int)na);
  auto p = [](int64_t x) { return (x + 255) / 256 * 256; };
  int64_t w = e.bytes_raw;                               // Gam in raw's columns
  w += p(8 * na * no * no) + 3 * p(8 * na * na);         // b, M, L^-T M and its transpose
  w += 2 * p(8 * n * (int64_t)q * no + 64) + p(8 * (int64_t)q * n * n);  // X, D X, the dense chunk
  w += 6 * p(8 * n * n) + p(8 * n * no) * 3 + p(8 * na) + p(8 * (2 * ncb + na + 8));  // D, W, C, gamma, J work
  w += 2 * p(4 * ncb) + (int64_t)(half_transform_f64_work(JKArgs{nullptr, nullptr, (int)na, (int)n,
                                                                  tiled_cols((int)n), PREC_FP64},
                                                           std::max(1, nocc)));
  // partial sums: per class launch at most 9 ket groups x 6 (centre, axis) x
  // (2048 x 128 lane slots + ket shells x workgroups), reused from class to class
  const int64_t slots = 2048 * 128 + 2048 + (int64_t)a.nsh * (npall / 128 + 2) + npall;
  w += p(8 * 9 * 6 * slots);
  // one-electron: Cartesian weights (two arrays) and partial sums
  w += 2 * p(8 * npall * 100) + p(8 * 6 * npall) + p(8 * (npall / 64 + 16) * natom * 3) + 64 * 256;
  const int64_t top = std::max(e.setup, w);
  return e.bottom + top + top / 64 + ((int64_t)32 << 20);
}

}  // namespace dfx

using namespace dfx;

extern "C" {

int dfx_grad_plan(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, int natom, int nocc,
                  int64_t* bytes) {
  return guard([&] {
    if (!bytes || natom <= 0 || nocc <= 0) throw Error(DFX_EINVAL, "dfx_grad_plan: bad argument");
    const HostShells hb = make_shells(shells, nsh, 3, "orbital basis");
    const HostShells ha = make_shells(aux, nauxsh, 4, "auxiliary basis");
    *bytes = grad_need(hb, ha, natom, nocc);
  });
}

int dfx_rhf_grad(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
                 const dfx_scf_opts* opts_in, const double* C_occ, const double* eps_occ, int nocc, double* grad,
                 dfx_grad_info* info) {
  return guard([&] {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (!geom || !C_occ || !eps_occ || !grad) throw Error(DFX_EINVAL, "dfx_rhf_grad: NULL argument");
    if (geom->natom <= 0 || !geom->xyz || !geom->Z) throw Error(DFX_EINVAL, "dfx_rhf_grad: bad geometry");
    dfx_scf_opts o;
    dfx_scf_default_opts(&o);
    if (opts_in) o = *opts_in;
    HostShells hb = make_shells(shells, nsh, 3, "orbital basis");
    HostShells ha = make_shells(aux, nauxsh, 4, "auxiliary basis");
    const int n = hb.nbf, naux = ha.nbf, natom = geom->natom;
    if (nocc <= 0 || nocc > n) throw Error(DFX_EINVAL, "dfx_rhf_grad: bad nocc");
    if (nocc > 512) throw Error(DFX_EUNSUPPORTED, "dfx_rhf_grad: more than 512 occupied orbitals");
    const std::vector<int> atb = shell_atoms(hb, geom, "orbital"), ata = shell_atoms(ha, geom, "auxiliary");
    std::unique_ptr<Arena> arena;
    if (o.workspace) {
      const int64_t need = grad_need(hb, ha, natom, nocc);
      if ((int64_t)o.ws_bytes < need)
        throw Error(DFX_ENOMEM, "dfx_rhf_grad: workspace of " + std::to_string(o.ws_bytes) + " bytes, " +
                                    std::to_string(need) + " needed (dfx_grad_plan)");
      arena = std::make_unique<Arena>(o.workspace, o.ws_bytes);
    }
    ArenaScope scope(arena.get());
    hipStream_t st = thread_ctx().st;
    const int64_t n2 = (int64_t)n * n;
    dfx_grad_info inf{};
    inf.natom = natom;
    EventSpans sp_w, sp_3, sp_2, sp_1;
    sp_w.st = sp_3.st = sp_2.st = sp_1.st = st;

    // ---- B, with L kept
    std::unique_ptr<dfx_B> B = build_B(std::move(hb), std::move(ha), o.tau, DFX_KEEP_METRIC, st);
    const HostShells& bas = B->bas;
    const HostShells& axs = B->aux;
    const int64_t ncols = B->ncols_p;
    const double* L = B->L.as<double>();
    inf.t_setup = B->info.eri_seconds + B->info.metric_seconds + B->info.trsm_seconds;

    // ---- D, W, gamma
    sp_w.begin();
    std::vector<double> eps_h(eps_occ, eps_occ + nocc);
    DevMem Cd(8 * (size_t)n * nocc), ed = upload(eps_h, st), Ce(8 * (size_t)n * nocc), D(8 * n2), Wm(8 * n2);
    DFX_HIP(hipMemcpyAsync(Cd.p, C_occ, Cd.n, hipMemcpyHostToDevice, st));
    auto gemm = [&](int M, int N, int K, const double* A, int64_t lda, bool ta, const double* Bm, int64_t ldb,
                    bool tb, double* C, int64_t ldc, double alpha, int batch = 1, int64_t sA = 0, int64_t sB = 0,
                    int64_t sC = 0) {
      GemmF64 g{};
      g.M = M; g.N = N; g.K = K;
      g.A = A; g.lda = lda; g.ta = ta; g.sA = sA;
      g.B = Bm; g.ldb = ldb; g.tb = tb; g.sB = sB;
      g.C = C; g.ldc = ldc; g.sC = sC;
      g.alpha = alpha; g.beta = 0.0; g.batch = batch;
      dgemm(g, st);
    };
    gemm(n, n, nocc, Cd.as<double>(), nocc, false, Cd.as<double>(), nocc, true, D.as<double>(), n, 1.0);
    scale_cols(Cd.as<double>(), ed.as<double>(), n, nocc, Ce.as<double>(), st);
    gemm(n, n, nocc, Ce.as<double>(), nocc, false, Cd.as<double>(), nocc, true, Wm.as<double>(), n, 1.0);
    const JKArgs ja{B->hi.as<float>(), B->lo.as<float>(), naux, n, B->ncols_t, PREC_FP64};
    DevMem gam(8 * (size_t)naux), dvec(8 * (size_t)B->ncols_t);
    j_gamma(ja, D.as<double>(), gam.as<double>(), dvec.as<double>(), st);
    dvec.release();

    // ---- Gam~ in raw's packed columns, b_Q = C^T X_Q, chunk by chunk of Q
    // (mu, nu) of every raw column (class by class, pair by pair, as the ERIs store it)
    std::vector<int> cmu(ncols), cnu(ncols);
    for (int cls = 0; cls < 16; ++cls) {
      const int SA = 2 * (cls / 4) + 1, SB = 2 * (cls % 4) + 1;
      const int64_t npc = (int64_t)B->cls_f[cls].size();
      for (int64_t p = 0; p < npc; ++p)
        for (int ma = 0; ma < SA; ++ma)
          for (int mb = 0; mb < SB; ++mb) {
            const int64_t col = B->cls_base[cls] + p * (SA * SB) + (ma * SB + mb);
            cmu[col] = bas.foff[B->cls_f[cls][p]] + ma;
            cnu[col] = bas.foff[B->cls_s[cls][p]] + mb;
          }
    }
    DevMem cmu_d = upload(cmu, st), cnu_d = upload(cnu, st);
    DevMem Gam(8 * (size_t)naux * std::max<int64_t>(ncols, 1));
    const int64_t nsq = (int64_t)nocc * nocc;
    DevMem bmat(8 * (size_t)naux * nsq);
    {
      const int qc = grad_qchunk(n, nocc, naux);
      const int64_t ldx = (int64_t)qc * nocc;
      DevMem X(8 * (size_t)n * ldx + 64), U(8 * (size_t)n * ldx + 64), T(8 * (size_t)qc * n2),
          hw(half_transform_f64_work(ja, nocc));
      for (int q0 = 0; q0 < naux; q0 += qc) {
        const int nq = std::min(qc, naux - q0);
        const int64_t kw = (int64_t)nq * nocc;
        half_transform_f64(ja, Cd.as<double>(), nocc, q0, nq, X.as<double>(), ldx, hw.p, st);
        gemm(n, (int)kw, n, D.as<double>(), n, false, X.as<double>(), ldx, false, U.as<double>(), ldx, 1.0);
        // -2 (D X_Q) C^T per Q, then + 4 gamma_Q D, packed
        gemm(n, n, nocc, U.as<double>(), ldx, false, Cd.as<double>(), nocc, true, T.as<double>(), n, -2.0, nq, nocc, 0,
             n2);
        gam_pack(T.as<double>(), D.as<double>(), n, gam.as<double>() + q0, cmu_d.as<int>(), cnu_d.as<int>(), ncols, nq,
                 Gam.as<double>() + (int64_t)q0 * ncols, st);
        // b_Q = C^T X_Q
        gemm(nocc, nocc, n, Cd.as<double>(), nocc, true, X.as<double>(), ldx, false,
             bmat.as<double>() + (int64_t)q0 * nsq, nocc, 1.0, nq, 0, nocc, nsq);
      }
    }
    // M = sum_ij b_ij b_ij^T - 2 gamma gamma^T, Gam2 = L^-T M L^-1, Gam = L^-T Gam~
    DevMem M(8 * (size_t)naux * naux), Y(8 * (size_t)naux * naux);
    gemm(naux, naux, (int)nsq, bmat.as<double>(), nsq, false, bmat.as<double>(), nsq, true, M.as<double>(), naux, 1.0);
    bmat.release();
    rank1_sub2(M.as<double>(), gam.as<double>(), naux, st);
    trsm_solve_t(L, naux, M.as<double>(), naux, st);                // L^-T M
    transpose_sq(M.as<double>(), Y.as<double>(), naux, st);         // (L^-T M)^T = M L^-1
    trsm_solve_t(L, naux, Y.as<double>(), naux, st);                // L^-T M L^-1
    trsm_solve_t(L, naux, Gam.as<double>(), ncols, st);
    sp_w.end();

    std::vector<double> g((size_t)natom * 3, 0.0);
    const double* rys = rys_table_device();

    // ---- three-index derivatives, class by class
    {
      const double tau = o.tau;
      std::vector<std::vector<int>> auxby(5);
      for (int c = 0; c < axs.nsh; ++c) auxby[axs.l[c]].push_back(c);
      std::vector<DevMem> auxby_d(5), qcl_d(5);
      for (int l = 0; l <= 4; ++l) {
        auxby_d[l] = upload(auxby[l], st);
        std::vector<double> q;
        for (int c : auxby[l]) q.push_back(B->QC[c]);
        qcl_d[l] = upload(q, st);
      }
      const std::vector<std::vector<int>>& cf = B->cls_f;
      const std::vector<std::vector<int>>& cs = B->cls_s;
      std::vector<std::vector<double>> cq(16);
      for (int cls = 0; cls < 16; ++cls)
        for (size_t p = 0; p < cf[cls].size(); ++p) cq[cls].push_back(B->Qab[(size_t)cf[cls][p] * bas.nsh + cs[cls][p]]);
      sp_3.begin();
      for (int cls = 0; cls < 16; ++cls) {
        if (cf[cls].empty()) continue;
        DevMem f_d = upload(cf[cls], st), s_d = upload(cs[cls], st), q_d = upload(cq[cls], st);
        const int LA = cls / 4, LB = cls % 4;
        for (int lc = 0; lc <= 4; ++lc) {
          if (auxby[lc].empty()) continue;
          GradArgs ga{};
          Eri3Args& e = ga.e;
          e.F = B->dbas.view();
          e.S = B->dbas.view();
          e.K = B->daux.view();
          e.pf = f_d.as<int>();
          e.ps = s_d.as<int>();
          e.pq = q_d.as<double>();
          e.cbase = B->cls_base[cls];
          e.npairs = (int)cf[cls].size();
          e.kl = auxby_d[lc].as<int>();
          e.kq = qcl_d[lc].as<double>();
          e.nk = (int)auxby[lc].size();
          e.tau = tau;
          e.rys = rys;
          const dim3 grid = eri3_grid(e);
          ga.gam = Gam.as<double>();
          ga.ldg = ncols;
          ga.scale_off = 2.0;
          const int ng = grad_groups_of(LA, LB, lc);
          const int64_t ps = (int64_t)grid.y * e.npairs, ks = (int64_t)e.nk * grid.x;
          const int64_t per = (int64_t)ng * (ps + ks);
          DevMem part(8 * (size_t)per * 6);
          for (int w = 0; w < 2; ++w)
            for (int ax = 0; ax < 3; ++ax) {
              double* base = part.as<double>() + (int64_t)(w * 3 + ax) * per;
              ga.pbuf = base;
              ga.kbuf = base + (int64_t)ng * ps;
              grad3_dispatch(LA, LB, lc, w, ax, ga, grid, ps, ks, st);
            }
          DFX_HIP(hipGetLastError());
          std::vector<double> h((size_t)per * 6);
          DFX_HIP(hipMemcpyAsync(h.data(), part.p, 8 * h.size(), hipMemcpyDeviceToHost, st));
          DFX_HIP(hipStreamSynchronize(st));
          for (int w = 0; w < 2; ++w)
            for (int ax = 0; ax < 3; ++ax) {
              const double* base = h.data() + (int64_t)(w * 3 + ax) * per;
              for (int gi = 0; gi < ng; ++gi) {
                const double* pb = base + gi * ps;
                for (unsigned y = 0; y < grid.y; ++y)
                  for (int p = 0; p < e.npairs; ++p) {
                    const int sh = w == 0 ? cf[cls][p] : cs[cls][p];
                    g[3 * atb[sh] + ax] += pb[(int64_t)y * e.npairs + p];
                  }
                const double* kb = base + (int64_t)ng * ps + gi * ks;
                for (int ci = 0; ci < e.nk; ++ci)
                  for (unsigned x = 0; x < grid.x; ++x) g[3 * ata[auxby[lc][ci]] + ax] += kb[(int64_t)ci * grid.x + x];
              }
            }
        }
      }
      sp_3.end();

      // ---- metric derivatives: (P|Q) with the first auxiliary shell moved
      sp_2.begin();
      for (int la = 0; la <= 4; ++la)
        for (int lc = 0; lc <= 4; ++lc) {
          if (auxby[la].empty() || auxby[lc].empty()) continue;
          GradArgs ga{};
          Eri3Args& e = ga.e;
          e.F = B->daux.view();
          e.S = B->daux.view();
          e.K = B->daux.view();
          e.pf = auxby_d[la].as<int>();
          e.npairs = (int)auxby[la].size();
          e.kl = auxby_d[lc].as<int>();
          e.nk = (int)auxby[lc].size();
          e.tau = -1.0;
          e.rys = rys;
          const dim3 grid = eri3_grid(e);
          ga.gam = Y.as<double>();
          ga.ldg = naux;
          ga.scale_off = 1.0;
          const int ng = grad_groups_of(la, 0, lc);
          const int64_t ps = (int64_t)grid.y * e.npairs, ks = (int64_t)e.nk * grid.x;
          const int64_t per = (int64_t)ng * (ps + ks);
          DevMem part(8 * (size_t)per * 3);
          for (int ax = 0; ax < 3; ++ax) {
            double* base = part.as<double>() + (int64_t)ax * per;
            ga.pbuf = base;
            ga.kbuf = base + (int64_t)ng * ps;
            grad2_dispatch(la, lc, ax, ga, grid, ps, ks, st);
          }
          DFX_HIP(hipGetLastError());
          std::vector<double> h((size_t)per * 3);
          DFX_HIP(hipMemcpyAsync(h.data(), part.p, 8 * h.size(), hipMemcpyDeviceToHost, st));
          DFX_HIP(hipStreamSynchronize(st));
          for (int ax = 0; ax < 3; ++ax) {
            const double* base = h.data() + (int64_t)ax * per;
            for (int gi = 0; gi < ng; ++gi) {
              const double* pb = base + gi * ps;
              for (unsigned y = 0; y < grid.y; ++y)
                for (int p = 0; p < e.npairs; ++p) g[3 * ata[auxby[la][p]] + ax] += pb[(int64_t)y * e.npairs + p];
              const double* kb = base + (int64_t)ng * ps + gi * ks;
              for (int ci = 0; ci < e.nk; ++ci)
                for (unsigned x = 0; x < grid.x; ++x) g[3 * ata[auxby[lc][ci]] + ax] += kb[(int64_t)ci * grid.x + x];
            }
          }
        }
      sp_2.end();
    }
    Gam.release();
    M.release();
    Y.release();

    // ---- one-electron terms: weights 2D (h) and 2W (S)
    sp_1.begin();
    {
      std::vector<double> xyz(geom->xyz, geom->xyz + 3 * natom), Zd(natom);
      for (int i = 0; i < natom; ++i) Zd[i] = geom->Z[i];
      DevMem xyz_d = upload(xyz, st), Z_d = upload(Zd, st);
      for (int la = 0; la <= 3; ++la)
        for (int lb = 0; lb <= 3; ++lb) {
          std::vector<int> pf, ps;
          std::vector<int64_t> wo;
          int64_t off = 0;
          for (int a = 0; a < bas.nsh; ++a)
            for (int b = 0; b <= a; ++b)
              if (bas.l[a] == la && bas.l[b] == lb) {
                pf.push_back(a);
                ps.push_back(b);
                wo.push_back(off);
                off += (int64_t)ncart(la) * ncart(lb);
              }
          if (pf.empty()) continue;
          const int np = (int)pf.size(), nblk = (np + 63) / 64;
          DevMem pf_d = upload(pf, st), ps_d = upload(ps, st), wo_d = upload(wo, st);
          DevMem wD(8 * (size_t)off), wW(8 * (size_t)off), pb(8 * (size_t)np * 6),
              nb(8 * (size_t)nblk * natom * 3);
          OneEGradArgs a1{};
          a1.sh = B->dbas.view();
          a1.pf = pf_d.as<int>();
          a1.ps = ps_d.as<int>();
          a1.npairs = np;
          a1.woff = wo_d.as<int64_t>();
          a1.wD = wD.as<double>();
          a1.wW = wW.as<double>();
          a1.xyz = xyz_d.as<double>();
          a1.Z = Z_d.as<double>();
          a1.natom = natom;
          a1.rys = rys;
          a1.pbuf = pb.as<double>();
          a1.nbuf = nb.as<double>();
          onee_grad_dispatch(la, lb, a1, D.as<double>(), Wm.as<double>(), n, 2.0, wD.as<double>(), wW.as<double>(),
                             st);
          DFX_HIP(hipGetLastError());
          std::vector<double> hp((size_t)np * 6), hn((size_t)nblk * natom * 3);
          DFX_HIP(hipMemcpyAsync(hp.data(), pb.p, 8 * hp.size(), hipMemcpyDeviceToHost, st));
          DFX_HIP(hipMemcpyAsync(hn.data(), nb.p, 8 * hn.size(), hipMemcpyDeviceToHost, st));
          DFX_HIP(hipStreamSynchronize(st));
          for (int p = 0; p < np; ++p)
            for (int k = 0; k < 3; ++k) {
              g[3 * atb[pf[p]] + k] += hp[(size_t)p * 6 + k];
              g[3 * atb[ps[p]] + k] += hp[(size_t)p * 6 + 3 + k];
            }
          for (int bl = 0; bl < nblk; ++bl)
            for (int c = 0; c < natom; ++c)
              for (int k = 0; k < 3; ++k) g[3 * c + k] += hn[((size_t)bl * natom + c) * 3 + k];
        }
    }
    sp_1.end();
    DFX_HIP(hipStreamSynchronize(st));

    // ---- nuclear repulsion
    for (int a = 0; a < natom; ++a)
      for (int b = 0; b < natom; ++b) {
        if (a == b) continue;
        const double* A = geom->xyz + 3 * a;
        const double* Bx = geom->xyz + 3 * b;
        const double d[3] = {A[0] - Bx[0], A[1] - Bx[1], A[2] - Bx[2]};
        const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int k = 0; k < 3; ++k) g[3 * a + k] -= (double)geom->Z[a] * geom->Z[b] * d[k] / (r * r * r);
      }
    std::copy(g.begin(), g.end(), grad);
    inf.t_weights = sp_w.seconds();
    inf.t_deriv3 = sp_3.seconds();
    inf.t_deriv2 = sp_2.seconds();
    inf.t_onee = sp_1.seconds();
    inf.t_total = std::chrono::duration<double>(clk::now() - t0).count();
    if (info) *info = inf;
  });
}

}  // extern "C"
