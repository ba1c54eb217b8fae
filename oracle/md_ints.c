/*
 * ORACLE -- test infrastructure only.  Nothing in the product path may link,
 * load or call this file; it exists to check the GPU path.
 *
 * Plain FP64 McMurchie-Davidson Gaussian integrals (Hermite expansion
 * coefficients E^{ij}_t and Hermite Coulomb integrals R_{tuv}), the textbook
 * route of Helgaker, Jorgensen & Olsen, "Molecular Electronic-Structure
 * Theory", ch. 9.  The paper evaluates electron-repulsion integrals by Rys
 * quadrature (section "Molecular integrals"); the oracle deliberately uses a
 * different exact algorithm so that the two share nothing but the definition
 *
 *     (ab|c) = int int phi_a(r1) phi_b(r1) |r1 - r2|^-1 phi_c(r2) dr1 dr2 .
 *
 * Shells arrive already normalised: coef[k] multiplies the *unnormalised*
 * Cartesian primitive x^i y^j z^k exp(-alpha r^2), and sph[l] maps Cartesian
 * monomials (lexicographic order, x-power descending) to real solid harmonics
 * m = -l..l.  Both tables are made by the Python side of the oracle.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LMAX 6          /* highest l of any single shell the oracle accepts */
#define LTOT 24         /* highest total l of an integral (4 * LMAX) */

static const double PI = 3.14159265358979323846264338327950288;

typedef struct {
  int nsh;
  const double *ctr;     /* [nsh][3] */
  const int *l;          /* [nsh] */
  const int *nprim;      /* [nsh] */
  const int *poff;       /* [nsh] offset into exps/coef */
  const double *exps;
  const double *coef;    /* normalised primitive coefficients */
  const int *foff;       /* [nsh] first spherical function */
} obasis;

/* sph tables: for each l, a (2l+1) x ncart(l) row-major matrix */
static const double *g_sph[LMAX + 1];

void oracle_set_sph(int l, const double *tab) { g_sph[l] = tab; }

static inline int ncart(int l) { return (l + 1) * (l + 2) / 2; }

static void cart_powers(int l, int (*p)[3]) {
  int n = 0;
  for (int i = l; i >= 0; --i)
    for (int j = l - i; j >= 0; --j) {
      p[n][0] = i; p[n][1] = j; p[n][2] = l - i - j; ++n;
    }
}

/* ---- Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt, m = 0..mmax ---- */
void oracle_boys(int mmax, double T, double *F) {
  if (T < 1e-15) {
    /* F_m(T) = sum_k (-T)^k / (k! (2m+2k+1)); two terms suffice here */
    for (int m = 0; m <= mmax; ++m) F[m] = 1.0 / (2 * m + 1) - T / (2 * m + 3);
    return;
  }
  const double eT = exp(-T);
  if (T < 50.0) {
    /* series: F_m(T) = e^{-T} sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)),
       all terms positive; then downward recursion, which is stable */
    double term = 1.0 / (2 * mmax + 1), sum = term;
    for (int k = 1; k < 4000; ++k) {
      term *= 2.0 * T / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    F[mmax] = eT * sum;
    for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + eT) / (2 * m + 1);
  } else {
    /* F_0 from the error function, then upward recursion (stable for T > m) */
    F[0] = 0.5 * sqrt(PI / T) * erf(sqrt(T));
    for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - eT) / (2.0 * T);
  }
}

/* ---- Hermite expansion coefficients for one Cartesian direction ----
 * E[i][j][t], i <= la, j <= lb, t <= i + j, for the product
 * x_A^i exp(-a x_A^2) x_B^j exp(-b x_B^2), with XAB = A - B.          */
#define ED (2 * LMAX + 3)
static void hermite_E(int la, int lb, double a, double b, double XAB,
                      double E[ED][ED][2 * ED]) {
  const double p = a + b, mu = a * b / p;
  const double XPA = -b / p * XAB, XPB = a / p * XAB, h = 0.5 / p;
  for (int i = 0; i <= la; ++i)
    for (int j = 0; j <= lb; ++j)
      for (int t = 0; t <= i + j + 1; ++t) E[i][j][t] = 0.0;
  E[0][0][0] = exp(-mu * XAB * XAB);
  for (int i = 0; i <= la; ++i) {
    for (int j = 0; j <= lb; ++j) {
      if (i == 0 && j == 0) continue;
      for (int t = 0; t <= i + j; ++t) {
        double v;
        if (i > 0) {
          v = XPA * E[i - 1][j][t];
          if (t > 0) v += h * E[i - 1][j][t - 1];
          if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
        } else {
          v = XPB * E[i][j - 1][t];
          if (t > 0) v += h * E[i][j - 1][t - 1];
          if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
        }
        E[i][j][t] = v;
      }
    }
  }
}

/* ---- Hermite Coulomb integrals R_{tuv} = R^0_{tuv}(alpha, X,Y,Z), t+u+v <= L ----
 * R^n_{000} = (-2 alpha)^n F_n(alpha R^2) and
 * R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v} (likewise u, v). */
#define RD (LTOT + 1)
static void hermite_R(int L, double alpha, double X, double Y, double Z, double *R) {
  double F[LTOT + 1];
  oracle_boys(L, alpha * (X * X + Y * Y + Z * Z), F);
  double *cur = (double *)malloc(sizeof(double) * RD * RD * RD);
  double *nxt = (double *)malloc(sizeof(double) * RD * RD * RD);
#define IX(t, u, v) (((t) * RD + (u)) * RD + (v))
  double f = 1.0;
  for (int n = 0; n < L; ++n) f *= -2.0 * alpha;
  cur[IX(0, 0, 0)] = f * F[L];
  for (int n = L - 1; n >= 0; --n) {
    f /= -2.0 * alpha;
    nxt[IX(0, 0, 0)] = f * F[n];
    const int N = L - n;
    for (int tot = 1; tot <= N; ++tot)
      for (int t = 0; t <= tot; ++t)
        for (int u = 0; u <= tot - t; ++u) {
          const int v = tot - t - u;
          double r;
          if (t > 0) {
            r = X * cur[IX(t - 1, u, v)];
            if (t > 1) r += (t - 1) * cur[IX(t - 2, u, v)];
          } else if (u > 0) {
            r = Y * cur[IX(t, u - 1, v)];
            if (u > 1) r += (u - 1) * cur[IX(t, u - 2, v)];
          } else {
            r = Z * cur[IX(t, u, v - 1)];
            if (v > 1) r += (v - 1) * cur[IX(t, u, v - 2)];
          }
          nxt[IX(t, u, v)] = r;
        }
    double *tmp = cur; cur = nxt; nxt = tmp;
  }
  for (int t = 0; t <= L; ++t)
    for (int u = 0; u <= L - t; ++u)
      for (int v = 0; v <= L - t - u; ++v) R[IX(t, u, v)] = cur[IX(t, u, v)];
  free(cur);
  free(nxt);
#undef IX
}
#define RIX(t, u, v) (((t) * RD + (u)) * RD + (v))

/* Hermite expansion of one (bra) product in all three directions */
/* The product centre P = (a A + b B) / p is kept as A and P - A = b (B - A) / p:
   differences of product centres are then formed from centre differences, so
   they vanish exactly for concentric functions and do not depend on where the
   origin lies (P itself, rounded, carries an error of the size of the
   coordinates' last digit). */
typedef struct {
  double Ex[ED][ED][2 * ED], Ey[ED][ED][2 * ED], Ez[ED][ED][2 * ED];
  double p, A[3], PA[3];
} hprod;

static void make_prod(hprod *h, int la, int lb, double a, const double *A, double b,
                      const double *B) {
  h->p = a + b;
  for (int k = 0; k < 3; ++k) {
    h->A[k] = A[k];
    h->PA[k] = b / h->p * (B[k] - A[k]);
  }
  hermite_E(la, lb, a, b, A[0] - B[0], h->Ex);
  hermite_E(la, lb, a, b, A[1] - B[1], h->Ey);
  hermite_E(la, lb, a, b, A[2] - B[2], h->Ez);
}

/* P - Q of a bra and a ket product */
static void pq_diff(const hprod *b, const hprod *k, double d[3]) {
  for (int i = 0; i < 3; ++i) d[i] = (b->A[i] - k->A[i]) + (b->PA[i] - k->PA[i]);
}

/* P - C for a point C */
static void pc_diff(const hprod *h, const double *C, double d[3]) {
  for (int i = 0; i < 3; ++i) d[i] = (h->A[i] - C[i]) + h->PA[i];
}

/* ---- spherical transform of one index of a contracted Cartesian block ----
 * in:  [pre][ncart(l)][post]   out: [pre][2l+1][post]                      */
static void sph_index(const double *in, double *out, int pre, int l, int post) {
  const int nc = ncart(l), ns = 2 * l + 1;
  const double *T = g_sph[l];
  for (int i = 0; i < pre; ++i)
    for (int m = 0; m < ns; ++m)
      for (int k = 0; k < post; ++k) {
        double s = 0.0;
        for (int c = 0; c < nc; ++c) s += T[m * nc + c] * in[(i * nc + c) * post + k];
        out[(i * ns + m) * post + k] = s;
      }
}

/* ---- generic two-electron integral over up to four shells ----
 * (ab|cd), with b and/or d replaced by an l = 0, alpha = 0 "unit" function
 * for three- and two-centre integrals.  Result: spherical block
 * [2la+1][2lb+1][2lc+1][2ld+1] (unit shells count as size 1).           */
typedef struct { double ctr[3]; int l, nprim, unit; const double *exps, *coef; } oshell;

static oshell get_shell(const obasis *bs, int s) {
  oshell o;
  for (int k = 0; k < 3; ++k) o.ctr[k] = bs->ctr[3 * s + k];
  o.l = bs->l[s];
  o.nprim = bs->nprim[s];
  o.exps = bs->exps + bs->poff[s];
  o.coef = bs->coef + bs->poff[s];
  o.unit = 0;
  return o;
}

static const double UNIT_EXP = 0.0, UNIT_COEF = 1.0;
static oshell unit_shell(const double *ctr) {
  oshell o;
  for (int k = 0; k < 3; ++k) o.ctr[k] = ctr[k];
  o.l = 0; o.nprim = 1; o.exps = &UNIT_EXP; o.coef = &UNIT_COEF;
  o.unit = 1;  /* the constant function 1: no solid-harmonic factor */
  return o;
}

static void eri_generic(const oshell *A, const oshell *B, const oshell *C, const oshell *D,
                        double *out) {
  const int la = A->l, lb = B->l, lc = C->l, ld = D->l;
  const int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
  int pa[28][3], pb[28][3], pc[28][3], pd[28][3];
  cart_powers(la, pa); cart_powers(lb, pb); cart_powers(lc, pc); cart_powers(ld, pd);
  const int ntot = na * nb * nc * nd;
  double *cart = (double *)calloc(ntot, sizeof(double));
  double *R = (double *)malloc(sizeof(double) * RD * RD * RD);
  hprod *hb = (hprod *)malloc(sizeof(hprod));
  hprod *hk = (hprod *)malloc(sizeof(hprod));
  const int L = la + lb + lc + ld;
  for (int ia = 0; ia < A->nprim; ++ia)
    for (int ib = 0; ib < B->nprim; ++ib) {
      make_prod(hb, la, lb, A->exps[ia], A->ctr, B->exps[ib], B->ctr);
      const double cab = A->coef[ia] * B->coef[ib];
      for (int ic = 0; ic < C->nprim; ++ic)
        for (int id = 0; id < D->nprim; ++id) {
          make_prod(hk, lc, ld, C->exps[ic], C->ctr, D->exps[id], D->ctr);
          const double p = hb->p, q = hk->p, alpha = p * q / (p + q);
          double d[3];
          pq_diff(hb, hk, d);
          hermite_R(L, alpha, d[0], d[1], d[2], R);
          const double pref = cab * C->coef[ic] * D->coef[id] * 2.0 * pow(PI, 2.5) /
                              (p * q * sqrt(p + q));
          int idx = 0;
          for (int a = 0; a < na; ++a)
            for (int b = 0; b < nb; ++b)
              for (int c = 0; c < nc; ++c)
                for (int d = 0; d < nd; ++d, ++idx) {
                  const int ax = pa[a][0] + 0, ay = pa[a][1], az = pa[a][2];
                  const int bx = pb[b][0], by = pb[b][1], bz = pb[b][2];
                  const int cx = pc[c][0], cy = pc[c][1], cz = pc[c][2];
                  const int dx = pd[d][0], dy = pd[d][1], dz = pd[d][2];
                  double s = 0.0;
                  for (int t = 0; t <= ax + bx; ++t)
                    for (int u = 0; u <= ay + by; ++u)
                      for (int v = 0; v <= az + bz; ++v) {
                        const double eb = hb->Ex[ax][bx][t] * hb->Ey[ay][by][u] * hb->Ez[az][bz][v];
                        if (eb == 0.0) continue;
                        double sk = 0.0;
                        for (int tt = 0; tt <= cx + dx; ++tt)
                          for (int uu = 0; uu <= cy + dy; ++uu)
                            for (int vv = 0; vv <= cz + dz; ++vv) {
                              const double ek = hk->Ex[cx][dx][tt] * hk->Ey[cy][dy][uu] *
                                                hk->Ez[cz][dz][vv];
                              const double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                              sk += sg * ek * R[RIX(t + tt, u + uu, v + vv)];
                            }
                        s += eb * sk;
                      }
                  cart[idx] += pref * s;
                }
        }
    }
  /* spherical transforms, index by index */
  const int sa = 2 * la + 1, sb = 2 * lb + 1, sc = 2 * lc + 1, sd = 2 * ld + 1;
  double *t1 = (double *)malloc(sizeof(double) * ntot);
  double *t2 = (double *)malloc(sizeof(double) * ntot);
  sph_index(cart, t1, 1, la, nb * nc * nd);
  if (B->unit) memcpy(t2, t1, sizeof(double) * sa * nc * nd);
  else sph_index(t1, t2, sa, lb, nc * nd);
  sph_index(t2, t1, sa * sb, lc, nd);
  if (D->unit) memcpy(out, t1, sizeof(double) * sa * sb * sc);
  else sph_index(t1, out, sa * sb * sc, ld, 1);
  free(t1); free(t2); free(cart); free(R); free(hb); free(hk);
}

/* ---- public entry points (blocks and whole matrices) ---- */

/* (ab|cd) spherical block */
void oracle_eri4_block(const obasis *bs, int a, int b, int c, int d, double *out) {
  oshell A = get_shell(bs, a), B = get_shell(bs, b), C = get_shell(bs, c), D = get_shell(bs, d);
  eri_generic(&A, &B, &C, &D, out);
}

/* (ab|P) spherical block [na][nb][nP] */
void oracle_eri3_block(const obasis *bs, int a, int b, const obasis *ax, int c, double *out) {
  oshell A = get_shell(bs, a), B = get_shell(bs, b), C = get_shell(ax, c);
  oshell D = unit_shell(C.ctr);
  eri_generic(&A, &B, &C, &D, out);
}

/* (P|Q) spherical block */
void oracle_eri2_block(const obasis *ax, int p, int q, double *out) {
  oshell A = get_shell(ax, p), C = get_shell(ax, q);
  oshell B = unit_shell(A.ctr), D = unit_shell(C.ctr);
  eri_generic(&A, &B, &C, &D, out);
}

static int nsph_of(const obasis *bs, int s) { return 2 * bs->l[s] + 1; }

/* full metric (P|Q), naux x naux row-major */
void oracle_eri2(const obasis *ax, int naux, double *J) {
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < ax->nsh; ++p) {
    double blk[81 * 4];
    for (int q = 0; q <= p; ++q) {
      oracle_eri2_block(ax, p, q, blk);
      const int np = nsph_of(ax, p), nq = nsph_of(ax, q);
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < nq; ++j) {
          const double v = blk[i * nq + j];
          J[(size_t)(ax->foff[p] + i) * naux + ax->foff[q] + j] = v;
          J[(size_t)(ax->foff[q] + j) * naux + ax->foff[p] + i] = v;
        }
    }
  }
}

/* raw (mu nu|P) for a list of shell pairs, packed aux-major:
 * out[P][col_off[k] + i*nb + j] for pair k = (a_k, b_k).  Pairs whose
 * triplet (a,b,C) is screened (skip[k*nauxsh + C] != 0) are left as zero. */
void oracle_eri3_packed(const obasis *bs, const obasis *ax, int npairs, const int *pa,
                        const int *pb, const long long *col_off, long long ncols,
                        const unsigned char *skip, double *out) {
#pragma omp parallel for schedule(dynamic)
  for (int k = 0; k < npairs; ++k) {
    const int a = pa[k], b = pb[k];
    const int na = nsph_of(bs, a), nb = nsph_of(bs, b);
    double *blk = (double *)malloc(sizeof(double) * na * nb * 13 * 13);
    for (int C = 0; C < ax->nsh; ++C) {
      if (skip && skip[(size_t)k * ax->nsh + C]) continue;
      const int nc = nsph_of(ax, C);
      oracle_eri3_block(bs, a, b, ax, C, blk);
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j)
          for (int m = 0; m < nc; ++m)
            out[(size_t)(ax->foff[C] + m) * ncols + col_off[k] + i * nb + j] =
                blk[(i * nb + j) * nc + m];
    }
    free(blk);
  }
}

/* Schwarz factors: Qab[a*nsh+b] = sqrt(max_{mu in a, nu in b} (mu nu|mu nu)),
 * QC[C] = sqrt(max_{P in C} (P|P)). */
void oracle_schwarz(const obasis *bs, const obasis *ax, double *Qab, double *QC) {
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < bs->nsh; ++a) {
    const int na = nsph_of(bs, a);
    for (int b = 0; b <= a; ++b) {
      const int nb = nsph_of(bs, b);
      double *blk = (double *)malloc(sizeof(double) * na * nb * na * nb);
      oracle_eri4_block(bs, a, b, a, b, blk);
      double mx = 0.0;
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          const double v = blk[((i * nb + j) * na + i) * nb + j];
          if (v > mx) mx = v;
        }
      Qab[a * bs->nsh + b] = Qab[b * bs->nsh + a] = sqrt(mx);
      free(blk);
    }
  }
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < ax->nsh; ++c) {
    const int nc = nsph_of(ax, c);
    double blk[81 * 4];
    oracle_eri2_block(ax, c, c, blk);
    double mx = 0.0;
    for (int i = 0; i < nc; ++i)
      if (blk[i * nc + i] > mx) mx = blk[i * nc + i];
    QC[c] = sqrt(mx);
  }
}

/* full 4-index (mu nu|la si), nbf^4 -- tiny systems only */
void oracle_eri4(const obasis *bs, int nbf, double *G) {
  const int n = bs->nsh;
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < n; ++a) {
    double *blk = (double *)malloc(sizeof(double) * 13 * 13 * 13 * 13);
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c)
        for (int d = 0; d < n; ++d) {
          oracle_eri4_block(bs, a, b, c, d, blk);
          const int na = nsph_of(bs, a), nb = nsph_of(bs, b), nc = nsph_of(bs, c),
                    nd = nsph_of(bs, d);
          for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j)
              for (int k = 0; k < nc; ++k)
                for (int l = 0; l < nd; ++l)
                  G[(((size_t)(bs->foff[a] + i) * nbf + bs->foff[b] + j) * nbf + bs->foff[c] + k) *
                        nbf + bs->foff[d] + l] = blk[((i * nb + j) * nc + k) * nd + l];
        }
    free(blk);
  }
}

/* ---- one-electron integrals: overlap, kinetic, nuclear attraction ---- */
static void onee_block(const oshell *A, const oshell *B, int natom, const double *xyz,
                       const double *Z, double *S, double *T, double *V) {
  const int la = A->l, lb = B->l, na = ncart(la), nb = ncart(lb);
  int pa[28][3], pb[28][3];
  cart_powers(la, pa); cart_powers(lb, pb);
  double *cs = (double *)calloc(na * nb, sizeof(double));
  double *ct = (double *)calloc(na * nb, sizeof(double));
  double *cv = (double *)calloc(na * nb, sizeof(double));
  double *R = (double *)malloc(sizeof(double) * RD * RD * RD);
  hprod *h = (hprod *)malloc(sizeof(hprod));
  for (int ia = 0; ia < A->nprim; ++ia)
    for (int ib = 0; ib < B->nprim; ++ib) {
      const double a = A->exps[ia], b = B->exps[ib], p = a + b;
      const double w = A->coef[ia] * B->coef[ib];
      /* E up to lb + 2 for the kinetic energy */
      make_prod(h, la, lb + 2, a, A->ctr, b, B->ctr);
      const double s1 = sqrt(PI / p);
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          const int *e = pa[i], *f = pb[j];
          double S1[3], D1[3];
          for (int k = 0; k < 3; ++k) {
            double (*E)[ED][2 * ED] = k == 0 ? h->Ex : (k == 1 ? h->Ey : h->Ez);
            const int ii = e[k], jj = f[k];
            S1[k] = E[ii][jj][0] * s1;
            /* <i| d^2/dx^2 |j> = 4b^2 S(i,j+2) - 2b(2j+1) S(i,j) + j(j-1) S(i,j-2) */
            double d = 4.0 * b * b * E[ii][jj + 2][0] * s1 - 2.0 * b * (2 * jj + 1) * S1[k];
            if (jj >= 2) d += jj * (jj - 1) * E[ii][jj - 2][0] * s1;
            D1[k] = d;
          }
          cs[i * nb + j] += w * S1[0] * S1[1] * S1[2];
          ct[i * nb + j] += w * -0.5 *
                            (D1[0] * S1[1] * S1[2] + S1[0] * D1[1] * S1[2] + S1[0] * S1[1] * D1[2]);
        }
      for (int C = 0; C < natom; ++C) {
        double d[3];
        pc_diff(h, xyz + 3 * C, d);
        hermite_R(la + lb, p, d[0], d[1], d[2], R);
        const double pref = -Z[C] * 2.0 * PI / p * w;
        for (int i = 0; i < na; ++i)
          for (int j = 0; j < nb; ++j) {
            const int *e = pa[i], *f = pb[j];
            double s = 0.0;
            for (int t = 0; t <= e[0] + f[0]; ++t)
              for (int u = 0; u <= e[1] + f[1]; ++u)
                for (int v = 0; v <= e[2] + f[2]; ++v)
                  s += h->Ex[e[0]][f[0]][t] * h->Ey[e[1]][f[1]][u] * h->Ez[e[2]][f[2]][v] *
                       R[RIX(t, u, v)];
            cv[i * nb + j] += pref * s;
          }
      }
    }
  const int sa = 2 * la + 1;
  double *tmp = (double *)malloc(sizeof(double) * na * nb);
  sph_index(cs, tmp, 1, la, nb); sph_index(tmp, S, sa, lb, 1);
  sph_index(ct, tmp, 1, la, nb); sph_index(tmp, T, sa, lb, 1);
  sph_index(cv, tmp, 1, la, nb); sph_index(tmp, V, sa, lb, 1);
  free(tmp); free(cs); free(ct); free(cv); free(R); free(h);
}

void oracle_int1e(const obasis *bs, int nbf, int natom, const double *xyz, const double *Z,
                  double *S, double *T, double *V) {
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < bs->nsh; ++a) {
    double s[169], t[169], v[169];
    oshell A = get_shell(bs, a);
    for (int b = 0; b <= a; ++b) {
      oshell B = get_shell(bs, b);
      onee_block(&A, &B, natom, xyz, Z, s, t, v);
      const int na = nsph_of(bs, a), nb = nsph_of(bs, b);
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          const size_t r = bs->foff[a] + i, c = bs->foff[b] + j;
          S[r * nbf + c] = S[c * nbf + r] = s[i * nb + j];
          T[r * nbf + c] = T[c * nbf + r] = t[i * nb + j];
          V[r * nbf + c] = V[c * nbf + r] = v[i * nb + j];
        }
    }
  }
}

/* ======================================================================
 * Nuclear-coordinate derivatives (the analytic gradient of DF-RHF).
 *
 * Moving the centre A of a Cartesian Gaussian x_A^i exp(-alpha x_A^2)
 * differentiates it into
 *     d/dA_x = 2 alpha x_A^{i+1} e^{..} - i x_A^{i-1} e^{..},
 * so every derivative integral is a combination of ordinary integrals with
 * one power raised or lowered on the moved centre, primitive by primitive.
 * The contractions below weight the derivative blocks of all shell pairs and
 * triplets with dense spherical weight arrays and sum into per-atom
 * gradients.  Each centre is differentiated directly (no translational
 * shortcut), so the translational sum rule is a test of the code.
 * ====================================================================== */

/* primitive Cartesian (ab|cd) without the 2 pi^{5/2}/(p q sqrt(p+q)) prefactor,
   for arbitrary power triples, from the Hermite expansions and R */
static double prim_eri(const hprod *hb, const hprod *hk, const double *R, const int *a, const int *b,
                       const int *c, const int *d) {
  double s = 0.0;
  for (int t = 0; t <= a[0] + b[0]; ++t)
    for (int u = 0; u <= a[1] + b[1]; ++u)
      for (int v = 0; v <= a[2] + b[2]; ++v) {
        const double eb = hb->Ex[a[0]][b[0]][t] * hb->Ey[a[1]][b[1]][u] * hb->Ez[a[2]][b[2]][v];
        if (eb == 0.0) continue;
        double sk = 0.0;
        for (int tt = 0; tt <= c[0] + d[0]; ++tt)
          for (int uu = 0; uu <= c[1] + d[1]; ++uu)
            for (int vv = 0; vv <= c[2] + d[2]; ++vv) {
              const double ek = hk->Ex[c[0]][d[0]][tt] * hk->Ey[c[1]][d[1]][uu] * hk->Ez[c[2]][d[2]][vv];
              const double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
              sk += sg * ek * R[RIX(t + tt, u + uu, v + vv)];
            }
        s += eb * sk;
      }
  return s;
}

/* d(ab|cd)/d(centre `which`)_k, k = x, y, z, spherical: out [3][sa][sb][sc][sd].
   which: 0 = A, 1 = B, 2 = C, 3 = D.  A unit shell (the constant 1) has no
   derivative and is never the moved shell here. */
static void eri_generic_deriv(const oshell *A, const oshell *B, const oshell *C, const oshell *D, int which,
                              double *out) {
  const oshell *S[4] = {A, B, C, D};
  int l[4], n[4];
  for (int s = 0; s < 4; ++s) { l[s] = S[s]->l; n[s] = ncart(l[s]); }
  int pw[4][28][3];
  for (int s = 0; s < 4; ++s) cart_powers(l[s], pw[s]);
  const int ntot = n[0] * n[1] * n[2] * n[3];
  double *cart = (double *)calloc(3 * ntot, sizeof(double));
  double *R = (double *)malloc(sizeof(double) * RD * RD * RD);
  hprod *hb = (hprod *)malloc(sizeof(hprod));
  hprod *hk = (hprod *)malloc(sizeof(hprod));
  const int L = l[0] + l[1] + l[2] + l[3] + 1;
  const int up0 = which == 0, up1 = which == 1, up2 = which == 2, up3 = which == 3;
  for (int ia = 0; ia < A->nprim; ++ia)
    for (int ib = 0; ib < B->nprim; ++ib) {
      make_prod(hb, l[0] + up0, l[1] + up1, A->exps[ia], A->ctr, B->exps[ib], B->ctr);
      const double cab = A->coef[ia] * B->coef[ib];
      for (int ic = 0; ic < C->nprim; ++ic)
        for (int id = 0; id < D->nprim; ++id) {
          make_prod(hk, l[2] + up2, l[3] + up3, C->exps[ic], C->ctr, D->exps[id], D->ctr);
          const double p = hb->p, q = hk->p, alpha = p * q / (p + q);
          double d[3];
          pq_diff(hb, hk, d);
          hermite_R(L, alpha, d[0], d[1], d[2], R);
          const double pref = cab * C->coef[ic] * D->coef[id] * 2.0 * pow(PI, 2.5) / (p * q * sqrt(p + q));
          const double ex = which == 0 ? A->exps[ia] : which == 1 ? B->exps[ib] : which == 2 ? C->exps[ic]
                                                                                              : D->exps[id];
          int idx = 0;
          for (int a = 0; a < n[0]; ++a)
            for (int b = 0; b < n[1]; ++b)
              for (int c = 0; c < n[2]; ++c)
                for (int d = 0; d < n[3]; ++d, ++idx) {
                  int q4[4][3];
                  memcpy(q4[0], pw[0][a], sizeof q4[0]);
                  memcpy(q4[1], pw[1][b], sizeof q4[1]);
                  memcpy(q4[2], pw[2][c], sizeof q4[2]);
                  memcpy(q4[3], pw[3][d], sizeof q4[3]);
                  for (int k = 0; k < 3; ++k) {
                    int *w = q4[which];
                    const int i0 = w[k];
                    w[k] = i0 + 1;
                    double v = 2.0 * ex * prim_eri(hb, hk, R, q4[0], q4[1], q4[2], q4[3]);
                    if (i0 > 0) {
                      w[k] = i0 - 1;
                      v -= i0 * prim_eri(hb, hk, R, q4[0], q4[1], q4[2], q4[3]);
                    }
                    w[k] = i0;
                    cart[k * ntot + idx] += pref * v;
                  }
                }
        }
    }
  const int sa = 2 * l[0] + 1, sb = B->unit ? 1 : 2 * l[1] + 1, sc = 2 * l[2] + 1, sd = D->unit ? 1 : 2 * l[3] + 1;
  const int nsph = sa * sb * sc * sd;
  double *t1 = (double *)malloc(sizeof(double) * ntot);
  double *t2 = (double *)malloc(sizeof(double) * ntot);
  for (int k = 0; k < 3; ++k) {
    sph_index(cart + k * ntot, t1, 1, l[0], n[1] * n[2] * n[3]);
    if (B->unit) memcpy(t2, t1, sizeof(double) * sa * n[2] * n[3]);
    else sph_index(t1, t2, sa, l[1], n[2] * n[3]);
    sph_index(t2, t1, sa * sb, l[2], n[3]);
    if (D->unit) memcpy(out + k * nsph, t1, sizeof(double) * nsph);
    else sph_index(t1, out + k * nsph, sa * sb * sc, l[3], 1);
  }
  free(t1); free(t2); free(cart); free(R); free(hb); free(hk);
}

/* d(ab|P)/dR of one triplet: out [3 centres A, B, P][3 axes][na][nb][nP] */
void oracle_eri3_deriv_block(const obasis *bs, int a, int b, const obasis *ax, int c, double *out) {
  oshell A = get_shell(bs, a), B = get_shell(bs, b), C = get_shell(ax, c);
  oshell D = unit_shell(C.ctr);
  const int blk = 3 * nsph_of(bs, a) * nsph_of(bs, b) * nsph_of(ax, c);
  eri_generic_deriv(&A, &B, &C, &D, 0, out);
  eri_generic_deriv(&A, &B, &C, &D, 1, out + blk);
  eri_generic_deriv(&A, &B, &C, &D, 2, out + 2 * blk);
}

/* d(P|Q)/dR: out [2 centres P, Q][3 axes][nP][nQ] */
void oracle_eri2_deriv_block(const obasis *ax, int p, int q, double *out) {
  oshell A = get_shell(ax, p), C = get_shell(ax, q);
  oshell B = unit_shell(A.ctr), D = unit_shell(C.ctr);
  const int blk = 3 * nsph_of(ax, p) * nsph_of(ax, q);
  eri_generic_deriv(&A, &B, &C, &D, 0, out);
  eri_generic_deriv(&A, &B, &C, &D, 2, out + blk);
}

/* grad[atom][k] += sum_{mu nu P} Gam[P][mu][nu] d(mu nu|P)/dR_atom,k over all
   shells a, b (both orders) and auxiliary shells C; Gam dense [naux][nbf][nbf]. */
void oracle_eri3_grad(const obasis *bs, int nbf, const obasis *ax, int naux, const int *atom_bs,
                      const int *atom_ax, int natom, const double *Gam, double *grad) {
  for (int i = 0; i < 3 * natom; ++i) grad[i] = 0.0;
#pragma omp parallel
  {
    double *g = (double *)calloc((size_t)3 * (size_t)(natom > 0 ? natom : 0), sizeof(double));
    double *blk = (double *)malloc(sizeof(double) * 9 * 13 * 13 * 9);
#pragma omp for schedule(dynamic) collapse(2)
    for (int a = 0; a < bs->nsh; ++a)
      for (int b = 0; b < bs->nsh; ++b) {
        const int na = nsph_of(bs, a), nb = nsph_of(bs, b);
        for (int C = 0; C < ax->nsh; ++C) {
          const int nc = nsph_of(ax, C), bl = na * nb * nc;
          oracle_eri3_deriv_block(bs, a, b, ax, C, blk);
          const int at[3] = {atom_bs[a], atom_bs[b], atom_ax[C]};
          for (int w = 0; w < 3; ++w)
            for (int k = 0; k < 3; ++k) {
              double s = 0.0;
              for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j)
                  for (int m = 0; m < nc; ++m)
                    s += Gam[((size_t)(ax->foff[C] + m) * nbf + bs->foff[a] + i) * nbf + bs->foff[b] + j] *
                         blk[(w * 3 + k) * bl + (i * nb + j) * nc + m];
              g[3 * at[w] + k] += s;
            }
        }
      }
#pragma omp critical
    for (int i = 0; i < 3 * natom; ++i) grad[i] += g[i];
    free(g); free(blk);
  }
}

/* grad[atom][k] += sum_{PQ} Gam2[P][Q] d(P|Q)/dR_atom,k; Gam2 dense [naux][naux] */
void oracle_eri2_grad(const obasis *ax, int naux, const int *atom_ax, int natom, const double *Gam2,
                      double *grad) {
  for (int i = 0; i < 3 * natom; ++i) grad[i] = 0.0;
#pragma omp parallel
  {
    double *g = (double *)calloc((size_t)3 * (size_t)(natom > 0 ? natom : 0), sizeof(double));
    double blk[2 * 3 * 81];
#pragma omp for schedule(dynamic) collapse(2)
    for (int p = 0; p < ax->nsh; ++p)
      for (int q = 0; q < ax->nsh; ++q) {
        const int np = nsph_of(ax, p), nq = nsph_of(ax, q), bl = np * nq;
        oracle_eri2_deriv_block(ax, p, q, blk);
        const int at[2] = {atom_ax[p], atom_ax[q]};
        for (int w = 0; w < 2; ++w)
          for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int i = 0; i < np; ++i)
              for (int j = 0; j < nq; ++j)
                s += Gam2[(size_t)(ax->foff[p] + i) * naux + ax->foff[q] + j] * blk[(w * 3 + k) * bl + i * nq + j];
            g[3 * at[w] + k] += s;
          }
      }
#pragma omp critical
    for (int i = 0; i < 3 * natom; ++i) grad[i] += g[i];
    free(g);
  }
}

/* ---- one-electron derivatives ----
 * Primitive Cartesian S, T and V_C for arbitrary powers i (on A) and j (on B),
 * from the Hermite expansion of the product (E up to i + 1 and j + 3). */
static double prim_S(const hprod *h, const int *i, const int *j) {
  const double s1 = sqrt(PI / h->p);
  return h->Ex[i[0]][j[0]][0] * h->Ey[i[1]][j[1]][0] * h->Ez[i[2]][j[2]][0] * s1 * s1 * s1;
}

static double prim_T(const hprod *h, const int *i, const int *j, double b) {
  /* <i| -1/2 d^2/dx^2 |j> per axis: 4b^2 S(i,j+2) - 2b(2j+1) S(i,j) + j(j-1) S(i,j-2) */
  const double s1 = sqrt(PI / h->p);
  double S1[3], D1[3];
  for (int k = 0; k < 3; ++k) {
    double (*E)[ED][2 * ED] = (double (*)[ED][2 * ED])(k == 0 ? h->Ex : (k == 1 ? h->Ey : h->Ez));
    const int ii = i[k], jj = j[k];
    S1[k] = E[ii][jj][0] * s1;
    double d = 4.0 * b * b * E[ii][jj + 2][0] * s1 - 2.0 * b * (2 * jj + 1) * S1[k];
    if (jj >= 2) d += jj * (jj - 1) * E[ii][jj - 2][0] * s1;
    D1[k] = d;
  }
  return -0.5 * (D1[0] * S1[1] * S1[2] + S1[0] * D1[1] * S1[2] + S1[0] * S1[1] * D1[2]);
}

static double prim_V(const hprod *h, const double *R, const int *i, const int *j) {
  /* <i| 1/|r - C| |j> without the charge: 2 pi / p sum E E E R */
  double s = 0.0;
  for (int t = 0; t <= i[0] + j[0]; ++t)
    for (int u = 0; u <= i[1] + j[1]; ++u)
      for (int v = 0; v <= i[2] + j[2]; ++v)
        s += h->Ex[i[0]][j[0]][t] * h->Ey[i[1]][j[1]][u] * h->Ez[i[2]][j[2]][v] * R[RIX(t, u, v)];
  return 2.0 * PI / h->p * s;
}

/* d/dC_k of <i| 1/|r - C| |j>: R_tuv depends on P - C, and d R_tuv / dC_x = -R_t+1,u,v */
static double prim_V_dC(const hprod *h, const double *R, const int *i, const int *j, int k) {
  double s = 0.0;
  for (int t = 0; t <= i[0] + j[0]; ++t)
    for (int u = 0; u <= i[1] + j[1]; ++u)
      for (int v = 0; v <= i[2] + j[2]; ++v)
        s += h->Ex[i[0]][j[0]][t] * h->Ey[i[1]][j[1]][u] * h->Ez[i[2]][j[2]][v] *
             R[RIX(t + (k == 0), u + (k == 1), v + (k == 2))];
  return -2.0 * PI / h->p * s;
}

/* Gradient of 2 tr(D h) - 2 tr(W S) over all shell pairs (both orders), h = T + V,
   V = -sum_C Z_C / |r - C|: the derivatives of the basis functions on both
   centres, and of the operator on every nucleus C (moving C by itself).
   Dw, Ww dense [nbf][nbf], already carrying their factors (2 D, 2 W). */
void oracle_int1e_grad(const obasis *bs, int nbf, const int *atom_bs, int natom, const double *xyz,
                       const double *Z, const double *Dw, const double *Ww, double *grad) {
  for (int i = 0; i < 3 * natom; ++i) grad[i] = 0.0;
#pragma omp parallel
  {
    double *g = (double *)calloc((size_t)3 * (size_t)(natom > 0 ? natom : 0), sizeof(double));
    double *R = (double *)malloc(sizeof(double) * RD * RD * RD);
    hprod *h = (hprod *)malloc(sizeof(hprod));
#pragma omp for schedule(dynamic) collapse(2)
    for (int sa = 0; sa < bs->nsh; ++sa)
      for (int sb = 0; sb < bs->nsh; ++sb) {
        const oshell A = get_shell(bs, sa), B = get_shell(bs, sb);
        const int la = A.l, lb = B.l, na = ncart(la), nb = ncart(lb), ma = 2 * la + 1, mb = 2 * lb + 1;
        int pa[28][3], pb[28][3];
        cart_powers(la, pa); cart_powers(lb, pb);
        /* Cartesian weights: Wd = T_a^T Dw_block T_b, likewise Ws */
        double cd[28 * 28], cs[28 * 28];
        for (int i = 0; i < na; ++i)
          for (int j = 0; j < nb; ++j) {
            double sd = 0.0, ss = 0.0;
            for (int m = 0; m < ma; ++m)
              for (int nn = 0; nn < mb; ++nn) {
                const double t = g_sph[la][m * na + i] * g_sph[lb][nn * nb + j];
                const size_t o = (size_t)(bs->foff[sa] + m) * nbf + bs->foff[sb] + nn;
                sd += t * Dw[o];
                ss += t * Ww[o];
              }
            cd[i * nb + j] = sd;
            cs[i * nb + j] = ss;
          }
        for (int ia = 0; ia < A.nprim; ++ia)
          for (int ib = 0; ib < B.nprim; ++ib) {
            const double a = A.exps[ia], b = B.exps[ib], w = A.coef[ia] * B.coef[ib];
            make_prod(h, la + 1, lb + 3, a, A.ctr, b, B.ctr);
            /* basis-function derivatives on A and on B: S, T, and V of every nucleus */
            for (int i = 0; i < na; ++i)
              for (int j = 0; j < nb; ++j) {
                const double wd = cd[i * nb + j], ws = cs[i * nb + j];
                for (int mv = 0; mv < 2; ++mv) {          /* 0: centre A moves, 1: centre B */
                  const double ex = mv == 0 ? a : b;
                  const int at = mv == 0 ? atom_bs[sa] : atom_bs[sb];
                  for (int k = 0; k < 3; ++k) {
                    int ii[3] = {pa[i][0], pa[i][1], pa[i][2]}, jj[3] = {pb[j][0], pb[j][1], pb[j][2]};
                    int *q = mv == 0 ? ii : jj;
                    const int i0 = q[k];
                    q[k] = i0 + 1;
                    double dS = 2.0 * ex * prim_S(h, ii, jj), dT = 2.0 * ex * prim_T(h, ii, jj, b);
                    if (i0 > 0) {
                      q[k] = i0 - 1;
                      dS -= i0 * prim_S(h, ii, jj);
                      dT -= i0 * prim_T(h, ii, jj, b);
                    }
                    g[3 * at + k] += w * (wd * dT - ws * dS);
                  }
                }
              }
            for (int C = 0; C < natom; ++C) {
              const double *Cc = xyz + 3 * C;
              double d[3];
              pc_diff(h, Cc, d);
              hermite_R(la + lb + 1, h->p, d[0], d[1], d[2], R);
              for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                  const double wd = cd[i * nb + j];
                  if (wd == 0.0) continue;
                  double dv[2][3];
                  for (int mv = 0; mv < 2; ++mv) {
                    const double ex = mv == 0 ? a : b;
                    for (int k = 0; k < 3; ++k) {
                      int ii[3] = {pa[i][0], pa[i][1], pa[i][2]}, jj[3] = {pb[j][0], pb[j][1], pb[j][2]};
                      int *q = mv == 0 ? ii : jj;
                      const int i0 = q[k];
                      q[k] = i0 + 1;
                      double v = 2.0 * ex * prim_V(h, R, ii, jj);
                      if (i0 > 0) {
                        q[k] = i0 - 1;
                        v -= i0 * prim_V(h, R, ii, jj);
                      }
                      dv[mv][k] = -Z[C] * v;
                    }
                  }
                  const int ii[3] = {pa[i][0], pa[i][1], pa[i][2]}, jj[3] = {pb[j][0], pb[j][1], pb[j][2]};
                  for (int k = 0; k < 3; ++k) {
                    g[3 * atom_bs[sa] + k] += w * wd * dv[0][k];
                    g[3 * atom_bs[sb] + k] += w * wd * dv[1][k];
                    /* the operator's own derivative: nucleus C moving alone */
                    g[3 * C + k] += w * wd * -Z[C] * prim_V_dC(h, R, ii, jj, k);
                  }
                }
            }
          }
      }
#pragma omp critical
    for (int i = 0; i < 3 * natom; ++i) grad[i] += g[i];
    free(g); free(R); free(h);
  }
}
