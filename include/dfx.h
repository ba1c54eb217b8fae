/*
 * dfx -- density-fitted Hartree-Fock hot path on AMD MI355X (gfx950).
 *
 * C-ABI of libdfx.so.  Plain pointers and sizes only.  The operations follow
 * the paper (T. Shiozaki, "BAGEL: Brilliantly Advanced General
 * Electronic-structure Library", arXiv:1707.03771):
 *   - three-index integrals kept in memory, Rys-quadrature ERIs
 *     (section "Molecular integrals"; "Introduction" on in-memory storage);
 *   - the density-fitting tensor operations of section "Density fitting
 *     utilities", Eqs. (1)-(3);
 *   - a DF-based restricted Hartree-Fock Fock builder (section "Standard
 *     algorithms"), and on the same fitted tensor the unrestricted and
 *     restricted open-shell variants and the MP2 correlation energy that
 *     section lists beside it.
 *
 * Conventions (all entry points):
 *   units       bohr and hartree.
 *   basis       spherical (real solid harmonic) functions; within a shell
 *               m = -l..l; m > 0 ~ cos(m phi), m < 0 ~ sin(|m| phi), no
 *               Condon-Shortley phase; function order = caller's shell order.
 *   shells      exps/coefs are host arrays of length nprim; coefs multiply
 *               normalised primitives and the contracted function is
 *               renormalised to unit norm.  Orbital shells: l <= 3; auxiliary
 *               shells: l <= 4.
 *   matrices    row-major FP64.  D, J, K, S, T, V: nbf x nbf.  C_occ: nbf x nocc.
 *   streams     `stream` is a hipStream_t (NULL = default stream); calls
 *               enqueue work on it and return, except where stated.
 *   errors      every call returns 0 (DFX_OK) or a negative DFX_E* code;
 *               dfx_last_error() returns the message of the calling thread's
 *               last failure.  No C++ exception crosses this boundary.
 *   ownership   device memory is the caller's.  Device pointers passed in are
 *               never freed by the library.  dfx_eri3 builds B inside a
 *               workspace the caller allocates (sized by dfx_eri3_plan); the
 *               dfx_B handle only describes it and draws dfx_jk's work from the
 *               same workspace, so the library allocates no device memory for
 *               them.  dfx_scf / dfx_uhf / dfx_rohf do the same with
 *               dfx_scf_opts.workspace (sized by dfx_scf_plan); without one
 *               they allocate per call.  The remaining entry points
 *               (dfx_mp2, dfx_lowdin, dfx_int1e, dfx_metric, dfx_cholesky, dfx_eigh, the
 *               learned guess) allocate their own scratch and free it before
 *               returning, except a guess model's weights, which it holds
 *               until dfx_guess_free.
 */
#ifndef DFX_H
#define DFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define DFX_OK 0
#define DFX_EINVAL (-1)        /* bad argument (null pointer, negative size, ...) */
#define DFX_ENOMEM (-2)        /* device allocation failed, or caller buffer too small */
#define DFX_EHIP (-3)          /* a HIP runtime call failed */
#define DFX_ENOTPOSDEF (-4)    /* fitting metric not positive definite */
#define DFX_ENOCONV (-5)       /* SCF did not converge (outputs still written) */
#define DFX_EUNSUPPORTED (-6)  /* angular momentum beyond the compiled classes */

/* ---- precisions / kinds ---------------------------------------------------- */
/* precision of K; J always reads B = hi + lo with FP64 accumulation */
#define DFX_FP64 0   /* B as hi + lo (FP64-equivalent), FP64 MFMA */
#define DFX_FP32 1   /* B hi word only, FP32 MFMA, FP32 sums of 32 products added in FP64 */
#define DFX_BF16 2   /* B hi word rounded to BF16, BF16 MFMA, the same accumulation */

#define DFX_DENSITY 0  /* dfx_jk input is D (nbf x nbf) */
#define DFX_COCC 1     /* dfx_jk input is C_occ (nbf x nocc); D = C_occ C_occ^T */

/* ---- inputs ------------------------------------------------------------------ */
typedef struct {
  double xyz[3];         /* centre (bohr) */
  int32_t l;             /* angular momentum */
  int32_t nprim;         /* number of primitives */
  const double* exps;    /* [nprim] host */
  const double* coefs;   /* [nprim] host */
} dfx_shell;

typedef struct {
  int32_t natom;
  const double* xyz;     /* [natom][3] host, bohr */
  const int32_t* Z;      /* [natom] host, nuclear charges */
  int32_t charge;        /* total molecular charge */
} dfx_geom;

/* ---- the fitted three-index tensor ---------------------------------------- */
typedef struct dfx_B dfx_B;

#define DFX_KEEP_RAW 1      /* keep the raw (mu nu|P) after the transform (tests) */
#define DFX_KEEP_METRIC 2   /* keep J_PQ and L (tests) */

typedef struct {
  double tau;            /* Schwarz threshold: (a,b,C) evaluated iff Q_ab Q_C >= tau */
  int32_t flags;         /* DFX_KEEP_* */
} dfx_eri3_opts;

typedef struct {
  int32_t nbf, naux;     /* basis and auxiliary function counts */
  int32_t nsh, nauxsh;   /* shell counts */
  int32_t npairs;        /* kept shell pairs a >= b */
  int64_t ncols;         /* canonical packed columns = sum over kept pairs of n_a n_b */
  int64_t ncols_tiled;   /* internal storage columns */
  int64_t ntriplets;     /* evaluated (a, b, C) triplets */
  int64_t nintegrals;    /* unique evaluated integrals: sum over triplets of n_a n_b n_C (a > b), n_a (n_a + 1)/2 n_C (a = b) */
  double eri_seconds;    /* GPU time of the three-index ERI kernels */
  double metric_seconds; /* metric + Cholesky + inverse */
  double trsm_seconds;   /* B = L^-1 raw (blocked forward substitution) with the FP32 split */
  double kappa_lb;       /* lower bound (max L_ii / min L_ii)^2 of cond(J_PQ) */
  double trsm_update_seconds;  /* the substitution's block updates R_i -= L_i,<i B_<i alone */
  double trsm_update_flops;    /* their FLOPs, 2 M K N summed */
  int32_t trsm_update_launches;
} dfx_B_info;

/*
 * dfx_eri3 -- raw integrals (mu nu|P) (section "Molecular integrals", Rys
 * quadrature), metric J_PQ = (P|Q), J_PQ = L L^T (plain Cholesky), and the
 * fitted tensor B_Q = sum_P (L^-1)_QP (mu nu|P) (Eq. (1c) with M' = L^-1),
 * stored as two FP32 words per element (hi = fl32(B), lo = fl32(B - hi)).
 *
 *   shells/nsh, aux/nauxsh   orbital and auxiliary shells (host)
 *   opts                     may be NULL (tau = 1e-12, flags = 0)
 *   dev_workspace, ws_bytes  device memory owned by the caller, at least
 *                            dfx_eri3_plan's bytes_workspace for the same
 *                            shells and flags; any alignment.  It must stay
 *                            allocated and untouched until dfx_B_free: B, the
 *                            setup's scratch and dfx_jk's work all live in it,
 *                            and the library allocates no device memory for
 *                            them.  The call checks the size before any device
 *                            work: smaller -> DFX_ENOMEM, nothing written.
 *   stream                   hipStream_t; the call synchronises it
 *   out                      receives a new handle (free with dfx_B_free)
 *
 * Screening: Q_ab = sqrt(max_{mu in a, nu in b} (mu nu|mu nu)), Q_C =
 * sqrt(max_{P in C} (P|P)); pair a >= b kept iff Q_ab max_C Q_C >= tau; its
 * block with C evaluated iff Q_ab Q_C >= tau, else zero.
 * Errors: DFX_EINVAL (also a NULL workspace), DFX_EUNSUPPORTED, DFX_ENOTPOSDEF
 * (no handle returned), DFX_ENOMEM, DFX_EHIP.
 */
int dfx_eri3(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, const dfx_eri3_opts* opts,
             void* dev_workspace, size_t ws_bytes, void* stream, dfx_B** out);

int dfx_B_info_get(const dfx_B* b, dfx_B_info* info);

/*
 * dfx_eri3_plan -- the workspace dfx_eri3 needs, host only (no GPU work, no
 * screening): function counts and upper bounds in bytes.  opts may be NULL
 * (its flags matter: kept raw integrals or metric stay in the workspace).
 * Errors as dfx_eri3.
 */
typedef struct {
  int32_t nbf, naux;
  int64_t ncols_tiled;      /* storage columns of B */
  int64_t bytes_B;          /* B's two FP32 words over the packed 32x32 tile layout */
  int64_t bytes_raw;        /* raw integrals during setup, as if no pair were screened */
  int64_t bytes_metric;     /* J_PQ and L during setup */
  int64_t bytes_persistent; /* in use from dfx_eri3's return until dfx_B_free: shells,
                               B, the metric's slot, kept metric / raw */
  int64_t bytes_jk;         /* the largest work of dfx_jk on this B (any kind,
                               precision, nocc <= 512) */
  int64_t bytes_workspace;  /* what to pass to dfx_eri3: persistent + the larger of
                               the setup scratch and dfx_jk's work, plus slack */
} dfx_eri3_sizes;
int dfx_eri3_plan(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, const dfx_eri3_opts* opts,
                  dfx_eri3_sizes* out);

/*
 * dfx_B_unpack -- rows q0..q1-1 of B as dense symmetric matrices,
 * dev_out[(q - q0) nbf nbf + mu nbf + nu] = B_q,mu nu (FP64 = hi + lo), device
 * memory of (q1 - q0) nbf^2 doubles owned by the caller.  Enqueued on stream.
 */
int dfx_B_unpack(const dfx_B* b, int q0, int q1, double* dev_out, void* stream);

/*
 * Integer lists of the screening (host buffers, the bit-exact contract):
 *   pairs   [2 * npairs]  (a, b) of each kept pair, canonical order a = 0..,
 *                         b = 0..a, a-major
 *   col_off [npairs + 1]  prefix sums of n_a n_b (int64)
 *   keep    [npairs * nauxsh] (may be NULL) 1 iff triplet (a, b, C) evaluated
 *   Qab     [nsh * nsh] (may be NULL) Schwarz factors, symmetric
 *   QC      [nauxsh]    (may be NULL)
 */
int dfx_B_lists(const dfx_B* b, int32_t* pairs, int64_t* col_off, uint8_t* keep, double* Qab,
                double* QC);

#define DFX_EXPORT_B 0     /* hi + lo (FP64 value) */
#define DFX_EXPORT_BHI 1   /* hi word only */
#define DFX_EXPORT_RAW 2   /* raw (mu nu|P), needs DFX_KEEP_RAW */
/*
 * Rows q0..q1-1 of B (or raw) in the canonical packed column order (pair
 * blocks n_a x n_b row-major in kept-pair order) into dev_out
 * [(q1 - q0) * ncols] FP64, device memory.
 */
int dfx_B_export(const dfx_B* b, int what, int q0, int q1, double* dev_out, void* stream);

/* J_PQ (what = 0) or L (what = 1), naux x naux, into dev_out; needs DFX_KEEP_METRIC. */
int dfx_B_metric(const dfx_B* b, int what, double* dev_out, void* stream);

int dfx_B_free(dfx_B* b);

/*
 * dfx_jk -- Coulomb and exchange matrices from B (section "Density fitting
 * utilities"): J = sum_Q B_Q gamma_Q with gamma_Q = sum B_Q D (Eqs. 3a, 3b);
 * K = sum_Q X_Q X_Q^T with X_Q = B_Q C_occ (Eqs. 1a, 2a).
 *   dev_in     kind = DFX_COCC: C_occ [nbf][nocc]; DFX_DENSITY: D [nbf][nbf]
 *              (symmetric).  For a density, K = sum_Q B_Q D B_Q through the
 *              signed factorisation D = C+ C+^T - C- C-^T from D's
 *              eigenvectors (eigenvalues below 1e-14 of the largest dropped);
 *              that call synchronises the stream.
 *   precision  DFX_FP64 | DFX_FP32 | DFX_BF16, for K.  J reads both words of B
 *              in every precision: it is bandwidth-bound, and from the hi word
 *              alone its error, amplified by the conditioning of the metric,
 *              would exceed that of the FP32 K (by about 100x on (H2O)64)
 *   dev_J, dev_K  nbf x nbf outputs, either may be NULL
 * Errors: DFX_EINVAL, DFX_ENOMEM, DFX_EHIP, DFX_EUNSUPPORTED.
 */
int dfx_jk(const dfx_B* b, const double* dev_in, int kind, int nocc, int precision, double* dev_J,
           double* dev_K, void* stream);

/*
 * dfx_jk_noalloc -- dfx_jk for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same J and K, from C_occ only, with the builds' scratch in a device array
 * that the library holds on every GPU it runs on, DFX_NOALLOC_SCRATCH_MIB
 * mebibytes per GPU, until the process ends.  It calls no hipMalloc / hipFree
 * and no allocating library routine, and does not touch B's workspace.
 *   dev_C      C_occ [nbf][nocc] device, 1 <= nocc <= min(nbf, 512)
 *   precision  as dfx_jk; dev_J, dev_K outputs as dfx_jk (either may be NULL)
 * The exchange build cuts the auxiliary index into as many chunks as the array
 * takes (more launches than dfx_jk for large systems; the sums run in another
 * order, so K agrees with dfx_jk to rounding, J bit for bit).  Sizes beyond
 * the array (about nbf > 2000) are rejected with DFX_ENOMEM before any work.
 * Every call on one GPU shares the array and it keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * GPU, on different streams or host threads, race and must be serialised by
 * the caller.  Enqueued on stream.
 * Errors: DFX_EINVAL, DFX_EUNSUPPORTED (nocc > 512), DFX_ENOMEM, DFX_EHIP.
 */
#define DFX_NOALLOC_SCRATCH_MIB 256
int dfx_jk_noalloc(const dfx_B* b, const double* dev_C, int nocc, int precision, double* dev_J, double* dev_K,
                   void* stream);

/*
 * dfx_mp2 -- DF-MP2 correlation energy of a closed-shell RHF reference (section
 * "Standard algorithms": MP2 as a post-HF method, on the density-fitting
 * operations of Eqs. (1) and (2)):
 *   (ia|Q) = sum C_mu,i B_Q,mu nu C_nu,a,  (ia|jb) = sum_Q (ia|Q)(jb|Q),
 *   E2 = sum_{ij,ab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b),
 * i, j over occupied orbitals nfrozen..nocc-1, a, b over nocc..nmo-1.  FP64.
 *   dev_C   device [nbf][nmo] row-major, column p = canonical orbital p (as dfx_scf
 *           returns C, its first nmo = nbf - ndropped columns)
 *   eps     host [nmo] orbital energies, ascending
 *   E2      host scalar out
 * Allocates device memory for (ia|Q) (nocc' x nvir x naux doubles) and one
 * block of (ia|jb) (nvir x nocc' x nvir doubles), nocc' = nocc - nfrozen <= 512.
 * Synchronises the stream.  Errors: DFX_EINVAL, DFX_ENOMEM, DFX_EHIP,
 * DFX_EUNSUPPORTED (more than 512 correlated occupied orbitals).
 */
int dfx_mp2(const dfx_B* b, const double* dev_C, int nmo, const double* eps, int nocc, int nfrozen, double* E2,
            void* stream);

/*
 * dfx_int1e -- overlap S, kinetic T and nuclear attraction
 * V = -sum_A Z_A <mu| 1/|r - R_A| |nu> (device outputs, nbf x nbf).
 */
int dfx_int1e(const dfx_shell* shells, int nsh, const dfx_geom* geom, double* dev_S, double* dev_T,
              double* dev_V, void* stream);

/*
 * dfx_metric -- the two-centre Coulomb metric J_PQ = (P|Q) of the auxiliary
 * basis (naux x naux, device output), by the same Rys kernels as dfx_eri3.
 */
int dfx_metric(const dfx_shell* aux, int nauxsh, double* dev_J, void* stream);

/*
 * dfx_cholesky -- J = L L^T for a symmetric positive definite n x n matrix
 * (device, row-major; only its lower triangle is read).  On return dev_A
 * holds L (upper triangle zeroed) and dev_Linv holds L^-1.  Plain blocked
 * Cholesky, no pivoting.  DFX_ENOTPOSDEF if a pivot falls below 1e-14 of its
 * original diagonal element.  Synchronises the stream.
 */
int dfx_cholesky(double* dev_A, int n, double* dev_Linv, void* stream);

/*
 * dfx_eigh -- all eigenpairs of a symmetric n x n matrix (device, row-major;
 * its symmetric part (A + A^T) / 2 is used), the eigen-decomposition behind
 * the SCF's orthogonaliser and orbitals (section "Standard algorithms").  On
 * return the rows of dev_A are orthonormal eigenvectors and dev_w (device, n)
 * holds the eigenvalues in ascending order, row k belonging to dev_w[k].
 * Two-sided block Jacobi (32 x 32 blocks, cyclic parallel ordering) until a
 * sweep finds every off-diagonal element below 1e-15 sqrt(|a_ii a_jj|).
 * Allocates its scratch (two padded copies of the matrix) and frees it
 * before returning; synchronises the stream.  *sweeps (may be NULL) gets the
 * number of Jacobi sweeps.  DFX_EHIP if 40 sweeps do not converge.
 */
int dfx_eigh(double* dev_A, int n, double* dev_w, int* sweeps, void* stream);

/* ---- SCF ---------------------------------------------------------------------- */
#define DFX_GUESS_CORE 0
#define DFX_GUESS_CINIT 1     /* start from C_init */
#define DFX_GUESS_DENSITY 2   /* start from D_init (projected to its top nocc natural orbitals) */
#define DFX_GUESS_LEARNED 3   /* Loewdin-basis density predicted by opts->model (see below) */

typedef struct dfx_guess dfx_guess;  /* trained starting-guess model, see below */

#define DFX_SCHED_FP64 0      /* every iteration in FP64 */
#define DFX_SCHED_MIXED 1     /* FP32/BF16 K until switch_err, then FP64 */

typedef struct {
  double tau;            /* Schwarz threshold (1e-12) */
  double conv_dE;        /* |E_k - E_k-1| threshold (1e-10) */
  double conv_err;       /* max |X^T (FDS - SDF) X| threshold (1e-7) */
  double ortho_thresh;   /* drop eigenvalues of S below this (1e-8) */
  double switch_err;     /* mixed schedule: go to FP64 when the DIIS error is below (1e-5) */
  int32_t max_iter;      /* 100 */
  int32_t diis_size;     /* 8 */
  int32_t schedule;      /* DFX_SCHED_* */
  int32_t mixed_prec;    /* DFX_FP32 or DFX_BF16 for the mixed phase */
  int32_t guess;         /* DFX_GUESS_* */
  int32_t verbose;
  const dfx_guess* model;  /* DFX_GUESS_LEARNED: the model (not owned), else NULL */
  int32_t switch_auto;   /* mixed schedule (1, default): once a reduced-precision stage's
                            error is below 1e-2, estimate its floor: K in that precision
                            and in FP64 on every 16th auxiliary function, the DIIS-error
                            commutator of the difference scaled by sqrt(16); the stage
                            ends once its error is below max(switch_err, estimate).  Into
                            FP64 from a stage with an estimate <= 1e-3 the DIIS history
                            carries over; otherwise DIIS restarts.  A BF16 stage is also
                            estimated on entry and skipped if its floor is above its 1e-2
                            threshold (a nearly linearly dependent basis amplifies BF16's
                            rounding); floor_est[DFX_BF16] then holds that estimate */
  int32_t purify;        /* 1 (default): after the first iteration, the occupied orbitals of
                            X^T F X come from trace-correcting purification (Niklasson,
                            Phys. Rev. B 66, 155115 (2002)) and a Cholesky QR of the
                            projector times the previous ones; the full eigen-decomposition
                            (dfx_eigh's block Jacobi) where it does not settle.  0: the
                            eigen-decomposition every iteration.  C and eps are the
                            eigenvectors and eigenvalues of the last X^T F X either way */
  double level_shift;    /* dfx_uhf / dfx_rohf only (dfx_scf: must be 0): b >= 0 added to the
                            virtual levels before each diagonalisation (Saunders and Hillier,
                            Int. J. Quantum Chem. 7, 699 (1973)).  UHF: F_s + b (S - S D_s S);
                            ROHF, in the orthonormal basis: F_eff + b (I - D/2), i.e. b on the
                            virtual and b/2 on the open levels.  The shift commutes with the
                            density at self-consistency, so it moves the path, not the
                            converged state; the DIIS error is that of the unshifted matrices.
                            0 (default): none */
  void* workspace;       /* device memory owned by the caller (NULL, the default: the call
                            allocates its own): at least dfx_scf_plan's bytes, any alignment.
                            Every device buffer of the call (B, the one-electron matrices,
                            the DIIS history, J/K work) lives in it; the library allocates
                            no device memory then, apart from a rocBLAS handle's scratch
                            that the calling thread keeps for the process.  Read and
                            written only during the call.  Too small: DFX_ENOMEM before
                            any device work */
  size_t ws_bytes;
} dfx_scf_opts;

#define DFX_MAXHIST 256
typedef struct {
  int32_t niter;         /* Fock builds performed */
  int32_t converged;
  int32_t n_mixed;       /* iterations in the reduced-precision phase */
  int32_t ndropped;      /* orthogonaliser eigenvalues dropped */
  int32_t nbf, naux, nocc;
  double E_nuc;
  double err_max;        /* final DIIS error */
  double t_setup;        /* seconds: integrals + fitting + one-electron + guess */
  double t_scf;          /* seconds: the iterations */
  double t_total;
  /* GPU time per phase (HIP events on the SCF stream), seconds */
  double t_eri;          /* three-index ERI kernels */
  double t_metric;       /* metric, Schwarz, Cholesky and L^-1 */
  double t_trsm;         /* B = L^-1 (mu nu|P) with the FP32 split */
  double t_j;            /* all J builds */
  double t_kx;           /* all K half-transforms X_Q = B_Q C_occ */
  double t_ksyrk;        /* all K contractions sum_Q X_Q X_Q^T (incl. reduction) */
  double t_eig;          /* all occupied-space updates (X^T F X, purification or eigen-decomposition,
                            C_occ and D) and the overlap eigensolve */
  int32_t n_jk;          /* J/K builds performed */
  int32_t n_kx_launch;   /* half-transform kernel launches */
  /* the same K figures split by precision, index DFX_FP64 / DFX_FP32 / DFX_BF16 */
  double t_kx_p[3];
  double t_ksyrk_p[3];
  int32_t n_jk_p[3];
  int32_t n_kx_launch_p[3];
  int64_t nintegrals;    /* unique evaluated three-index integrals */
  int64_t ncols;         /* packed pair columns of B */
  double E_hist[DFX_MAXHIST];
  double err_hist[DFX_MAXHIST];
  int8_t prec_hist[DFX_MAXHIST];  /* DFX_FP64 / DFX_FP32 / DFX_BF16 of each Fock build */
  double t_guess;        /* seconds of wall time for the starting guess (inside t_setup) */
  double floor_est[3];   /* switch_auto: estimated DIIS-error floor per precision (0 if none) */
  int32_t guess_fallback; /* DFX_GUESS_LEARNED: 0 used; 1 non-finite prediction, core guess
                             used instead; 2 no convergence from it in max_iter, restarted
                             from the core guess (niter and the histories count both passes) */
  int32_t n_purified;    /* occupied-space updates by purification */
  int32_t n_eigh;        /* occupied-space updates by eigen-decomposition (the final C/eps solve excluded) */
  int32_t purify_steps;  /* purification steps (matrix squarings) over all updates */
  double t_trsm_update;  /* the B transform's block update products alone (inside t_trsm) */
  double trsm_update_flops;
  int32_t n_trsm_update; /* their launches */
  double t_purify;       /* the purifications of the occupied-space updates alone (inside t_eig;
                            failed attempts included), seconds */
} dfx_scf_info;

void dfx_scf_default_opts(dfx_scf_opts* o);

/*
 * dfx_scf_plan -- bytes of dfx_scf_opts.workspace for dfx_scf, dfx_uhf or
 * dfx_rohf on these shells (an upper bound; host only).  natom: atoms of the
 * geometry (the learned guess's inputs scale with the atom pairs); opts may be
 * NULL (defaults; only diis_size matters).
 */
int dfx_scf_plan(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, int natom,
                 const dfx_scf_opts* opts, int64_t* bytes);

/*
 * dfx_scf -- DF-RHF: D = C_occ C_occ^T, F = h + 2J - K, E = tr D (h + F) + E_nn,
 * Pulay DIIS on e = X^T (F D S - S D F) X, aufbau on the lowest nocc levels.
 *   init    host [nbf][nbf] C (guess = CINIT) or D (guess = DENSITY), else NULL
 *   E       host scalar out; C host [nbf][nbf] out (may be NULL); eps [nbf] (may be NULL)
 * Synchronous.  DFX_ENOCONV: not converged within max_iter (E, C written).
 */
int dfx_scf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
            const dfx_scf_opts* opts, const double* init, double* E, double* C, double* eps,
            dfx_scf_info* info);

/*
 * dfx_rhf_grad -- analytic nuclear gradient of the DF-RHF energy (section
 * "Standard algorithms" lists analytic gradients of the SCF methods; section
 * "Molecular integrals" the integral derivatives) at converged orbitals:
 *   dE/dR = 2 tr(D h^x) - 2 tr(W S^x) + dE_nn/dx
 *         + sum Gam_P,mu nu (mu nu|P)^x + sum Gam2_PQ (P|Q)^x,
 *   D = C_occ C_occ^T, W = C_occ diag(eps_occ) C_occ^T,
 *   Gam = L^-T (4 gamma_Q D - 2 C_occ b_Q C_occ^T), b_Q = C_occ^T B_Q C_occ, gamma = B d,
 *   Gam2 = L^-T (-2 gamma gamma^T + sum_ij b_ij b_ij^T) L^-1,
 * for the fitted tensor of dfx_eri3 with opts->tau (the integrals of screened
 * triplets are dropped from the derivative as from the energy).  Every shell
 * moves with the atom of geom whose coordinates equal its centre exactly.
 *   opts        tau and workspace as for dfx_scf (workspace sized by dfx_grad_plan)
 *   C_occ       host [nbf][nocc]: the occupied orbitals of a converged dfx_scf
 *               (its C's first nocc columns), eps_occ host [nocc] their levels
 *   grad        host [natom][3] out, Eh/bohr
 *   info        may be NULL: GPU times of the weights, the three-index and metric
 *               derivatives and the one-electron terms, and the wall time
 * FP64 throughout.  Synchronous.  Errors: DFX_EINVAL (NULL, bad nocc, a shell
 * off every atom), DFX_EUNSUPPORTED (nocc > 512, l beyond the compiled
 * classes), DFX_ENOMEM, DFX_EHIP, DFX_ENOTPOSDEF.
 */
typedef struct {
  int32_t natom;
  double t_setup;        /* B (integrals, metric, fit) */
  double t_weights;      /* D, W, gamma, Gam and Gam2 */
  double t_deriv3;       /* three-index derivative integrals with their contraction */
  double t_deriv2;       /* metric derivative integrals */
  double t_onee;         /* one-electron derivative terms */
  double t_total;        /* wall time of the call */
} dfx_grad_info;
int dfx_rhf_grad(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
                 const dfx_scf_opts* opts, const double* C_occ, const double* eps_occ, int nocc, double* grad,
                 dfx_grad_info* info);
/* bytes of dfx_scf_opts.workspace for dfx_rhf_grad (an upper bound; host only) */
int dfx_grad_plan(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, int natom, int nocc,
                  int64_t* bytes);

/*
 * dfx_uhf -- DF-UHF (section "Standard algorithms" lists unrestricted Hartree-Fock
 * among the SCF methods): the Pople-Nesbet equations on the same fitted tensor as
 * dfx_scf.  With n_alpha = (nelec + multiplicity - 1) / 2 and n_beta = nelec - n_alpha,
 *   D_s = C_s,occ C_s,occ^T,  F_s = h + J[D_alpha + D_beta] - K[D_s]  (s = alpha, beta),
 *   E = 1/2 sum_s tr D_s (h + F_s) + E_nn,
 * one Pulay DIIS over both spins (error overlaps summed, both Fock matrices
 * extrapolated with the same coefficients), aufbau per spin (from the second iteration
 * on by purification, as for dfx_scf; the first update, a purification that does not
 * settle and the returned orbitals by the block Jacobi eigen-decomposition), start
 * from the core Hamiltonian for both spins.  FP64 J and K throughout.
 *   opts          as for dfx_scf; guess must be DFX_GUESS_CORE and schedule
 *                 DFX_SCHED_FP64 (DFX_EINVAL otherwise); the learned guess and
 *                 precision switches do not apply; purify and level_shift apply
 *   multiplicity  2S + 1 >= 1; DFX_EINVAL if its parity does not match the electron
 *                 count, or if it exceeds nelec + 1
 *   E             host scalar out
 *   C             host [2][nbf][nbf] out (may be NULL): alpha then beta orbitals whose
 *                 densities gave E, columns in ascending level order; the last
 *                 ndropped columns are zero (canonical orthogonalisation)
 *   eps           host [2][nbf] out (may be NULL): the levels of those orbitals, the
 *                 eigenvalues of the (DIIS-extrapolated, level-shifted) X^T F_s X
 *                 last diagonalised; zero beyond nbf - ndropped
 *   info          may be NULL: niter, converged, nbf, naux, nocc (= n_alpha), E_nuc,
 *                 err_max (larger of the two spins), E_hist / err_hist, timings
 * Synchronous.  DFX_ENOCONV: not converged within max_iter (E, C and eps written).
 * A closed shell (multiplicity 1) gives the dfx_scf energy for the same options.
 */
int dfx_uhf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
            const dfx_scf_opts* opts, int multiplicity, double* E, double* C, double* eps, dfx_scf_info* info);

/*
 * dfx_rohf -- DF-ROHF (section "Standard algorithms" lists restricted open-shell
 * Hartree-Fock among the SCF methods): one orbital set C, the n_beta lowest doubly
 * occupied (core), the next n_alpha - n_beta singly (open), n_alpha and n_beta as
 * for dfx_uhf.  D_alpha = C_(core+open) C_(core+open)^T, D_beta = C_core C_core^T;
 * F_s and E as for dfx_uhf.  The orbitals are the eigenvectors of Roothaan's
 * effective Fock matrix: in the basis of the current orbitals its core-open block
 * is that of F_beta, its open-virtual block that of F_alpha, every other block that
 * of (F_alpha + F_beta) / 2.  It is formed in the orthonormal basis of X from the
 * projectors onto the core, open and virtual spaces of the last update, and Pulay
 * DIIS extrapolates it with the error F_eff D - D F_eff of D = D_alpha + D_beta in
 * that basis (zero exactly when the core-open, core-virtual and open-virtual blocks
 * are).  From the second iteration on the core and core + open spaces of the
 * extrapolated matrix come by purification at n_beta and n_alpha (opts.purify);
 * otherwise, and for the returned orbitals, by its eigen-decomposition.  Arguments, options, errors and info as for
 * dfx_uhf (err_max: the one error matrix), except that C is one set, host
 * [nbf][nbf] (core, open, virtual columns in that order), and eps host [nbf], the
 * eigenvalues of the effective Fock matrix last diagonalised (Roothaan's
 * canonicalisation: unlike E and D they depend on the diagonal-block choice).  A closed shell gives the dfx_scf
 * energy; with n_beta = 0 it is the dfx_uhf determinant.
 */
int dfx_rohf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
             const dfx_scf_opts* opts, int multiplicity, double* E, double* C, double* eps, dfx_scf_info* info);

/* ---- learned starting guess ---------------------------------------------------
 * Replaces the core-Hamiltonian start of the SCF ("Standard algorithms") with a
 * density predicted block by block: for every atom pair (a, b) closer than the
 * pair cutoff rc, and for every atom (a, a), an FP32 multilayer perceptron of
 * that pair's element types maps invariant descriptors of the local geometry
 * to the block P_ab written in a local frame; the block is rotated to the
 * laboratory frame with real-solid-harmonic rotation matrices.
 *
 * P is the density in the symmetrically orthogonalised (Loewdin) basis,
 * P = S^1/2 D S^1/2 with D = C_occ C_occ^T (dfx_lowdin): its entries are
 * bounded by one, and an error in P reaches the orthonormal-basis density of
 * the SCF unamplified, whereas AO blocks of a nearly linearly dependent basis
 * are large and cancel each other.  The SCF takes the top nocc eigenvectors of
 * U^T P U, U the kept eigenvectors of S.
 *
 * Local frame of pair (a, b): z along a -> b; x from the nearest further
 * neighbour of a at least 0.1 rad off the z axis, projected off z (else the
 * laboratory axis least aligned with z); y = z x x.  Atom frame: z toward the
 * nearest neighbour, x from the next as above.  Neighbours ranked by distance
 * rounded to 1e-8 bohr, ties by index.
 * Descriptors of a pair (a, b), Z_a >= Z_b:  one-hot(Z_a) [3], one-hot(Z_b) [3],
 *   16 Gaussians of |r_ab| with centres evenly spaced on [0.5, rc] (width =
 *   spacing), then for a and for b the environment
 *   sum_k g_n(r) f_c(r) Y_lm(F r_ak / r)  over neighbours k within rc_env other
 *   than the pair partner, per element channel H, C, O [3 x 8 x 9]: 8 Gaussians
 *   on [0.5, rc_env], real spherical harmonics l <= 2, f_c(r) = (cos(pi r /
 *   rc_env) + 1) / 2.  Pairs of equal elements are evaluated in both
 *   orientations and averaged.
 * Descriptors of an atom: one-hot(Z_a) [3], its environment [3 x 8 x 9].
 * Network: widths (d_in, hidden x depth, block size), SiLU between layers,
 *   inputs and targets standardised per component on the training set (input
 *   scales floored at 0.1, target scales at 1e-6),
 *   mean-squared-error loss, Adam (beta 0.9 / 0.999, eps 1e-8).
 * All arrays host-side and row-major unless stated.  Not thread-safe per model.
 */
typedef struct {
  int32_t nelem;          /* elements the model covers (H, C, O only) */
  const int32_t* Z;       /* [nelem] */
  const int32_t* nshell;  /* [nelem] shells per atom of that element */
  const int32_t* shell_l; /* concatenated l of those shells, in basis order (l <= 3) */
  double rc;              /* pair cutoff, bohr (<= 0: 8) */
  double rc_env;          /* environment cutoff, bohr (<= 0: 6) */
  int32_t hidden;         /* hidden width (<= 0: 256) */
  int32_t depth;          /* hidden layers (<= 0: 3) */
  uint64_t seed;          /* weight initialisation and minibatch order */
} dfx_guess_spec;

/*
 * dfx_lowdin -- P = S^1/2 D S^1/2 for the orbital basis `shells` (S from the
 * same kernels as dfx_int1e, S^1/2 from its eigendecomposition, negative
 * eigenvalues clamped to zero).  D, P host [nbf][nbf].  Synchronous.
 */
int dfx_lowdin(const dfx_geom* geom, const dfx_shell* shells, int nsh, const double* D, double* P, void* stream);

int dfx_guess_create(const dfx_guess_spec* spec, dfx_guess** out);
int dfx_guess_free(dfx_guess* g);
/* add the samples of one converged geometry: P host [nbf][nbf], its Loewdin-basis
 * density (dfx_lowdin), basis ordered atom by atom with the shells of the spec;
 * adding to a trained type: DFX_EINVAL */
int dfx_guess_add(dfx_guess* g, const dfx_geom* geom, const double* P);
/* train every pair type for `epochs` passes of minibatches of `batch` samples
 * (a ragged last minibatch is skipped); loss_out [epochs] (may be NULL): mean
 * standardised MSE per epoch over all types.  Synchronous, on the GPU. */
int dfx_guess_train(dfx_guess* g, int epochs, int batch, double lr, double* loss_out);
/* predicted Loewdin-basis density P host [nbf][nbf] (symmetric; zero beyond rc);
 * DFX_EINVAL if a pair type is unknown or untrained */
int dfx_guess_predict(const dfx_guess* g, const dfx_geom* geom, double* P);
/* the stored training samples of one type: X [samples][d_in] descriptors,
 * T [samples][d_out] local-frame blocks (either may be NULL) */
int dfx_guess_samples(const dfx_guess* g, int type, double* X, double* T);
/* number of pair types; desc (may be NULL) [ntypes][6] = is_atom, Z_a, Z_b,
 * d_in, d_out, samples */
int dfx_guess_info(const dfx_guess* g, int* ntypes, int32_t* desc);
/* trained parameters of one type: theta (FP32, per layer W[out][in] then b),
 * input mean/std [d_in], target mean/std [d_out]; any pointer may be NULL */
int dfx_guess_export(const dfx_guess* g, int type, float* theta, double* fmean, double* fstd, double* tmean,
                     double* tstd);
/* set the parameters of one type (created if absent; is_atom: Z_a == Z_b, else
 * Z_a >= Z_b), with the layout of dfx_guess_export; the type counts as trained */
int dfx_guess_import(dfx_guess* g, int is_atom, int za, int zb, const float* theta, const double* fmean,
                     const double* fstd, const double* tmean, const double* tstd);
/* descriptors [d_in] and frame rows [3][3] of pair (a, b) (a == b: atom a), as used
 * for training and prediction; nfeat receives d_in.  Any output may be NULL. */
int dfx_guess_features(const dfx_guess* g, const dfx_geom* geom, int a, int b, double* feat, double* frame,
                       int* nfeat);
/* U [(2l+1)][(2l+1)] with Y_m(F^T u) = sum_m' U[m][m'] Y_m'(u), F [3][3] orthogonal */
int dfx_sh_rotation(int l, const double* F, double* U);
int dfx_guess_save(const dfx_guess* g, const char* path);
int dfx_guess_load(const char* path, dfx_guess** out);

/* ---- the network kernels (FP32, device arrays, on `stream`) ------------------
 * widths [nlayers + 1]; theta as in dfx_guess_export; X [batch][widths[0]];
 * Y, T [batch][widths[nlayers]].
 * dfx_mlp_forward: Y = network(X); synchronises the stream.
 * dfx_mlp_loss_grad: grad [nparams] = d/dtheta of mean((Y - T)^2); *loss the
 *   mean (accumulated in FP64); synchronises the stream.
 * dfx_mlp_adam: one Adam step (beta 0.9 / 0.999, eps 1e-8) of theta, with
 *   moment buffers m, v [n] (zero before step 1). */
int dfx_mlp_forward(const int32_t* widths, int nlayers, const float* theta, const float* X, int batch, float* Y,
                    void* stream);
int dfx_mlp_loss_grad(const int32_t* widths, int nlayers, const float* theta, const float* X, const float* T,
                      int batch, float* grad, double* loss, void* stream);
int dfx_mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t n, int step, float lr, void* stream);

const char* dfx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFX_H */
