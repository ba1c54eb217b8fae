"""ORACLE -- test infrastructure only.

Plain, slow, FP64 CPU reference for the density-fitted restricted Hartree-Fock
hot path.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
GPU library: integrals are McMurchie-Davidson (``md_ints.c``) rather than Rys
quadrature, solid harmonics come from a closed formula rather than a
recursion, and the linear algebra is NumPy/SciPy.

What it computes, and where the paper states it (section "Density fitting
utilities", Eqs. (1)-(3); section "Molecular integrals"; section "Standard
algorithms" for DF-based RHF):

* three-index integrals (mu nu|P) and the two-centre metric J_PQ = (P|Q);
* the fitted tensor B with B_Q = sum_P (L^-1)_QP (mu nu|P), J_PQ = L L^T --
  Eq. (1c) with M' = L^-1;
* J = sum_Q B_Q gamma_Q with gamma_Q = sum_{mu nu} B_Q,mu nu D_mu nu -- Eq. (3a)
  then (3b);
* K = sum_Q (B_Q C)(B_Q C)^T -- Eq. (1a) then (2a);
* a DIIS-accelerated restricted SCF built on these;
* the analytic nuclear gradient of that SCF energy (``grad.py``, with the
  McMurchie-Davidson derivative integrals of ``md_ints.c``).

Textbook parts the paper does not spell out (Boys function, Hermite
recursions, Pulay DIIS, canonical orthogonalisation) follow Helgaker,
Jorgensen & Olsen, "Molecular Electronic-Structure Theory", ch. 6 and 9, and
Pulay (1980).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        # DFX_ORACLE_LIB: another build of md_ints.c (the sanitizer test's)
        path = os.environ.get("DFX_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: WPS433 (oracle-local build step)
            _b.build()
        _LIB = ctypes.CDLL(path)
        for l in range(7):
            t = solid_harmonics(l)
            _keep.append(t)
            _LIB.oracle_set_sph(ctypes.c_int(l), t.ctypes.data_as(ctypes.c_void_p))
    return _LIB


_keep: list = []


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Boys function
# --------------------------------------------------------------------------

def boys(mmax, T):
    """F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt for m = 0..mmax (C series / recursion)."""
    F = np.zeros(mmax + 1)
    lib().oracle_boys(ctypes.c_int(mmax), ctypes.c_double(T), _p(F))
    return F


# --------------------------------------------------------------------------
# Real solid harmonics, closed formula (Helgaker et al. eqs. 6.4.47-6.4.50)
# --------------------------------------------------------------------------

def cart_powers(l):
    """Cartesian monomials of degree l, x-power descending, then y descending."""
    return [(i, j, l - i - j) for i in range(l, -1, -1) for j in range(l - i, -1, -1)]


def solid_harmonics(l):
    """Matrix T[m + l, c] with r^l Y_lm = sum_c T x^i y^j z^k, Y_lm orthonormal on
    the unit sphere, m = -l..l; m > 0 ~ cos(m phi), m < 0 ~ sin(|m| phi), no
    Condon-Shortley phase."""
    pw = cart_powers(l)
    idx = {p: n for n, p in enumerate(pw)}
    T = np.zeros((2 * l + 1, len(pw)))
    for m in range(-l, l + 1):
        am = abs(m)
        vm = 0.0 if m >= 0 else 0.5
        N = (1.0 / (2 ** am * math.factorial(l))) * math.sqrt(
            2.0 * math.factorial(l + am) * math.factorial(l - am) / (2.0 if m == 0 else 1.0))
        for t in range((l - am) // 2 + 1):
            for u in range(t + 1):
                v = vm
                vmax = math.floor(am / 2.0 - vm) + vm
                while v <= vmax + 1e-9:
                    c = ((-1.0) ** (t + v - vm) * 0.25 ** t * math.comb(l, t)
                         * math.comb(l - t, am + t) * math.comb(t, u) * math.comb(am, int(round(2 * v))))
                    px = int(round(2 * t + am - 2 * (u + v)))
                    py = int(round(2 * (u + v)))
                    pz = l - 2 * t - am
                    T[m + l, idx[(px, py, pz)]] += N * c
                    v += 1.0
    # S_lm above is Racah-normalised: r^l Y_lm = sqrt((2l+1)/(4 pi)) S_lm
    return np.ascontiguousarray(T * math.sqrt((2 * l + 1) / (4.0 * math.pi)))


def prim_norm(l, a):
    """N with int |N r^l Y_lm exp(-a r^2)|^2 = 1 for orthonormal Y_lm."""
    return math.sqrt(2.0 * (2.0 * a) ** (l + 1.5) / math.gamma(l + 1.5))


def normalized_coefs(l, exps, coefs):
    """Coefficients of unnormalised Cartesian primitives such that the contracted
    spherical function has unit norm; input coefs multiply normalised primitives."""
    exps = np.asarray(exps, float)
    c = np.asarray(coefs, float)
    s = (2.0 * np.sqrt(np.outer(exps, exps)) / np.add.outer(exps, exps)) ** (l + 1.5)
    nrm = math.sqrt(float(c @ s @ c))
    return np.array([ci * prim_norm(l, a) for ci, a in zip(c, exps)]) / nrm


# --------------------------------------------------------------------------
# Basis packing for the C engine
# --------------------------------------------------------------------------

class _OBasis(ctypes.Structure):
    _fields_ = [("nsh", ctypes.c_int), ("ctr", ctypes.c_void_p), ("l", ctypes.c_void_p),
                ("nprim", ctypes.c_void_p), ("poff", ctypes.c_void_p),
                ("exps", ctypes.c_void_p), ("coef", ctypes.c_void_p),
                ("foff", ctypes.c_void_p)]


class Basis:
    """A list of shells (dicts from ``workloads``) packed for the C engine."""

    def __init__(self, shells):
        self.shells = shells
        self.nsh = len(shells)
        self.ctr = np.ascontiguousarray(np.array([s["center"] for s in shells], float).reshape(-1, 3))
        self.l = np.array([s["l"] for s in shells], np.int32)
        self.nprim = np.array([len(s["exps"]) for s in shells], np.int32)
        self.poff = np.zeros(self.nsh, np.int32)
        self.poff[1:] = np.cumsum(self.nprim)[:-1]
        self.exps = np.concatenate([np.asarray(s["exps"], float) for s in shells]) if shells else np.zeros(0)
        self.coef = (np.concatenate([normalized_coefs(s["l"], s["exps"], s["coefs"]) for s in shells])
                     if shells else np.zeros(0))
        self.size = 2 * self.l + 1
        self.foff = np.zeros(self.nsh, np.int32)
        self.foff[1:] = np.cumsum(self.size)[:-1]
        self.nbf = int(self.size.sum())
        self.c = _OBasis(self.nsh, _p(self.ctr), _p(self.l), _p(self.nprim), _p(self.poff),
                         _p(self.exps), _p(self.coef), _p(self.foff))

    @property
    def ref(self):
        return ctypes.byref(self.c)


# --------------------------------------------------------------------------
# Integrals
# --------------------------------------------------------------------------

def eri3_block(bas, a, b, aux, c):
    """(ab|C) spherical block [n_a][n_b][n_C]."""
    out = np.zeros((bas.size[a], bas.size[b], aux.size[c]))
    lib().oracle_eri3_block(bas.ref, a, b, aux.ref, c, _p(out))
    return out


def eri2_block(aux, p, q):
    out = np.zeros((aux.size[p], aux.size[q]))
    lib().oracle_eri2_block(aux.ref, p, q, _p(out))
    return out


def eri4_block(bas, a, b, c, d):
    out = np.zeros((bas.size[a], bas.size[b], bas.size[c], bas.size[d]))
    lib().oracle_eri4_block(bas.ref, a, b, c, d, _p(out))
    return out


def eri2(aux):
    """Coulomb metric J_PQ = (P|Q)."""
    J = np.zeros((aux.nbf, aux.nbf))
    lib().oracle_eri2(aux.ref, aux.nbf, _p(J))
    return J


def eri4(bas):
    """Full (mu nu|la si) -- tiny systems only."""
    G = np.zeros((bas.nbf,) * 4)
    lib().oracle_eri4(bas.ref, bas.nbf, _p(G))
    return G


def int1e(bas, xyz, Z):
    """Overlap S, kinetic T and nuclear attraction V = -sum_A Z_A (mu|1/r_A|nu)."""
    n = bas.nbf
    S, T, V = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    xyz = np.ascontiguousarray(np.asarray(xyz, float))
    Zd = np.ascontiguousarray(np.asarray(Z, float))
    lib().oracle_int1e(bas.ref, n, len(Zd), _p(xyz), _p(Zd), _p(S), _p(T), _p(V))
    return S, T, V


def nuclear_repulsion(xyz, Z):
    xyz = np.asarray(xyz, float)
    e = 0.0
    for i in range(len(Z)):
        for j in range(i):
            e += Z[i] * Z[j] / np.linalg.norm(xyz[i] - xyz[j])
    return float(e)


def schwarz(bas, aux):
    """Q_ab = sqrt(max (mu nu|mu nu)) per shell pair, Q_C = sqrt(max (P|P)) per aux shell."""
    Qab = np.zeros((bas.nsh, bas.nsh))
    QC = np.zeros(aux.nsh)
    lib().oracle_schwarz(bas.ref, aux.ref, _p(Qab), _p(QC))
    return Qab, QC


# --------------------------------------------------------------------------
# Screening and indexing (integer lists are part of the parity contract)
# --------------------------------------------------------------------------

@dataclass
class Screen:
    pairs: np.ndarray          # int32 [npairs, 2], canonical a >= b, a-major
    col_off: np.ndarray        # int64 [npairs + 1], prefix sum of n_a * n_b
    keep: np.ndarray           # bool  [npairs, nauxsh]: triplet (a,b,C) evaluated
    tau: float
    margin: float = field(default=np.inf)  # smallest |Q_ab Q_C / tau - 1|


def screen(bas, aux, Qab, QC, tau=1e-12):
    """Keep pair (a>=b) iff Q_ab * max_C Q_C >= tau; evaluate (a,b,C) iff Q_ab*Q_C >= tau."""
    qmax = QC.max() if len(QC) else 0.0
    pairs = [(a, b) for a in range(bas.nsh) for b in range(a + 1) if Qab[a, b] * qmax >= tau]
    pairs = np.array(pairs, np.int32).reshape(-1, 2)
    sizes = bas.size[pairs[:, 0]].astype(np.int64) * bas.size[pairs[:, 1]]
    col_off = np.zeros(len(pairs) + 1, np.int64)
    col_off[1:] = np.cumsum(sizes)
    prod = Qab[pairs[:, 0], pairs[:, 1]][:, None] * QC[None, :]
    keep = prod >= tau
    with np.errstate(divide="ignore", invalid="ignore"):
        margin = float(np.min(np.abs(prod / tau - 1.0))) if prod.size else np.inf
    return Screen(pairs, col_off, keep, tau, margin)


def eri3_packed(bas, aux, scr):
    """Raw (mu nu|P), aux-major packed: [naux][ncols], column blocks n_a x n_b
    (row-major, mu in shell a) for each kept pair in canonical order."""
    ncols = int(scr.col_off[-1])
    out = np.zeros((aux.nbf, ncols))
    pa = np.ascontiguousarray(scr.pairs[:, 0])
    pb = np.ascontiguousarray(scr.pairs[:, 1])
    skip = np.ascontiguousarray((~scr.keep).astype(np.uint8))
    co = np.ascontiguousarray(scr.col_off)
    lib().oracle_eri3_packed(bas.ref, aux.ref, ctypes.c_int(len(pa)), _p(pa), _p(pb), _p(co),
                             ctypes.c_longlong(ncols), _p(skip), _p(out))
    return out


def pair_index(bas, scr):
    """(mu, nu) of every packed column."""
    mus, nus = [], []
    for (a, b), off in zip(scr.pairs, scr.col_off[:-1]):
        na, nb = bas.size[a], bas.size[b]
        i, j = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
        mus.append(bas.foff[a] + i.ravel())
        nus.append(bas.foff[b] + j.ravel())
    if not mus:
        return np.zeros(0, int), np.zeros(0, int)
    return np.concatenate(mus), np.concatenate(nus)


def unpack(Bp, bas, scr, rows=None):
    """Packed [nq][ncols] -> dense symmetric [nq][nbf][nbf]."""
    mu, nu = pair_index(bas, scr)
    if rows is not None:
        Bp = Bp[rows]
    out = np.zeros((Bp.shape[0], bas.nbf, bas.nbf))
    out[:, mu, nu] = Bp
    out[:, nu, mu] = Bp
    return out


# --------------------------------------------------------------------------
# Density fitting: Eq. (1c) with M' = L^-1, and Eqs. (1a), (2a), (3a), (3b)
# --------------------------------------------------------------------------

def fit(raw, J2):
    """B = L^-1 raw with J_PQ = L L^T (plain Cholesky, no pivoting)."""
    L = sla.cholesky(J2, lower=True)
    B = sla.solve_triangular(L, raw, lower=True)
    return L, B


@dataclass
class DF:
    bas: Basis
    aux: Basis
    scr: Screen
    B: np.ndarray              # packed [naux][ncols]
    L: np.ndarray
    mu: np.ndarray = None
    nu: np.ndarray = None

    def __post_init__(self):
        self.mu, self.nu = pair_index(self.bas, self.scr)

    def dense_rows(self, q0, q1):
        n = self.bas.nbf
        out = np.zeros((q1 - q0, n, n))
        out[:, self.mu, self.nu] = self.B[q0:q1]
        out[:, self.nu, self.mu] = self.B[q0:q1]
        return out


def build_df(bas, aux, tau=1e-12):
    Qab, QC = schwarz(bas, aux)
    scr = screen(bas, aux, Qab, QC, tau)
    raw = eri3_packed(bas, aux, scr)
    J2 = eri2(aux)
    L, B = fit(raw, J2)
    return DF(bas, aux, scr, B, L)


def jk(df, D=None, C=None, chunk=128, want_j=True, want_k=True):
    """J = sum_Q B_Q tr(B_Q D) (Eqs. 3a, 3b).  K = sum_Q (B_Q C)(B_Q C)^T when the
    occupied block C is given (Eqs. 1a, 2a), else K = sum_Q B_Q D B_Q."""
    n = df.bas.nbf
    if D is None:
        D = C @ C.T
    J = np.zeros((n, n))
    K = np.zeros((n, n))
    naux = df.B.shape[0]
    for q0 in range(0, naux, chunk):
        q1 = min(naux, q0 + chunk)
        Bq = df.dense_rows(q0, q1)
        if want_j:
            gam = np.einsum("qmn,mn->q", Bq, D)
            J += np.einsum("q,qmn->mn", gam, Bq)
        if want_k:
            if C is not None:
                X = Bq @ C                      # [q][mu][i]
                K += np.einsum("qmi,qni->mn", X, X)
            else:
                K += np.einsum("qml,ls,qsn->mn", Bq, D, Bq)
    return J, K


# --------------------------------------------------------------------------
# Restricted Hartree-Fock with Pulay DIIS
# --------------------------------------------------------------------------

def orthogonalizer(S, thresh=1e-8):
    """Canonical orthogonalisation X = U s^-1/2, dropping eigenvalues of S below thresh."""
    s, U = np.linalg.eigh(S)
    keep = s >= thresh
    return U[:, keep] / np.sqrt(s[keep]), int((~keep).sum())


@dataclass
class SCFResult:
    E: float
    C: np.ndarray
    eps: np.ndarray
    D: np.ndarray
    F: np.ndarray
    niter: int
    converged: bool
    history: list
    ndropped: int


def rhf(S, h, Enuc, nocc, jk_fn, C_init=None, diis_size=8, conv_dE=1e-10, conv_err=1e-8,
        max_iter=100, ortho_thresh=1e-8):
    """DF-RHF: D = C_occ C_occ^T, F = h + 2J - K, E = tr D(h + F) + E_nn,
    DIIS on e = X^T (F D S - S D F) X, aufbau on the lowest nocc orbitals."""
    X, ndrop = orthogonalizer(S, ortho_thresh)

    def diag(F):
        eps, Cp = np.linalg.eigh(X.T @ F @ X)
        return eps, X @ Cp

    if C_init is None:
        eps, C = diag(h)
    else:
        C, eps = np.array(C_init, float), None
    D = C[:, :nocc] @ C[:, :nocc].T
    Fs, es, hist = [], [], []
    E_old, converged, it = None, False, 0
    F = h
    for it in range(1, max_iter + 1):
        J, K = jk_fn(D, C[:, :nocc])
        F = h + 2.0 * J - K
        E = float(np.sum(D * (h + F))) + Enuc
        err = X.T @ (F @ D @ S - S @ D @ F) @ X
        emax = float(np.max(np.abs(err)))
        hist.append((E, emax))
        if E_old is not None and abs(E - E_old) < conv_dE and emax < conv_err:
            converged = True
            break
        E_old = E
        Fs.append(F)
        es.append(err)
        if len(Fs) > diis_size:
            Fs.pop(0)
            es.pop(0)
        Fbar = F
        while len(Fs) > 1:
            m = len(Fs)
            Bm = -np.ones((m + 1, m + 1))
            Bm[m, m] = 0.0
            for i in range(m):
                for j in range(m):
                    Bm[i, j] = float(np.sum(es[i] * es[j]))
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            if 1.0 / np.linalg.cond(Bm[:m, :m]) < 1e-14:
                Fs.pop(0)
                es.pop(0)
                continue
            c = np.linalg.solve(Bm, rhs)[:m]
            Fbar = sum(ci * Fi for ci, Fi in zip(c, Fs))
            break
        eps, C = diag(Fbar)
        D = C[:, :nocc] @ C[:, :nocc].T
    return SCFResult(E, C, eps, D, F, it, converged, hist, ndrop)


def df_rhf(elems_Z, xyz, shells, aux_shells, nocc, tau=1e-12, **kw):
    """End-to-end oracle DF-RHF: integrals, fitting and SCF."""
    bas, aux = Basis(shells), Basis(aux_shells)
    S, T, V = int1e(bas, xyz, elems_Z)
    df = build_df(bas, aux, tau)
    Enuc = nuclear_repulsion(xyz, elems_Z)
    res = rhf(S, T + V, Enuc, nocc, lambda D, C: jk(df, D=D, C=C), **kw)
    return res, df
