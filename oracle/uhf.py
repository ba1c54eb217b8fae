"""ORACLE -- test infrastructure only (see oracle/__init__.py for who may use it).

Unrestricted Hartree-Fock on the density-fitted J and K of the oracle (the
paper lists UHF among its standard SCF algorithms, section "Standard
algorithms").  Textbook equations (Szabo & Ostlund, "Modern Quantum Chemistry",
sec. 3.8, Pople-Nesbet):

    D_s  = C_s,occ C_s,occ^T,  s = alpha, beta (n_alpha >= n_beta occupied)
    F_s  = h + J[D_alpha + D_beta] - K[D_s]
    E    = 1/2 sum_s tr D_s (h + F_s) + E_nn

with Pulay DIIS on the two spin blocks together: the error vector is the pair
(e_alpha, e_beta), e_s = X^T (F_s D_s S - S D_s F_s) X, and one set of
coefficients extrapolates both Fock matrices.  Aufbau per spin from the core
guess.
"""
from dataclasses import dataclass

import numpy as np

from . import (Basis, build_df, int1e, jk, nuclear_repulsion, orthogonalizer)


@dataclass
class UHFResult:
    E: float
    C: tuple           # (C_alpha, C_beta)
    eps: tuple
    D: tuple
    niter: int
    converged: bool
    history: list


def uhf(S, h, Enuc, nalpha, nbeta, jk_fn, diis_size=8, conv_dE=1e-10, conv_err=1e-8, max_iter=200,
        ortho_thresh=1e-8):
    """jk_fn(D, C_occ) -> (J[D], K[C_occ C_occ^T]); J and K of each spin are built
    from that spin's occupied orbitals, J from the total density."""
    X, _ = orthogonalizer(S, ortho_thresh)

    def diag(F):
        eps, Cp = np.linalg.eigh(X.T @ F @ X)
        return eps, X @ Cp

    nocc = (nalpha, nbeta)
    eps0, C0 = diag(h)
    C, eps = [C0, C0.copy()], [eps0, eps0.copy()]
    Fs, es, hist = [], [], []
    E_old, converged, it, E = None, False, 0, 0.0
    for it in range(1, max_iter + 1):
        D = [C[s][:, :nocc[s]] @ C[s][:, :nocc[s]].T for s in range(2)]
        J, _ = jk_fn(D[0] + D[1], None)
        K = [jk_fn(None, C[s][:, :nocc[s]])[1] if nocc[s] > 0 else np.zeros_like(h) for s in range(2)]
        F = [h + J - K[s] for s in range(2)]
        E = 0.5 * sum(float(np.sum(D[s] * (h + F[s]))) for s in range(2)) + Enuc
        err = [X.T @ (F[s] @ D[s] @ S - S @ D[s] @ F[s]) @ X for s in range(2)]
        emax = max(float(np.max(np.abs(e))) for e in err)
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
                    Bm[i, j] = sum(float(np.sum(es[i][s] * es[j][s])) for s in range(2))
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            if 1.0 / np.linalg.cond(Bm[:m, :m]) < 1e-14:
                Fs.pop(0)
                es.pop(0)
                continue
            c = np.linalg.solve(Bm, rhs)[:m]
            Fbar = [sum(ci * Fi[s] for ci, Fi in zip(c, Fs)) for s in range(2)]
            break
        for s in range(2):
            eps[s], C[s] = diag(Fbar[s])
    D = [C[s][:, :nocc[s]] @ C[s][:, :nocc[s]].T for s in range(2)]
    return UHFResult(E, tuple(C), tuple(eps), tuple(D), it, converged, hist)


def df_uhf(elems_Z, xyz, shells, aux_shells, nalpha, nbeta, tau=1e-12, **kw):
    """End-to-end oracle DF-UHF: integrals, fitting and SCF."""
    bas, aux = Basis(shells), Basis(aux_shells)
    S, T, V = int1e(bas, xyz, elems_Z)
    df = build_df(bas, aux, tau)
    Enuc = nuclear_repulsion(xyz, elems_Z)

    def jk_fn(D, C):
        if D is not None:
            return jk(df, D=D, want_k=False)
        return jk(df, C=C, want_j=False)

    return uhf(S, T + V, Enuc, nalpha, nbeta, jk_fn, **kw), df
