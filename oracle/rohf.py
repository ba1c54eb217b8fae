"""ORACLE -- test infrastructure only (see oracle/__init__.py for who may use it).

Restricted open-shell Hartree-Fock on the density-fitted J and K of the oracle
(the paper lists ROHF beside RHF and UHF among its standard SCF algorithms,
section "Standard algorithms").  One set of orbitals C; the n_beta lowest are
doubly occupied (core, c), the next n_alpha - n_beta singly (open, o), the rest
empty (virtual, v).  The spin densities and Fock matrices are the
unrestricted ones built from those orbitals,

    D_alpha = C_(c+o) C_(c+o)^T,  D_beta = C_c C_c^T,
    F_s = h + J[D_alpha + D_beta] - K[D_s],
    E   = 1/2 sum_s tr D_s (h + F_s) + E_nn,

and the orbitals are the eigenvectors of one effective Fock matrix (Roothaan's
coupling-operator construction; the diagonal blocks take the average
F_c = (F_alpha + F_beta) / 2, the Guest-Saunders choice).  In the basis of the
current orbitals its blocks are

    cc, oo, vv, cv:  F_c     co:  F_beta     ov:  F_alpha

so that its c-o, c-v and o-v blocks vanish exactly where the energy is
stationary under rotations between the three spaces.  In the AO basis
F_eff = S C R C^T S.  Pulay DIIS extrapolates F_eff with the error
X^T (F_eff D S - S D F_eff) X, D = D_alpha + D_beta: D has the eigenvalues
2, 1, 0 on c, o, v, so the error is zero exactly when the coupling blocks are.
"""
from dataclasses import dataclass

import numpy as np

from . import (Basis, build_df, int1e, jk, nuclear_repulsion, orthogonalizer)


@dataclass
class ROHFResult:
    E: float
    C: np.ndarray
    eps: np.ndarray
    D: tuple           # (D_alpha, D_beta)
    niter: int
    converged: bool
    history: list


def rohf_energy(C, h, Enuc, nalpha, nbeta, jk_fn):
    """E and (F_alpha, F_beta) of the determinant with orbitals C."""
    D = (C[:, :nalpha] @ C[:, :nalpha].T, C[:, :nbeta] @ C[:, :nbeta].T)
    J, _ = jk_fn(D[0] + D[1], None)
    K = [jk_fn(None, C[:, :n])[1] if n > 0 else np.zeros_like(h) for n in (nalpha, nbeta)]
    F = (h + J - K[0], h + J - K[1])
    E = 0.5 * sum(float(np.sum(D[s] * (h + F[s]))) for s in range(2)) + Enuc
    return E, F, D


def effective_fock(S, C, Fa, Fb, nalpha, nbeta):
    """S C R C^T S with R the block matrix of the module docstring (C square or
    the m kept columns of X rotations)."""
    Fc = 0.5 * (Fa + Fb)
    R = C.T @ Fc @ C
    Ra, Rb = C.T @ Fa @ C, C.T @ Fb @ C
    c, o = slice(0, nbeta), slice(nbeta, nalpha)
    v = slice(nalpha, C.shape[1])
    R[c, o] = Rb[c, o]
    R[o, c] = Rb[o, c]
    R[o, v] = Ra[o, v]
    R[v, o] = Ra[v, o]
    SC = S @ C
    return SC @ R @ SC.T


def rohf(S, h, Enuc, nalpha, nbeta, jk_fn, diis_size=8, conv_dE=1e-10, conv_err=1e-8, max_iter=200,
         ortho_thresh=1e-8):
    """jk_fn(D, C_occ) -> (J[D], K[C_occ C_occ^T]); n_alpha >= n_beta."""
    assert nalpha >= nbeta >= 0
    X, _ = orthogonalizer(S, ortho_thresh)

    def diag(F):
        eps, Cp = np.linalg.eigh(X.T @ F @ X)
        return eps, X @ Cp

    eps, C = diag(h)
    Fs, es, hist = [], [], []
    E_old, converged, it, E = None, False, 0, 0.0
    for it in range(1, max_iter + 1):
        E, (Fa, Fb), D = rohf_energy(C, h, Enuc, nalpha, nbeta, jk_fn)
        F = effective_fock(S, C, Fa, Fb, nalpha, nbeta)
        Dt = D[0] + D[1]
        err = X.T @ (F @ Dt @ S - S @ Dt @ F) @ X
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
            if 1.0 / np.linalg.cond(Bm[:m, :m]) < 1e-14:
                Fs.pop(0)
                es.pop(0)
                continue
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            c = np.linalg.solve(Bm, rhs)[:m]
            Fbar = sum(ci * Fi for ci, Fi in zip(c, Fs))
            break
        eps, C = diag(Fbar)
    D = (C[:, :nalpha] @ C[:, :nalpha].T, C[:, :nbeta] @ C[:, :nbeta].T)
    return ROHFResult(E, C, eps, D, it, converged, hist)


def df_rohf(elems_Z, xyz, shells, aux_shells, nalpha, nbeta, tau=1e-12, **kw):
    """End-to-end oracle DF-ROHF: integrals, fitting and SCF.  Also returns
    (S, h, E_nn, jk_fn) for tests that evaluate the energy of other orbitals."""
    bas, aux = Basis(shells), Basis(aux_shells)
    S, T, V = int1e(bas, xyz, elems_Z)
    df = build_df(bas, aux, tau)
    Enuc = nuclear_repulsion(xyz, elems_Z)

    def jk_fn(D, C):
        if D is not None:
            return jk(df, D=D, want_k=False)
        return jk(df, C=C, want_j=False)

    return rohf(S, T + V, Enuc, nalpha, nbeta, jk_fn, **kw), (S, T + V, Enuc, jk_fn)
