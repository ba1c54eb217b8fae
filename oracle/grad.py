"""ORACLE -- test infrastructure only.

Analytic nuclear gradient of the DF-RHF energy (section "Standard
algorithms": analytic gradients of the SCF methods; section "Molecular
integrals": the derivative integrals; the fitted integrals are those of
Eqs. (1)-(3) with the Coulomb metric).  Plain FP64, dense arrays: small
systems only.

With D = C_occ C_occ^T, W = C_occ diag(eps_occ) C_occ^T, the raw integrals
(mu nu|P), the metric J_PQ = (P|Q),

    v_P = sum (mu nu|P) D_mu nu,          c = J^-1 v,
    (ij|P) = sum C_mu i C_nu j (mu nu|P),  Z^ij = J^-1 (ij|.),

the energy E = 2 tr D h + 2 v^T c - sum_ij (ij|.)^T Z^ij + E_nn differentiates to

    dE/dx = 2 tr(D h^x) - 2 tr(W S^x)
          + sum_{mu nu P} Gam_P,mu nu (mu nu|P)^x,   Gam_P = 4 c_P D - 2 C Z_P C^T
          + sum_{PQ} Gam2_PQ (P|Q)^x,               Gam2 = -2 c c^T + sum_ij Z^ij Z^ij^T
          + dE_nn/dx,

where ^x differentiates the integrals (basis functions move with their atoms;
the nuclear attraction operator moves with its nucleus) and the orbital
response enters only through the energy-weighted density W, since the
energy is stationary in the orbitals.  The derivative integrals are
McMurchie-Davidson (md_ints.c), contracted there.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import Basis, _p, eri2, eri3_packed, lib, screen, unpack


def atoms_of(shells, xyz):
    """Atom index of every shell: the atom whose coordinates equal the centre."""
    xyz = np.asarray(xyz, float)
    out = np.zeros(len(shells), np.int32)
    for k, s in enumerate(shells):
        d = np.linalg.norm(xyz - np.asarray(s["center"], float)[None, :], axis=1)
        i = int(np.argmin(d))
        if d[i] > 1e-10:
            raise ValueError(f"shell {k} is not centred on an atom")
        out[k] = i
    return out


def dense_raw(bas, aux):
    """(mu nu|P) for every pair, dense [naux][nbf][nbf] (no screening)."""
    npair = bas.nsh * (bas.nsh + 1) // 2
    keep = np.ones((npair, aux.nsh), bool)
    pairs = np.array([(a, b) for a in range(bas.nsh) for b in range(a + 1)], np.int32).reshape(-1, 2)
    sizes = bas.size[pairs[:, 0]].astype(np.int64) * bas.size[pairs[:, 1]]
    col_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    from . import Screen
    scr = Screen(pairs, col_off, keep, 0.0)
    return unpack(eri3_packed(bas, aux, scr), bas, scr)


def nuclear_gradient(xyz, Z):
    xyz = np.asarray(xyz, float)
    g = np.zeros_like(xyz)
    for a in range(len(Z)):
        for b in range(len(Z)):
            if a != b:
                r = xyz[a] - xyz[b]
                g[a] -= Z[a] * Z[b] * r / np.linalg.norm(r) ** 3
    return g


def weights(bas, aux, C, eps):
    """The contraction weights D, W, Gam (dense [naux][nbf][nbf]) and Gam2."""
    D = C @ C.T
    W = (C * eps[None, :]) @ C.T
    raw = dense_raw(bas, aux)
    J2 = eri2(aux)
    cf = sla.cho_factor(J2, lower=True)
    v = np.einsum("pmn,mn->p", raw, D)
    c = sla.cho_solve(cf, v)
    rij = np.einsum("mi,pmn,nj->pij", C, raw, C)
    no = C.shape[1]
    Zij = sla.cho_solve(cf, rij.reshape(aux.nbf, -1)).reshape(aux.nbf, no, no)
    Gam = 4.0 * c[:, None, None] * D[None] - 2.0 * np.einsum("mi,pij,nj->pmn", C, Zij, C)
    Gam2 = -2.0 * np.outer(c, c) + np.einsum("pij,qij->pq", Zij, Zij)
    return D, W, np.ascontiguousarray(Gam), np.ascontiguousarray(Gam2)


def df_rhf_gradient(Z, xyz, shells, aux_shells, C_occ, eps_occ):
    """dE/dR [natom][3] of DF-RHF at the converged occupied orbitals C_occ
    (nbf x nocc) with levels eps_occ, and its parts (one-electron, three-index,
    metric, nuclear)."""
    xyz = np.ascontiguousarray(np.asarray(xyz, float))
    Zd = np.ascontiguousarray(np.asarray(Z, float))
    natom = len(Zd)
    bas, aux = Basis(shells), Basis(aux_shells)
    at_b = np.ascontiguousarray(atoms_of(shells, xyz))
    at_a = np.ascontiguousarray(atoms_of(aux_shells, xyz))
    C = np.asarray(C_occ, float)
    D, W, Gam, Gam2 = weights(bas, aux, C, np.asarray(eps_occ, float))
    Dw, Ww = np.ascontiguousarray(2.0 * D), np.ascontiguousarray(2.0 * W)
    g1 = np.zeros((natom, 3))
    lib().oracle_int1e_grad(bas.ref, bas.nbf, _p(at_b), natom, _p(xyz), _p(Zd), _p(Dw), _p(Ww), _p(g1))
    g3 = np.zeros((natom, 3))
    lib().oracle_eri3_grad(bas.ref, bas.nbf, aux.ref, aux.nbf, _p(at_b), _p(at_a), natom, _p(Gam), _p(g3))
    g2 = np.zeros((natom, 3))
    lib().oracle_eri2_grad(aux.ref, aux.nbf, _p(at_a), natom, _p(Gam2), _p(g2))
    gn = nuclear_gradient(xyz, Zd)
    return g1 + g3 + g2 + gn, {"one_electron": g1, "three_index": g3, "metric": g2, "nuclear": gn}


def eri3_deriv_block(bas, a, b, aux, c):
    """d(ab|C)/dR: [3 centres a, b, C][3 axes][n_a][n_b][n_C]."""
    out = np.zeros((3, 3, bas.size[a], bas.size[b], aux.size[c]))
    lib().oracle_eri3_deriv_block(bas.ref, a, b, aux.ref, c, _p(out))
    return out


def eri2_deriv_block(aux, p, q):
    """d(P|Q)/dR: [2 centres P, Q][3 axes][n_P][n_Q]."""
    out = np.zeros((2, 3, aux.size[p], aux.size[q]))
    lib().oracle_eri2_deriv_block(aux.ref, p, q, _p(out))
    return out
