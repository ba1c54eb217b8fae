"""ORACLE -- test infrastructure only (see oracle/__init__.py for who may use it).

DF-MP2 correlation energy of a closed-shell RHF reference.  The paper lists MP2
as a post-HF method among its standard algorithms and provides the operations
it is built from (section "Density fitting utilities"): the two index
transformations of Eq. (1) applied to B give the mixed occupied-virtual
three-index tensor, and the contraction of two such tensors (Eq. (2), second
form) gives the four-index integrals.  The energy expression is the textbook
closed-shell second-order energy (Szabo & Ostlund, "Modern Quantum Chemistry",
eq. 6.74, written in spatial orbitals):

    (ia|Q)  = sum_{mu nu} C_mu,i B_Q,mu nu C_nu,a
    (ia|jb) = sum_Q (ia|Q) (jb|Q)
    E2      = sum_{ij} sum_{ab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)

with i, j over the correlated occupied orbitals (the first nfrozen are left
out) and a, b over the virtual ones.
"""
import numpy as np


def ov_tensor(df, C, nocc, nfrozen=0, chunk=64):
    """(ia|Q) as an array [i][a][Q], from B in chunks of auxiliary rows."""
    Co, Cv = C[:, nfrozen:nocc], C[:, nocc:]
    naux = df.aux.nbf
    out = np.zeros((Co.shape[1], Cv.shape[1], naux))
    for q0 in range(0, naux, chunk):
        q1 = min(naux, q0 + chunk)
        Bd = df.dense_rows(q0, q1)                              # [Q][mu][nu]
        out[:, :, q0:q1] = np.einsum("qmn,mi,na->iaq", Bd, Co, Cv, optimize=True)
    return out


def df_mp2(df, C, eps, nocc, nfrozen=0):
    """E2 of the module docstring; C holds the canonical orbitals as columns
    (occupied first) and eps their energies."""
    iaQ = ov_tensor(df, C, nocc, nfrozen)
    eo, ev = np.asarray(eps[nfrozen:nocc]), np.asarray(eps[nocc:C.shape[1]])
    E = 0.0
    for i in range(iaQ.shape[0]):
        for j in range(iaQ.shape[0]):
            g = iaQ[i] @ iaQ[j].T                               # (ia|jb) as [a][b]
            d = eo[i] + eo[j] - ev[:, None] - ev[None, :]
            E += float(np.sum(g * (2.0 * g - g.T) / d))
    return E


def mp2_from_mo_integrals(G, eps, nocc, nfrozen=0):
    """The same energy from a full four-index MO integral array G[p][q][r][s] =
    (pq|rs), by explicit loops (for tiny cases: a check of the contraction)."""
    n = G.shape[0]
    E = 0.0
    for i in range(nfrozen, nocc):
        for j in range(nfrozen, nocc):
            for a in range(nocc, n):
                for b in range(nocc, n):
                    E += G[i, a, j, b] * (2.0 * G[i, a, j, b] - G[i, b, j, a]) / (eps[i] + eps[j] - eps[a] - eps[b])
    return E
