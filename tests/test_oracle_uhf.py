"""Pins for the oracle's DF-UHF (oracle/uhf.py): the one-electron case is the
lowest eigenvalue of the core Hamiltonian (self-interaction cancels exactly in
Hartree-Fock, and in DF too, since J and K come from the same B); a closed
shell reproduces RHF; the minimal-basis H2 triplet equals its determinant
energy from the four-index integrals."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import systems
from oracle import uhf as U

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _shell(ctr, l, exps, coefs=None):
    return {"center": np.asarray(ctr, float), "l": l, "exps": list(exps),
            "coefs": list(coefs) if coefs is not None else [1.0] * len(exps)}


def test_one_electron_is_the_core_ground_state():
    xyz, Z, sh, ax, nocc = systems.h4()
    r, df = U.df_uhf(Z, xyz, sh, ax, 1, 0)            # H4^3+: one electron
    assert r.converged
    bas = O.Basis(sh)
    S, T, V = O.int1e(bas, xyz, Z)
    lam = sla.eigh(T + V, S, eigvals_only=True)[0]
    assert r.E == pytest.approx(lam + O.nuclear_repulsion(xyz, Z), abs=1e-10)


def test_closed_shell_equals_rhf():
    xyz, Z, sh, ax, nocc = systems.h4()
    r, df = U.df_uhf(Z, xyz, sh, ax, nocc, nocc)
    ref, _ = O.df_rhf(Z, xyz, sh, ax, nocc)
    assert r.converged and abs(r.E - ref.E) < 1e-9
    assert np.abs(r.D[0] - r.D[1]).max() < 1e-7


def test_h2_triplet_against_four_index_integrals():
    """Both spin-up electrons fill the two-function space: one determinant, whose
    energy sum_i h_ii + 1/2 sum_ij [(ii|jj) - (ij|ji)] + E_nn is basis-invariant."""
    g = json.load(open(os.path.join(GOLD, "h2_sto3g.json")))
    xyz = np.array([[0, 0, 0], [0, 0, g["R_bohr"]]], float)
    prims = [(xyz[i], e) for i in range(2) for e in g["exps"]]
    aux = [_shell((a * A + b * B) / (a + b), 0, [a + b])
           for i, (A, a) in enumerate(prims) for (B, b) in prims[:i + 1]]
    sh = [_shell(xyz[i], 0, g["exps"], g["coefs"]) for i in range(2)]
    r, df = U.df_uhf([1, 1], xyz, sh, aux, 2, 0, tau=0.0)
    assert r.converged
    bas = O.Basis(sh)
    S, T, V = O.int1e(bas, xyz, [1, 1])
    G = O.eri4(bas)
    Xs = sla.inv(sla.sqrtm(S)).real                    # any orthonormal basis of the space
    h = Xs.T @ (T + V) @ Xs
    Gm = np.einsum("mnls,mp,nq,lr,st->pqrt", G, Xs, Xs, Xs, Xs)
    E = sum(h[i, i] for i in range(2)) + 0.5 * sum(Gm[i, i, j, j] - Gm[i, j, j, i] for i in range(2) for j in range(2))
    assert r.E == pytest.approx(E + 1.0 / g["R_bohr"], abs=1e-9)


def test_doublet_lies_below_its_restricted_counterpart():
    """H4+ doublet: the unrestricted energy is variational, at or below the
    restricted-open-shell-like start where alpha and beta share orbitals."""
    xyz, Z, sh, ax, nocc = systems.h4()
    r, df = U.df_uhf(Z, xyz, sh, ax, 2, 1)             # H4+: 3 electrons
    assert r.converged
    # a single UHF iteration from the common core orbitals gives an upper bound
    r1, _ = U.df_uhf(Z, xyz, sh, ax, 2, 1, max_iter=1)
    assert r.E <= r1.history[0][0] + 1e-12
