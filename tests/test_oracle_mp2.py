"""Pins for the oracle's DF-MP2 energy (oracle/mp2.py): textbook values for
minimal-basis H2, the two-orbital closed form, an independent loop over the
four-index MO integrals, frozen-core bookkeeping, sign and rotational
invariance."""
import json
import os

import numpy as np
import pytest

import oracle as O
import systems
import workloads as W
from oracle import mp2 as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _shell(ctr, l, exps, coefs=None):
    return {"center": np.asarray(ctr, float), "l": l, "exps": list(exps),
            "coefs": list(coefs) if coefs is not None else [1.0] * len(exps)}


def _h2_exact_df():
    """H2 STO-3G with every primitive product as an auxiliary function: DF is exact."""
    g = json.load(open(os.path.join(GOLD, "h2_sto3g.json")))
    xyz = np.array([[0, 0, 0], [0, 0, g["R_bohr"]]], float)
    prims = [(xyz[i], e) for i in range(2) for e in g["exps"]]
    aux = []
    for i in range(len(prims)):
        for j in range(i + 1):
            (A, a), (B, b) = prims[i], prims[j]
            aux.append(_shell((a * A + b * B) / (a + b), 0, [a + b]))
    sh = [_shell(xyz[i], 0, g["exps"], g["coefs"]) for i in range(2)]
    return O.df_rhf([1, 1], xyz, sh, aux, 1, tau=0.0)


def _mo_integrals(df, C):
    Bd = df.dense_rows(0, df.aux.nbf)
    G = np.einsum("qmn,qls->mnls", Bd, Bd)                 # (mu nu|la si), Eq. (2) second form
    return np.einsum("mnls,mp,nq,lr,st->pqrt", G, C, C, C, C, optimize=True)


def test_h2_sto3g_mp2_textbook():
    g = json.load(open(os.path.join(GOLD, "h2_sto3g_mp2.json")))
    res, df = _h2_exact_df()
    assert res.converged
    Gm = _mo_integrals(df, res.C)
    tol = g["tol"]
    assert abs(Gm[0, 0, 0, 0] - g["J11"]) < tol and abs(Gm[0, 0, 1, 1] - g["J12"]) < tol
    assert abs(Gm[1, 1, 1, 1] - g["J22"]) < tol and abs(Gm[0, 1, 1, 0] - g["K12"]) < tol
    E2 = M.df_mp2(df, res.C, res.eps, 1)
    assert abs(E2 - g["E2"]) < tol
    # two orbitals: E2 = K12^2 / (2 (e1 - e2)) exactly
    assert E2 == pytest.approx(Gm[0, 1, 1, 0] ** 2 / (2.0 * (res.eps[0] - res.eps[1])), rel=1e-12)


@pytest.fixture(scope="module")
def h4_mp2():
    xyz, Z, sh, ax, nocc = systems.h4()
    res, df = O.df_rhf(Z, xyz, sh, ax, nocc)
    assert res.converged
    return xyz, Z, sh, ax, nocc, res, df


@pytest.mark.parametrize("nfrozen", [0, 1])
def test_mp2_against_four_index_loops(h4_mp2, nfrozen):
    *_, nocc, res, df = h4_mp2
    Gm = _mo_integrals(df, res.C)
    E_loops = M.mp2_from_mo_integrals(Gm, res.eps, nocc, nfrozen)
    E = M.df_mp2(df, res.C, res.eps, nocc, nfrozen)
    assert E == pytest.approx(E_loops, rel=1e-12, abs=1e-14)
    assert E < 0.0


def test_mp2_frozen_core_drops_the_core_pairs(h4_mp2):
    *_, nocc, res, df = h4_mp2
    E0 = M.df_mp2(df, res.C, res.eps, nocc, 0)
    E1 = M.df_mp2(df, res.C, res.eps, nocc, 1)
    assert E1 > E0          # fewer negative pair energies


def test_mp2_rotation_invariance(h4_mp2):
    xyz, Z, sh, ax, nocc, res, df = h4_mp2
    E = M.df_mp2(df, res.C, res.eps, nocc)
    rng = np.random.default_rng(3)
    q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    new = xyz @ q.T + rng.normal(size=3)
    r2, df2 = O.df_rhf(Z, new, W.shells_at(sh, xyz, new), W.shells_at(ax, xyz, new), nocc)
    assert abs(M.df_mp2(df2, r2.C, r2.eps, nocc) - E) < 1e-9
