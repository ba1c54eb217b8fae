"""DF-MP2 through the C-ABI (dfx_mp2) against the oracle (oracle/mp2.py).

The orbitals and energies fed to both sides are the oracle's own converged RHF
ones, so the comparison isolates the MP2 step: the GPU uses its B (Rys
integrals, FP64 transform), the oracle its own (McMurchie-Davidson).  Then an
end-to-end case: GPU SCF followed by GPU MP2 against oracle SCF + oracle MP2.
Tolerance 1e-10 Eh on E2 (FP64 throughout; B agrees to 1e-9 absolute).
"""
import numpy as np
import pytest

import oracle as O
import systems
import workloads as W
from oracle import mp2 as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


def _case(name):
    if name == "h4":
        xyz, Z, sh, ax, nocc = systems.h4()
    elif name == "mixed":
        xyz, Z, sh, ax = systems.mixed_molecule(seed=3, natom=6, lorb=2, laux=3)
        Z = np.array([1] * len(Z), np.int32)
        nocc = 3
    else:
        e, xyz, sh, ax = W.workload("water2")
        Z, nocc = W.charges(e), W.nocc_of(e)
    res, df = O.df_rhf(Z, xyz, sh, ax, nocc, max_iter=200)
    assert res.converged
    return xyz, Z, sh, ax, nocc, res, df


@pytest.mark.parametrize("name,nfrozen", [("h4", 0), ("h4", 1), ("mixed", 0), ("mixed", 2), ("water2", 0),
                                          ("water2", 8)])
def test_mp2_matches_oracle(dfx, name, nfrozen):
    """water2: 40 occupied (one 64-column block), 152 virtual (two 128-row tiles)."""
    xyz, Z, sh, ax, nocc, res, df = _case(name)
    E_ref = M.df_mp2(df, res.C, res.eps, nocc, nfrozen)
    B = dfx.eri3(sh, ax)
    try:
        E = dfx.mp2(B, torch.tensor(res.C, device="cuda"), res.eps, nocc, nfrozen)
    finally:
        B.free()
    print(f"{name} nfrozen {nfrozen}: E2 {E:.12f} oracle {E_ref:.12f} diff {E - E_ref:.2e}")
    assert abs(E - E_ref) <= 1e-10


def test_scf_then_mp2_end_to_end(dfx):
    xyz, Z, sh, ax, nocc, res, df = _case("mixed")
    E_ref = M.df_mp2(df, res.C, res.eps, nocc)
    E, C, eps, info = dfx.scf(xyz, Z, sh, ax, conv_dE=1e-11, conv_err=1e-9, max_iter=200)
    assert info["converged"]
    nmo = info["nbf"] - info["ndropped"]
    B = dfx.eri3(sh, ax)
    try:
        E2 = dfx.mp2(B, torch.tensor(np.ascontiguousarray(C[:, :nmo]), device="cuda"), eps, nocc)
    finally:
        B.free()
    assert abs(E - res.E) <= 1e-8 and abs(E2 - E_ref) <= 1e-8


def test_mp2_rejects_bad_counts(dfx):
    xyz, Z, sh, ax, nocc, res, df = _case("h4")
    B = dfx.eri3(sh, ax)
    try:
        C = torch.tensor(res.C, device="cuda")
        for args in ((nocc, nocc), (C.shape[1], 0), (0, 0)):
            with pytest.raises(dfx.DfxError):
                dfx.mp2(B, C, res.eps, *args)
    finally:
        B.free()


def test_h2_sto3g_textbook_mp2(dfx):
    """Szabo & Ostlund's minimal-basis H2 (tests/golden/h2_sto3g_mp2.json) through
    the GPU SCF and MP2, with exact DF (the 21 products of the six primitives as
    the auxiliary basis): E2 to the book's 4 decimals, and to 1e-9 of the
    two-orbital closed form K12^2 / (2 (e1 - e2)) evaluated from the oracle's
    four-index integrals in the GPU's own orbitals (the fit is exact up to
    kappa u of a metric with kappa = 2.8e7)."""
    import json
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    g = json.load(open(os.path.join(gold, "h2_sto3g.json")))
    gm = json.load(open(os.path.join(gold, "h2_sto3g_mp2.json")))
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, g["R_bohr"]]])
    prims = [(xyz[i], e) for i in range(2) for e in g["exps"]]
    aux = [systems.shell((a * A + b * B) / (a + b), 0, [a + b])
           for i, (A, a) in enumerate(prims) for (B, b) in prims[:i + 1]]
    sh = [systems.shell(xyz[i], 0, g["exps"], g["coefs"]) for i in range(2)]
    Z = np.array([1, 1], np.int32)
    E, C, eps, info = dfx.scf(xyz, Z, sh, aux, tau=0.0, conv_dE=1e-12, conv_err=1e-10)
    assert info["converged"]
    B = dfx.eri3(sh, aux, tau=0.0)
    try:
        E2 = dfx.mp2(B, torch.tensor(C, device="cuda"), eps, 1)
    finally:
        B.free()
    assert abs(E2 - gm["E2"]) < gm["tol"]
    G = np.einsum("mnls,mp,nq,lr,st->pqrt", O.eri4(O.Basis(sh)), C, C, C, C)
    assert abs(E2 - G[0, 1, 0, 1] ** 2 / (2.0 * (eps[0] - eps[1]))) <= 1e-9
