"""Invariances of the whole GPU path, independent of the oracle, on a molecule
whose orbital shells reach f and auxiliary shells g (solid harmonics up to
l = 3 and 4; 210 functions, 330 auxiliary, several ragged tiles).

- rotating and translating the molecule leaves the DF-RHF energy unchanged:
  every m-component of every shell class must transform consistently;
- permuting the atoms (so the shell, tile and pair order of B) leaves the
  DF-RHF and DF-MP2 energies unchanged.
Energies are converged to |dE| < 1e-11 and agree to 1e-9 Eh.
"""
import numpy as np
import pytest

import systems
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CONV = dict(conv_dE=1e-11, conv_err=1e-9, max_iter=200)


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


@pytest.fixture(scope="module")
def mol(dfx):
    xyz, _, sh, ax = systems.mixed_molecule(seed=3, natom=6, lorb=3, laux=4)
    Z = np.ones(len(xyz), np.int32)
    E, C, eps, info = dfx.scf(xyz, Z, sh, ax, **CONV)
    assert info["converged"] and info["nbf"] == 210 and info["naux"] == 330
    return xyz, Z, sh, ax, E, C, eps, info


def _mp2(dfx, sh, ax, C, eps, info):
    nmo = info["nbf"] - info["ndropped"]
    B = dfx.eri3(sh, ax)
    try:
        return dfx.mp2(B, torch.tensor(np.ascontiguousarray(C[:, :nmo]), device="cuda"), eps, info["nocc"])
    finally:
        B.free()


def test_rotation_and_translation(dfx, mol):
    xyz, Z, sh, ax, E, C, eps, info = mol
    rng = np.random.default_rng(11)
    q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    new = xyz @ q.T + rng.normal(size=3)
    E2, _, eps2, i2 = dfx.scf(new, Z, W.shells_at(sh, xyz, new), W.shells_at(ax, xyz, new), **CONV)
    print(f"rotated: dE = {E2 - E:.2e}, max |d eps| = {np.abs(eps2 - eps).max():.2e}")
    assert i2["converged"] and abs(E2 - E) <= 1e-9
    assert np.abs(eps2 - eps).max() <= 1e-7


def test_atom_permutation_scf_and_mp2(dfx, mol):
    xyz, Z, sh, ax, E, C, eps, info = mol
    perm = np.array([4, 1, 5, 0, 3, 2])

    def by_atom(shells):
        groups = [[s for s in shells if np.linalg.norm(s["center"] - xyz[a]) < 1e-12] for a in range(len(xyz))]
        assert sum(len(g) for g in groups) == len(shells)
        return [s for a in perm for s in groups[a]]

    shp, axp = by_atom(sh), by_atom(ax)
    Ep, Cp, epsp, ip = dfx.scf(xyz[perm], Z[perm], shp, axp, **CONV)
    assert ip["converged"] and abs(Ep - E) <= 1e-9
    E2 = _mp2(dfx, sh, ax, C, eps, info)
    E2p = _mp2(dfx, shp, axp, Cp, epsp, ip)
    print(f"permuted: dE = {Ep - E:.2e}, E2 = {E2:.12f}, dE2 = {E2p - E2:.2e}")
    assert E2 < 0.0 and abs(E2p - E2) <= 1e-9
