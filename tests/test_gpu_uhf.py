"""DF-UHF through the C-ABI (dfx_uhf) against the oracle's (oracle/uhf.py).

Both sides start from the core Hamiltonian for both spins and run Pulay DIIS
over both spins with summed error overlaps, so they follow the same path to
the same state; the GPU uses its own B (Rys integrals, FP64 transform).
Energies agree to 1e-8 Eh (the fitted tensors differ by about 1e-9 absolute,
and both converge to |dE| < 1e-11).
"""
import numpy as np
import pytest

import oracle as O
import systems
import workloads as W
from oracle import uhf as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CONV = dict(conv_dE=1e-11, conv_err=1e-9, max_iter=200)


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


def _spins(Z, charge, mult):
    nelec = int(np.sum(Z)) - charge
    na = (nelec + mult - 1) // 2
    return na, nelec - na


def _mixed():
    xyz, Z, sh, ax = systems.mixed_molecule(seed=3, natom=6, lorb=2, laux=3)
    return xyz, np.array([1] * len(Z), np.int32), sh, ax


@pytest.mark.parametrize("name,charge,mult", [("h4", 1, 2), ("h4", 0, 3), ("h4", 3, 2), ("mixed", 1, 2),
                                              ("mixed", 0, 3), ("water1", 1, 2)])
def test_uhf_matches_oracle(dfx, name, charge, mult):
    """h4 +3: one electron (n_beta = 0, K_beta = 0).  mixed: 126 functions,
    three full 32-wide tiles and a ragged one.  water1: H2O+, 5 alpha and 4 beta."""
    if name == "h4":
        xyz, Z, sh, ax, _ = systems.h4()
    elif name == "mixed":
        xyz, Z, sh, ax = _mixed()
    else:
        e, xyz, sh, ax = W.workload("water1")
        Z = W.charges(e)
    na, nb = _spins(Z, charge, mult)
    ref, _ = U.df_uhf(Z, xyz, sh, ax, na, nb, **CONV)
    assert ref.converged
    print(f"{name} q={charge} 2S+1={mult}: n_alpha {na} n_beta {nb}", flush=True)
    E, C, eps, info = dfx.uhf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, **CONV)
    print(f"  E {E:.12f} oracle {ref.E:.12f} diff {E - ref.E:.2e} it {info['niter']} / {ref.niter}")
    assert info["status"] == dfx.OK and info["converged"]
    assert info["nocc"] == na
    assert abs(E - ref.E) <= 1e-8
    # the spin densities (projectors: unique) and the occupied levels
    for s_, n_ in enumerate((na, nb)):
        D = C[s_][:, :n_] @ C[s_][:, :n_].T
        assert np.abs(D - ref.D[s_]).max() <= 1e-6 * max(1.0, np.abs(ref.D[s_]).max())
        assert np.abs(eps[s_][:n_] - ref.eps[s_][:n_]).max(initial=0.0) <= 1e-6


def test_closed_shell_equals_rhf(dfx):
    xyz, Z, sh, ax = _mixed()
    E_u, _, _, iu = dfx.uhf(xyz, Z, sh, ax, multiplicity=1, want_c=False, **CONV)
    E_r, _, _, ir = dfx.scf(xyz, Z, sh, ax, want_c=False, **CONV)
    print(f"UHF {E_u:.12f} RHF {E_r:.12f} diff {E_u - E_r:.2e}")
    assert iu["converged"] and ir["converged"]
    assert abs(E_u - E_r) <= 1e-9


def test_one_electron_is_core_ground_state(dfx):
    """A single electron feels no two-electron energy: J and K of B cancel exactly."""
    xyz, Z, sh, ax, _ = systems.h4()
    E, _, _, info = dfx.uhf(xyz, Z, sh, ax, charge=3, multiplicity=2, want_c=False, **CONV)
    bas = O.Basis(sh)
    S, T, V = O.int1e(bas, xyz, Z)
    import scipy.linalg as sla
    lam = sla.eigh(T + V, S, eigvals_only=True)[0]
    assert abs(E - (lam + O.nuclear_repulsion(xyz, Z))) <= 1e-9


@pytest.mark.parametrize("charge,mult", [(0, 2), (0, 6), (-46, 1)])
def test_bad_spin_state_raises(dfx, charge, mult):
    """h4 (4 electrons, 24 functions): a doublet has the wrong parity, a sextet
    needs 5 unpaired electrons; 50 electrons put 25 alpha in 24 functions."""
    xyz, Z, sh, ax, _ = systems.h4()
    with pytest.raises(dfx.DfxError):
        dfx.uhf(xyz, Z, sh, ax, charge=charge, multiplicity=mult)


def test_options_outside_uhf_raise(dfx):
    xyz, Z, sh, ax, _ = systems.h4()
    with pytest.raises(dfx.DfxError):
        dfx.uhf(xyz, Z, sh, ax, charge=1, multiplicity=2, schedule=dfx.SCHED_MIXED)


@pytest.mark.parametrize("method", ["uhf", "rohf"])
def test_h2_triplet_single_determinant(dfx, method):
    """Minimal-basis H2 triplet (tests/golden/h2_sto3g.json geometry and basis,
    exact DF with the primitive-product auxiliary basis): both alpha electrons
    fill the two-function space, so the UHF and ROHF energies are that one
    determinant's,
    sum_i h_ii + 1/2 sum_ij [(ii|jj) - (ij|ji)] + E_nn in any orthonormal basis,
    from the oracle's four-index integrals."""
    import json
    import os
    import scipy.linalg as sla
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "h2_sto3g.json")))
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, g["R_bohr"]]])
    prims = [(xyz[i], e) for i in range(2) for e in g["exps"]]
    aux = [systems.shell((a * A + b * B) / (a + b), 0, [a + b])
           for i, (A, a) in enumerate(prims) for (B, b) in prims[:i + 1]]
    sh = [systems.shell(xyz[i], 0, g["exps"], g["coefs"]) for i in range(2)]
    Z = np.array([1, 1], np.int32)
    E, _, _, info = getattr(dfx, method)(xyz, Z, sh, aux, multiplicity=3, tau=0.0, want_c=False, **CONV)
    assert info["converged"]
    bas = O.Basis(sh)
    S, T, V = O.int1e(bas, xyz, Z)
    Xs = sla.inv(sla.sqrtm(S)).real
    h = Xs.T @ (T + V) @ Xs
    Gm = np.einsum("mnls,mp,nq,lr,st->pqrt", O.eri4(bas), Xs, Xs, Xs, Xs)
    Ed = sum(h[i, i] for i in range(2)) + 0.5 * sum(Gm[i, i, j, j] - Gm[i, j, j, i] for i in range(2)
                                                    for j in range(2))
    assert abs(E - (Ed + 1.0 / g["R_bohr"])) <= 1e-8   # exact fit up to kappa u, kappa = 2.8e7


@pytest.mark.parametrize("charge,mult", [(1, 2), (0, 3)])
def test_uhf_purification_matches_eigensolver(dfx, charge, mult):
    """From the second iteration on, each spin's occupied space comes from
    trace-correcting purification (purify = 1, the default): the energy, the spin
    densities and the occupied levels equal those of a run with an
    eigen-decomposition of both Fock matrices every iteration."""
    xyz, Z, sh, ax = _mixed()
    na, nb = _spins(Z, charge, mult)
    kw = dict(conv_dE=1e-10, conv_err=1e-8, max_iter=200)
    E0, C0, e0, i0 = dfx.uhf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, purify=0, **kw)
    E1, C1, e1, i1 = dfx.uhf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, purify=1, **kw)
    assert i0["converged"] and i1["converged"]
    assert i0["n_purified"] == 0 and i1["n_purified"] >= 2
    assert abs(E1 - E0) <= 1e-10
    for s_, n_ in enumerate((na, nb)):
        D0, D1 = C0[s_][:, :n_] @ C0[s_][:, :n_].T, C1[s_][:, :n_] @ C1[s_][:, :n_].T
        assert np.abs(D1 - D0).max() <= 1e-7 * max(1.0, np.abs(D0).max())
        assert np.abs(e1[s_][:n_] - e0[s_][:n_]).max(initial=0.0) <= 1e-7
    print(f"q={charge} 2S+1={mult}: {i1['n_purified']} purified spin updates, {i1['n_eigh']} eigen-decompositions")
