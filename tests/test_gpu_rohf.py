"""DF-ROHF through the C-ABI (dfx_rohf) against the oracle's (oracle/rohf.py).

Same start (core Hamiltonian), same effective Fock matrix and DIIS on both
sides, so the same path to the same state; energies agree to 1e-8 Eh.  Plus
the properties that hold at any size: a closed shell is RHF, no beta electrons
is UHF, and UHF is a lower bound.
"""
import numpy as np
import pytest

import systems
import workloads as W
from oracle import rohf as R

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


def _system(name):
    if name == "h4":
        xyz, Z, sh, ax, _ = systems.h4()
    elif name == "mixed":
        xyz, Z, sh, ax = systems.mixed_molecule(seed=3, natom=6, lorb=2, laux=3)
        Z = np.array([1] * len(Z), np.int32)
    else:
        e, xyz, sh, ax = W.workload("water1")
        Z = W.charges(e)
    return xyz, Z, sh, ax


@pytest.mark.parametrize("name,charge,mult", [("h4", 1, 2), ("h4", 0, 3), ("h4", 3, 2), ("mixed", 1, 2),
                                              ("mixed", 0, 3), ("water1", 1, 2)])
def test_rohf_matches_oracle(dfx, name, charge, mult):
    """mixed: 126 functions (three full 32-wide tiles and a ragged one), core,
    open and virtual spaces all present."""
    xyz, Z, sh, ax = _system(name)
    na, nb = _spins(Z, charge, mult)
    ref, _ = R.df_rohf(Z, xyz, sh, ax, na, nb, **CONV)
    assert ref.converged
    print(f"{name} q={charge} 2S+1={mult}: n_alpha {na} n_beta {nb}", flush=True)
    E, C, eps, info = dfx.rohf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, **CONV)
    print(f"  E {E:.12f} oracle {ref.E:.12f} diff {E - ref.E:.2e} it {info['niter']} / {ref.niter}")
    assert info["status"] == dfx.OK and info["converged"]
    assert abs(E - ref.E) <= 1e-8
    # spin densities from the one orbital set, and the effective Fock levels of the
    # occupied orbitals (same construction on both sides)
    for s_, n_ in enumerate((na, nb)):
        D = C[:, :n_] @ C[:, :n_].T
        assert np.abs(D - ref.D[s_]).max() <= 1e-6 * max(1.0, np.abs(ref.D[s_]).max())
    assert np.abs(eps[:na] - ref.eps[:na]).max() <= 1e-6


def test_closed_shell_equals_rhf(dfx):
    xyz, Z, sh, ax = _system("mixed")
    E_o, _, _, io = dfx.rohf(xyz, Z, sh, ax, multiplicity=1, want_c=False, **CONV)
    E_r, _, _, ir = dfx.scf(xyz, Z, sh, ax, want_c=False, **CONV)
    assert io["converged"] and ir["converged"]
    assert abs(E_o - E_r) <= 1e-9


@pytest.mark.parametrize("charge,mult", [(2, 3), (1, 4)])
def test_no_beta_electrons_equals_uhf(dfx, charge, mult):
    xyz, Z, sh, ax = _system("h4")
    assert _spins(Z, charge, mult)[1] == 0
    E_o, _, _, io = dfx.rohf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, want_c=False, **CONV)
    E_u, _, _, iu = dfx.uhf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, want_c=False, **CONV)
    assert io["converged"] and iu["converged"]
    assert abs(E_o - E_u) <= 1e-9


def test_uhf_is_a_lower_bound(dfx):
    xyz, Z, sh, ax = _system("mixed")
    E_o, _, _, io = dfx.rohf(xyz, Z, sh, ax, multiplicity=3, want_c=False, **CONV)
    E_u, _, _, iu = dfx.uhf(xyz, Z, sh, ax, multiplicity=3, want_c=False, **CONV)
    assert io["converged"] and iu["converged"]
    assert E_u <= E_o + 1e-10


@pytest.mark.parametrize("charge,mult", [(0, 2), (0, 6)])
def test_bad_spin_state_raises(dfx, charge, mult):
    xyz, Z, sh, ax = _system("h4")
    with pytest.raises(dfx.DfxError):
        dfx.rohf(xyz, Z, sh, ax, charge=charge, multiplicity=mult)


@pytest.mark.parametrize("method", ["uhf", "rohf"])
@pytest.mark.parametrize("name,charge,mult", [("h4", 1, 2), ("mixed", 0, 3), ("water1", 1, 2)])
def test_level_shift_keeps_the_converged_state(dfx, method, name, charge, mult):
    """A level shift changes the path, not the fixed point: the shifted runs reach
    the oracle's unshifted energy."""
    xyz, Z, sh, ax = _system(name)
    na, nb = _spins(Z, charge, mult)
    if method == "uhf":
        from oracle import uhf as U
        ref, _ = U.df_uhf(Z, xyz, sh, ax, na, nb, **CONV)
    else:
        ref, _ = R.df_rohf(Z, xyz, sh, ax, na, nb, **CONV)
    assert ref.converged
    E, _, _, info = getattr(dfx, method)(xyz, Z, sh, ax, charge=charge, multiplicity=mult, level_shift=0.5,
                                         want_c=False, **CONV)
    print(f"{method} {name}: shifted E {E:.12f} oracle {ref.E:.12f} diff {E - ref.E:.2e} it {info['niter']}")
    assert info["converged"]
    assert abs(E - ref.E) <= 1e-8


def test_level_shift_validation(dfx):
    xyz, Z, sh, ax = _system("h4")
    with pytest.raises(dfx.DfxError):
        dfx.rohf(xyz, Z, sh, ax, charge=1, multiplicity=2, level_shift=-0.1)
    with pytest.raises(dfx.DfxError):
        dfx.scf(xyz, Z, sh, ax, level_shift=0.2)


def test_open_shell_at_full_size(dfx):
    """C30H62 (730 functions, 3106 auxiliary; the size the alkane evaluation
    runs), where the oracle would take half an hour per SCF: the properties
    that hold at any size.  Closed-shell UHF and ROHF give the RHF energy; the
    triplet converges in both, to energies within 50 mEh of each other.  Plain
    DIIS takes the ROHF triplet on a long path here (85 iterations, or more than
    150 after a change of the fit at the 1e-9 level), so that run uses a level
    shift of 0.3 Eh, which leaves the converged state where it is (checked
    against the oracle on the small cases) and damps the path.  The two drivers
    can land on different triplet solutions from the core guess (measured: UHF
    -711.66033, shifted ROHF -711.66493), so UHF <= ROHF, which holds within one
    state, is checked against the oracle on the small systems instead."""
    elems, xyz, sh, ax = W.workload("alkane", seed=0)
    Z = W.charges(elems)
    conv = dict(conv_dE=1e-9, conv_err=1e-7, max_iter=150)
    E_r, _, _, ir = dfx.scf(xyz, Z, sh, ax, want_c=False, **conv)
    assert ir["converged"]
    for fn in (dfx.uhf, dfx.rohf):
        E, _, _, info = fn(xyz, Z, sh, ax, multiplicity=1, want_c=False, **conv)
        print(f"{fn.__name__} singlet: E - E_RHF = {E - E_r:.2e} ({info['niter']} iterations)", flush=True)
        assert info["converged"] and abs(E - E_r) <= 1e-8
    E_u, _, _, iu = dfx.uhf(xyz, Z, sh, ax, multiplicity=3, want_c=False, **conv)
    E_o, _, _, io = dfx.rohf(xyz, Z, sh, ax, multiplicity=3, want_c=False, level_shift=0.3,
                             **dict(conv, max_iter=300))
    print(f"triplet: UHF {E_u:.9f} ({iu['niter']} it), ROHF {E_o:.9f} ({io['niter']} it)")
    assert iu["converged"] and io["converged"]
    assert iu["nbf"] == 730 and abs(E_o - E_u) < 0.05


@pytest.mark.parametrize("charge,mult", [(1, 2), (0, 3)])
def test_rohf_purification_matches_eigensolver(dfx, charge, mult):
    """From the second iteration on, the core and core + open spaces come from
    trace-correcting purification of the effective Fock matrix at n_beta and
    n_alpha (purify = 1, the default): the energy, the spin densities and the
    occupied levels equal those of a run with an eigen-decomposition every
    iteration."""
    xyz, Z, sh, ax = _system("mixed")
    na, nb = _spins(Z, charge, mult)
    kw = dict(conv_dE=1e-10, conv_err=1e-8, max_iter=200)
    E0, C0, e0, i0 = dfx.rohf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, purify=0, **kw)
    E1, C1, e1, i1 = dfx.rohf(xyz, Z, sh, ax, charge=charge, multiplicity=mult, purify=1, **kw)
    assert i0["converged"] and i1["converged"]
    assert i0["n_purified"] == 0 and i1["n_purified"] >= 2
    assert abs(E1 - E0) <= 1e-10
    for n_ in (na, nb):
        D0, D1 = C0[:, :n_] @ C0[:, :n_].T, C1[:, :n_] @ C1[:, :n_].T
        assert np.abs(D1 - D0).max() <= 1e-7 * max(1.0, np.abs(D0).max())
    assert np.abs(e1[:na] - e0[:na]).max() <= 1e-7
    print(f"q={charge} 2S+1={mult}: {i1['n_purified']} purified updates, {i1['n_eigh']} eigen-decompositions")
