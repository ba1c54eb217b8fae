"""Pins for the oracle's DF-ROHF (oracle/rohf.py).

- a closed shell is RHF;
- with no beta electrons ROHF and UHF are the same determinant;
- the unrestricted energy is a lower bound (UHF has more freedom);
- the converged energy is stationary under rotations between the core, open
  and virtual spaces: E(theta) - E(0) is quadratic, not linear, in theta --
  a wrong coupling block converges to a point where it is linear;
- one electron: the lowest level of the core Hamiltonian.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import systems
from oracle import rohf as R
from oracle import uhf as U

CONV = dict(conv_dE=1e-12, conv_err=1e-10, max_iter=300)


def _h4():
    xyz, Z, sh, ax, nocc = systems.h4()
    return xyz, Z, sh, ax


def test_closed_shell_equals_rhf():
    xyz, Z, sh, ax = _h4()
    r, _ = R.df_rohf(Z, xyz, sh, ax, 2, 2, **CONV)
    ref, _ = O.df_rhf(Z, xyz, sh, ax, 2)
    assert r.converged and abs(r.E - ref.E) < 1e-9


@pytest.mark.parametrize("na", [1, 2, 3])
def test_all_alpha_equals_uhf(na):
    xyz, Z, sh, ax = _h4()
    r, _ = R.df_rohf(Z, xyz, sh, ax, na, 0, **CONV)
    u, _ = U.df_uhf(Z, xyz, sh, ax, na, 0, **CONV)
    assert r.converged and u.converged
    assert abs(r.E - u.E) < 1e-9


def test_one_electron_is_the_core_ground_state():
    xyz, Z, sh, ax = _h4()
    r, _ = R.df_rohf(Z, xyz, sh, ax, 1, 0, **CONV)
    S, T, V = O.int1e(O.Basis(sh), xyz, Z)
    lam = sla.eigh(T + V, S, eigvals_only=True)[0]
    assert r.E == pytest.approx(lam + O.nuclear_repulsion(xyz, Z), abs=1e-10)


@pytest.mark.parametrize("na,nb", [(2, 1), (3, 1)])
def test_uhf_is_a_lower_bound(na, nb):
    xyz, Z, sh, ax = _h4()
    r, _ = R.df_rohf(Z, xyz, sh, ax, na, nb, **CONV)
    u, _ = U.df_uhf(Z, xyz, sh, ax, na, nb, **CONV)
    assert r.converged and u.converged
    assert u.E <= r.E + 1e-10
    assert r.E - u.E < 0.05                      # same state, small spin-polarisation energy


def _stationarity(r, extra, na, nb, seed=0, theta=1e-4):
    """(linear, quadratic) parts of E(C expm(theta kappa)) - E(C) for a random
    kappa coupling only c-o, c-v and o-v.  The odd part is cubic, about 1e-5 of
    the even part at theta = 1e-4, at a stationary point."""
    S, h, Enuc, jk_fn = extra
    C = r.C
    m = C.shape[1]
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, m))
    occ = np.array([2] * nb + [1] * (na - nb) + [0] * (m - na))
    A[occ[:, None] == occ[None, :]] = 0.0         # no rotations inside a space
    kappa = np.tril(A, -1) - np.tril(A, -1).T
    E = lambda t: R.rohf_energy(C @ sla.expm(t * kappa), h, Enuc, na, nb, jk_fn)[0]
    e0, ep, em = E(0.0), E(theta), E(-theta)
    return abs(ep - em) / 2, abs(ep + em - 2 * e0) / 2


@pytest.mark.parametrize("na,nb", [(2, 1), (3, 1)])
def test_converged_energy_is_stationary(na, nb):
    xyz, Z, sh, ax = _h4()
    r, extra = R.df_rohf(Z, xyz, sh, ax, na, nb, **CONV)
    assert r.converged
    lin, quad = _stationarity(r, extra, na, nb)
    assert quad > 1e-9                           # the probe moves the energy
    assert lin < 1e-4 * quad


def test_wrong_coupling_block_is_not_stationary(monkeypatch):
    """Sensitivity of the stationarity pin: the core-open block taken from
    F_alpha instead of F_beta converges to a non-stationary point."""
    real = R.effective_fock

    def wrong(S, C, Fa, Fb, na, nb):
        return real(S, C, Fa, Fa, na, nb) * 0.5 + real(S, C, Fa, Fb, na, nb) * 0.5

    monkeypatch.setattr(R, "effective_fock", wrong)
    xyz, Z, sh, ax = _h4()
    r, extra = R.df_rohf(Z, xyz, sh, ax, 3, 1, **CONV)
    assert r.converged
    lin, quad = _stationarity(r, extra, 3, 1)
    assert lin > 1e-2 * quad
