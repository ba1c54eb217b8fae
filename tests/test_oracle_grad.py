"""Pins for the oracle's DF-RHF analytic gradient (oracle/grad.py and the
derivative integrals in md_ints.c), against things other than itself:

* central finite differences (four points, O(h^4)) of the oracle's own
  converged DF-RHF energy, with the basis functions moving with their atoms;
* the translational sum rule sum_A g_A = 0 and the torque-free rule
  sum_A R_A x g_A = 0 (every centre is differentiated directly, so neither
  holds by construction);
* every derivative-integral block against finite differences of the oracle's
  integral blocks (which are pinned to brute-force quadrature elsewhere);
* planted omissions (the energy-weighted overlap term, the metric term) are
  shown to fail the finite-difference pin.
"""
import numpy as np
import pytest

import oracle as O
import systems
import workloads as W
from oracle import grad as G

CONV = dict(tau=0.0, conv_dE=1e-13, conv_err=1e-11)


def _scf(Z, xyz, sh, ax, nocc):
    res, _ = O.df_rhf(Z, xyz, sh, ax, nocc, **CONV)
    assert res.converged
    return res


def _fd(Z, xyz, sh, ax, nocc, a, k, h=1e-3):
    def E(s):
        x = xyz.copy()
        x[a, k] += s
        return _scf(Z, x, W.shells_at(sh, xyz, x), W.shells_at(ax, xyz, x), nocc).E
    return (8.0 * (E(h) - E(-h)) - (E(2 * h) - E(-2 * h))) / (12.0 * h)


def _system(name):
    if name == "h4":
        elems, xyz, sh, ax = W.workload("h4")
        return W.charges(elems), xyz, sh, ax
    if name == "water1":
        elems, xyz, sh, ax = W.workload("water1")
        return W.charges(elems), xyz, sh, ax
    # two centres carrying s..f orbital and s..g auxiliary shells (one contracted p each)
    xyz, _, sh, ax = systems.mixed_molecule(seed=5, natom=2, lorb=3, laux=4)
    return np.array([2, 2], np.int32), xyz, sh, ax


def _gradient(name):
    Z, xyz, sh, ax = _system(name)
    nocc = int(np.sum(Z)) // 2
    res = _scf(Z, xyz, sh, ax, nocc)
    g, parts = G.df_rhf_gradient(Z, xyz, sh, ax, res.C[:, :nocc], res.eps[:nocc])
    return Z, xyz, sh, ax, nocc, g, parts


@pytest.mark.parametrize("name,coords", [
    ("h4", [(a, k) for a in range(4) for k in range(3)]),
    ("sf", [(0, 0), (0, 1), (1, 2), (1, 0)]),
    ("water1", [(0, 0), (0, 2), (1, 1), (2, 2)]),
])
def test_gradient_against_finite_differences(name, coords):
    """Bound: 2e-9 Eh/bohr plus the rounding of the energies themselves (a few
    ulps of |E|, converged far below that) carried through the difference
    quotient, 40 eps |E| / h: 2.7e-9 for the water molecule, 2.1e-9 for H4.
    The 2e-9 is noise, not truncation: for the water molecule the four-point
    differences at h and 2h scatter by up to 1.4e-9 around the analytic value
    with no trend between the two steps."""
    Z, xyz, sh, ax, nocc, g, _ = _gradient(name)
    E = _scf(Z, xyz, sh, ax, nocc).E
    h = 1e-3
    bound = 2e-9 + 40.0 * np.finfo(float).eps * abs(E) / h
    for a, k in coords:
        d = _fd(Z, xyz, sh, ax, nocc, a, k, h=h)
        assert abs(d - g[a, k]) <= bound, (name, a, k, d, g[a, k], bound)


@pytest.mark.parametrize("name", ["h4", "sf", "water1"])
def test_translation_and_rotation_sum_rules(name):
    Z, xyz, sh, ax, nocc, g, parts = _gradient(name)
    assert np.abs(g.sum(axis=0)).max() <= 1e-11
    torque = sum(np.cross(xyz[i], g[i]) for i in range(len(Z)))
    assert np.abs(torque).max() <= 1e-10
    # each part is an integral type of its own and obeys the rule by itself
    for p in parts.values():
        assert np.abs(p.sum(axis=0)).max() <= 1e-11 * max(1.0, np.abs(p).max())


def test_planted_omissions_fail_the_pin():
    """The finite-difference pin is sensitive to each weight: dropping the
    energy-weighted overlap term or the metric term moves the gradient far
    beyond the 1e-9 bound."""
    Z, xyz, sh, ax, nocc, g, parts = _gradient("water1")
    d = _fd(Z, xyz, sh, ax, nocc, 0, 2)
    assert abs(d - (g[0, 2] - parts["metric"][0, 2])) > 1e-4
    res = _scf(Z, xyz, sh, ax, nocc)
    # no energy-weighted density: W = 0
    g_noW, _ = G.df_rhf_gradient(Z, xyz, sh, ax, res.C[:, :nocc], 0.0 * res.eps[:nocc])
    assert abs(d - g_noW[0, 2]) > 1e-3


def test_derivative_integral_blocks_against_finite_differences():
    xyz, _, sh, ax = systems.mixed_molecule(seed=2, natom=3, lorb=3, laux=4)
    bas, aux = O.Basis(sh), O.Basis(ax)
    h = 1e-4
    rng = np.random.default_rng(1)
    for _ in range(6):
        a, b, c = int(rng.integers(bas.nsh)), int(rng.integers(bas.nsh)), int(rng.integers(aux.nsh))
        d = G.eri3_deriv_block(bas, a, b, aux, c)
        for w, (S, idx) in enumerate(((sh, a), (sh, b), (ax, c))):
            for k in range(3):
                def blk(s):
                    sh2 = [dict(q) for q in sh]
                    ax2 = [dict(q) for q in ax]
                    tgt = (sh2 if S is sh else ax2)[idx]
                    tgt["center"] = np.asarray(tgt["center"], float).copy()
                    tgt["center"][k] += s
                    return O.eri3_block(O.Basis(sh2), a, b, O.Basis(ax2), c)
                fd = (8 * (blk(h) - blk(-h)) - (blk(2 * h) - blk(-2 * h))) / (12 * h)
                if S is sh and a == b:
                    continue  # moving the shared shell moves both bra centres
                assert np.abs(fd - d[w, k]).max() <= 1e-8 * max(1.0, np.abs(d[w, k]).max()), (a, b, c, w, k)
    for _ in range(4):
        p, q = int(rng.integers(aux.nsh)), int(rng.integers(aux.nsh))
        if p == q:
            continue
        d = G.eri2_deriv_block(aux, p, q)
        for w, idx in enumerate((p, q)):
            for k in range(3):
                def blk(s):
                    ax2 = [dict(x) for x in ax]
                    ax2[idx]["center"] = np.asarray(ax2[idx]["center"], float).copy()
                    ax2[idx]["center"][k] += s
                    return O.eri2_block(O.Basis(ax2), p, q)
                fd = (8 * (blk(h) - blk(-h)) - (blk(2 * h) - blk(-2 * h))) / (12 * h)
                assert np.abs(fd - d[w, k]).max() <= 1e-8 * max(1.0, np.abs(d[w, k]).max()), (p, q, w, k)
