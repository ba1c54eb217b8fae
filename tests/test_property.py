"""Property tests over random shells (hypothesis, derandomised so every run
draws the same cases): random centres, exponents and contractions, orbital
l <= 3 and auxiliary l <= 4.

CPU (the oracle's McMurchie-Davidson integrals, section "Molecular integrals"):
translation invariance, the bra swap symmetry, invariance of a block's norm
under a rotation of all centres (complete shells of real solid harmonics
transform by orthogonal matrices), and the Schwarz inequality.

GPU (marked gpu): the library's Rys raw integrals (mu nu|P) for the same kind
of random shell sets against the oracle's, element by element, at the raw
parity bound (1e-13 of the largest element plus 1e-15).
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

import oracle as O
import systems

PROFILE = settings(max_examples=25, deadline=None, derandomize=True,
                   suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])

coord = st.floats(-1.5, 1.5, allow_nan=False, allow_infinity=False)
centre = st.tuples(coord, coord, coord)
expo = st.floats(0.15, 8.0, allow_nan=False, allow_infinity=False)
coef = st.floats(0.1, 1.0, allow_nan=False, allow_infinity=False)


@st.composite
def a_shell(draw, lmax):
    l = draw(st.integers(0, lmax))
    k = draw(st.integers(1, 3))
    exps = draw(st.lists(expo, min_size=k, max_size=k, unique=True))
    coefs = draw(st.lists(coef, min_size=k, max_size=k))
    return systems.shell(draw(centre), l, exps, coefs)


@st.composite
def triplet(draw):
    """Two orbital shells and one auxiliary shell."""
    return draw(a_shell(3)), draw(a_shell(3)), draw(a_shell(4))


def _block(a, b, c):
    return O.eri3_block(O.Basis([a, b]), 0, 1, O.Basis([c]), 0)


def _moved(s, R=np.eye(3), t=np.zeros(3)):
    out = dict(s)
    out["center"] = R @ np.asarray(s["center"], float) + t
    return out


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@PROFILE
@given(triplet(), st.tuples(coord, coord, coord))
def test_translation_invariance(t3, shift):
    a, b, c = t3
    t = np.array(shift) * 3.0
    ref = _block(a, b, c)
    mv = _block(_moved(a, t=t), _moved(b, t=t), _moved(c, t=t))
    assert np.abs(mv - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@PROFILE
@given(triplet())
def test_bra_swap(t3):
    a, b, c = t3
    ab = _block(a, b, c)
    ba = _block(b, a, c)
    assert np.abs(ab - ba.transpose(1, 0, 2)).max() <= 1e-13 * max(1.0, np.abs(ab).max())


@PROFILE
@given(triplet(), st.integers(0, 2 ** 31 - 1))
def test_rotation_keeps_block_norm(t3, seed):
    a, b, c = t3
    R = _rotation(seed)
    ref = _block(a, b, c)
    rot = _block(_moved(a, R), _moved(b, R), _moved(c, R))
    n0, n1 = np.linalg.norm(ref), np.linalg.norm(rot)
    assert abs(n1 - n0) <= 1e-12 * max(1.0, n0)
    # the rotation acts on the block, reshaped to [n_a n_b][n_C], by orthogonal
    # matrices on both sides, so its singular values are invariant as well
    s0 = np.linalg.svd(ref.reshape(-1, ref.shape[2]), compute_uv=False)
    s1 = np.linalg.svd(rot.reshape(-1, rot.shape[2]), compute_uv=False)
    assert np.abs(s1 - s0).max() <= 1e-12 * max(1.0, s0.max())


@PROFILE
@given(triplet())
def test_schwarz_inequality(t3):
    a, b, c = t3
    bas, aux = O.Basis([a, b]), O.Basis([c])
    blk = O.eri3_block(bas, 0, 1, aux, 0)
    abab = O.eri4_block(bas, 0, 1, 0, 1)
    cc = O.eri2_block(aux, 0, 0)
    na, nb, nc = blk.shape
    d_ab = np.array([[abab[i, j, i, j] for j in range(nb)] for i in range(na)])
    d_c = np.diag(cc)
    bound = np.sqrt(d_ab)[:, :, None] * np.sqrt(d_c)[None, None, :]
    assert np.all(np.abs(blk) <= bound * (1 + 1e-12) + 1e-15)


# ---- GPU: random shell sets, raw integrals against the oracle ---------------------

@st.composite
def shell_set(draw):
    """2 or 3 centres at least 1 bohr apart; 1-3 orbital shells each (l <= 3,
    1-3 primitives); at most one auxiliary shell per (centre, l), l <= 4, so
    the metric stays positive definite."""
    n = draw(st.integers(2, 3))
    ctrs = [np.array(draw(centre)) * 1.5 for _ in range(n)]
    assume(min(np.linalg.norm(ctrs[i] - ctrs[j]) for i in range(n) for j in range(i)) >= 1.0)
    sh, ax = [], []
    for r in ctrs:
        for _ in range(draw(st.integers(1, 3))):
            s = draw(a_shell(3))
            s["center"] = r
            sh.append(s)
        for l in draw(st.lists(st.integers(0, 4), min_size=1, max_size=3, unique=True)):
            ax.append(systems.shell(r, l, [draw(st.floats(0.3, 3.0))]))
    return sh, ax


@pytest.mark.gpu
@settings(max_examples=15, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large,
                                 HealthCheck.function_scoped_fixture])
@given(shell_set())
def test_gpu_raw_integrals_random_shells(shells):
    torch = pytest.importorskip("torch")
    import paper_1707_03771_amd as dfx
    sh, ax = shells
    bas, aux = O.Basis(sh), O.Basis(ax)
    Qab, QC = O.schwarz(bas, aux)
    scr = O.screen(bas, aux, Qab, QC, 0.0)
    raw = O.eri3_packed(bas, aux, scr)
    B = dfx.eri3(sh, ax, tau=0.0, flags=dfx.KEEP_RAW)
    try:
        g = B.export(what=2).detach().cpu().numpy()
    finally:
        B.free()
        torch.cuda.synchronize()
    assert g.shape == raw.shape
    assert np.abs(g - raw).max() <= 1e-13 * np.abs(raw).max() + 1e-15
