"""Reduced-precision J/K through the C-ABI against the oracle.

FP32 / BF16 are approximations: the GPU result is compared (a) with an FP64
emulation that rounds the same operands the same way (B to FP32, then C, B and
the half-transformed X to BF16, nearest even), which isolates accumulation
order, and (b) with the exact FP64 oracle, where the stated error scale is the
unit roundoff of the format.  J reads B = hi + lo in every precision and must
match the FP64 oracle.  The SCF energies of the mixed schedules must
equal the FP64 oracle's, because the last iterations run in FP64.
"""
import numpy as np
import pytest

import oracle as O
import systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module", params=["mixed", "mixed_d"])
def case(request, dfx):
    sh, ax = (systems.mixed_molecule() if request.param == "mixed"
              else systems.mixed_molecule(seed=3, natom=6, lorb=2, laux=3))[2:4]
    df = O.build_df(O.Basis(sh), O.Basis(ax))
    B = dfx.eri3(sh, ax)
    rng = np.random.default_rng(4)
    C = np.linalg.qr(rng.normal(size=(df.bas.nbf, 11)))[0]
    yield df, B, C
    B.free()


def test_k_fp32(dfx, case):
    df, B, C = case
    Bhi = B.export(what=dfx.EXPORT_BHI).cpu().numpy()          # B rounded to FP32 by the library
    assert np.array_equal(Bhi, Bhi.astype(np.float32).astype(np.float64))
    dfe = O.DF(df.bas, df.aux, df.scr, Bhi, df.L)
    Ce = C.astype(np.float32).astype(np.float64)
    _, Ke = O.jk(dfe, C=Ce)
    J, K = dfx.jk(B, torch.tensor(C, device="cuda"), precision=dfx.FP32)
    K = K.cpu().numpy()
    Jx, Kx = O.jk(df, C=C)
    assert np.abs(K - Ke).max() <= 2e-6 * np.abs(Ke).max()
    assert np.abs(K - Kx).max() <= 1e-5 * np.abs(Kx).max()
    # J reads both FP32 words of B in every precision: the exact FP64 result
    assert np.abs(J.cpu().numpy() - Jx).max() <= 1e-9 * max(1.0, np.abs(Jx).max())


def test_k_bf16(dfx, case):
    df, B, C = case
    Bhi = B.export(what=dfx.EXPORT_BHI).cpu().numpy()
    Bb = bf16(Bhi)
    Cb = bf16(C)
    n = df.bas.nbf
    Ke = np.zeros((n, n))
    for q0 in range(0, Bb.shape[0], 64):
        Bd = O.DF(df.bas, df.aux, df.scr, Bb[q0:q0 + 64], df.L).dense_rows(0, min(64, Bb.shape[0] - q0))
        X = bf16(Bd @ Cb)
        Ke += np.einsum("qmi,qni->mn", X, X)
    _, K = dfx.jk(B, torch.tensor(C, device="cuda"), precision=dfx.BF16, want_j=False)
    K = K.cpu().numpy()
    _, Kx = O.jk(df, C=C)
    assert np.abs(K - Ke).max() <= 2e-3 * np.abs(Ke).max()
    assert np.abs(K - Kx).max() <= 2e-2 * np.abs(Kx).max()
    assert np.abs(K - K.T).max() == 0.0


@pytest.mark.parametrize("prec", ["FP32", "BF16"])
def test_mixed_scf_energy_is_the_fp64_energy(dfx, prec):
    xyz, Z, sh, ax, nocc = systems.h4()
    ref, _ = O.df_rhf(Z, xyz, sh, ax, nocc)
    E, _, _, info = dfx.scf(xyz, Z, sh, ax, schedule=dfx.SCHED_MIXED, mixed_prec=getattr(dfx, prec))
    assert info["converged"] and info["n_mixed"] >= 1
    assert abs(E - ref.E) <= 1e-8
    if prec == "BF16":
        # a well-conditioned basis: the BF16 stage passes its entry check and runs
        assert 0.0 < info["floor_est"][dfx.BF16] <= 1e-2
        assert dfx.BF16 in info["prec_hist"]
