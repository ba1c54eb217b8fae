"""Stage-by-stage GPU checks through the C-ABI: the Coulomb metric and the
blocked Cholesky / inverse, each against the oracle on its own."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


@pytest.mark.parametrize("name", ["h4", "mixed"])
def test_metric(dfx, name):
    ax = systems.h4()[3] if name == "h4" else systems.mixed_molecule()[3]
    J = O.eri2(O.Basis(ax))
    g = dfx.metric(ax).cpu().numpy()
    assert np.abs(g - J).max() <= 1e-13 * np.abs(J).max()


@pytest.mark.parametrize("n", [1, 17, 64, 65, 100, 130, 300])
def test_cholesky_and_inverse(dfx, n):
    rng = np.random.default_rng(n)
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = Q @ np.diag(np.exp(rng.uniform(-6, 2, n))) @ Q.T
    A = (A + A.T) / 2
    L, Li = dfx.cholesky(torch.tensor(A, device="cuda"))
    L, Li = L.cpu().numpy(), Li.cpu().numpy()
    Lr = sla.cholesky(A, lower=True)
    assert np.abs(L - Lr).max() <= 1e-10 * np.abs(Lr).max()
    assert np.abs(np.triu(L, 1)).max() == 0.0 and np.abs(np.triu(Li, 1)).max() == 0.0
    assert np.abs(Li @ Lr - np.eye(n)).max() <= 1e-9


def test_cholesky_rejects_singular(dfx):
    rng = np.random.default_rng(0)
    X = rng.normal(size=(80, 40))
    with pytest.raises(dfx.DfxError) as e:
        dfx.cholesky(torch.tensor(X @ X.T, device="cuda"))
    assert e.value.code == dfx.ENOTPOSDEF
