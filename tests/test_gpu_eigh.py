"""dfx_eigh, the library's block Jacobi eigen-decomposition (through the C-ABI),
against LAPACK's (numpy.linalg.eigvalsh) on seeded symmetric matrices.

A valid result is an orthonormal V and ascending w with A V = V diag(w); the
eigenvectors of repeated eigenvalues are not unique, so the test checks that
definition (residual, orthogonality, order) plus the eigenvalues themselves
against LAPACK.  Bounds: a Jacobi method's backward error is a small multiple
of n eps ||A||, so with n <= 1536 the eigenvalues agree to 1e-12 ||A||_2 and
the residual and orthogonality stay below 5e-12 (relative to ||A||_2 and 1).
Sizes cover one block pair (n <= 64), ragged padding (65, 333) and the
(H2O)64 orbital count (1536); spectra: random (GOE), threefold-degenerate,
diagonal, decoupled blocks and a wide dynamic range.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


def _goe(n, seed):
    M = np.random.default_rng(seed).normal(size=(n, n))
    return (M + M.T) / 2.0


def _with_spectrum(w, seed):
    n = len(w)
    Q, R = np.linalg.qr(np.random.default_rng(seed).normal(size=(n, n)))
    Q = Q * np.sign(np.diag(R))[None, :]
    A = (Q * np.asarray(w)[None, :]) @ Q.T
    return (A + A.T) / 2.0


CASES = {
    "n1": lambda: np.array([[3.5]]),
    "n2": lambda: np.array([[1.0, 2.0], [2.0, -1.0]]),
    "goe31": lambda: _goe(31, 1),
    "goe64": lambda: _goe(64, 2),
    "goe65": lambda: _goe(65, 3),
    "goe333": lambda: _goe(333, 4),
    "degenerate96": lambda: _with_spectrum(np.repeat(np.arange(32, dtype=float), 3), 5),
    "diagonal100": lambda: np.diag(np.random.default_rng(6).normal(size=100)),
    "blocks130": lambda: np.kron(np.eye(2), _goe(65, 7)),
    "wide200": lambda: _with_spectrum(np.logspace(-8, 4, 200), 8),
    "goe1536": lambda: _goe(1536, 9),
}


@pytest.mark.parametrize("name", list(CASES))
def test_eigh_against_lapack(dfx, name):
    A = CASES[name]()
    n = A.shape[0]
    w, V, sweeps = dfx.eigh(torch.tensor(A, device="cuda"))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    norm = max(np.abs(ref).max(), 1e-300)
    dw = np.abs(w - ref).max() / norm
    orth = np.abs(V.T @ V - np.eye(n)).max()
    res = np.abs(A @ V - V * w[None, :]).max() / norm
    print(f"{name}: n {n}, sweeps {sweeps}, |dw|/|A| {dw:.1e}, orth {orth:.1e}, residual {res:.1e}")
    assert np.all(np.diff(w) >= 0.0)
    assert dw <= 1e-12 and orth <= 5e-12 and res <= 5e-12


def test_eigh_diagonal_needs_one_sweep_and_is_exact(dfx):
    d = np.array([3.0, -1.0, 2.0, 0.0, 5.0])
    w, V, sweeps = dfx.eigh(torch.tensor(np.diag(d), device="cuda"))
    assert sweeps == 1
    assert np.array_equal(w.cpu().numpy(), np.sort(d))
    assert np.array_equal(np.abs(V.cpu().numpy()), np.eye(5)[:, np.argsort(d)])


def test_eigh_repeatable_bitwise(dfx):
    A = torch.tensor(_goe(200, 10), device="cuda")
    w1, V1, _ = dfx.eigh(A)
    w2, V2, _ = dfx.eigh(A)
    assert torch.equal(w1, w2) and torch.equal(V1, V2)

