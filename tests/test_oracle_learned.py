"""Pins of the learned-guess oracle (oracle/learned.py) against closed forms,
textbook real spherical harmonics, group properties of rotations, finite
differences and exact round trips.  CPU only."""
import math

import numpy as np
import pytest

from oracle import learned as L
import workloads as W

WATER = {8: [0, 0, 0, 1, 1, 2], 1: [0, 0, 1]}
RC, RC_ENV = 8.0, 6.0


def rand_rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def rz(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


# ---- radial functions and cutoff ------------------------------------------------

def test_cutoff_values():
    assert L.cutoff(np.array(0.0), RC_ENV) == pytest.approx(1.0, abs=1e-15)
    assert L.cutoff(np.array(RC_ENV / 2), RC_ENV) == pytest.approx(0.5, abs=1e-15)
    assert L.cutoff(np.array(RC_ENV), RC_ENV) == 0.0
    assert L.cutoff(np.array(RC_ENV + 1.0), RC_ENV) == 0.0


@pytest.mark.parametrize("n,rmax", [(8, 6.0), (16, 8.0)])
def test_radial_centres_and_widths(n, rmax):
    w = (rmax - 0.5) / (n - 1)
    for k in range(n):
        mu = 0.5 + k * w
        g = L.radial(np.array(mu), n, rmax)
        assert g[k] == pytest.approx(1.0, abs=1e-15)
        g1 = L.radial(np.array(mu + w / 2), n, rmax)
        assert g1[k] == pytest.approx(math.exp(-0.25), rel=1e-14)


# ---- real solid harmonic rotations -----------------------------------------------

@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_rotation_about_z_closed_form(l):
    """With F = Rz(alpha), f(F^T u) turns phi into phi - alpha: the m > 0 (cosine)
    and m < 0 (sine) partners mix with cos(m alpha) and sin(m alpha)."""
    alpha = 0.7321
    U = L.sh_rotation(l, rz(alpha))
    ref = np.zeros((2 * l + 1, 2 * l + 1))
    ref[l, l] = 1.0
    for m in range(1, l + 1):
        c, s = math.cos(m * alpha), math.sin(m * alpha)
        ref[l + m, l + m] = c
        ref[l + m, l - m] = s
        ref[l - m, l - m] = c
        ref[l - m, l + m] = -s
    np.testing.assert_allclose(U, ref, atol=1e-12)


def test_rotation_l1_is_permuted_transpose():
    """l = 1 harmonics are proportional to (y, z, x) = P u, so U = P F^T P^T."""
    F = rand_rotation(5)
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], float)
    np.testing.assert_allclose(L.sh_rotation(1, F), P @ F.T @ P.T, atol=1e-12)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_rotation_group_properties(l):
    F1, F2 = rand_rotation(11), rand_rotation(12)
    U1, U2 = L.sh_rotation(l, F1), L.sh_rotation(l, F2)
    # orthogonal, U(F2 F1) = U(F1) U(F2), U(I) = I
    np.testing.assert_allclose(U1 @ U1.T, np.eye(2 * l + 1), atol=1e-12)
    np.testing.assert_allclose(L.sh_rotation(l, F2 @ F1), U1 @ U2, atol=1e-12)
    np.testing.assert_allclose(L.sh_rotation(l, np.eye(3)), np.eye(2 * l + 1), atol=1e-12)
    # trace is the SO(3) character sin((2l+1) t/2) / sin(t/2) of the rotation angle t
    t = math.acos((np.trace(F1) - 1) / 2)
    chi = math.sin((2 * l + 1) * t / 2) / math.sin(t / 2)
    assert np.trace(U1) == pytest.approx(chi, abs=1e-11)


# ---- frames and descriptors ---------------------------------------------------------

def small_water():
    elems, xyz = W.water_cluster(side=2, seed=3)
    return W.charges(elems), xyz


def test_frame_axes():
    Z, xyz = small_water()
    for a, b in [(0, 1), (0, 3), (4, 7), (5, 5)]:
        F = L.frame(xyz, a, b, RC)
        np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-13)
        assert np.linalg.det(F) == pytest.approx(1.0, abs=1e-13)
        if a != b:
            u = (xyz[b] - xyz[a]) / np.linalg.norm(xyz[b] - xyz[a])
            np.testing.assert_allclose(F[2], u, atol=1e-13)


def test_frame_of_linear_arrangement_uses_lab_axis():
    xyz = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 1.2], [0.6, 0.8, 2.4]])
    F = L.frame(xyz, 0, 1, RC)
    # every neighbour lies on the axis; x comes from the lab axis least aligned with z
    z = xyz[1] / np.linalg.norm(xyz[1])
    e = np.array([1.0, 0.0, 0.0])
    x = e - (e @ z) * z
    np.testing.assert_allclose(F[0], x / np.linalg.norm(x), atol=1e-13)


def ylm_textbook(u):
    """Orthonormal real spherical harmonics l <= 2 of a unit vector, m = -l..l."""
    x, y, z = u
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3 / (4 * math.pi))
    c2 = math.sqrt(15 / (4 * math.pi))
    c20 = math.sqrt(5 / (16 * math.pi))
    c22 = math.sqrt(15 / (16 * math.pi))
    return np.array([c0, c1 * y, c1 * z, c1 * x, c2 * x * y, c2 * y * z, c20 * (3 * z * z - 1),
                     c2 * x * z, c22 * (x * x - y * y)])


def test_pair_descriptor_closed_form():
    """Two atoms alone: one-hots, 16 Gaussians of the distance, empty environments."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 3.0, 4.0]])
    f, F = L.pair_features(xyz, np.array([8, 1]), 0, 1, RC)
    mus = [0.5 + i * 7.5 / 15 for i in range(16)]
    rad = [math.exp(-((5.0 - mu) / 0.5) ** 2) for mu in mus]
    np.testing.assert_allclose(f[:22], [0, 0, 1, 1, 0, 0] + rad, atol=1e-15)
    assert np.all(f[22:] == 0.0)
    np.testing.assert_allclose(F[2], [0.0, 0.6, 0.8], atol=1e-15)


def test_atom_descriptor_closed_form():
    """O at the origin, H1 on +z (nearest), H2 in the xz plane: the atom frame
    is the lab frame and each neighbour adds g_n(r) f_c(r) Y(u)."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.8], [1.7, 0.0, -0.6]])
    Z = np.array([8, 1, 1])
    f, F = L.pair_features(xyz, Z, 0, 0, RC)
    np.testing.assert_allclose(F, np.eye(3), atol=1e-15)
    assert list(f[:3]) == [0.0, 0.0, 1.0]
    env = np.zeros((3, 8, 9))
    for k in (1, 2):
        r = np.linalg.norm(xyz[k])
        fc = 0.5 * (math.cos(math.pi * r / RC_ENV) + 1)
        mus = [0.5 + i * 5.5 / 7 for i in range(8)]
        g = np.array([math.exp(-((r - mu) / (5.5 / 7)) ** 2) for mu in mus])
        env[0] += np.outer(g * fc, ylm_textbook(xyz[k] / r))
    np.testing.assert_allclose(f[3:], env.ravel(), atol=1e-14)


def test_descriptors_invariant_and_frames_covariant():
    Z, xyz = small_water()
    R = rand_rotation(21)
    t = np.array([1.0, -2.0, 0.5])
    xyz2 = xyz @ R.T + t
    for a, b in L.samples(xyz, Z, RC)[:60]:
        f1, F1 = L.pair_features(xyz, Z, a, b, RC)
        f2, F2 = L.pair_features(xyz2, Z, a, b, RC)
        np.testing.assert_allclose(f1, f2, atol=1e-11)
        np.testing.assert_allclose(F2, F1 @ R.T, atol=1e-11)


def test_sample_orientation_rules():
    Z, xyz = small_water()
    S = L.samples(xyz, Z, RC)
    assert sum(1 for a, b in S if a == b) == len(Z)
    for a, b in S:
        assert Z[a] >= Z[b]
        if a != b and Z[a] == Z[b]:
            assert (b, a) in S
        if a != b:
            assert np.linalg.norm(xyz[a] - xyz[b]) < RC


# ---- assembly ---------------------------------------------------------------------

def test_local_blocks_round_trip():
    """Local blocks of any symmetric D, rotated back and assembled, give D on
    every atom and pair block within the cutoff and zero elsewhere."""
    Z, xyz = small_water()
    off, n = L.offsets(Z, WATER)
    A = np.random.default_rng(0).normal(size=(n, n))
    D = A + A.T
    blocks = {}
    for a, b in L.samples(xyz, Z, RC):
        _, blocks[(a, b)] = L.local_block(D, xyz, Z, WATER, a, b, RC)
    D2 = L.assemble(blocks, xyz, Z, WATER, RC)
    mask = np.zeros((n, n), bool)
    for a in range(len(Z)):
        for b in range(len(Z)):
            if a == b or np.linalg.norm(xyz[a] - xyz[b]) < RC:
                mask[off[a]:off[a] + L.atom_nbf(WATER, Z[a]), off[b]:off[b] + L.atom_nbf(WATER, Z[b])] = True
    np.testing.assert_allclose(D2[mask], D[mask], atol=1e-12)
    assert np.all(D2[~mask] == 0.0)


def random_nets(Z, xyz, seed=0, hidden=16):
    nets = {}
    rng = np.random.default_rng(seed)
    for a, b in L.samples(xyz, Z, RC):
        k = L.type_key(Z, a, b)
        if k in nets:
            continue
        din = len(L.pair_features(xyz, Z, a, b, RC)[0])
        dout = L.atom_nbf(WATER, Z[a]) * L.atom_nbf(WATER, Z[b])
        widths = [din, hidden, hidden, dout]
        nets[k] = (widths, L.init_params(widths, seed + len(nets)), rng.normal(size=din) * 0.1,
                   1.0 + rng.random(din), rng.normal(size=dout) * 0.1, 0.1 + rng.random(dout))
    return nets


def test_prediction_equivariance():
    """A rotated molecule gets D' = U(R)^T D U(R) with U(R) the basis rotation."""
    Z, xyz = small_water()
    nets = random_nets(Z, xyz)
    D = L.predict(nets, xyz, Z, WATER, RC)
    np.testing.assert_allclose(D, D.T, atol=1e-13)
    R = rand_rotation(8)
    D2 = L.predict(nets, xyz @ R.T + 0.3, Z, WATER, RC)
    U = L.basis_rotation(Z, WATER, R)
    np.testing.assert_allclose(D2, U.T @ D @ U, atol=1e-10)


# ---- network -------------------------------------------------------------------------

def test_forward_closed_form():
    widths = [2, 2, 1]
    theta = L.flatten([np.eye(2), np.zeros(2), np.array([[1.0, -2.0]]), np.array([0.5])])
    X = np.array([[0.3, -1.2], [2.0, 0.0]])
    Y, _ = L.forward(theta, widths, X)
    s = lambda z: z / (1 + math.exp(-z))
    for i in range(2):
        assert Y[i, 0] == pytest.approx(s(X[i, 0]) - 2 * s(X[i, 1]) + 0.5, rel=1e-15)


def test_gradient_finite_differences():
    rng = np.random.default_rng(3)
    widths = [7, 11, 9, 4]
    theta = L.init_params(widths, 1) + 0.05 * rng.normal(size=L.init_params(widths, 1).size)
    X = rng.normal(size=(5, 7))
    T = rng.normal(size=(5, 4))
    _, g = L.loss_and_grad(theta, widths, X, T)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (L.loss_and_grad(tp, widths, X, T)[0] - L.loss_and_grad(tm, widths, X, T)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(g)


def test_adam_first_step_moves_by_lr():
    """Step 1: m_hat = g and v_hat = g^2, so each parameter moves by lr sign(g)."""
    g = np.array([1e-2, -3.0, 0.5, -1e-3])
    th, m, v = L.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    np.testing.assert_allclose(th, -1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-15)


def test_lowdin_density_is_a_projector():
    """For D = C C^T with C^T S C = 1 (k columns), P = S^1/2 D S^1/2 satisfies
    P^2 = P and tr P = k, and (S^1/2)^2 = S; a nearly singular S included."""
    rng = np.random.default_rng(2)
    n, k = 12, 5
    A = rng.normal(size=(n, n))
    S = A @ A.T + 1e-6 * np.eye(n)
    S /= np.sqrt(np.outer(np.diag(S), np.diag(S)))
    s, U = np.linalg.eigh(S)
    X = U / np.sqrt(s)
    Q, _ = np.linalg.qr(rng.normal(size=(n, k)))
    C = X @ Q
    P = L.lowdin(S, C @ C.T)
    np.testing.assert_allclose(P @ P, P, atol=1e-9)
    assert np.trace(P) == pytest.approx(k, abs=1e-9)
    Sh = L.lowdin(S, np.linalg.inv(S))      # S^1/2 S^-1 S^1/2 = 1
    np.testing.assert_allclose(Sh, np.eye(n), atol=1e-6)
