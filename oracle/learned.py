"""ORACLE -- test infrastructure only.

FP64 reference for the learned starting guess: a per-atom-pair multilayer
perceptron that maps invariant descriptors of a pair's local geometry to the
block of that pair of the density matrix in the symmetrically orthogonalised
(Loewdin) basis, expressed in a local frame.

Written from the definitions, independent of the library:
* local frames from the geometry (same stated rules, separate code);
* real-solid-harmonic rotation matrices fitted by least squares on sample
  points of the rotated harmonics (the library substitutes polynomials);
* descriptors: radial Gaussians times real solid harmonics of neighbour
  directions in the local frame, with a cosine cutoff;
* the network: Linear -> SiLU -> ... -> Linear, mean-squared error, Adam, with
  a hand-derived backward pass.
"""
from __future__ import annotations

import math

import numpy as np

from . import cart_powers, solid_harmonics

ELEMENTS = (1, 6, 8)          # H, C, O: one-hot / neighbour channels
NRAD = 8                      # radial Gaussians per neighbour channel, on [RMIN, rc_env]
NPAIR_RAD = 16                # radial Gaussians of the pair distance, on [RMIN, rc]
RMIN = 0.5
RC_PAIR, RC_ENV = 8.0, 6.0    # pair cutoff, neighbour-environment cutoff (bohr)


def cutoff(r, rc):
    return np.where(r < rc, 0.5 * (np.cos(np.pi * r / rc) + 1.0), 0.0)


def radial(r, n, rmax):
    """n Gaussians with centres evenly spaced on [RMIN, rmax], width = spacing."""
    mu = np.linspace(RMIN, rmax, n)
    w = (rmax - RMIN) / (n - 1)
    return np.exp(-((r - mu) / w) ** 2)


def _unit(v):
    return v / np.linalg.norm(v)


def frame(xyz, a, b, rc):
    """Rows (x, y, z) of the local frame of pair (a, b), or of atom a if b == a.
    z: a -> b (pair) or a -> nearest neighbour (atom); x: the nearest other
    neighbour of a whose direction is at least 0.1 rad from z, projected off z;
    with none, the lab axis least aligned with z.  Neighbours are ranked by
    distance (1e-8 bohr resolution), ties by index."""
    A = xyz[a]
    # rank by distance at a resolution of 1e-8 bohr, then by index: equal bond
    # lengths (a rigid water's two O-H) keep their order under rotation
    d = np.linalg.norm(xyz - A, axis=1)
    order = sorted((k for k in range(len(xyz)) if k != a), key=lambda k: (math.floor(d[k] * 1e8 + 0.5), k))
    if b != a:
        z = _unit(xyz[b] - A)
        cand = [k for k in order if k != b]
    else:
        if not order:
            return np.eye(3)
        z = _unit(xyz[order[0]] - A)
        cand = order[1:]
    xv = None
    for k in cand:
        v = xyz[k] - A
        s = np.linalg.norm(np.cross(_unit(v), z))
        if s > math.sin(0.1):
            xv = v - (v @ z) * z
            break
    if xv is None:
        ax = np.argmin(np.abs(z))
        e = np.zeros(3)
        e[ax] = 1.0
        xv = e - (e @ z) * z
    x = _unit(xv)
    y = np.cross(z, x)
    return np.array([x, y, z])


def sh_rotation(l, F):
    """U with f_m(F^T u) = sum_m' U[m, m'] f_m'(u) for the orthonormal real solid
    harmonics of degree l, by least squares on random unit vectors."""
    if l == 0:
        return np.ones((1, 1))
    T = solid_harmonics(l)
    pw = np.array(cart_powers(l))
    rng = np.random.default_rng(1234 + l)
    u = rng.normal(size=(6 * (2 * l + 1), 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)

    def ev(pts):
        return T @ np.prod(pts[:, None, :] ** pw[None, :, :], axis=2).T  # [m][k]

    Fm = ev(u @ F)          # rows of u @ F are (F^T u_k)^T
    G = ev(u)
    U, *_ = np.linalg.lstsq(G.T, Fm.T, rcond=None)
    return U.T


def shell_rotation(ls, F):
    """Block-diagonal rotation over an atom's shells."""
    blocks = [sh_rotation(l, F) for l in ls]
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n))
    o = 0
    for bl in blocks:
        k = bl.shape[0]
        out[o:o + k, o:o + k] = bl
        o += k
    return out


def env_features(xyz, Z, a, F, exclude, rc):
    """sum over neighbours k of a (k not in exclude, |r_ak| < rc):
    radial_n(r) f_c(r) Y_lm(unit(F (r_k - r_a))), l <= 2, per element channel,
    radial Gaussians on [RMIN, rc]."""
    out = np.zeros((len(ELEMENTS), NRAD, 9))
    Ys = [solid_harmonics(l) for l in range(3)]
    pws = [np.array(cart_powers(l)) for l in range(3)]
    for k in range(len(Z)):
        if k == a or k in exclude:
            continue
        v = xyz[k] - xyz[a]
        r = np.linalg.norm(v)
        if r >= rc:
            continue
        u = F @ (v / r)
        ylm = np.concatenate([Ys[l] @ np.prod(u[None, :] ** pws[l], axis=1) for l in range(3)])
        ch = ELEMENTS.index(int(Z[k]))
        out[ch] += np.outer(radial(r, NRAD, rc) * cutoff(r, rc), ylm)
    return out.ravel()


def pair_features(xyz, Z, a, b, rc=RC_PAIR, rc_env=RC_ENV):
    """Descriptors and local frame of sample (a, b); atom a alone when b == a.
    Pair: one-hot(Z_a), one-hot(Z_b), Gaussians of |r_ab| on [RMIN, rc], then
    the environments of a and of b (each without the other).  Atom: one-hot(Z_a)
    and its environment."""
    F = frame(xyz, a, b, rc)
    if a == b:
        onehot = np.array([float(Z[a] == e) for e in ELEMENTS])
        return np.concatenate([onehot, env_features(xyz, Z, a, F, (), rc_env)]), F
    r = np.linalg.norm(xyz[b] - xyz[a])
    ta = np.array([float(Z[a] == e) for e in ELEMENTS])
    tb = np.array([float(Z[b] == e) for e in ELEMENTS])
    rad = radial(r, NPAIR_RAD, rc)
    fa = env_features(xyz, Z, a, F, (b,), rc_env)
    fb = env_features(xyz, Z, b, F, (a,), rc_env)
    return np.concatenate([ta, tb, rad, fa, fb]), F


# ---------------------------------------------------------------------------
# network: theta = concatenation over layers of W (out x in, row-major), b (out)

def init_params(widths, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for i in range(len(widths) - 1):
        fan_in = widths[i]
        ps.append(rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=(widths[i + 1], widths[i])))
        ps.append(np.zeros(widths[i + 1]))
    return flatten(ps)


def flatten(ps):
    return np.concatenate([p.ravel() for p in ps])


def unflatten(theta, widths):
    ps, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        ps.append(theta[o:o + n_in * n_out].reshape(n_out, n_in))
        o += n_in * n_out
        ps.append(theta[o:o + n_out])
        o += n_out
    return ps


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, widths, X):
    ps = unflatten(theta, widths)
    a, cache = X, []
    nl = len(widths) - 1
    for i in range(nl):
        W, b = ps[2 * i], ps[2 * i + 1]
        z = a @ W.T + b
        cache.append((a, z))
        a = silu(z) if i < nl - 1 else z
    return a, cache


def loss_and_grad(theta, widths, X, T):
    """MSE = mean over all outputs of (y - t)^2 and its gradient in theta."""
    Y, cache = forward(theta, widths, X)
    diff = Y - T
    loss = float(np.mean(diff ** 2))
    g = 2.0 * diff / diff.size
    ps = unflatten(theta, widths)
    grads = [None] * len(ps)
    nl = len(widths) - 1
    for i in reversed(range(nl)):
        a_in, z = cache[i]
        if i < nl - 1:
            g = g * dsilu(z)
        grads[2 * i] = g.T @ a_in
        grads[2 * i + 1] = g.sum(axis=0)
        g = g @ ps[2 * i]
    return loss, flatten(grads)


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad ** 2
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# samples, local target blocks and assembly of the predicted density
#
# basis: {Z: [l of each shell of that element, in basis order]}; the molecular
# basis lists the shells atom by atom.  A sample is an ordered pair (a, b): the
# atom itself (a, a), and for every pair closer than rc the orientation with the
# heavier element first; pairs of equal elements give both orientations.

def atom_nbf(basis, z):
    return sum(2 * l + 1 for l in basis[int(z)])


def offsets(Z, basis):
    off = np.cumsum([0] + [atom_nbf(basis, z) for z in Z])
    return off[:-1], int(off[-1])


def type_key(Z, a, b):
    return ("atom", int(Z[a])) if a == b else ("pair", int(Z[a]), int(Z[b]))


def samples(xyz, Z, rc):
    out = []
    n = len(Z)
    for a in range(n):
        out.append((a, a))
        for b in range(a + 1, n):
            if np.linalg.norm(xyz[b] - xyz[a]) >= rc:
                continue
            if Z[a] > Z[b]:
                out.append((a, b))
            elif Z[a] < Z[b]:
                out.append((b, a))
            else:
                out.append((a, b))
                out.append((b, a))
    return out


def local_block(D, xyz, Z, basis, a, b, rc=RC_PAIR, rc_env=RC_ENV):
    """D_ab written in the local frame of (a, b): U_a^T D_ab U_b, and its descriptors."""
    f, F = pair_features(xyz, Z, a, b, rc, rc_env)
    off, _ = offsets(Z, basis)
    na, nb = atom_nbf(basis, Z[a]), atom_nbf(basis, Z[b])
    Ua = shell_rotation(basis[int(Z[a])], F)
    Ub = shell_rotation(basis[int(Z[b])], F)
    blk = D[off[a]:off[a] + na, off[b]:off[b] + nb]
    return f, Ua.T @ blk @ Ub


def training_set(geoms, basis, rc=RC_PAIR, rc_env=RC_ENV):
    """{type: (X [n, d_in], T [n, d_out])} from [(xyz, Z, P)], P the converged
    density in the Loewdin basis."""
    data = {}
    for xyz, Z, P in geoms:
        for a, b in samples(xyz, Z, rc):
            f, blk = local_block(P, xyz, Z, basis, a, b, rc, rc_env)
            xs, ts = data.setdefault(type_key(Z, a, b), ([], []))
            xs.append(f)
            ts.append(blk.ravel())
    return {k: (np.array(x), np.array(t)) for k, (x, t) in data.items()}


def assemble(blocks, xyz, Z, basis, rc=RC_PAIR):
    """D from local-frame blocks {(a, b): P}: rotate each to the lab frame,
    U_a P U_b^T, place it at (a, b) and its transpose at (b, a); orientations of
    equal-element pairs are averaged and atom blocks symmetrised."""
    off, n = offsets(Z, basis)
    D = np.zeros((n, n))
    for (a, b), P in blocks.items():
        F = frame(xyz, a, b, rc)
        Ua = shell_rotation(basis[int(Z[a])], F)
        Ub = shell_rotation(basis[int(Z[b])], F)
        M = Ua @ P @ Ub.T
        w = 0.5 if (a == b or Z[a] == Z[b]) else 1.0
        na, nb = M.shape
        D[off[a]:off[a] + na, off[b]:off[b] + nb] += w * M
        D[off[b]:off[b] + nb, off[a]:off[a] + na] += w * M.T
    return D


def predict(nets, xyz, Z, basis, rc=RC_PAIR, rc_env=RC_ENV):
    """Loewdin-basis density predicted by nets[type] = (widths, theta, fmean,
    fstd, tmean, tstd)."""
    blocks = {}
    for a, b in samples(xyz, Z, rc):
        widths, theta, fm, fs, tm, ts = nets[type_key(Z, a, b)]
        f, _ = pair_features(xyz, Z, a, b, rc, rc_env)
        y, _ = forward(np.asarray(theta, np.float64), widths, ((f - fm) / fs)[None, :])
        na, nb = atom_nbf(basis, Z[a]), atom_nbf(basis, Z[b])
        blocks[(a, b)] = (y[0] * ts + tm).reshape(na, nb)
    return assemble(blocks, xyz, Z, basis, rc)


def basis_rotation(Z, basis, R):
    """Block-diagonal U(R) over the molecular basis (R orthogonal 3 x 3)."""
    mats = [shell_rotation(basis[int(z)], R) for z in Z]
    n = sum(m.shape[0] for m in mats)
    out = np.zeros((n, n))
    o = 0
    for m in mats:
        k = m.shape[0]
        out[o:o + k, o:o + k] = m
        o += k
    return out


def lowdin(S, D):
    """P = S^1/2 D S^1/2: the density in the symmetrically orthogonalised basis.
    Its entries are bounded by one and its errors reach the orthonormal-basis
    density unamplified, whereas AO-basis blocks of a nearly linearly dependent
    basis are large and cancel each other."""
    s, U = np.linalg.eigh(S)
    Sh = (U * np.sqrt(np.clip(s, 0.0, None))) @ U.T
    return Sh @ D @ Sh
