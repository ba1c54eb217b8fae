"""Seeded synthetic inputs: molecular geometries and even-tempered basis recipes.

This module is shared by the oracle and the GPU path *only* as an input source.
It holds no integral, fitting or SCF arithmetic: it places atoms and lists raw
Gaussian exponents and (unnormalised) contraction coefficients.  Each consumer
normalises and evaluates on its own.

Units are bohr.  A shell is a dict ``{"center": (3,), "l": int, "exps": [...],
"coefs": [...]}``; ``coefs`` multiply *normalised* primitives and the consumer
renormalises the contracted function to one.

Workloads (all seeded, all synthetic):

* ``h4``      -- H4 chain, 1.8 bohr spacing; orbital 3s1p / aux 6s3p2d per H.
* ``c40``     -- 40 C atoms uniform in a 20 bohr cube (min. separation 2.5),
                 orbital [4s3p2d1f], aux [8s6p5d3f2g]; plus a random orthonormal
                 1200x120 occupied block.
* ``alkane``  -- zigzag C30H62 (C-C 2.91, C-H 2.06 bohr, tetrahedral angles,
                 +-0.05 bohr uniform jitter); C [3s2p1d]/[7s5p4d2f], H [2s1p]/[4s3p2d].
* ``ring``    -- crown C8H16 (C-C 2.91, angle CCC 116 deg, C-H 2.06), Gaussian
                 displacements sigma 0.1 bohr; C as ``c40``, H [2s1p]/[4s3p2d].
* ``water``   -- (H2O)_n on a jittered cubic lattice (5.5 bohr), random
                 orientations; O [3s2p1d]/[8s6p4d2f], H [2s1p]/[4s3p2d].

Even-tempered exponents: orbital alpha_{l,k} = 0.15 * 3**k, auxiliary
alpha_{l,k} = 0.1 * 2.5**k, k = 0 .. n_l - 1 (the H4 chain has its own values).
"""
from __future__ import annotations

import math

import numpy as np

Z_OF = {"H": 1, "He": 2, "C": 6, "N": 7, "O": 8}

# -- basis recipes ---------------------------------------------------------

ORB_BASE, ORB_RATIO = 0.15, 3.0
AUX_BASE, AUX_RATIO = 0.1, 2.5

# number of shells per angular momentum, index = l
ORB_SHAPE = {
    "c40": {"C": [4, 3, 2, 1]},
    "alkane": {"C": [3, 2, 1], "H": [2, 1]},
    "ring": {"C": [4, 3, 2, 1], "H": [2, 1]},
    "water": {"O": [3, 2, 1], "H": [2, 1]},
}
AUX_SHAPE = {
    "c40": {"C": [8, 6, 5, 3, 2]},
    "alkane": {"C": [7, 5, 4, 2], "H": [4, 3, 2]},
    "ring": {"C": [8, 6, 5, 3, 2], "H": [4, 3, 2]},
    "water": {"O": [8, 6, 4, 2], "H": [4, 3, 2]},
}


def even_tempered(shape, base, ratio):
    """[(l, alpha), ...] for an even-tempered set; shape[l] = number of shells."""
    out = []
    for l, n in enumerate(shape):
        for k in range(n):
            out.append((l, base * ratio ** k))
    return out


def _shells_for(elems, xyz, recipe):
    shells = []
    for e, r in zip(elems, xyz):
        for l, a in recipe[e]:
            shells.append({"center": np.array(r, dtype=np.float64), "l": int(l),
                           "exps": [float(a)], "coefs": [1.0]})
    return shells


def basis_for(kind, elems, xyz):
    """Orbital and auxiliary shell lists for a named workload family."""
    if kind == "h4":
        orb = {"H": [(0, 0.1 * 3 ** k) for k in range(3)] + [(1, 0.8)]}
        aux = {"H": [(0, 0.05 * 2.5 ** k) for k in range(6)]
                    + [(1, 0.2 * 2.5 ** k) for k in range(3)]
                    + [(2, 0.5 * 2.5 ** k) for k in range(2)]}
    else:
        orb = {e: even_tempered(s, ORB_BASE, ORB_RATIO) for e, s in ORB_SHAPE[kind].items()}
        aux = {e: even_tempered(s, AUX_BASE, AUX_RATIO) for e, s in AUX_SHAPE[kind].items()}
    return _shells_for(elems, xyz, orb), _shells_for(elems, xyz, aux)


# -- geometries ------------------------------------------------------------

def h4_chain(spacing=1.8):
    xyz = np.array([[0.0, 0.0, spacing * k] for k in range(4)])
    return ["H"] * 4, xyz


def random_carbons(n=40, box=20.0, min_sep=2.5, seed=0):
    """Rejection sampling, uniform in [0, box]^3, attempts from one RNG stream."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        c = rng.uniform(0.0, box, size=3)
        if all(np.linalg.norm(c - p) >= min_sep for p in pts):
            pts.append(c)
    return ["C"] * n, np.array(pts)


def _unit(v):
    return v / np.linalg.norm(v)


def _two_h(c, n1, n2, bond, half=math.radians(109.4712206) / 2):
    """Two H on a carbon bonded to n1, n2: H-C-H bisects the open side."""
    u = -_unit(_unit(n1 - c) + _unit(n2 - c))
    w = _unit(np.cross(n1 - c, n2 - c))
    return [c + bond * (math.cos(half) * u + s * math.sin(half) * w) for s in (1.0, -1.0)]


def zigzag_alkane(ncarbon=30, cc=2.91, ch=2.06, jitter=0.05, seed=0):
    """Planar zigzag backbone in the xy plane, CH2 groups, CH3 ends."""
    th = math.radians(109.4712206)
    dx, dy = cc * math.sin(th / 2), cc * math.cos(th / 2)
    C = [np.array([k * dx, (k % 2) * dy, 0.0]) for k in range(ncarbon)]
    H = []
    for k in range(1, ncarbon - 1):
        H += _two_h(C[k], C[k - 1], C[k + 1], ch)
    for k, nb in ((0, 1), (ncarbon - 1, ncarbon - 2)):
        e = _unit(C[nb] - C[k])
        p = _unit(np.cross(np.cross(e, [0.0, 0.0, 1.0]), e))  # in-plane, perpendicular to the bond
        q = np.cross(e, p)
        for j in range(3):
            ph = 2.0 * math.pi * j / 3.0
            d = -e / 3.0 + (math.sqrt(8.0) / 3.0) * (math.cos(ph) * p + math.sin(ph) * q)
            H.append(C[k] + ch * d)
    xyz = np.array(C + H)
    rng = np.random.default_rng(seed)
    xyz = xyz + rng.uniform(-jitter, jitter, size=xyz.shape)
    return ["C"] * ncarbon + ["H"] * len(H), xyz


def crown_ring(n=8, cc=2.91, ch=2.06, angle_deg=116.0, sigma=0.1, seed=0):
    """Crown C_nH_2n: carbons alternate z = +-h on a circle, then N(0, sigma^2) noise."""
    ca = math.cos(math.radians(angle_deg))
    c1, c2 = math.cos(2 * math.pi / n), math.cos(4 * math.pi / n)
    # with R the ring radius and 2h the z offset between neighbours:
    #   |C_k - C_k+1|^2       = R^2 (2 - 2 c1) + 4 h^2 = cc^2
    #   (C_k-1 - C_k).(C_k+1 - C_k) = R^2 (c2 - 2 c1 + 1) + 4 h^2 = cc^2 cos(angle)
    R2 = cc ** 2 * (1.0 - ca) / (1.0 - c2)
    R, h = math.sqrt(R2), math.sqrt((cc ** 2 - (2 - 2 * c1) * R2) / 4.0)
    C = [np.array([R * math.cos(2 * math.pi * k / n), R * math.sin(2 * math.pi * k / n),
                   h if k % 2 == 0 else -h]) for k in range(n)]
    H = []
    for k in range(n):
        H += _two_h(C[k], C[k - 1], C[(k + 1) % n], ch)
    xyz = np.array(C + H)
    rng = np.random.default_rng(seed)
    xyz = xyz + rng.normal(0.0, sigma, size=xyz.shape)
    return ["C"] * n + ["H"] * (2 * n), xyz


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_cluster(side=4, spacing=5.5, sigma=0.1, oh=1.81, hoh_deg=104.5, seed=0):
    """side^3 waters: O on a jittered lattice, each molecule randomly oriented."""
    rng = np.random.default_rng(seed)
    half = math.radians(hoh_deg) / 2
    mono = np.array([[0.0, 0.0, 0.0],
                     [oh * math.sin(half), 0.0, oh * math.cos(half)],
                     [-oh * math.sin(half), 0.0, oh * math.cos(half)]])
    elems, xyz = [], []
    for i in range(side):
        for j in range(side):
            for k in range(side):
                o = spacing * np.array([i, j, k], dtype=float) + rng.normal(0.0, sigma, 3)
                Rm = _random_rotation(rng)
                for e, r in zip("OHH", mono):
                    elems.append(e)
                    xyz.append(o + Rm @ r)
    return elems, np.array(xyz)


def trajectory(xyz, nframes, step_sigma=0.02, seed=1):
    """Frames f+1 = f + N(0, step_sigma^2) per coordinate."""
    rng = np.random.default_rng(seed)
    frames = [np.array(xyz, dtype=float)]
    for _ in range(nframes - 1):
        frames.append(frames[-1] + rng.normal(0.0, step_sigma, size=xyz.shape))
    return frames


def random_orthonormal(n, k, seed=1):
    """QR of an N(0,1) n x k matrix with sign fix diag(R) > 0 (Euclidean orthonormal)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(n, k)))
    return q * np.sign(np.diag(r))[None, :]


# Benzene of the paper's sample input (Fig. 1), coordinates in bohr.
BENZENE_FIG1 = (["C"] * 6 + ["H"] * 6, np.array([
    [-0.07, 2.54, 0.00], [2.55, 2.54, 0.00], [3.87, 4.82, 0.00],
    [2.55, 7.10, 0.00], [-0.07, 7.10, 0.00], [-1.39, 4.82, 0.00],
    [-1.11, 0.74, 0.00], [3.59, 0.74, 0.00], [5.95, 4.82, 0.00],
    [3.59, 8.90, 0.00], [-1.11, 8.90, 0.00], [-3.47, 4.82, 0.00]]))


def workload(name, seed=None):
    """Return (elems, xyz, shells, aux) for a named workload."""
    if name == "h4":
        elems, xyz = h4_chain()
        kind = "h4"
    elif name == "c40":
        elems, xyz = random_carbons(seed=0 if seed is None else seed)
        kind = "c40"
    elif name == "alkane":
        elems, xyz = zigzag_alkane(seed=0 if seed is None else seed)
        kind = "alkane"
    elif name == "ring":
        elems, xyz = crown_ring(seed=0 if seed is None else seed)
        kind = "ring"
    elif name.startswith("water"):
        side = int(name[5:] or 4)
        elems, xyz = water_cluster(side=side, seed=0 if seed is None else seed)
        kind = "water"
    else:
        raise ValueError(f"unknown workload {name!r}")
    shells, aux = basis_for(kind, elems, xyz)
    return elems, xyz, shells, aux


def charges(elems):
    return np.array([Z_OF[e] for e in elems], dtype=np.int32)


def nocc_of(elems, charge=0):
    ne = int(sum(Z_OF[e] for e in elems)) - charge
    if ne % 2:
        raise ValueError("closed-shell reference needs an even electron count")
    return ne // 2


def shells_at(shells, xyz_old, xyz_new):
    """Move every shell with its atom (used for trajectories and invariance tests)."""
    out = []
    for s in shells:
        d = np.linalg.norm(xyz_old - s["center"][None, :], axis=1)
        a = int(np.argmin(d))
        out.append(dict(s, center=np.array(xyz_new[a], dtype=np.float64) + (s["center"] - xyz_old[a])))
    return out
