"""Brute-force Coulomb integrals, independent of the Boys function and of any
integral recursion.

Uses 1/r12 = (2/sqrt(pi)) int_0^inf exp(-u^2 r12^2) du.  For fixed u the six-
dimensional integral of Gaussians times polynomials factorises into three
two-dimensional (x1, x2) integrals, each evaluated exactly by completing the
square and a tensor Gauss-Hermite rule.  The outer u integral runs through
scipy's adaptive quadrature after u = s / (1 - s).
"""
import math

import numpy as np
from scipy import integrate

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(12)


def _axis(u, A, B, C, a, b, g, i, j, k):
    """int int (x1-A)^i (x1-B)^j (x2-C)^k exp(-a(x1-A)^2 - b(x1-B)^2
    - u^2 (x1-x2)^2 - g (x2-C)^2) dx1 dx2, exactly."""
    M = np.array([[a + b + u * u, -u * u], [-u * u, g + u * u]])
    bv = np.array([a * A + b * B, g * C])
    c = a * A * A + b * B * B + g * C * C
    m = np.linalg.solve(M, bv)
    L = np.linalg.cholesky(M)
    Linv_T = np.linalg.inv(L).T
    y1, y2 = np.meshgrid(_GH_X, _GH_X, indexing="ij")
    w = np.outer(_GH_W, _GH_W)
    x1 = m[0] + Linv_T[0, 0] * y1 + Linv_T[0, 1] * y2
    x2 = m[1] + Linv_T[1, 0] * y1 + Linv_T[1, 1] * y2
    poly = (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k
    return math.exp(-(c - bv @ m)) / np.prod(np.diag(L)) * float(np.sum(w * poly))


def eri3_cart(A, a, pa, B, b, pb, C, g, pc):
    """(a b|c) over unnormalised Cartesian primitives: centres A, B, C,
    exponents a, b, g and power triples pa, pb, pc."""
    A, B, C = (np.asarray(v, float) for v in (A, B, C))

    def f(s):
        if s <= 0.0:
            u = 0.0
        elif s >= 1.0:
            return 0.0
        else:
            u = s / (1.0 - s)
        val = 2.0 / math.sqrt(math.pi)
        for ax in range(3):
            val *= _axis(u, A[ax], B[ax], C[ax], a, b, g, pa[ax], pb[ax], pc[ax])
        return val / (1.0 - s) ** 2

    pts = [0.05, 0.2, 0.5, 0.8, 0.95]
    v, err = integrate.quad(f, 0.0, 1.0, epsabs=0.0, epsrel=2e-14, limit=400, points=pts)
    return v


def overlap_cart(A, a, pa, B, b, pb):
    """int (r-A)^pa (r-B)^pb exp(-a|r-A|^2 - b|r-B|^2) d^3r by Gauss-Hermite."""
    A, B = np.asarray(A, float), np.asarray(B, float)
    p = a + b
    P = (a * A + b * B) / p
    K = math.exp(-a * b / p * float(np.sum((A - B) ** 2)))
    x, w = np.polynomial.hermite.hermgauss(16)
    out = K
    for ax in range(3):
        t = P[ax] + x / math.sqrt(p)
        out *= float(np.sum(w * (t - A[ax]) ** pa[ax] * (t - B[ax]) ** pb[ax])) / math.sqrt(p)
    return out


def kinetic_cart(A, a, pa, B, b, pb):
    """<a| -1/2 nabla^2 |b> over unnormalised Cartesian primitives, in the
    symmetric form 1/2 int grad(phi_a) . grad(phi_b) d^3r (integration by
    parts).  Each first derivative is written out, d/dx [(x-A)^i e^(-a(x-A)^2)]
    = [i (x-A)^(i-1) - 2a (x-A)^(i+1)] e^(-a(x-A)^2), and every axis integral is
    an exact Gauss-Hermite sum, so nothing is shared with a second-derivative
    recursion on one side."""
    A, B = np.asarray(A, float), np.asarray(B, float)
    p = a + b
    P = (a * A + b * B) / p
    K = math.exp(-a * b / p * float(np.sum((A - B) ** 2)))
    x, w = np.polynomial.hermite.hermgauss(16)
    s_ax, d_ax = [], []
    for ax in range(3):
        t = P[ax] + x / math.sqrt(p)
        u, v = t - A[ax], t - B[ax]
        i, j = pa[ax], pb[ax]
        fa, fb = u ** i, v ** j
        ga = (i * u ** (i - 1) if i > 0 else 0.0) - 2.0 * a * u ** (i + 1)
        gb = (j * v ** (j - 1) if j > 0 else 0.0) - 2.0 * b * v ** (j + 1)
        s_ax.append(float(np.sum(w * fa * fb)) / math.sqrt(p))
        d_ax.append(float(np.sum(w * ga * gb)) / math.sqrt(p))
    tot = (d_ax[0] * s_ax[1] * s_ax[2] + s_ax[0] * d_ax[1] * s_ax[2] + s_ax[0] * s_ax[1] * d_ax[2])
    return 0.5 * K * tot
