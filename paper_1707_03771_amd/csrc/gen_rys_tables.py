"""Generate the Rys quadrature root/weight tables used by the integral kernels.

    python paper_1707_03771_amd/csrc/gen_rys_tables.py [--check]

The Rys quadrature (Dupuis, Rys & King, J. Chem. Phys. 65, 111 (1976); the
paper's section "Molecular integrals" names it as its ERI algorithm) replaces
the Boys-function sum of an integral over Gaussians with total angular momentum
L by an n-point Gauss rule, n = floor(L/2) + 1, for the weight exp(-T t^2) on
t in [0, 1] and polynomials in u = t^2:

    int_0^1 u^m exp(-T u) dt = sum_i w_i(T) u_i(T)^m,   m = 0 .. 2n-1.

Ground truth: at 60 significant digits (mpmath) the moments F_m(T) build a
Hankel matrix whose Cholesky factor gives the three-term recurrence of the
orthogonal polynomials; the Jacobi matrix's eigen-decomposition (Golub-Welsch)
gives u_i and w_i.

Table: on [0, T_max(n)) the functions u_i(T), w_i(T) are interpolated on
intervals of width H by degree-DEG polynomials (Chebyshev nodes, converted
exactly to monomials in the local variable x in [-1, 1]; coefficients stored
highest power first for Horner's rule).  Above T_max(n) the large-T limit
u_i = x_i^2 / T, w_i = W_i / sqrt(T) holds to double precision, with x_i > 0
the roots of the Hermite polynomial H_2n and W_i its Gauss weights.

Output: ``rys_tables.inc`` beside this script (committed; regenerate after any
change here).  ``--check`` re-validates the written tables against fresh
ground truth at random T and the moment identity.
"""
import argparse
import os
import sys

import mpmath as mp
import numpy as np

NMAX = 7          # up to (ff|ff) Schwarz diagonals and (ff|g) three-index classes
H_OF = {1: 1.0, 2: 4.0, 3: 4.0, 4: 4.0, 5: 4.0, 6: 4.0, 7: 4.0}   # interval width per root count
H = 4.0           # step of the large-T threshold search
DEG = 16
TOL_ASYM = 2e-15
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "rys_tables.inc")

mp.mp.dps = 60


def boys_mp(m, T):
    T = mp.mpf(T)
    if T == 0:
        return mp.mpf(1) / (2 * m + 1)
    return mp.gammainc(m + mp.mpf(1) / 2, 0, T) / (2 * T ** (m + mp.mpf(1) / 2))


def rys_mp(n, T):
    """Roots u_i (ascending) and weights w_i, as mpf."""
    mom = [boys_mp(k, T) for k in range(2 * n + 1)]
    Hk = mp.matrix(n + 1, n + 1)
    for i in range(n + 1):
        for j in range(n + 1):
            Hk[i, j] = mom[i + j]
    R = mp.cholesky(Hk).T       # upper triangular, Hk = R^T R
    J = mp.matrix(n, n)
    for k in range(n):
        J[k, k] = R[k, k + 1] / R[k, k] - (R[k - 1, k] / R[k - 1, k - 1] if k > 0 else 0)
        if k < n - 1:
            J[k, k + 1] = J[k + 1, k] = R[k + 1, k + 1] / R[k, k]
    E, Q = mp.eigsy(J)
    pairs = sorted((E[i], mom[0] * Q[0, i] ** 2) for i in range(n))
    return [p[0] for p in pairs], [p[1] for p in pairs]


def hermite_asym(n):
    """Positive roots x_i of H_2n (squared, ascending) and their Gauss-Hermite
    weights, by Golub-Welsch on the Hermite Jacobi matrix (beta_k = k/2) at
    60 digits."""
    m = 2 * n
    J = mp.matrix(m, m)
    for k in range(1, m):
        J[k - 1, k] = J[k, k - 1] = mp.sqrt(mp.mpf(k) / 2)
    E, Q = mp.eigsy(J)
    pts = sorted((E[i] ** 2, mp.sqrt(mp.pi) * Q[0, i] ** 2) for i in range(m) if E[i] > 0)
    return np.array([float(p[0]) for p in pts]), np.array([float(p[1]) for p in pts])


def asym_error(n, T):
    r, w = rys_mp(n, T)
    x2, W = hermite_asym(n)
    er = max(abs(float(r[i]) - x2[i] / T) / float(r[i]) for i in range(n))
    ew = max(abs(float(w[i]) - W[i] / np.sqrt(T)) / float(w[i]) for i in range(n))
    return max(er, ew)


def tmax_for(n):
    """Smallest multiple of H from which the large-T form is within TOL_ASYM."""
    T = H * np.ceil(30.0 / H)
    while T < 400.0:
        if all(asym_error(n, T + d) <= TOL_ASYM for d in (0.0, 0.5 * H, 2.0 * H, 6.0 * H)):
            return T
        T += H
    raise RuntimeError(f"large-T limit never reached {TOL_ASYM} for n={n}")


def fit_interval(n, a, h):
    """Monomial coefficients (highest first) in x = (T - c) / (H/2), c = a + H/2,
    for the 2n functions [u_1..u_n, w_1..w_n], from interpolation at DEG+1
    Chebyshev nodes, all in 60-digit arithmetic."""
    m = DEG + 1
    xs = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / m) for k in range(m)]
    c = mp.mpf(a) + mp.mpf(h) / 2
    vals = [rys_mp(n, c + mp.mpf(h) / 2 * x) for x in xs]
    out = []
    for f in range(2 * n):
        y = [vals[k][0][f] if f < n else vals[k][1][f - n] for k in range(m)]
        # Chebyshev coefficients by the discrete cosine sum
        cc = []
        for j in range(m):
            s = mp.fsum(y[k] * mp.cos(mp.pi * j * (k + mp.mpf(1) / 2) / m) for k in range(m))
            cc.append(s * 2 / m)
        cc[0] /= 2
        # T_j(x) -> monomials
        mono = [mp.mpf(0)] * m
        Tprev, Tcur = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
        for j in range(m):
            if j == 0:
                Tj = Tprev
            elif j == 1:
                Tj = Tcur
            else:
                Tn = [mp.mpf(0)] * (j + 1)
                for i, v in enumerate(Tcur):
                    Tn[i + 1] += 2 * v
                for i, v in enumerate(Tprev):
                    Tn[i] -= v
                Tprev, Tcur = Tcur, Tn
                Tj = Tn
            for i, v in enumerate(Tj):
                mono[i] += cc[j] * v
        out.append([float(v) for v in reversed(mono)])
    return out


def horner(cs, x):
    r = 0.0
    for c in cs:
        r = r * x + c
    return r


def evaluate(tab, n, T):
    """Double-precision evaluation exactly as the kernels do it."""
    if T >= tab["tmax"][n]:
        x2, W = tab["x2"][n], tab["W"][n]
        return [x / T for x in x2], [w / np.sqrt(T) for w in W]
    h = tab["h"][n]
    k = int(T / h)
    x = (T - (k * h + h / 2)) / (h / 2)
    blk = tab["coef"][n][k]
    return [horner(blk[f], x) for f in range(n)], [horner(blk[n + f], x) for f in range(n)]


def generate():
    tab = {"tmax": {}, "coef": {}, "x2": {}, "W": {}, "h": dict(H_OF)}
    for n in range(1, NMAX + 1):
        tm = tmax_for(n)
        nint = int(round(tm / H_OF[n]))
        tab["tmax"][n] = tm
        tab["coef"][n] = [fit_interval(n, k * H_OF[n], H_OF[n]) for k in range(nint)]
        x2, W = hermite_asym(n)
        tab["x2"][n], tab["W"][n] = list(x2), list(W)
        print(f"n={n}: T_max={tm:g}, {nint} intervals", file=sys.stderr)
    return tab


def write(tab):
    L = ["/* Rys quadrature tables -- GENERATED by gen_rys_tables.py, do not edit.",
         f" * Interval width RYS_HN[n], Horner degree {DEG} in x = (T - centre)/(h/2);",
         " * layout per root count n: [interval][2n functions: u_1..u_n, w_1..w_n][DEG+1],",
         " * highest power first.  T >= RYS_TMAX[n]: u_i = RYS_X2[n][i]/T, w_i = RYS_W[n][i]/sqrt(T). */",
         f"#define RYS_NMAX {NMAX}", f"#define RYS_DEG {DEG}", ""]
    L.append("static constexpr double RYS_HN[RYS_NMAX + 1] = {0.0, " +
             ", ".join(repr(float(H_OF[n])) for n in range(1, NMAX + 1)) + "};")
    L.append("static constexpr int RYS_NINT[RYS_NMAX + 1] = {0, " +
             ", ".join(str(len(tab["coef"][n])) for n in range(1, NMAX + 1)) + "};")
    L.append("static constexpr double RYS_TMAX[RYS_NMAX + 1] = {0.0, " +
             ", ".join(repr(float(tab["tmax"][n])) for n in range(1, NMAX + 1)) + "};")
    L.append("static constexpr int RYS_OFF[RYS_NMAX + 1] = {0, " + ", ".join(
        str(sum(len(tab["coef"][m]) * 2 * m * (DEG + 1) for m in range(1, n))) for n in range(1, NMAX + 1)) + "};")
    L.append("static constexpr double RYS_X2[RYS_NMAX + 1][RYS_NMAX] = {{0}, " + ", ".join(
        "{" + ", ".join(repr(float(v)) for v in tab["x2"][n]) + "}" for n in range(1, NMAX + 1)) + "};")
    L.append("static constexpr double RYS_W[RYS_NMAX + 1][RYS_NMAX] = {{0}, " + ", ".join(
        "{" + ", ".join(repr(float(v)) for v in tab["W"][n]) + "}" for n in range(1, NMAX + 1)) + "};")
    flat = []
    for n in range(1, NMAX + 1):
        for blk in tab["coef"][n]:
            for f in blk:
                flat.extend(f)
    L.append(f"#define RYS_TABLE_SIZE {len(flat)}")
    L.append("/* initializer list for the coefficient table (one translation unit defines it) */")
    L.append("#define RYS_TABLE_INIT { \\")
    for i in range(0, len(flat), 4):
        L.append("  " + ", ".join(repr(float(v)) for v in flat[i:i + 4]) + ", \\")
    L.append("}")
    with open(OUT, "w") as f:
        f.write("\n".join(L) + "\n")


def read():
    """Parse the written .inc back (for --check)."""
    txt = open(OUT).read()

    def arr(name):
        s = txt[txt.index("static constexpr"):]
        s = s[s.index(name):]
        s = s[s.index("=") + 1:s.index(";")]
        return s

    nint = [int(v) for v in arr("RYS_NINT[").strip(" {}").split(",")]
    tmax = [float(v) for v in arr("RYS_TMAX[").strip(" {}").split(",")]

    def nested(name):
        s = arr(name).strip()[1:-1]
        rows = [r.strip(" {},") for r in s.split("}")]
        return [[float(v) for v in r.split(",") if v.strip()] for r in rows if r != ""]

    x2 = nested("RYS_X2[")
    W = nested("RYS_W[")
    body = txt[txt.index("#define RYS_TABLE_INIT"):]
    body = body[body.index("{") + 1:body.rindex("}")].replace("\\", " ").replace("\n", " ")
    flat = [float(v) for v in body.split(",") if v.strip()]
    hn = [float(v) for v in arr("RYS_HN[").strip(" {}").split(",")]
    tab = {"tmax": {}, "coef": {}, "x2": {}, "W": {}, "h": {n: hn[n] for n in range(1, NMAX + 1)}}
    pos = 0
    for n in range(1, NMAX + 1):
        tab["tmax"][n] = tmax[n]
        tab["x2"][n], tab["W"][n] = x2[n - 1 + (1 if len(x2) > NMAX else 0)], W[n - 1 + (1 if len(W) > NMAX else 0)]
        blocks = []
        for _ in range(nint[n]):
            blk = []
            for _ in range(2 * n):
                blk.append(flat[pos:pos + DEG + 1])
                pos += DEG + 1
            blocks.append(blk)
        tab["coef"][n] = blocks
    return tab


def check(tab, npts=40, seed=0):
    rng = np.random.default_rng(seed)
    worst = 0.0
    for n in range(1, NMAX + 1):
        Ts = np.concatenate([[0.0, 1e-9, tab["h"][n], tab["tmax"][n] - 1e-9, tab["tmax"][n]],
                             rng.uniform(0, tab["tmax"][n] * 1.3, npts)])
        for T in Ts:
            r, w = rys_mp(n, float(T))
            u, wt = evaluate(tab, n, float(T))
            for i in range(n):
                worst = max(worst, abs(u[i] - float(r[i])) / float(r[i]),
                            abs(wt[i] - float(w[i])) / float(w[i]))
            # moment identity sum_i w_i u_i^m = F_m(T), m < 2n
            for m in range(2 * n):
                s = sum(wt[i] * u[i] ** m for i in range(n))
                f = float(boys_mp(m, float(T)))
                worst = max(worst, abs(s - f) / f)
    return worst


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--check", action="store_true")
    a = ap.parse_args()
    if not a.check:
        write(generate())
    err = check(read())
    print(f"max relative error (roots, weights, moments): {err:.3e}")
    if err > 2e-14:
        sys.exit(1)
