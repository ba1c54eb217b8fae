"""Pins for the CPU oracle: each test checks it against something other than
itself -- printed textbook values, closed forms, brute-force quadrature,
invariances and identities -- so that a dropped term, wrong sign or index, or a
transposed operand fails at least one of them."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import bruteforce as bf
import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _shell(ctr, l, exps, coefs=None):
    return {"center": np.asarray(ctr, float), "l": l, "exps": list(exps),
            "coefs": list(coefs) if coefs is not None else [1.0] * len(exps)}


# --------------------------------------------------------------------- Boys

def _boys_mp(m, T):
    mpmath.mp.dps = 40
    if T == 0:
        return mpmath.mpf(1) / (2 * m + 1)
    return mpmath.gammainc(m + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (m + 0.5))


@pytest.mark.parametrize("T", [0.0, 1e-13, 1e-7, 0.3, 2.0, 9.7, 29.9, 30.1, 49.99, 50.0, 75.0, 140.0, 1e4])
def test_boys_against_incomplete_gamma(T):
    F = O.boys(16, T)
    for m in range(17):
        ref = float(_boys_mp(m, T))
        assert abs(F[m] - ref) <= 2e-15 * ref, (m, T)


def test_boys_f0_is_erf():
    for T in (0.01, 1.0, 7.0, 33.0):
        assert O.boys(0, T)[0] == pytest.approx(0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T)),
                                                rel=1e-15)


# ------------------------------------------------------- solid harmonics

def _sphere_monomial(px, py, pz):
    if px % 2 or py % 2 or pz % 2:
        return 0.0
    g = lambda k: math.gamma((k + 1) / 2)  # noqa: E731
    return 2.0 * g(px) * g(py) * g(pz) / math.gamma((px + py + pz + 3) / 2)


@pytest.mark.parametrize("l", range(7))
def test_solid_harmonics_orthonormal_and_harmonic(l):
    T = O.solid_harmonics(l)
    pw = O.cart_powers(l)
    G = np.array([[_sphere_monomial(*np.add(p, q)) for q in pw] for p in pw])
    assert np.abs(T @ G @ T.T - np.eye(2 * l + 1)).max() < 5e-15
    # each row is a harmonic polynomial: its Laplacian vanishes
    for row in T:
        lap = {}
        for c, (i, j, k) in zip(row, pw):
            for ax, e in enumerate((i, j, k)):
                if e >= 2:
                    q = [i, j, k]
                    q[ax] -= 2
                    lap[tuple(q)] = lap.get(tuple(q), 0.0) + c * e * (e - 1)
        assert max([abs(v) for v in lap.values()] + [0.0]) < 1e-12


def test_solid_harmonics_convention():
    # m = -l..l; m>0 ~ cos(m phi), m<0 ~ sin(|m| phi); positive leading coefficients
    rng = np.random.default_rng(3)
    for l in range(1, 5):
        T = O.solid_harmonics(l)
        pw = np.array(O.cart_powers(l))
        for _ in range(5):
            th, ph = rng.uniform(0.1, 3.0), rng.uniform(0, 2 * math.pi)
            r = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
            vals = T @ np.prod(r[None, :] ** pw, axis=1)
            for m in range(-l, l + 1):
                am = abs(m)
                Plm = float(mpmath.legenp(l, am, math.cos(th))) * (-1) ** am  # drop Condon-Shortley
                norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
                ang = (math.cos(m * ph) if m >= 0 else math.sin(am * ph)) * (math.sqrt(2) if m else 1.0)
                assert vals[m + l] == pytest.approx(norm * Plm * ang, rel=1e-11, abs=1e-13)


# ---------------------------------------------------------- one-electron

@pytest.mark.parametrize("l", range(5))
def test_overlap_within_shell_is_identity(l):
    bas = O.Basis([_shell([0.3, -0.1, 0.2], l, [0.4, 1.7, 6.0], [0.3, 0.5, 0.4])])
    S, T, V = O.int1e(bas, np.zeros((1, 3)), [1])
    assert np.abs(S - np.eye(2 * l + 1)).max() < 2e-14


def test_overlap_against_gauss_hermite():
    A, B = np.array([0.1, 0.2, -0.3]), np.array([-0.5, 0.9, 0.4])
    bas = O.Basis([_shell(A, 2, [0.7]), _shell(B, 3, [1.9])])
    S, _, _ = O.int1e(bas, np.zeros((1, 3)), [0])
    ca, cb = bas.coef[0], bas.coef[1]
    pa, pb = O.cart_powers(2), O.cart_powers(3)
    cart = np.array([[bf.overlap_cart(A, 0.7, p, B, 1.9, q) for q in pb] for p in pa]) * ca * cb
    ref = O.solid_harmonics(2) @ cart @ O.solid_harmonics(3).T
    assert np.abs(S[:5, 5:] - ref).max() < 1e-14


@pytest.mark.parametrize("la,lb", [(0, 2), (2, 2), (1, 3), (3, 2), (3, 3)])
def test_kinetic_against_gauss_hermite(la, lb):
    """d and f shells on both sides: the ket's j (j - 1) S(i, j - 2) term of
    the kinetic recursion only appears for Cartesian powers j >= 2."""
    A, B = np.array([0.2, -0.4, 0.1]), np.array([-0.3, 0.5, 0.6])
    a, b = 0.9, 1.4
    bas = O.Basis([_shell(A, la, [a]), _shell(B, lb, [b])])
    _, T, _ = O.int1e(bas, np.zeros((1, 3)), [0])
    na = 2 * la + 1
    ca, cb = bas.coef[0], bas.coef[1]
    pa, pb = O.cart_powers(la), O.cart_powers(lb)
    cart = np.array([[bf.kinetic_cart(A, a, p, B, b, q) for q in pb] for p in pa]) * ca * cb
    ref = O.solid_harmonics(la) @ cart @ O.solid_harmonics(lb).T
    assert np.abs(T[:na, na:] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    # the diagonal block of one shell: <phi| T |phi> against the same quadrature
    cart_aa = np.array([[bf.kinetic_cart(A, a, p, A, a, q) for q in pa] for p in pa]) * ca * ca
    ref_aa = O.solid_harmonics(la) @ cart_aa @ O.solid_harmonics(la).T
    assert np.abs(T[:na, :na] - ref_aa).max() < 1e-13 * max(1.0, np.abs(ref_aa).max())


def test_kinetic_pin_catches_a_dropped_term():
    """The quadrature is sensitive to the term a dropped j (j - 1) S(i, j - 2)
    would lose: for x^2 e^(-b x^2) against itself that term is 2 S(2, 0), which
    is not small next to the total."""
    A = np.zeros(3)
    full = bf.kinetic_cart(A, 1.1, (2, 0, 0), A, 1.1, (2, 0, 0))
    dropped = full - (-0.5) * 2 * bf.overlap_cart(A, 1.1, (2, 0, 0), A, 1.1, (0, 0, 0))
    assert abs(full - dropped) > 1e-2 * abs(full)


def test_h2_sto3g_textbook():
    g = json.load(open(os.path.join(GOLD, "h2_sto3g.json")))
    xyz = np.array([[0, 0, 0], [0, 0, g["R_bohr"]]], float)
    sh = [_shell(xyz[i], 0, g["exps"], g["coefs"]) for i in range(2)]
    bas = O.Basis(sh)
    S, T, V = O.int1e(bas, xyz, [1, 1])
    G = O.eri4(bas)
    tol = g["tol"]
    assert abs(S[0, 1] - g["S12"]) < tol and abs(T[0, 0] - g["T11"]) < tol and abs(T[0, 1] - g["T12"]) < tol
    assert abs(V[0, 0] - g["V11_total"]) < tol
    assert abs(G[0, 0, 0, 0] - g["eri_1111"]) < tol and abs(G[0, 0, 1, 1] - g["eri_1122"]) < tol
    assert abs(G[1, 0, 1, 0] - g["eri_2121"]) < tol and abs(G[1, 0, 0, 0] - g["eri_2111"]) < tol
    jkf = lambda D, C: (np.einsum("mnls,ls->mn", G, D), np.einsum("mlns,ls->mn", G, D))  # noqa: E731
    r = O.rhf(S, T + V, 1.0 / g["R_bohr"], 1, jkf)
    assert r.converged and abs(r.E - g["E_total"]) < tol
    assert np.allclose(r.eps, g["eps"], atol=tol)


def test_he_one_gaussian_closed_form_through_df():
    g = json.load(open(os.path.join(GOLD, "he_one_gaussian.json")))
    a = ((8 * math.sqrt(2) - 2) / (6 * math.sqrt(math.pi))) ** 2
    assert a == pytest.approx(g["alpha_star_value"], rel=1e-10)
    # DF with the single product aux function (exponent 2a) is exact here
    res, df = O.df_rhf([2], np.zeros((1, 3)), [_shell([0, 0, 0], 0, [a])],
                       [_shell([0, 0, 0], 0, [2 * a])], nocc=1)
    assert abs(res.E - g["E_star"]) < g["tol"]
    bas = O.Basis([_shell([0, 0, 0], 0, [a])])
    S, T, V = O.int1e(bas, np.zeros((1, 3)), [2])
    assert abs(2 * T[0, 0] - g["T_star"]) < g["tol"]


def test_nuclear_attraction_s_closed_form():
    A, C = np.array([0.2, -0.1, 0.5]), np.array([1.1, 0.4, -0.3])
    a = 0.9
    bas = O.Basis([_shell(A, 0, [a])])
    _, _, V = O.int1e(bas, C[None, :], [3])
    p = 2 * a
    T = p * np.sum((A - C) ** 2)
    F0 = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    ref = -3 * (2 * a / math.pi) ** 1.5 * 2 * math.pi / p * F0
    assert V[0, 0] == pytest.approx(ref, rel=1e-14)


# ---------------------------------------------------------- two-electron

def test_ss_s_closed_form():
    A, B, C = np.array([0.1, -0.2, 0.3]), np.array([1.0, 0.5, -0.4]), np.array([-0.7, 1.1, 0.9])
    a, b, g = 0.8, 1.3, 0.6
    bas = O.Basis([_shell(A, 0, [a]), _shell(B, 0, [b])])
    aux = O.Basis([_shell(C, 0, [g])])
    v = O.eri3_block(bas, 1, 0, aux, 0)[0, 0, 0]
    p = a + b
    P = (a * A + b * B) / p
    T = p * g / (p + g) * np.sum((P - C) ** 2)
    F0 = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    N = lambda x: (2 * x / math.pi) ** 0.75  # noqa: E731
    ref = N(a) * N(b) * N(g) * 2 * math.pi ** 2.5 / (p * g * math.sqrt(p + g)) \
        * math.exp(-a * b / p * np.sum((A - B) ** 2)) * F0
    assert v == pytest.approx(ref, rel=1e-14)
    # two-centre (s|s)
    J = O.eri2(O.Basis([_shell(A, 0, [a]), _shell(C, 0, [g])]))
    T2 = a * g / (a + g) * np.sum((A - C) ** 2)
    F0 = 0.5 * math.sqrt(math.pi / T2) * math.erf(math.sqrt(T2))
    ref2 = N(a) * N(g) * 2 * math.pi ** 2.5 / (a * g * math.sqrt(a + g)) * F0
    assert J[0, 1] == pytest.approx(ref2, rel=1e-14)


@pytest.mark.parametrize("la,lb,lc", [(1, 0, 0), (0, 1, 2), (1, 1, 1), (2, 1, 0), (2, 0, 2), (1, 2, 3)])
def test_eri3_against_brute_force(la, lb, lc):
    A, B, C = np.array([0.1, -0.2, 0.3]), np.array([0.9, 0.5, -0.4]), np.array([-0.6, 0.8, 0.7])
    a, b, g = 0.8, 1.3, 0.6
    bas = O.Basis([_shell(A, la, [a]), _shell(B, lb, [b])])
    aux = O.Basis([_shell(C, lc, [g])])
    blk = O.eri3_block(bas, 0, 1, aux, 0)
    pa, pb, pc = O.cart_powers(la), O.cart_powers(lb), O.cart_powers(lc)
    cart = np.zeros((len(pa), len(pb), len(pc)))
    for i, p in enumerate(pa):
        for j, q in enumerate(pb):
            for k, r in enumerate(pc):
                cart[i, j, k] = bf.eri3_cart(A, a, p, B, b, q, C, g, r)
    cart *= bas.coef[0] * bas.coef[1] * aux.coef[0]
    ref = np.einsum("ai,bj,ck,ijk->abc", O.solid_harmonics(la), O.solid_harmonics(lb),
                    O.solid_harmonics(lc), cart)
    assert np.abs(blk - ref).max() <= 1e-12 * np.abs(ref).max()


def test_eri3_contracted_is_sum_of_primitives():
    A, B, C = np.array([0.0, 0.0, 0.0]), np.array([0.0, 1.2, 0.3]), np.array([0.7, 0.0, -0.5])
    e, c = [0.5, 2.0], [0.6, 0.5]
    sh = [_shell(A, 1, e, c), _shell(B, 2, [0.9])]
    bas = O.Basis(sh)
    aux = O.Basis([_shell(C, 1, [1.1])])
    tot = O.eri3_block(bas, 0, 1, aux, 0)
    parts = []
    for k in range(2):
        b1 = O.Basis([_shell(A, 1, [e[k]]), _shell(B, 2, [0.9])])
        parts.append(O.eri3_block(b1, 0, 1, aux, 0))
    # contracted = sum_k c_k N_k phi_k / norm; primitives normalised individually
    w = np.array(c)
    s = (2 * math.sqrt(e[0] * e[1]) / (e[0] + e[1])) ** 2.5
    nrm = math.sqrt(w[0] ** 2 + w[1] ** 2 + 2 * w[0] * w[1] * s)
    assert np.abs(tot - (w[0] * parts[0] + w[1] * parts[1]) / nrm).max() < 1e-14


def test_eri_permutational_symmetry():
    rng = np.random.default_rng(7)
    sh = [_shell(rng.normal(size=3), l, [rng.uniform(0.3, 2.0)]) for l in (0, 1, 2, 1)]
    bas = O.Basis(sh)
    G = O.eri4(bas)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0), (2, 3, 1, 0)]:
        assert np.abs(G - G.transpose(perm)).max() < 1e-14 * np.abs(G).max()
    aux = O.Basis([_shell(rng.normal(size=3), 2, [0.8])])
    b01 = O.eri3_block(bas, 0, 2, aux, 0)
    b10 = O.eri3_block(bas, 2, 0, aux, 0)
    # the two orders take the product centre from different first centres: equal
    # to rounding (a transposed operand would differ at O(1))
    assert np.abs(b01 - b10.transpose(1, 0, 2)).max() < 1e-14 * np.abs(b01).max() + 1e-18
    J = O.eri2(O.Basis([_shell(rng.normal(size=3), l, [rng.uniform(0.3, 2)]) for l in (0, 2, 4, 3)]))
    assert np.abs(J - J.T).max() == 0.0
    assert np.linalg.eigvalsh(J).min() > 0


def test_schwarz_inequality_and_factors():
    elems, xyz, shells, aux_sh = W.workload("h4")
    bas, aux = O.Basis(shells), O.Basis(aux_sh)
    Qab, QC = O.schwarz(bas, aux)
    for a in range(bas.nsh):
        for b in range(a + 1):
            for c in range(0, aux.nsh, 5):
                blk = O.eri3_block(bas, a, b, aux, c)
                assert np.abs(blk).max() <= Qab[a, b] * QC[c] * (1 + 1e-12)
    # Q_ab is the largest diagonal (mu nu|mu nu)
    G = O.eri4(bas)
    d = np.einsum("mnmn->mn", G)
    for a in range(bas.nsh):
        for b in range(bas.nsh):
            sa = slice(bas.foff[a], bas.foff[a] + bas.size[a])
            sb = slice(bas.foff[b], bas.foff[b] + bas.size[b])
            assert Qab[a, b] == pytest.approx(math.sqrt(d[sa, sb].max()), rel=1e-14)


# ----------------------------------------------------------- screening

def test_screen_rule_and_offsets():
    rng = np.random.default_rng(11)
    shells = [_shell(rng.normal(size=3), int(l), [1.0]) for l in rng.integers(0, 4, size=9)]
    auxs = [_shell(rng.normal(size=3), int(l), [1.0]) for l in rng.integers(0, 5, size=6)]
    bas, aux = O.Basis(shells), O.Basis(auxs)
    Qab = np.exp(rng.uniform(-40, 0, size=(9, 9)))
    Qab = (Qab + Qab.T) / 2
    QC = np.exp(rng.uniform(-10, 0, size=6))
    tau = 1e-9
    scr = O.screen(bas, aux, Qab, QC, tau)
    exp_pairs = [(a, b) for a in range(9) for b in range(a + 1) if Qab[a, b] * QC.max() >= tau]
    assert [tuple(p) for p in scr.pairs] == exp_pairs
    off = 0
    for k, (a, b) in enumerate(exp_pairs):
        assert scr.col_off[k] == off
        off += (2 * bas.l[a] + 1) * (2 * bas.l[b] + 1)
        for c in range(6):
            assert scr.keep[k, c] == (Qab[a, b] * QC[c] >= tau)
    assert scr.col_off[-1] == off and scr.col_off.dtype == np.int64


# ---------------------------------------------------- density fitting

def test_df_exact_with_product_aux_basis():
    """With every primitive product as aux function, DF reproduces (mu nu|la si)."""
    g = json.load(open(os.path.join(GOLD, "h2_sto3g.json")))
    xyz = np.array([[0, 0, 0], [0, 0, 1.4]])
    prims = [(xyz[i], e) for i in range(2) for e in g["exps"]]
    aux = []
    for i in range(len(prims)):
        for j in range(i + 1):
            (A, a), (B, b) = prims[i], prims[j]
            aux.append(_shell((a * A + b * B) / (a + b), 0, [a + b]))
    sh = [_shell(xyz[i], 0, g["exps"], g["coefs"]) for i in range(2)]
    bas, ab = O.Basis(sh), O.Basis(aux)
    Qab, QC = O.schwarz(bas, ab)
    scr = O.screen(bas, ab, Qab, QC, 0.0)
    raw = O.eri3_packed(bas, ab, scr)
    L, B = O.fit(raw, O.eri2(ab))
    df = O.DF(bas, ab, scr, B, L)
    Bd = df.dense_rows(0, ab.nbf)
    G_df = np.einsum("qmn,qls->mnls", Bd, Bd)
    assert np.abs(G_df - O.eri4(bas)).max() < 1e-9


def test_df_coulomb_energy_lower_bound_and_k_psd():
    elems, xyz, shells, aux_sh = W.workload("h4")
    df = O.build_df(O.Basis(shells), O.Basis(aux_sh))
    G = O.eri4(df.bas)
    rng = np.random.default_rng(2)
    C = np.linalg.qr(rng.normal(size=(df.bas.nbf, 2)))[0]
    D = C @ C.T
    J, K = O.jk(df, D=D, C=C)
    Jx = np.einsum("mnls,ls->mn", G, D)
    assert np.sum(D * J) <= np.sum(D * Jx) + 1e-12
    assert np.sum(D * J) > 0.99 * np.sum(D * Jx)   # a decent fit
    w = np.linalg.eigvalsh(K)
    assert w.min() >= -1e-12 * np.abs(w).max()
    # the density route gives the same K
    _, K2 = O.jk(df, D=D)
    assert np.abs(K - K2).max() < 1e-13


def test_jk_matches_four_index_with_fitted_integrals():
    """Cross-check Eqs. (3a,3b) and (1a,2a) against the rebuilt 4-index tensor (Eq. 2b)."""
    elems, xyz, shells, aux_sh = W.workload("h4")
    df = O.build_df(O.Basis(shells), O.Basis(aux_sh))
    Bd = df.dense_rows(0, df.aux.nbf)
    G = np.einsum("qmn,qls->mnls", Bd, Bd)
    rng = np.random.default_rng(5)
    C = rng.normal(size=(df.bas.nbf, 3))
    D = C @ C.T
    J, K = O.jk(df, D=D, C=C)
    assert np.abs(J - np.einsum("mnls,ls->mn", G, D)).max() < 1e-12
    assert np.abs(K - np.einsum("mlns,ls->mn", G, D)).max() < 1e-12


# ------------------------------------------------------------------ SCF

def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_h4_scf_converged_state_invariants():
    elems, xyz, shells, aux_sh = W.workload("h4")
    Z = W.charges(elems)
    res, df = O.df_rhf(Z, xyz, shells, aux_sh, nocc=2)
    assert res.converged
    bas = df.bas
    S, _, _ = O.int1e(bas, xyz, Z)
    D = res.D
    assert np.abs(D @ S @ D - D).max() < 1e-10
    assert abs(np.trace(D @ S) - 2) < 1e-10
    # restarting from the converged orbitals is a fixed point
    res2, _ = O.df_rhf(Z, xyz, shells, aux_sh, nocc=2, C_init=res.C)
    assert abs(res2.E - res.E) < 1e-10 and res2.niter <= 3


def test_energy_rotation_translation_invariance():
    elems, xyz, shells, aux_sh = W.workload("h4")
    Z = W.charges(elems)
    e0 = O.df_rhf(Z, xyz, shells, aux_sh, nocc=2)[0].E
    rng = np.random.default_rng(9)
    R = _rotation(rng)
    t = rng.normal(size=3)
    new = xyz @ R.T + t
    e1 = O.df_rhf(Z, new, W.shells_at(shells, xyz, new), W.shells_at(aux_sh, xyz, new), nocc=2)[0].E
    assert abs(e1 - e0) < 1e-10


def test_benzene_fig1_rotation_invariance():
    """Planar benzene of the paper's Fig. 1 (bohr), a small even-tempered basis."""
    elems, xyz = W.BENZENE_FIG1
    orb = {"C": [(0, 0.3), (0, 1.2), (1, 0.5)], "H": [(0, 0.4)]}
    auxr = {"C": [(0, 0.4), (0, 1.6), (1, 0.8), (2, 1.0)], "H": [(0, 0.6), (1, 0.9)]}
    sh = [_shell(r, l, [a]) for e, r in zip(elems, xyz) for l, a in orb[e]]
    ax = [_shell(r, l, [a]) for e, r in zip(elems, xyz) for l, a in auxr[e]]
    Z = W.charges(elems)
    e0 = O.df_rhf(Z, xyz, sh, ax, nocc=21, max_iter=200)[0]
    R = _rotation(np.random.default_rng(4))
    new = xyz @ R.T
    e1 = O.df_rhf(Z, new, W.shells_at(sh, xyz, new), W.shells_at(ax, xyz, new), nocc=21, max_iter=200)[0]
    assert e0.converged and e1.converged
    assert abs(e0.E - e1.E) < 1e-9
