"""Writes df_rhf_floors.json: for each named workload, the oracle's converged
DF-RHF energy and how far FP64 rounding in the fit alone can move it.  Calls
only the oracle.

Per workload (seeded geometry, Schwarz 1e-12, core guess, DIIS(8), converged to
|dE| < 1e-10 and max|e| < 1e-8):
  E            the oracle's energy;
  kappa        cond(J_PQ) from its eigenvalues;
  deltas       E(D*, B') - E(D*, B) for four metrics perturbed elementwise at
               the rounding level, J'_PQ = J_PQ (1 + 1.1e-16 (R + R^T)_PQ) with
               R uniform in [-1, 1] (seeds 0..3), B' = L'^-1 raw by the same
               Cholesky and triangular solve.  The energy is stationary in the
               density, so at the converged density D* the first-order change
               is the whole effect of the perturbation;
  floor        max |deltas|: the spread of FP64 energies that equally valid
               roundings of the metric give;
  d_explicit   the same difference for B = (L^-1) raw with L^-1 formed
               explicitly (one triangular solve against the identity), the
               other common way to apply the fit;
  d_integrals  the same difference for the metric and the raw integrals each
               perturbed element-wise by 2e-15 relative (seeds 10..13), the
               accuracy of two independent exact integral algorithms (the Rys
               root and weight tables agree with 60-digit values to 2.2e-15
               relative); integral_floor = max |d_integrals|;
  d_hilo       the same difference for B stored as two FP32 words, hi =
               fl32(B) and lo = fl32(B - hi), as the GPU holds it (about 2^-48
               relative);
  d_order      the same difference with the auxiliary functions taken in
               reverse order (metric and raw rows permuted, then the same
               Cholesky and solve): an exact symmetry of the fit, so the
               difference is rounding alone, as any other order of the
               factorisation's operations would give it;
  spread       max of floor, integral_floor, |d_hilo| and |d_order|: how far
               apart equally valid FP64 evaluations of this energy lie.

    python tests/golden/make_energy_floors.py water2 water3 alkane
"""
import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "df_rhf_floors.json")


def energy_at(df, h, C, Enuc):
    D = C @ C.T
    J, K = O.jk(df, C=C)
    F = h + 2.0 * J - K
    return float(np.sum(D * (h + F))) + Enuc


def run(name):
    t0 = time.time()
    elems, xyz, sh, ax = W.workload(name, seed=0) if name == "alkane" else W.workload(name)
    Z = W.charges(elems)
    nocc = W.nocc_of(elems)
    bas, aux = O.Basis(sh), O.Basis(ax)
    S, T, V = O.int1e(bas, xyz, Z)
    h = T + V
    Qab, QC = O.schwarz(bas, aux)
    scr = O.screen(bas, aux, Qab, QC, 1e-12)
    raw = O.eri3_packed(bas, aux, scr)
    J2 = O.eri2(aux)
    L, B = O.fit(raw, J2)
    df = O.DF(bas, aux, scr, B, L)
    Enuc = O.nuclear_repulsion(xyz, Z)
    res = O.rhf(S, h, Enuc, nocc, lambda D, C: O.jk(df, D=D, C=C), conv_dE=1e-10, conv_err=1e-8)
    t_scf = time.time() - t0
    print(f"{name}: E = {res.E:.12f} in {res.niter} iterations, {t_scf:.0f} s", flush=True)
    C = res.C[:, :nocc]
    E0 = energy_at(df, h, C, Enuc)
    deltas = []
    for seed in range(4):
        R = np.random.default_rng(seed).uniform(-1.0, 1.0, size=J2.shape)
        Lp = sla.cholesky(J2 * (1.0 + 1.1e-16 * (R + R.T)), lower=True)
        del R
        dfp = O.DF(bas, aux, scr, sla.solve_triangular(Lp, raw, lower=True), Lp)
        deltas.append(energy_at(dfp, h, C, Enuc) - E0)
        del dfp
        print(f"  metric perturbation {seed}: dE = {deltas[-1]:.3e}", flush=True)
    d_int = []
    for seed in range(10, 14):
        rng = np.random.default_rng(seed)
        R = rng.uniform(-1.0, 1.0, size=J2.shape)
        Lp = sla.cholesky(J2 * (1.0 + 2e-15 * (R + R.T) / 2.0), lower=True)
        del R
        rawp = raw * (1.0 + 2e-15 * rng.uniform(-1.0, 1.0, size=raw.shape))
        dfp = O.DF(bas, aux, scr, sla.solve_triangular(Lp, rawp, lower=True), Lp)
        del rawp
        d_int.append(energy_at(dfp, h, C, Enuc) - E0)
        del dfp
        print(f"  integral-level perturbation {seed}: dE = {d_int[-1]:.3e}", flush=True)
    perm = np.arange(aux.nbf)[::-1]
    Lr = sla.cholesky(J2[np.ix_(perm, perm)], lower=True)
    dfr = O.DF(bas, aux, scr, sla.solve_triangular(Lr, raw[perm], lower=True), Lr)
    d_order = energy_at(dfr, h, C, Enuc) - E0
    del dfr, Lr
    print(f"  auxiliary functions reversed: dE = {d_order:.3e}", flush=True)
    hi = B.astype(np.float32)
    B2 = hi.astype(np.float64) + (B - hi.astype(np.float64)).astype(np.float32).astype(np.float64)
    del hi
    d_hilo = energy_at(O.DF(bas, aux, scr, B2, L), h, C, Enuc) - E0
    del B2
    print(f"  hi + lo FP32 words: dE = {d_hilo:.3e}", flush=True)
    Linv = sla.solve_triangular(L, np.eye(aux.nbf), lower=True)
    dfi = O.DF(bas, aux, scr, Linv @ raw, L)
    d_explicit = energy_at(dfi, h, C, Enuc) - E0
    del dfi
    print(f"  explicit L^-1: dE = {d_explicit:.3e}", flush=True)
    w = np.linalg.eigvalsh(J2)
    return {"workload": name, "nbf": bas.nbf, "naux": aux.nbf, "nocc": nocc, "E": res.E,
            "E_at_Dstar": E0, "niter": res.niter, "converged": bool(res.converged), "tau": 1e-12,
            "conv": {"dE": 1e-10, "err": 1e-8}, "kappa": float(w[-1] / w[0]),
            "deltas": deltas, "floor": float(max(abs(d) for d in deltas)), "d_explicit": d_explicit,
            "d_hilo": d_hilo, "d_order": d_order, "d_integrals": d_int,
            "integral_floor": float(max(abs(d) for d in d_int)),
            "spread": float(max([abs(d) for d in deltas] + [abs(d) for d in d_int] + [abs(d_hilo), abs(d_order)])),
            "oracle_seconds": round(time.time() - t0, 1),
            "source": "oracle (McMurchie-Davidson integrals, scipy Cholesky and triangular solve, DIIS RHF)"}


def main():
    names = sys.argv[1:] or ["water2", "water3", "alkane"]
    for n in names:
        row = run(n)
        # re-read before writing: several workloads may run in parallel processes
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        data[n] = row
        json.dump(data, open(OUT + f".{n}.tmp", "w"), indent=1)
        os.replace(OUT + f".{n}.tmp", OUT)
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
