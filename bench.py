#!/usr/bin/env python
"""Benchmark of the density-fitted RHF hot path on one MI355X.

One step = one complete DF-RHF (dfx_scf through the C-ABI): Schwarz screening,
Rys three-index integrals, metric, Cholesky, B = L^-1 (mu nu|P), one-electron
integrals, the learned starting guess (descriptors, MLP inference, rotation,
projection) and every SCF iteration, on the (H2O)64 workload (seeded water
cluster, even-tempered O [3s2p1d] / H [2s1p], auxiliary O [8s6p4d2f] /
H [4s3p2d]; 1536 basis / 6784 auxiliary functions).  Prints ONE JSON line.

Before the timed steps (untimed, reported): the guess model is trained on the
GPU from converged densities of seeded 3x3x3 and 2x2x2 water clusters; a
core-guess run and a plain FP64 run of the same workload are timed for context.

    python bench.py [--steps K] [--warmup W] [--workload water4] [--schedule fp64|mixed]
                    [--guess learned|core] [--trajectory]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "DF-RHF wall time at |ΔE|≤1e-6 Eh, mixed+learned vs FP64 plain; 3-idx ERI/s"

# MI355X published peaks
PEAK_FP64 = 78.6e12       # vector and matrix, FLOP/s
PEAK_FP32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12         # B/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRSM_LABEL = "B transform block updates R_i -= L_i,<i B_<i (dgemm_kernel EPI_SUB)"
TRAFFIC_PROFILES = {"K half-transform X_Q = B_Q C, FP64": "kx64_water64_pmc.txt",
                    TRSM_LABEL: "trsm_update_water64_pmc.txt"}


def measured_traffic(kernel_label):
    """HBM bytes per launch from the committed counter summary of the kernel
    (the FP64 half transform or the B transform), or None if there is none or
    the kernel's source has changed since the counters were taken."""
    import hashlib
    name = next((f for k, f in TRAFFIC_PROFILES.items() if kernel_label.startswith(k)), None)
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, kv.get("source", ""))
    if not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv.get("source_sha256_16"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline(info, nbf, naux, nocc):
    """Roofline of the kernel with the largest GPU time, from the live HIP-event
    timings the library reports per kernel and precision: algorithmic FLOPs per
    launch / average launch time, against the peak of the precision used."""
    peaks = {0: ("FP64", PEAK_FP64), 1: ("FP32", PEAK_FP32_MFMA), 2: ("BF16", PEAK_BF16_MFMA)}
    # the B transform's block updates (the substitution's MFMA products): their
    # FLOPs as the library counts them, 2 M K N per launch, and their own GPU time
    cands = {f"{TRSM_LABEL}, FP64 MFMA":
             (info["t_trsm_update"], info["trsm_update_flops"], info["n_trsm_update"], PEAK_FP64)}
    for p, (pname, peak) in peaks.items():
        nj = info["n_jk_p"][p]
        nl = info["n_kx_launch_p"][p]
        if nj == 0:
            continue
        # X_Q = B_Q C_occ for every Q, per K build
        cands[f"K half-transform X_Q = B_Q C, {pname} MFMA"] = (info["t_kx_p"][p], 2.0 * nbf * nbf * nocc * naux * nj,
                                                               nl, peak)
        # sum_Q X_Q X_Q^T, lower triangle, per K build
        cands[f"K contraction sum_Q X_Q X_Q^T, {pname} MFMA"] = (info["t_ksyrk_p"][p],
                                                                nbf * (nbf + 1.0) * nocc * naux * nj, nl, peak)
    name, (t, flops, launches, peak) = max(cands.items(), key=lambda kv: kv[1][0])
    if t <= 0:
        return None
    launches = max(1, launches)
    achieved = (flops / launches) / (t / launches)
    return {"kernel": name, "bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(name),
            "flops_per_launch": flops / launches, "avg_launch_ms": 1e3 * t / launches,
            "all": {k: {"s": round(v[0], 4), "TFLOP/s": round(v[1] / v[0] / 1e12, 2) if v[0] > 0 else None,
                        "frac": round(v[1] / v[0] / v[3], 4) if v[0] > 0 else None} for k, v in cands.items()}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(elems, xyz, sh, ax, niter, budget_pairs=250, q_rows=16, seed=0):
    """The oracle, timed on bounded samples of the same workload and scaled to
    one full DF-RHF (an extrapolation, not a run): ERIs over a random sample of
    shell pairs, the fit on their columns, J/K on a sample of aux rows times
    niter (the iteration count of the plain FP64 schedule from the core guess,
    which is what the oracle runs), and the dense eigen/matrix work of one
    iteration times niter."""
    import oracle as O
    import scipy.linalg as sla
    import threadpoolctl  # noqa: F401  (BLAS threads = cores)
    rng = np.random.default_rng(seed)
    bas, aux = O.Basis(sh), O.Basis(ax)
    Z = W.charges(elems)
    nocc = W.nocc_of(elems)
    t_all = {}
    t0 = time.perf_counter()
    Qab, QC = O.schwarz(bas, aux)
    scr = O.screen(bas, aux, Qab, QC, 1e-12)
    t_all["schwarz"] = time.perf_counter() - t0
    npairs = len(scr.pairs)
    pick = np.sort(rng.choice(npairs, size=min(budget_pairs, npairs), replace=False))
    sub = O.Screen(scr.pairs[pick], np.concatenate([[0], np.cumsum(np.diff(scr.col_off)[pick])]).astype(np.int64),
                   scr.keep[pick], scr.tau)
    t0 = time.perf_counter()
    raw = O.eri3_packed(bas, aux, sub)
    t_eri = time.perf_counter() - t0
    t_all["eri"] = t_eri * npairs / len(pick)
    t0 = time.perf_counter()
    J2 = O.eri2(aux)
    L = sla.cholesky(J2, lower=True)
    t_all["metric"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Bs = sla.solve_triangular(L, raw, lower=True)
    t_all["fit"] = (time.perf_counter() - t0) * scr.col_off[-1] / max(1, raw.shape[1])
    del raw
    # J/K on q_rows rows of B (same cost per row as the real tensor)
    n = bas.nbf
    rows = rng.normal(size=(q_rows, int(scr.col_off[-1]))) * 1e-2
    dfs = O.DF(bas, aux, scr, rows, L[:q_rows, :q_rows])
    C = np.linalg.qr(rng.normal(size=(n, nocc)))[0]
    t0 = time.perf_counter()
    O.jk(dfs, C=C, chunk=16)
    t_all["jk"] = (time.perf_counter() - t0) * aux.nbf / q_rows * niter
    # one iteration's dense work: X^T F X, eigh, C, D, F D S, X^T e X
    S, T, V = O.int1e(bas, xyz, Z)
    X, _ = O.orthogonalizer(S)
    Fm = T + V
    t0 = time.perf_counter()
    e = X.T @ (Fm @ S @ S - S @ S @ Fm) @ X
    w, Cp = np.linalg.eigh(X.T @ Fm @ X)
    Cf = X @ Cp
    D = Cf[:, :nocc] @ Cf[:, :nocc].T
    t_all["dense"] = (time.perf_counter() - t0) * niter
    del e, w, D
    total = sum(t_all.values())
    return {"value": total, "unit": "s", "cores": os.cpu_count(), "kind": "oracle",
            "extrapolated": True, "cpu_model": cpu_model(),
            "sample": (f"estimate, extrapolated from bounded samples of the oracle on the same workload: ERIs "
                       f"of {len(pick)} random shell pairs of {npairs} (scaled), metric + Cholesky in full, "
                       f"triangular solve on their columns (scaled), J/K on {q_rows} of {aux.nbf} aux rows "
                       f"(scaled) x {niter} iterations (plain FP64 from the core guess), one iteration's "
                       f"dense eigen/matrix work x {niter}"),
            "phases_s": {k: round(v, 3) for k, v in t_all.items()}}


def train_guess(dfx, n27=8, n8=16, epochs=80, batch=128, seed=5, sigma=0.04):
    """Guess model for water from converged GPU densities of seeded clusters:
    3x3x3 clusters hold every coordination a water has in the 4x4x4 cluster
    (corner to fully surrounded), 2x2x2 clusters add surface environments.
    Every atom is displaced by N(0, sigma^2) per coordinate, so that bond
    lengths and angles vary as they do along a trajectory."""
    basis = {8: [0, 0, 0, 1, 1, 2], 1: [0, 0, 1]}
    m = dfx.GuessModel(basis, rc=8.0, rc_env=6.0, hidden=256, depth=3, seed=seed)
    t0 = time.perf_counter()
    ngeom = 0
    for side, seeds in ((3, range(1, 1 + n27)), (2, range(1, 1 + n8))):
        for sd in seeds:
            elems, xyz = W.water_cluster(side=side, seed=1000 + sd)
            xyz = xyz + np.random.default_rng(5000 + sd).normal(0.0, sigma, size=xyz.shape)
            sh, ax = W.basis_for("water", elems, xyz)
            Z = W.charges(elems)
            E, C, _, info = dfx.scf(xyz, Z, sh, ax, schedule=dfx.SCHED_MIXED, conv_dE=1e-8, conv_err=1e-6)
            nocc = info["nocc"]
            m.add(xyz, Z, dfx.lowdin(xyz, Z, sh, C[:, :nocc] @ C[:, :nocc].T))
            ngeom += 1
        log(f"guess training data: {ngeom} geometries, {time.perf_counter() - t0:.1f} s")
    t_data = time.perf_counter() - t0
    t1 = time.perf_counter()
    loss = m.train(epochs=epochs, batch=batch, lr=1e-3)
    t_train = time.perf_counter() - t1
    log(f"guess training: {epochs} epochs in {t_train:.1f} s, loss {loss[0]:.3f} -> {loss[-1]:.4f}")
    return m, {"geometries": f"{n27} x (H2O)27 + {n8} x (H2O)8, seeds 1001.., per-atom sigma {sigma} bohr",
               "data_s": round(t_data, 2),
               "train_s": round(t_train, 2), "epochs": epochs, "batch": batch,
               "samples": sum(t["samples"] for t in m.types()), "loss_first": round(float(loss[0]), 4),
               "loss_last": round(float(loss[-1]), 4)}


def profile_jk(dfx, torch, sh, ax, nocc, prec):
    """One J/K build on the workload's B with a seeded orthonormal C_occ, then a
    copy of 2^28 floats (1 GiB read, 1 GiB written) whose counters calibrate
    the per-dispatch HBM byte counts.  B is built twice: the first build loads
    the integral kernels' code objects, the second is the one to read."""
    dfx.eri3(sh, ax).free()
    B = dfx.eri3(sh, ax)
    C = torch.tensor(W.random_orthonormal(B.nbf, nocc, seed=1), device="cuda")
    J, K = dfx.jk(B, C, precision=prec)
    torch.cuda.synchronize()
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"profile-jk: nbf {B.nbf} naux {B.naux} nocc {nocc}; copy calibration 1 GiB read + 1 GiB written")
    B.free()


def _shape_ls(kind, elem):
    return [l for l, n in enumerate(W.ORB_SHAPE[kind][elem]) for _ in range(n)]


def _stats(v):
    v = np.asarray(v, float)
    return {"mean": round(float(v.mean()), 4), "median": round(float(np.median(v)), 4),
            "min": round(float(v.min()), 4), "max": round(float(v.max()), 4)}


def eval_ring_guess(dfx, ntrain, ntest, epochs, batch):
    """Seeded C8H16 crowns: train the guess on ntrain converged densities (seeds
    0..), then on ntest unseen crowns (seeds 1600..) compare plain FP64 DF-RHF
    from the learned guess with the core guess at |dE| < 1e-8."""
    m = dfx.GuessModel({6: _shape_ls("ring", "C"), 1: _shape_ls("ring", "H")}, rc=8.0, rc_env=6.0,
                       hidden=256, depth=3, seed=4)
    conv = dict(conv_dE=1e-8, conv_err=1e-7)
    elems, xyz, sh, ax = W.workload("ring", seed=0)
    dfx.scf(xyz, W.charges(elems), sh, ax, want_c=False, **conv)          # warm-up
    t0 = time.perf_counter()
    for sd in range(ntrain):
        elems, xyz, sh, ax = W.workload("ring", seed=sd)
        Z = W.charges(elems)
        _, C, _, info = dfx.scf(xyz, Z, sh, ax, **conv)
        nocc = info["nocc"]
        m.add(xyz, Z, dfx.lowdin(xyz, Z, sh, C[:, :nocc] @ C[:, :nocc].T))
        if sd % 100 == 99:
            log(f"ring training data: {sd + 1} geometries, {time.perf_counter() - t0:.1f} s")
    t_data = time.perf_counter() - t0
    t1 = time.perf_counter()
    loss = m.train(epochs=epochs, batch=batch, lr=1e-3)
    t_train = time.perf_counter() - t1
    log(f"ring guess training: {epochs} epochs in {t_train:.1f} s, loss {loss[0]:.3f} -> {loss[-1]:.4f}")
    it_c, it_l, w_c, w_l, dE, nfb = [], [], [], [], [], 0
    for sd in range(1600, 1600 + ntest):
        elems, xyz, sh, ax = W.workload("ring", seed=sd)
        Z = W.charges(elems)
        ta = time.perf_counter()
        Ec, _, _, ic = dfx.scf(xyz, Z, sh, ax, want_c=False, **conv)
        tb = time.perf_counter()
        El, _, _, il = dfx.scf(xyz, Z, sh, ax, want_c=False, model=m, **conv)
        tc = time.perf_counter()
        it_c.append(ic["niter"])
        it_l.append(il["niter"])
        w_c.append(tb - ta)
        w_l.append(tc - tb)
        dE.append(abs(El - Ec))
        nfb += il["guess_fallback"] != 0
    out = {"metric": "learned-guess gain, C8H16 crowns (plain FP64 DF-RHF, |dE| < 1e-8)",
           "workload": "ring: crown C8H16, C [4s3p2d1f] / [8s6p5d3f2g], H [2s1p] / [4s3p2d], sigma 0.1 bohr",
           "train": {"geometries": ntrain, "seeds": f"0..{ntrain - 1}", "data_s": round(t_data, 2),
                     "train_s": round(t_train, 2), "epochs": epochs, "batch": batch,
                     "samples": sum(t["samples"] for t in m.types()), "loss_first": round(float(loss[0]), 4),
                     "loss_last": round(float(loss[-1]), 4)},
           "test": {"geometries": ntest, "seeds": f"1600..{1600 + ntest - 1}",
                    "iterations_core": _stats(it_c), "iterations_learned": _stats(it_l),
                    "wall_core_s": _stats(w_c), "wall_learned_s": _stats(w_l),
                    "max_abs_dE_learned_vs_core": float(max(dE)), "fallbacks": nfb}}
    print(json.dumps(out))


def eval_alkane(dfx):
    """C30H62: plain FP64 against the mixed schedules (FP32 -> FP64 and
    BF16 -> FP32 -> FP64), each |dE| against the oracle's stored energy."""
    elems, xyz, sh, ax = W.workload("alkane", seed=0)
    Z = W.charges(elems)
    gold = os.path.join(ROOT, "tests", "golden", "df_rhf_floors.json")
    E_or = json.load(open(gold))["alkane"]["E"] if os.path.exists(gold) else None
    conv = dict(conv_dE=1e-9, conv_err=1e-7)
    dfx.scf(xyz, Z, sh, ax, want_c=False, **conv)                                     # warm-up
    runs = {}
    for tag, kw in (("plain_fp64", {}), ("mixed_fp32", dict(schedule=dfx.SCHED_MIXED, mixed_prec=dfx.FP32)),
                    ("mixed_bf16", dict(schedule=dfx.SCHED_MIXED, mixed_prec=dfx.BF16))):
        t0 = time.perf_counter()
        E, _, _, i = dfx.scf(xyz, Z, sh, ax, want_c=False, **conv, **kw)
        runs[tag] = {"wall_s": round(time.perf_counter() - t0, 3), "E": E, "niter": i["niter"],
                     "n_mixed": i["n_mixed"], "dE_vs_oracle": (E - E_or) if E_or is not None else None}
        log(f"alkane {tag}: E = {E:.10f} iters {i['niter']} wall {runs[tag]['wall_s']:.2f} s")
    print(json.dumps({"metric": "C30H62 DF-RHF: plain FP64 vs mixed, |dE| vs the oracle",
                      "workload": "alkane: zigzag C30H62 seed 0, C [3s2p1d] / [7s5p4d2f], H [2s1p] / [4s3p2d]",
                      "oracle_E": E_or, "runs": runs}))


def eval_mp2(dfx, workloads=("alkane", "water4")):
    """DF-MP2 (FP64) after a converged plain FP64 SCF: energy, time and the
    FP64 MFMA rate of the whole MP2 step (both transformations and the pair
    products, 2 nbf^2 o Q + 2 v nbf o Q + v^2 Q o (o + 1) FLOP, o = correlated
    occupied, v = virtual, Q = auxiliary functions)."""
    import torch
    rows = []
    for wl in workloads:
        elems, xyz, sh, ax = W.workload(wl, seed=0) if wl == "alkane" else W.workload(wl)
        Z = W.charges(elems)
        E, C, eps, info = dfx.scf(xyz, Z, sh, ax, conv_dE=1e-9, conv_err=1e-7)
        # the SCF's cached workspace back to the device: B and MP2's work need it
        dfx.release_scf_workspace()
        torch.cuda.empty_cache()
        nocc, nbf, naux = info["nocc"], info["nbf"], info["naux"]
        nmo = nbf - info["ndropped"]
        nfrozen = sum(1 for z in Z if z > 2)  # 1s cores of C and O
        Ct = torch.tensor(np.ascontiguousarray(C[:, :nmo]), device="cuda")
        B = dfx.eri3(sh, ax)
        dfx.mp2(B, Ct, eps, nocc, nfrozen)                                    # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E2 = dfx.mp2(B, Ct, eps, nocc, nfrozen)
        dt = time.perf_counter() - t0
        B.free()
        o, v = nocc - nfrozen, nmo - nocc
        flop = 2.0 * nbf * nbf * o * naux + 2.0 * v * nbf * o * naux + float(v) * v * naux * o * (o + 1)
        row = {"workload": wl, "nbf": nbf, "naux": naux, "nocc": nocc, "nfrozen": nfrozen, "nvir": v,
               "E_scf": E, "E2": E2, "mp2_s": round(dt, 4), "TFLOP/s": round(flop / dt / 1e12, 2),
               "frac_fp64_peak": round(flop / dt / PEAK_FP64, 4)}
        log(json.dumps(row))
        rows.append(row)
    print(json.dumps({"metric": "DF-MP2 correlation energy after DF-RHF, FP64 MFMA", "runs": rows}))


def eval_open_shell(dfx, runs=(("alkane", 0, 1, 150, 0.0), ("alkane", 0, 3, 150, 0.0), ("alkane", 1, 2, 150, 0.0),
                                 ("water4", 1, 2, 30, 0.0), ("water4", 1, 2, 80, 0.3))):
    """DF-UHF and DF-ROHF (FP64, core guess) at full size: energy, iterations and
    seconds per iteration beside the DF-RHF of the same molecule.  Closed shells
    must give the RHF energy and UHF must lie at or below ROHF.  The (H2O)64
    cation runs a fixed 30 iterations for the per-iteration time only: from the
    core guess with plain DIIS it does not converge (the oracle does not on the
    (H2O)8 cation either); the last row adds a level shift of 0.3 Eh."""
    rows, rhf = [], {}
    for wl, charge, mult, max_iter, shift in runs:
        conv = dict(conv_dE=1e-9, conv_err=1e-7, max_iter=max_iter)
        elems, xyz, sh, ax = W.workload(wl, seed=0) if wl == "alkane" else W.workload(wl)
        Z = W.charges(elems)
        if wl not in rhf:
            Er, _, _, ir = dfx.scf(xyz, Z, sh, ax, want_c=False, **conv)
            rhf[wl] = (Er, ir)
        Er, ir = rhf[wl]
        ne = int(Z.sum()) - charge
        row = {"workload": wl, "charge": charge, "multiplicity": mult, "n_alpha": (ne + mult - 1) // 2,
               "n_beta": ne - (ne + mult - 1) // 2, "max_iter": max_iter, "level_shift": shift, "E_rhf": Er,
               "rhf_s_per_iter": round(ir["t_scf"] / max(1, ir["niter"]), 4)}
        for name, fn in (("uhf", dfx.uhf), ("rohf", dfx.rohf)):
            t0 = time.perf_counter()
            E, _, _, info = fn(xyz, Z, sh, ax, charge=charge, multiplicity=mult, level_shift=shift, want_c=False,
                               **conv)
            dt = time.perf_counter() - t0
            row.update({"nbf": info["nbf"], f"E_{name}": E, f"{name}_converged": info["converged"],
                        f"{name}_iters": info["niter"], f"{name}_s": round(dt, 3),
                        f"{name}_s_per_iter": round(info["t_scf"] / max(1, info["niter"]), 4)})
            if charge == 0 and mult == 1:
                row[f"E_{name}_minus_E_rhf"] = E - Er
        if row["uhf_converged"] and row["rohf_converged"]:
            row["E_rohf_minus_E_uhf"] = row["E_rohf"] - row["E_uhf"]
        log(json.dumps(row))
        rows.append(row)
    print(json.dumps({"metric": "DF-UHF and DF-ROHF (FP64 J and K, core guess, DIIS)", "runs": rows}))


def eval_grad(dfx, workloads=("alkane", "water4")):
    """DF-RHF analytic nuclear gradient (FP64) after a converged plain FP64 SCF
    at full size: wall and GPU times of its phases, the translational and
    torque sum rules, and the largest component."""
    import torch
    rows = []
    for wl in workloads:
        elems, xyz, sh, ax = W.workload(wl, seed=0) if wl == "alkane" else W.workload(wl)
        Z = W.charges(elems)
        E, C, eps, info = dfx.scf(xyz, Z, sh, ax, conv_dE=1e-9, conv_err=1e-7)
        # the SCF's cached workspace back to the device for the gradient's own
        dfx.release_scf_workspace()
        torch.cuda.empty_cache()
        nocc = info["nocc"]
        dfx.rhf_grad(xyz, Z, sh, ax, C[:, :nocc], eps[:nocc])                     # warm-up
        t0 = time.perf_counter()
        g, gi = dfx.rhf_grad(xyz, Z, sh, ax, C[:, :nocc], eps[:nocc])
        dt = time.perf_counter() - t0
        ctr = np.asarray(xyz).mean(axis=0)
        torque = sum(np.cross(xyz[i] - ctr, g[i]) for i in range(len(Z)))  # about the centroid
        row = {"workload": wl, "natom": len(Z), "nbf": info["nbf"], "naux": info["naux"], "nocc": nocc,
               "E": E, "grad_s": round(dt, 4), "phases_s": {k: round(v, 4) for k, v in gi.items() if k != "natom"},
               "max_abs_g": float(np.abs(g).max()), "sum_rule": float(np.abs(g.sum(axis=0)).max()),
               "torque": float(np.abs(torque).max()), "scf_s": round(info["t_total"], 3)}
        log(json.dumps(row))
        rows.append(row)
    print(json.dumps({"metric": "DF-RHF analytic nuclear gradient, FP64", "runs": rows}))


def eval_trajectory(dfx, nframes):
    """(H2O)64 over a seeded trajectory: per frame, mixed + learned (timed) and
    plain FP64 from the core guess; as context, mixed from the previous frame's
    orbitals."""
    model, learned = train_guess(dfx)
    elems, xyz, sh, ax = W.workload("water4")
    Z = W.charges(elems)
    frames = W.trajectory(xyz, nframes, seed=1)
    conv = dict(conv_dE=1e-7, conv_err=1e-5)
    rows, C_prev = [], None
    for k, x in enumerate(frames):
        shx, axx = W.shells_at(sh, xyz, x), W.shells_at(ax, xyz, x)
        t0 = time.perf_counter()
        El, _, _, il = dfx.scf(x, Z, shx, axx, want_c=False, schedule=dfx.SCHED_MIXED, model=model, **conv)
        t1 = time.perf_counter()
        Ep, Cp, _, ip = dfx.scf(x, Z, shx, axx, **conv)
        t2 = time.perf_counter()
        row = {"frame": k, "learned_mixed_s": round(t1 - t0, 3), "learned_mixed_iters": il["niter"],
               "plain_fp64_s": round(t2 - t1, 3), "plain_fp64_iters": ip["niter"], "dE": El - Ep}
        if C_prev is not None:
            t3 = time.perf_counter()
            Eq, _, _, iq = dfx.scf(x, Z, shx, axx, want_c=False, schedule=dfx.SCHED_MIXED, init=C_prev,
                                   guess=dfx.GUESS_CINIT, **conv)
            row.update(prev_frame_mixed_s=round(time.perf_counter() - t3, 3), prev_frame_mixed_iters=iq["niter"],
                       dE_prev=Eq - Ep)
        C_prev = Cp
        rows.append(row)
        log(json.dumps(row))
    tl = sum(r["learned_mixed_s"] for r in rows)
    tp = sum(r["plain_fp64_s"] for r in rows)
    print(json.dumps({"metric": "(H2O)64 trajectory: mixed + learned vs plain FP64, per frame",
                      "frames": nframes, "learned_guess": learned, "total_learned_mixed_s": round(tl, 3),
                      "total_plain_fp64_s": round(tp, 3), "speedup": round(tp / tl, 3),
                      "max_abs_dE": max(abs(r["dE"]) for r in rows), "per_frame": rows}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="water4")
    ap.add_argument("--schedule", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--mixed-prec", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--guess", default="learned", choices=["learned", "core"])
    ap.add_argument("--trajectory", action="store_true",
                    help="step k runs frame k of a seeded trajectory (per-atom sigma 0.02 bohr)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 reference run")
    ap.add_argument("--no-context", action="store_true", help="skip the core-guess context run")
    ap.add_argument("--eval", default=None,
                    choices=["ring-guess", "alkane", "trajectory", "mp2", "open-shell", "grad"],
                    help="evaluation runs beside the benchmark line (each prints its own JSON line)")
    ap.add_argument("--ntrain", type=int, default=1600)
    ap.add_argument("--ntest", type=int, default=400)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--frames", type=int, default=10)
    ap.add_argument("--profile-jk", default=None, choices=["fp64", "fp32", "bf16"],
                    help="counter-run driver: build B, one J/K build in this precision with the SCF's "
                         "launch configuration, and a 1 GiB elementwise copy as the HBM calibration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--run-log", default=None, help="append one JSON line per SCF / gradient call to this file")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; run with --gpus 1 (sharding the "
                                   "auxiliary index over several GPUs is designed, not implemented)"}))
        sys.exit(2)

    import torch
    import paper_1707_03771_amd as dfx
    if a.run_log:
        dfx.set_run_log(a.run_log)

    elems, xyz, sh, ax = W.workload(a.workload)
    Z = W.charges(elems)
    nocc = W.nocc_of(elems)
    if a.eval == "ring-guess":
        eval_ring_guess(dfx, a.ntrain, a.ntest, a.epochs, 256)
        return
    if a.eval == "alkane":
        eval_alkane(dfx)
        return
    if a.eval == "mp2":
        eval_mp2(dfx)
        return
    if a.eval == "open-shell":
        eval_open_shell(dfx)
        return
    if a.eval == "grad":
        eval_grad(dfx)
        return
    if a.eval == "trajectory":
        eval_trajectory(dfx, a.frames)
        return
    if a.profile_jk:
        profile_jk(dfx, torch, sh, ax, nocc, {"fp64": dfx.FP64, "fp32": dfx.FP32, "bf16": dfx.BF16}[a.profile_jk])
        return
    nbf = sum(2 * s["l"] + 1 for s in sh)
    naux = sum(2 * s["l"] + 1 for s in ax)
    sched = dfx.SCHED_MIXED if a.schedule == "mixed" else dfx.SCHED_FP64
    mp = dfx.BF16 if a.mixed_prec == "bf16" else dfx.FP32
    # converged = |E_k - E_k-1| < 1e-7 and max|e| < 1e-5 for every run: with the
    # superlinear end of the iterations this leaves the energy within ~1e-8 of a
    # tightly converged FP64 solution, well inside the 1e-6 Eh the metric asks for
    opts = dict(conv_dE=1e-7, conv_err=1e-5, schedule=sched, mixed_prec=mp, max_iter=100)
    log(f"workload {a.workload}: {len(elems)} atoms, nbf {nbf}, naux {naux}, nocc {nocc}")

    model, learned = (None, None)
    if a.guess == "learned":
        model, learned = train_guess(dfx)
    frames = W.trajectory(xyz, a.steps + a.warmup, seed=1) if a.trajectory else None

    def step(tag, k=None, **kw):
        x = xyz if frames is None or k is None else frames[k]
        shx, axx = (sh, ax) if x is xyz else (W.shells_at(sh, xyz, x), W.shells_at(ax, xyz, x))
        o = dict(opts, **kw)
        t0 = time.perf_counter()
        E, _, _, info = dfx.scf(x, Z, shx, axx, want_c=False, **o)
        dt = time.perf_counter() - t0
        log(f"{tag}: E = {E:.10f}  iters {info['niter']} (mixed {info['n_mixed']})  "
            f"wall {dt:.2f} s  guess {info['t_guess']:.3f} eri {info['t_eri']:.3f} trsm {info['t_trsm']:.3f} "
            f"(updates {info['t_trsm_update']:.3f}) "
            f"j {info['t_j']:.3f} kx {info['t_kx']:.3f} ksyrk {info['t_ksyrk']:.3f} eig {info['t_eig']:.3f} "
            f"(purification {info['t_purify']:.3f} over {info['n_purified']} updates, "
            f"{info['purify_steps']} squarings)")
        pn = {0: "d", 1: "s", 2: "b"}
        log("   history: " + " ".join(f"{pn.get(p, '?')}{e:.1e}" for p, e in zip(info["prec_hist"], info["err_hist"])))
        eh = info["E_hist"]
        log("   |dE|:    " + " ".join(f"{abs(eh[k] - eh[k - 1]):.1e}" for k in range(1, len(eh))))
        if info["guess_fallback"]:
            log(f"   learned guess fell back to the core guess (code {info['guess_fallback']})")
        return E, info, dt

    gk = {"model": model} if model is not None else {}
    for w in range(a.warmup):
        step(f"warmup {w}", a.steps + w, **gk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step(f"step {k}", k, **gk) for k in range(a.steps)]
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / max(1, a.steps)
    walls = [r[2] for r in res]
    # the roofline and the reported phases come from the step of median wall time
    k_med = int(np.argsort(walls)[(len(walls) - 1) // 2])
    E, info, _ = res[k_med]
    k_last = a.steps - 1

    context = None
    if model is not None and not a.no_context:
        Ec, ic, tc = step("context: same schedule, core guess", k_last)
        context = {"guess": "core", "wall_s": round(tc, 3), "niter": ic["niter"], "n_mixed": ic["n_mixed"],
                   "dE_vs_learned": Ec - E}
    plain = None
    if sched != dfx.SCHED_FP64 and not a.no_plain:
        Ep, ip, tp = step("plain fp64, core guess", k_last, schedule=dfx.SCHED_FP64)
        plain = {"wall_s": round(tp, 3), "E": Ep, "niter": ip["niter"], "dE_vs_plain": E - Ep,
                 "speedup": round(tp / T, 3)}

    out = {
        "metric": METRIC,
        "value": round(T, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * T, 2),
        "step_wall_s": {"mean": round(float(np.mean(walls)), 4), "median": round(float(np.median(walls)), 4),
                        "min": round(float(np.min(walls)), 4), "max": round(float(np.max(walls)), 4),
                        "median_step": k_med},
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if sched == dfx.SCHED_FP64 else f"{a.mixed_prec}+f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: (H2O)_{len(elems) // 3} DF-RHF, O[3s2p1d] H[2s1p] / "
                               f"O[8s6p4d2f] H[4s3p2d] even-tempered", "nbf": nbf, "naux": naux,
                   "nocc": nocc, "schedule": a.schedule, "guess": a.guess, "tau": 1e-12,
                   "trajectory": bool(a.trajectory)},
        "E": E,
        "niter": info["niter"],
        "n_mixed": info["n_mixed"],
        # per iteration of the timed step: precision of K (0 FP64, 1 FP32, 2 BF16),
        # energy and largest DIIS error element
        "iterations": [{"prec": int(p), "E": e, "err": float(r)}
                       for p, e, r in zip(info["prec_hist"], info["E_hist"], info["err_hist"])],
        "t_guess_s": round(info["t_guess"], 4),
        "floor_est": info["floor_est"],
        "learned_guess": learned,
        "context_core_guess": context,
        "eri_per_s": info["nintegrals"] / info["t_eri"] if info["t_eri"] > 0 else None,
        "phases_s": {k: round(info[k], 4) for k in ("t_setup", "t_scf", "t_eri", "t_metric", "t_trsm",
                                                     "t_trsm_update", "t_j", "t_kx", "t_ksyrk", "t_eig",
                                                     "t_purify")},
        # occupied-space updates by purification: count, squarings and GPU time each
        "purification": {"updates": info["n_purified"], "squarings": info["purify_steps"],
                         "ms_per_update": round(1e3 * info["t_purify"] / info["n_purified"], 3)
                         if info["n_purified"] else None},
        "roofline": roofline(info, nbf, naux, nocc),
        "plain_fp64": plain,
    }
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle on samples) ...")
        out["cpu_baseline"] = cpu_baseline(elems, xyz, sh, ax, plain["niter"] if plain else info["niter"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
