"""Writes alkane_df_rhf.json: the oracle's DF-RHF energy of the zigzag C30H62
workload (seed 0; C [3s2p1d] / [7s5p4d2f], H [2s1p] / [4s3p2d], even-tempered;
Schwarz 1e-12), converged to |dE| < 1e-10 and max|e| < 1e-8 from the core
guess.  Calls only the oracle.

    python tests/golden/make_alkane_energy.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    elems, xyz, sh, ax = W.workload("alkane", seed=0)
    Z = W.charges(elems)
    nocc = W.nocc_of(elems)
    t0 = time.time()
    res, df = O.df_rhf(Z, xyz, sh, ax, nocc, tau=1e-12, conv_dE=1e-10, conv_err=1e-8)
    out = {"workload": "alkane (C30H62 zigzag, seed 0)", "nbf": df.bas.nbf, "naux": df.aux.nbf, "nocc": nocc,
           "E": res.E, "niter": res.niter, "converged": bool(res.converged), "tau": 1e-12,
           "conv": {"dE": 1e-10, "err": 1e-8}, "oracle_seconds": round(time.time() - t0, 1),
           "source": "oracle.df_rhf (McMurchie-Davidson integrals, scipy Cholesky, DIIS RHF)"}
    json.dump(out, open(os.path.join(HERE, "alkane_df_rhf.json"), "w"), indent=1)
    print(out)


if __name__ == "__main__":
    main()
