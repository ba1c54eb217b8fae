"""Small seeded test systems shared by the parity tests (inputs only)."""
import numpy as np

import workloads as W


def shell(ctr, l, exps, coefs=None):
    return {"center": np.asarray(ctr, float), "l": int(l), "exps": list(exps),
            "coefs": list(coefs) if coefs is not None else [1.0] * len(exps)}


def mixed_molecule(seed=0, natom=4, lorb=3, laux=4):
    """A few atoms carrying every orbital l <= lorb and aux l <= laux, plus one
    contracted shell per atom, so that every integral class and the primitive
    loops are exercised.  nbf spans several 32-function tiles with a ragged tail."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-2.0, 2.0, size=(natom, 3))
    sh, ax = [], []
    for r in xyz:
        for l in range(lorb + 1):
            sh.append(shell(r, l, [0.4 + 0.3 * l]))
            sh.append(shell(r, l, [1.6 + 0.5 * l]))
        sh.append(shell(r, 1, [3.0, 0.9, 0.25], [0.2, 0.5, 0.4]))
        for l in range(laux + 1):
            ax.append(shell(r, l, [0.3 + 0.2 * l]))
            ax.append(shell(r, l, [1.5 + 0.7 * l]))
        ax.append(shell(r, 2, [4.0, 1.1], [0.6, 0.5]))
    Z = np.array([6] * natom, np.int32)
    return xyz, Z, sh, ax


def h4():
    elems, xyz, sh, ax = W.workload("h4")
    return xyz, W.charges(elems), sh, ax, W.nocc_of(elems)
