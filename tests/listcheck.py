"""Comparison of the GPU's screening lists with the oracle's (inputs and
bookkeeping only; no integral arithmetic).

The integer lists are a bit-exact contract.  The one place where two correct
FP64 evaluations may legitimately disagree is a product Q_ab Q_C (or Q_ab
max_C Q_C for a pair) that lies within rounding of the threshold: both sides
compute Q to about 1e-15 relative, so an element whose product is within
TIE (relative) of tau may fall either way.  Such elements, counted from the
oracle's own Q values, are the only ones excluded; everything else is compared
exactly, and the result says which branch ran.
"""
import numpy as np

TIE = 1e-12


def compare_lists(bas, scr, Qab, QC, pairs, off, keep=None, tie=TIE):
    tau = scr.tau
    qmax = float(QC.max())
    nsh = Qab.shape[0]
    a, b = np.tril_indices(nsh)                 # canonical order: a-major, b = 0..a
    with np.errstate(divide="ignore", invalid="ignore"):
        tie_pair = np.abs(Qab[a, b] * qmax / tau - 1.0) < tie
    tie_pairs = set(zip(a[tie_pair].tolist(), b[tie_pair].tolist()))
    gset = set(map(tuple, np.asarray(pairs).tolist()))
    oset = set(map(tuple, np.asarray(scr.pairs).tolist()))
    diff = gset ^ oset
    assert diff <= tie_pairs, f"pairs differ outside the tie zone: {sorted(diff - tie_pairs)[:10]}"
    sizes = bas.size.astype(np.int64)
    gp = np.asarray(pairs).reshape(-1, 2)
    if not diff:
        assert np.array_equal(gp, scr.pairs)
        assert np.array_equal(off, scr.col_off)
    else:
        # canonical order and offsets consistent with the GPU's own pair list
        order = gp[:, 0].astype(np.int64) * (gp[:, 0] + 1) // 2 + gp[:, 1]
        assert np.all(np.diff(order) > 0)
        ref_off = np.concatenate([[0], np.cumsum(sizes[gp[:, 0]] * sizes[gp[:, 1]])])
        assert np.array_equal(off, ref_off)
    ntie_trip = 0
    if keep is not None:
        keep = np.asarray(keep).astype(bool)
        gidx = {p: i for i, p in enumerate(map(tuple, gp.tolist()))}
        rows = [(gidx[p], k) for k, p in enumerate(map(tuple, np.asarray(scr.pairs).tolist())) if p in gidx]
        gi = np.array([r[0] for r in rows], np.int64)
        oi = np.array([r[1] for r in rows], np.int64)
        q = Qab[scr.pairs[oi, 0], scr.pairs[oi, 1]][:, None] * QC[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            tie_trip = np.abs(q / tau - 1.0) < tie
        ntie_trip = int(tie_trip.sum())
        mism = keep[gi] != scr.keep[oi]
        assert not np.any(mism & ~tie_trip), f"{int((mism & ~tie_trip).sum())} triplets differ outside the tie zone"
        if not diff and ntie_trip == 0:
            assert np.array_equal(keep, scr.keep)
    npairs_all = nsh * (nsh + 1) // 2
    out = {"mode": "exact" if not diff and ntie_trip == 0 and not tie_pair.any() else "tie-zone",
           "tie_pairs": int(tie_pair.sum()), "tie_pairs_differing": len(diff), "tie_triplets": ntie_trip,
           "screened_pairs": npairs_all - len(scr.pairs),
           "screened_triplets": int((~scr.keep).sum())}
    print("screening lists:", out)
    return out
