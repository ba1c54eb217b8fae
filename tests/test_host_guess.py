"""CPU checks of the learned guess's host logic in libdfx.so (descriptors, local
frames, real-solid-harmonic rotations, model bookkeeping, save/load) against
the oracle.  None of these calls touches the GPU."""
import os

import numpy as np
import pytest

from oracle import learned as L
import workloads as W

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1707_03771_amd", "libdfx.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdfx.so not built")

WATER = {8: [0, 0, 0, 1, 1, 2], 1: [0, 0, 1]}
RC = 8.0


def model():
    import paper_1707_03771_amd as dfx
    return dfx.GuessModel(WATER, rc=RC, rc_env=6.0, hidden=32, depth=2, seed=1)


@pytest.mark.parametrize("seed", [0, 3])
def test_descriptors_and_frames_match_oracle(seed):
    elems, xyz = W.water_cluster(side=2, seed=seed)
    Z = W.charges(elems)
    m = model()
    for a, b in L.samples(xyz, Z, RC):
        f, F = m.features(xyz, Z, a, b)
        fo, Fo = L.pair_features(xyz, Z, a, b, RC)
        assert f.shape == fo.shape
        np.testing.assert_allclose(f, fo, atol=1e-13, rtol=0)
        np.testing.assert_allclose(F, Fo, atol=1e-13, rtol=0)


def test_descriptors_of_mixed_elements():
    """C, H, O together (every channel populated), a linear fragment included."""
    rng = np.random.default_rng(4)
    xyz = rng.uniform(0, 7, size=(12, 3))
    xyz[1] = xyz[0] + np.array([0.0, 0.0, 2.0])
    xyz[2] = xyz[0] + np.array([0.0, 0.0, 4.1])
    Z = np.array([6, 6, 6, 1, 8, 1, 6, 8, 1, 1, 6, 1], np.int32)
    import paper_1707_03771_amd as dfx
    m = dfx.GuessModel({6: [0, 0, 1, 1, 2], 8: [0, 0, 0, 1, 1, 2], 1: [0, 0, 1]}, rc=RC)
    for a in range(len(Z)):
        for b in range(len(Z)):
            if a != b and np.linalg.norm(xyz[a] - xyz[b]) >= RC:
                continue
            f, F = m.features(xyz, Z, a, b)
            fo, Fo = L.pair_features(xyz, Z, a, b, RC)
            np.testing.assert_allclose(f, fo, atol=1e-13, rtol=0)
            np.testing.assert_allclose(F, Fo, atol=1e-13, rtol=0)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_sh_rotation_matches_oracle(l):
    import paper_1707_03771_amd as dfx
    for seed in range(4):
        q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
        if np.linalg.det(q) < 0:
            q[:, 0] *= -1
        np.testing.assert_allclose(dfx.sh_rotation(l, q), L.sh_rotation(l, q), atol=1e-13, rtol=0)


def test_types_and_sample_counts():
    elems, xyz = W.water_cluster(side=2, seed=1)
    Z = W.charges(elems)
    off, n = L.offsets(Z, WATER)
    m = model()
    m.add(xyz, Z, np.eye(n))
    got = {(t["atom"], t["Za"], t["Zb"]): t for t in m.types()}
    want = {}
    for a, b in L.samples(xyz, Z, RC):
        k = L.type_key(Z, a, b)
        key = (k[0] == "atom", k[1], k[-1])
        want[key] = want.get(key, 0) + 1
    assert {k: v["samples"] for k, v in got.items()} == want
    for (atom, za, zb), t in got.items():
        assert t["d_out"] == L.atom_nbf(WATER, za) * L.atom_nbf(WATER, zb)
        assert t["d_in"] == (3 + 3 * 8 * 9 if atom else 6 + 16 + 2 * 3 * 8 * 9)


def test_stored_samples_match_oracle():
    """Descriptors and local-frame target blocks the library stores for training
    equal the oracle's for the same (symmetric) density."""
    elems, xyz = W.water_cluster(side=2, seed=2)
    Z = W.charges(elems)
    _, n = L.offsets(Z, WATER)
    A = np.random.default_rng(1).normal(size=(n, n))
    P = A + A.T
    m = model()
    m.add(xyz, Z, P)
    ref = L.training_set([(xyz, Z, P)], WATER, RC)
    types = m.types()
    assert len(types) == len(ref)
    for t, ty in enumerate(types):
        key = ("atom", ty["Za"]) if ty["atom"] else ("pair", ty["Za"], ty["Zb"])
        X, T = m.samples(t)
        np.testing.assert_allclose(X, ref[key][0], atol=1e-13, rtol=0)
        np.testing.assert_allclose(T, ref[key][1], atol=1e-12, rtol=0)


def test_errors_are_status_codes(tmp_path):
    import paper_1707_03771_amd as dfx
    m = model()
    with pytest.raises(dfx.DfxError) as e:
        m.add(np.zeros((1, 3)), [7], np.zeros((1, 1)))     # nitrogen: no descriptor channel
    assert e.value.code == dfx.EUNSUPPORTED
    with pytest.raises(dfx.DfxError) as e:
        dfx.GuessModel({8: [0, 4]})                          # l = 4 orbital shell
    assert e.value.code == dfx.EUNSUPPORTED
    with pytest.raises(dfx.DfxError) as e:
        dfx.GuessModel.load(str(tmp_path / "missing.bin"))
    assert e.value.code == dfx.EINVAL
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a model file")
    with pytest.raises(dfx.DfxError):
        dfx.GuessModel.load(str(bad))


def test_import_save_load_round_trip(tmp_path):
    """Imported parameters survive save and load unchanged (no GPU involved)."""
    import paper_1707_03771_amd as dfx
    m = model()
    rng = np.random.default_rng(0)
    din, dout = 3 + 3 * 8 * 9, 14 * 14
    widths = [din, 32, 32, dout]
    npar = sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(3))
    th = rng.normal(size=npar).astype(np.float32)
    fm, fs, tm, ts = rng.normal(size=din), 1 + rng.random(din), rng.normal(size=dout), 1 + rng.random(dout)
    m.import_type(True, 8, 8, th, fm, fs, tm, ts)
    p = tmp_path / "m.bin"
    m.save(str(p))
    m2 = dfx.GuessModel.load(str(p))
    assert m2.types() == m.types()
    got = m2.export(0, widths)
    for x, y in zip(got, (th, fm, fs, tm, ts)):
        assert np.array_equal(x, y)


def test_stored_samples_do_not_depend_on_thread_count(monkeypatch):
    """The training samples are computed on a pool of host threads, one sample
    at a time each and stored in sample order: one thread and eight store the
    same descriptors and blocks, bit for bit, in the same order."""
    elems, xyz = W.water_cluster(side=3, seed=5)
    Z = W.charges(elems)
    _, n = L.offsets(Z, WATER)
    A = np.random.default_rng(2).normal(size=(n, n))
    P = A + A.T
    got = []
    for nt in ("1", "8"):
        monkeypatch.setenv("OMP_NUM_THREADS", nt)
        m = model()
        m.add(xyz, Z, P)
        got.append([m.samples(t) for t in range(len(m.types()))])
    assert len(got[0]) == len(got[1])
    for (X1, T1), (X8, T8) in zip(*got):
        assert X1.shape[0] > 16
        assert np.array_equal(X1, X8) and np.array_equal(T1, T8)
