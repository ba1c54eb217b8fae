"""GPU tests of the learned starting guess through the C-ABI.

* MLP kernels (FP32) against the oracle's FP64 network on the same FP32
  weights and batch.  Tolerances from FP32 arithmetic: a dot product of
  length n carries a relative error of about sqrt(n) * 6e-8 per layer, so
  1e-5 (forward, norm-wise), 1e-4 (gradient, norm-wise) and 1e-6 lr (Adam).
* The whole prediction (descriptors -> network -> rotation -> assembly) with
  seeded imported weights against the oracle's predict; |dD| <= 1e-4.
* Equivariance, training, save/load, the iteration gain over the core guess
  at the same energy, and both fallbacks to the core guess.
"""
import numpy as np
import pytest

from oracle import learned as L
import workloads as W

pytestmark = pytest.mark.gpu

WATER = {8: [0, 0, 0, 1, 1, 2], 1: [0, 0, 1]}
RC = 8.0


def dev(x, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype or torch.float32, device="cuda")


def widths_cases():
    return [([13, 70, 33, 5], 37), ([454, 256, 256, 256, 196], 300), ([7, 3], 1), ([219, 256, 256, 256, 25], 65)]


def seeded_net(widths, seed):
    rng = np.random.default_rng(seed)
    th = L.init_params(widths, seed) + 0.01 * rng.normal(size=sum(
        widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1)))
    return th.astype(np.float32)


@pytest.mark.parametrize("widths,batch", widths_cases())
def test_mlp_forward_matches_oracle(widths, batch):
    import paper_1707_03771_amd as dfx
    rng = np.random.default_rng(1)
    th = seeded_net(widths, 2)
    X = rng.normal(size=(batch, widths[0])).astype(np.float32)
    Y = dfx.mlp_forward(widths, dev(th), dev(X)).cpu().numpy()
    Yo, _ = L.forward(th.astype(np.float64), widths, X.astype(np.float64))
    assert np.linalg.norm(Y - Yo) <= 1e-5 * np.linalg.norm(Yo)


@pytest.mark.parametrize("widths,batch", widths_cases())
def test_mlp_gradient_matches_oracle(widths, batch):
    import paper_1707_03771_amd as dfx
    rng = np.random.default_rng(3)
    th = seeded_net(widths, 4)
    X = rng.normal(size=(batch, widths[0])).astype(np.float32)
    T = rng.normal(size=(batch, widths[-1])).astype(np.float32)
    loss, g = dfx.mlp_loss_grad(widths, dev(th), dev(X), dev(T))
    lo, go = L.loss_and_grad(th.astype(np.float64), widths, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * lo
    g = g.cpu().numpy()
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    # every layer on its own, so that a small layer's error is not hidden
    o = 0
    for i in range(len(widths) - 1):
        k = widths[i] * widths[i + 1] + widths[i + 1]
        assert np.linalg.norm(g[o:o + k] - go[o:o + k]) <= 1e-4 * np.linalg.norm(go[o:o + k]) + 1e-12
        o += k


def test_mlp_adam_matches_oracle():
    import paper_1707_03771_amd as dfx
    rng = np.random.default_rng(5)
    n = 100003
    th = rng.normal(size=n).astype(np.float32)
    t, m, v = dev(th), dev(np.zeros(n)), dev(np.zeros(n))
    tho, mo, vo = th.astype(np.float64), np.zeros(n), np.zeros(n)
    lr = 1e-3
    for step in range(1, 4):
        g = (rng.normal(size=n) * 10 ** rng.uniform(-2, 0, size=n)).astype(np.float32)
        dfx.mlp_adam(t, dev(g), m, v, step, lr)
        tho, mo, vo = L.adam(tho, g.astype(np.float64), mo, vo, step, lr=lr)
    # compare the change, so that the FP32 rounding of theta itself does not count
    dt = t.cpu().numpy().astype(np.float64) - th.astype(np.float64)
    assert np.abs(dt - (tho - th.astype(np.float64))).max() <= 1e-6 * lr * 3 + 2 * np.spacing(np.abs(th)).max()


def test_mlp_argument_errors():
    import paper_1707_03771_amd as dfx
    import ctypes
    w = np.array([3, 2], np.int32)
    assert dfx._lib.dfx_mlp_forward(w.ctypes.data, 1, None, None, 4, None, None) == dfx.EINVAL
    assert dfx._lib.dfx_mlp_adam(None, None, None, None, 0, 1, ctypes.c_float(1e-3), None) == dfx.EINVAL


# ---- the whole prediction with seeded weights --------------------------------------

def seeded_model(dfx, Z, xyz, seed=0, hidden=256, depth=3):
    m = dfx.GuessModel(WATER, rc=RC, rc_env=6.0, hidden=hidden, depth=depth, seed=seed)
    nets = {}
    rng = np.random.default_rng(seed)
    for a, b in L.samples(xyz, Z, RC):
        k = L.type_key(Z, a, b)
        if k in nets:
            continue
        din = len(L.pair_features(xyz, Z, a, b, RC)[0])
        dout = L.atom_nbf(WATER, Z[a]) * L.atom_nbf(WATER, Z[b])
        widths = [din] + [hidden] * depth + [dout]
        th = seeded_net(widths, seed + 17 * len(nets))
        fm, fs = rng.normal(size=din) * 0.1, 0.5 + rng.random(din)
        tm, ts = rng.normal(size=dout) * 0.05, 0.05 + 0.1 * rng.random(dout)
        m.import_type(k[0] == "atom", k[1], k[-1], th, fm, fs, tm, ts)
        nets[k] = (widths, th.astype(np.float64), fm, fs, tm, ts)
    return m, nets


def test_prediction_matches_oracle():
    import paper_1707_03771_amd as dfx
    elems, xyz = W.water_cluster(side=2, seed=7)
    Z = W.charges(elems)
    _, n = L.offsets(Z, WATER)
    m, nets = seeded_model(dfx, Z, xyz)
    D = m.predict(xyz, Z, n)
    Do = L.predict(nets, xyz, Z, WATER, RC)
    assert np.abs(D - D.T).max() == 0.0
    assert np.abs(D - Do).max() <= 1e-4, np.abs(D - Do).max()


def test_prediction_equivariance_on_gpu():
    import paper_1707_03771_amd as dfx
    elems, xyz = W.water_cluster(side=2, seed=9)
    Z = W.charges(elems)
    _, n = L.offsets(Z, WATER)
    m, _ = seeded_model(dfx, Z, xyz, seed=3)
    q, r = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))
    R = q if np.linalg.det(q) > 0 else -q
    D = m.predict(xyz, Z, n)
    D2 = m.predict(xyz @ R.T + np.array([0.2, -1.0, 3.0]), Z, n)
    U = L.basis_rotation(Z, WATER, R)
    assert np.abs(D2 - U.T @ D @ U).max() <= 1e-5


# ---- training, the gain over the core guess and the fallbacks ----------------------

def water_system(seed, side=2):
    elems, xyz = W.water_cluster(side=side, seed=seed)
    shells, aux = W.basis_for("water", elems, xyz)
    return W.charges(elems), xyz, shells, aux


def converged(dfx, Z, xyz, shells, aux):
    E, C, eps, info = dfx.scf(xyz, Z, shells, aux)
    assert info["converged"]
    nocc = info["nocc"]
    return E, C[:, :nocc] @ C[:, :nocc].T, info


def test_lowdin_matches_oracle():
    """P = S^1/2 D S^1/2 on the GPU against the oracle's overlap and eigh; D has
    entries of a few hundred here, P entries below one: |dP| <= 1e-9."""
    import oracle as O
    import paper_1707_03771_amd as dfx
    Z, xyz, sh, ax = water_system(4)
    E, D, info = converged(dfx, Z, xyz, sh, ax)
    P = dfx.lowdin(xyz, Z, sh, D)
    S, _, _ = O.int1e(O.Basis(sh), xyz, Z)
    Po = L.lowdin(S, D)
    assert np.abs(P - Po).max() <= 1e-9, np.abs(P - Po).max()
    assert abs(np.trace(P) - info["nocc"]) <= 1e-8
    assert np.abs(P @ P - P).max() <= 1e-8


@pytest.fixture(scope="module")
def trained(tmp_path_factory):
    import paper_1707_03771_amd as dfx
    m = dfx.GuessModel(WATER, rc=RC, rc_env=6.0, hidden=256, depth=3, seed=11)
    for seed in range(1, 13):
        Z, xyz, sh, ax = water_system(seed)
        _, D, _ = converged(dfx, Z, xyz, sh, ax)
        m.add(xyz, Z, dfx.lowdin(xyz, Z, sh, D))
    loss = m.train(epochs=150, batch=32, lr=1e-3)
    return m, loss


def test_training_reduces_loss(trained):
    _, loss = trained
    print("loss per epoch (first, 10th, last):", loss[0], loss[9], loss[-1])
    assert np.all(np.isfinite(loss))
    assert loss[-1] < 0.05 * loss[0]


def test_saved_model_predicts_bitwise_identically(trained, tmp_path):
    import paper_1707_03771_amd as dfx
    m, _ = trained
    Z, xyz, _, _ = water_system(101)
    _, n = L.offsets(Z, WATER)
    p = tmp_path / "water.dfxg"
    m.save(str(p))
    m2 = dfx.GuessModel.load(str(p))
    assert np.array_equal(m.predict(xyz, Z, n), m2.predict(xyz, Z, n))


def test_learned_guess_gain(trained):
    """Unseen geometries: fewer iterations than the core guess, same energy."""
    import paper_1707_03771_amd as dfx
    m, _ = trained
    it_core, it_learn = [], []
    for seed in (101, 102, 103):
        Z, xyz, sh, ax = water_system(seed)
        E0, D0, i0 = converged(dfx, Z, xyz, sh, ax)
        E1, C1, _, i1 = dfx.scf(xyz, Z, sh, ax, model=m)
        assert i1["converged"] and i1["guess_fallback"] == 0
        assert abs(E1 - E0) <= 1e-8, (seed, E1 - E0)
        # the learned start's first energy is nearer the converged one than the core start's
        assert abs(i1["E_hist"][0] - E0) < abs(i0["E_hist"][0] - E0)
        print(f"seed {seed}: first-iteration error core {i0['E_hist'][0] - E0:.3e}, "
              f"learned {i1['E_hist'][0] - E0:.3e}; t_guess {i1['t_guess'] * 1e3:.1f} ms")
        it_core.append(i0["niter"])
        it_learn.append(i1["niter"])
    print("iterations core:", it_core, "learned:", it_learn)
    assert sum(it_learn) <= 0.75 * sum(it_core)


def test_non_finite_prediction_falls_back_to_core():
    import paper_1707_03771_amd as dfx
    Z, xyz, sh, ax = water_system(5)
    m, nets = seeded_model(dfx, Z, xyz, seed=1, hidden=16, depth=1)
    widths, th, fm, fs, tm, ts = nets[("atom", 8)]
    bad = th.astype(np.float32)
    bad[3] = np.nan
    m.import_type(True, 8, 8, bad, fm, fs, tm, ts)
    E0, _, i0 = converged(dfx, Z, xyz, sh, ax)
    E1, _, _, i1 = dfx.scf(xyz, Z, sh, ax, model=m)
    assert i1["guess_fallback"] == 1 and i1["converged"]
    assert E1 == E0 and i1["niter"] == i0["niter"]


def test_unconverged_learned_start_restarts_from_core():
    import paper_1707_03771_amd as dfx
    Z, xyz, sh, ax = water_system(5)
    m, _ = seeded_model(dfx, Z, xyz, seed=1, hidden=16, depth=1)
    E, C, eps, info = dfx.scf(xyz, Z, sh, ax, model=m, max_iter=2)
    assert info["status"] == dfx.ENOCONV and info["guess_fallback"] == 2
    assert info["niter"] == 4 and len(info["E_hist"]) == 4


def test_learned_guess_checks_the_basis():
    import paper_1707_03771_amd as dfx
    Z, xyz, sh, ax = water_system(5)
    m, _ = seeded_model(dfx, Z, xyz, seed=1, hidden=16, depth=1)
    with pytest.raises(dfx.DfxError) as e:
        dfx.scf(xyz, Z, sh[:-1], ax, model=m)
    assert e.value.code == dfx.EINVAL
