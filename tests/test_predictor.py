"""Learned refinement predictor: library kernels against the CPU oracle.

Features are checked bitwise (same FP64 summation order, one rounding to FP32);
forward pass, loss and gradients against the FP64 oracle within FP32 rounding;
Adam over an epoch of three ragged batches; the partial refinement against the
oracle's refinement of marked blocks (topology bit-exact, values bitwise); the
guided step in its two limits against the plain step and against an unrefined
step; horizon labels against the oracle's definition.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp as OM

M = pytest.importorskip("paper_1902_00088_amd")


def _keyset(lv, co):
    return {(int(l),) + tuple(int(v) for v in c) for l, c in zip(lv, co)}


@pytest.mark.parametrize("dim,seed", [(2, s) for s in range(6)] + [(3, 10), (3, 11)])
def test_horizon_labels_match_oracle(dim, seed):
    """Host logic (no GPU): the library's labels equal the oracle's on random forests."""
    try:
        M.lib()
    except Exception as e:  # library not built
        pytest.skip(str(e))
    jmax = 5 if dim == 2 else 3
    a = W.random_graded_forest(dim, jmax, seed)
    b = W.random_graded_forest(dim, jmax, seed + 100)
    got = M.horizon_labels(dim, a[0], a[1], b[0], b[1])
    want = OM.horizon_labels(a[0], a[1], b[0], b[1], dim=dim)
    assert np.array_equal(got, want)
    assert set(np.unique(got)) <= {0, 1, 2}
    # against itself: everything is kept
    same = M.horizon_labels(dim, a[0], a[1], a[0], a[1])
    assert np.all(same == OM.KEEP)


# ---------------------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------------------

def _pair(cfg, nsteps):
    s = M.Solver(cfg)
    o = oracle.Oracle(cfg)
    s.init_grid()
    o.init_grid()
    t = 0.0
    for _ in range(nsteps):
        s.step(t, cfg.dt)
        o.step(t, cfg.dt)
        t += cfg.dt
    return s, o


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["C1", "C3"])
def test_features_bitwise_vs_oracle_pool(which):
    if which == "C1":
        cfg, n = W.C1(jmax=4), 6
    else:
        cfg, n = W.C3(jmax=4, eps=1e-4), 2
    s, o = _pair(cfg, n)
    lv, co = s.read_forest()
    lo, coo = o.read_forest()
    assert np.array_equal(lv, lo) and np.array_equal(co, coo)
    assert len(np.unique(lv)) > 1 or which == "C3"
    got = s.mlp_features()
    want = OM.pool_features(o.read_blocks(), cfg.bs, cfg.nf).astype(np.float32)
    print(which, "blocks", len(lv), "levels", np.unique(lv))
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    s.close()


def _model(nf, seed=5):
    nin = 64 * nf
    p = W.mlp_init_params(nin, seed)
    mean = np.linspace(-0.3, 0.4, nf).astype(np.float32)
    std = np.linspace(0.5, 2.0, nf).astype(np.float32)
    return nin, p, mean, std


def _inputs(n, nin, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((n, nin)) * 1.5 + 0.2).astype(np.float32)
    y = rng.integers(0, 3, n).astype(np.int8)
    return x, y


@pytest.mark.gpu
@pytest.mark.parametrize("nf,n", [(4, 300), (1, 1), (1, 97)])
def test_forward_loss_and_gradient_vs_oracle(nf, n):
    cfg = W.C3(jmax=3) if nf == 4 else W.C1(jmax=3)
    s = M.Solver(cfg)
    nin, p, mean, std = _model(nf)
    s.mlp_init(p, mean, std)
    x, y = _inputs(n, nin, 7)
    cw = W.class_weights(y).astype(np.float32)
    xn = OM.normalise(x.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), nf)
    z3, _ = OM.forward(p.astype(np.float64), xn, nin)
    got = s.mlp_forward(x)
    scale = max(1.0, float(np.abs(z3).max()))
    assert np.abs(got - z3).max() <= 1e-4 * scale, np.abs(got - z3).max()
    loss, g = s.mlp_grad(x, y, cw)
    lref, gref = OM.loss_and_grad(p.astype(np.float64), xn, y, cw.astype(np.float64), nin)
    assert abs(loss - lref) <= 1e-5 * max(1.0, abs(lref))
    err = np.abs(g - gref)
    gmax = float(np.abs(gref).max())
    assert np.linalg.norm(g - gref) <= 1e-4 * np.linalg.norm(gref)
    assert err.max() <= 1e-4 * gmax, (err.max(), gmax)
    # deterministic: the reduction order is fixed
    loss2, g2 = s.mlp_grad(x, y, cw)
    assert loss2 == loss and np.array_equal(g, g2)
    s.close()


@pytest.mark.gpu
def test_adam_epoch_vs_oracle():
    """Three ragged batches (1024, 1024, 452), one Adam step each."""
    cfg = W.C3(jmax=3)
    s = M.Solver(cfg)
    nin, p, mean, std = _model(4, seed=9)
    s.mlp_init(p, mean, std)
    x, y = _inputs(2500, nin, 8)
    cw = W.class_weights(y).astype(np.float32)
    lr = 1e-3
    mloss = s.mlp_train_epoch(x, y, cw, batch=1024, lr=lr)
    got = s.mlp_params()
    xn = OM.normalise(x.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), 4)
    q = p.astype(np.float64)
    opt = OM.Adam(len(q), lr=lr)
    well = np.ones(len(q), bool)
    losses = []
    for off in range(0, 2500, 1024):
        sl = slice(off, min(off + 1024, 2500))
        lb, gb = OM.loss_and_grad(q, xn[sl], y[sl], cw.astype(np.float64), nin)
        losses.append(lb)
        well &= np.abs(gb) >= 1e-3 * np.abs(gb).max()
        q = opt.step(q, gb)
    d = np.abs(got.astype(np.float64) - q)
    assert abs(mloss - np.mean(losses)) <= 1e-5 * max(1.0, abs(np.mean(losses)))
    assert well.sum() > 0.5 * len(q)
    assert d[well].max() <= 2e-3 * lr * 3, d[well].max()
    assert d.max() <= 2.0 * lr * 3 + 1e-6
    # Adam moves every well-conditioned parameter by about lr per step
    moved = np.abs(got.astype(np.float64) - p)
    assert np.median(moved[well]) > 0.5 * lr
    s.close()


@pytest.mark.gpu
def test_training_learns_a_teacher():
    """A seeded teacher MLP labels random inputs; the GPU training loop fits them."""
    cfg = W.C1(jmax=3)
    s = M.Solver(cfg)
    nin = 64
    teacher = W.mlp_init_params(nin, 21) * 4.0
    rng = np.random.default_rng(22)
    x = rng.standard_normal((4096, nin)).astype(np.float32)
    z3, _ = OM.forward(teacher.astype(np.float64), x.astype(np.float64), nin)
    y = np.argmax(z3, axis=1).astype(np.int8)
    from paper_1902_00088_amd import predictor as P
    losses = P.train(s, x, y, W.mlp_init_params(nin, 5), epochs=30, batch=256, lr=3e-3)
    cm, acc = P.evaluate(s, x, y)
    print("teacher fit: loss", losses[0], "->", losses[-1], "acc", acc)
    assert losses[-1] < 0.5 * losses[0]
    assert acc > 0.85
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("which,seed", [("C1", 0), ("C1", 1), ("C3", 2), ("C4", 3)])
def test_refine_marked_vs_oracle(which, seed):
    if which == "C4":
        # 3D: a random graded forest with sampled blob data (no time steps)
        cfg = W.C4(jmax=3)
        s, o = M.Solver(cfg), oracle.Oracle(cfg)
        o.init_forest(*W.random_graded_forest(3, 3, seed))
        lv, co = o.read_forest()
        s.init_forest(lv, co)
        data = W.sample(cfg, lv, co)
        s.load_blocks(data)
        o.load_blocks(data)
    else:
        cfg, n = (W.C1(jmax=5), 4) if which == "C1" else (W.C3(jmax=5, eps=1e-4), 1)
        s, o = _pair(cfg, n)
    nb = s.num_blocks()
    mask = (np.random.default_rng(seed).random(nb) < 0.2).astype(np.int8)
    k1 = s.refine_marked(mask)
    k2 = o.refine_marked(mask)
    print(which, "blocks", nb, "refined", k1)
    assert k1 == k2 and k1 > 0
    lv, co = s.read_forest()
    lo, coo = o.read_forest()
    assert np.array_equal(lv, lo) and np.array_equal(co, coo)
    assert np.array_equal(s.read_blocks(), o.read_blocks())
    if which == "C4":
        s.close()
        return
    # and the step after it
    s.rk4(0.0, cfg.dt)
    o.rk4(0.0, cfg.dt)
    s.adapt()
    o.adapt()
    assert np.array_equal(s.read_forest()[0], o.read_forest()[0])
    assert np.array_equal(s.read_blocks(), o.read_blocks())
    s.close()


def _constant_model(nf, b3):
    nin = 64 * nf
    p = np.zeros(OM.n_params(nin), np.float32)
    p[-3:] = b3
    return p, np.zeros(nf, np.float32), np.ones(nf, np.float32)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["refine", "unsure", "keep", "guard"])
def test_step_predicted_limits(mode):
    """Confident 'refine' everywhere, or probability below tau everywhere, is the plain
    step; confident 'keep' everywhere is RK4 on the unrefined grid plus adaptation;
    confident 'keep' with a detail guard refines exactly the blocks whose last detail
    maximum reaches guard x eps."""
    cfg = W.C1(jmax=5)
    s, o = _pair(cfg, 3)
    b3 = {"refine": (30.0, 0.0, 0.0), "unsure": (0.0, 0.0, 0.0), "keep": (0.0, 30.0, 0.0),
          "guard": (0.0, 30.0, 0.0)}[mode]
    guard = 0.05 if mode == "guard" else 0.0
    s.mlp_init(*_constant_model(1, b3))
    t = 3 * cfg.dt
    for _ in range(3):
        k = s.step_predicted(t, cfg.dt, 0.9, guard)
        if mode == "keep":
            assert k == 0
            o.rk4(t, cfg.dt)
            o.adapt()
        elif mode == "guard":
            _, md = o.mr_pass()
            mask = (md >= guard * cfg.eps).any(axis=1).astype(np.int8)
            assert 0 < mask.sum() < len(mask)
            assert o.refine_marked(mask) == k
            o.rk4(t, cfg.dt)
            o.adapt()
        else:
            o.step(t, cfg.dt)
        t += cfg.dt
        lv, co = s.read_forest()
        lo, coo = o.read_forest()
        assert np.array_equal(lv, lo) and np.array_equal(co, coo)
        assert np.array_equal(s.read_blocks(), o.read_blocks())
    s.close()


@pytest.mark.gpu
def test_predictor_errors():
    cfg = W.C1(jmax=3)
    s = M.Solver(cfg)
    s.init_grid()
    with pytest.raises(M.MrbError):
        s.mlp_predict()                 # no model yet
    p, m, sd = _constant_model(1, (0, 0, 0))
    with pytest.raises(M.MrbError):
        s.mlp_init(p, m, np.zeros(1, np.float32))   # std must be positive
    s.mlp_init(p, m, sd)
    x = np.zeros((4, 64), np.float32)
    with pytest.raises(M.MrbError):
        s.mlp_grad(x, np.array([0, 1, 3, 0], np.int8), np.ones(3, np.float32))
    pred, prob = s.mlp_predict()
    assert len(pred) == s.num_blocks() and np.allclose(prob, 1.0 / 3.0)
    s.close()
    c4 = M.Solver(W.C4(jmax=2))
    with pytest.raises(M.MrbError):
        c4.mlp_init(*_constant_model(1, (0, 0, 0)))   # 2D blocks only
    c4.close()


@pytest.mark.gpu
def test_guided_run_gain_on_advected_blob():
    """Record 1000 plain steps of the advected blob (Jmax 6, eps 1e-4), train on the
    first 800, guide a rerun from the same grid with a shadow plain step every 10 steps: fewer
    block updates than the plain method, solution within 10 eps of the plain one."""
    from paper_1902_00088_amd import predictor as P
    cfg = W.C1(jmax=6, eps=1e-4)
    s = M.Solver(cfg)
    s.init_grid()
    r = P.gain_study(s, W.mlp_init_params(64, 5), nsteps=1000, shadow_every=10)
    print({k: r[k] for k in ("labels_train", "test_accuracy", "block_updates_saved", "rel_err_vs_plain")},
          r["guided"])
    assert r["labels_train"][0] > 0 and r["labels_train"][2] > 0     # all three classes occur
    assert r["loss_first_last"][1] < r["loss_first_last"][0]
    assert r["block_updates_saved"] > 0.1
    assert r["guided"]["mispredicted_steps"] <= 0.1 * r["guided"]["shadowed"]
    assert r["within_bound"], r["rel_err_vs_plain"]
    s.close()
