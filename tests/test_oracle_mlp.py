"""Pins of the predictor oracle (oracle/mlp.py): closed forms and finite differences."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mlp as O


def test_gelu_values_and_derivative():
    # GELU(x) = x * Phi(x): Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert abs(O.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert O.gelu(np.array([0.0]))[0] == 0.0
    assert abs(O.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(O.gelu(np.array([-10.0]))[0]) < 1e-12
    z = np.linspace(-4, 4, 33)
    h = 1e-6
    fd = (O.gelu(z + h) - O.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - O.gelu_grad(z))) < 1e-8


def _problem(nin=16, n=12, seed=0):
    rng = np.random.default_rng(seed)
    p = W.mlp_init_params(nin, seed).astype(np.float64)
    x = rng.normal(size=(n, nin))
    y = rng.integers(0, 3, n)
    cw = np.array([2.0, 0.5, 1.5])
    return p, x, y, cw


def test_gradient_matches_central_differences():
    nin = 16
    p, x, y, cw = _problem(nin)
    loss, g = O.loss_and_grad(p, x, y, cw, nin)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(p), 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (O.loss_and_grad(p + e, x, y, cw, nin)[0] - O.loss_and_grad(p - e, x, y, cw, nin)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_softmax_ce_identities():
    """Sum over classes of dL/dz is zero per sample, so the output-bias gradient sums to zero;
    equal logits give loss log(3)."""
    nin = 16
    p, x, y, cw = _problem(nin)
    _, g = O.loss_and_grad(p, x, y, cw, nin)
    db3 = g[-3:]
    assert abs(db3.sum()) < 1e-15
    p0 = p.copy()
    p0[-3 - 64 * 3:] = 0.0  # W3 = 0, b3 = 0 -> uniform softmax
    loss, _ = O.loss_and_grad(p0, x, y, cw, nin)
    assert abs(loss - math.log(3.0)) < 1e-14


def test_adam_first_step_closed_form():
    """After one step the bias-corrected moments are g and g^2, so the update is
    -lr g / (|g| + eps): about lr times the sign of the gradient."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = O.Adam(50, lr=1e-3)
    p1 = opt.step(p, g)
    want = -1e-3 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs((p1 - p) - want)) < 1e-15
    assert np.all(np.sign(p1 - p) == -np.sign(g))


def test_pooling_is_exact_for_linear_data():
    bs = 33
    a, b, c = 0.3, -1.2, 0.7
    i = np.arange(bs)
    X, Y = np.meshgrid(i, i)
    blk = (a + b * X + c * Y).reshape(1, 1, -1)
    f = O.pool_features(blk, bs, 1)
    w = (bs - 1) // 8
    for by in range(8):
        for bx in range(8):
            cx = bx * w + (w - 1) / 2
            cy = by * w + (w - 1) / 2
            assert abs(f[0, by * 8 + bx] - (a + b * cx + c * cy)) < 1e-12


def test_horizon_labels_by_construction():
    now_l = np.array([2, 2, 2, 2, 1, 1, 1], np.int8)
    now_c = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [1, 0], [0, 1], [1, 1]], np.int32)
    # later: first family merged to level 1; block (1,0) of level 1 refined; others unchanged
    lat_l = np.array([1] + [2, 2, 2, 2] + [1, 1], np.int8)
    lat_c = np.array([[0, 0], [2, 0], [3, 0], [2, 1], [3, 1], [0, 1], [1, 1]], np.int32)
    lab = O.horizon_labels(now_l, now_c, lat_l, lat_c)
    assert list(lab) == [O.COARSEN] * 4 + [O.REFINE, O.KEEP, O.KEEP]
