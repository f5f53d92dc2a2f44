"""Pins of the oracle MLP: closed forms, the paper's printed parameter totals,
finite differences of the hand-derived backward, and Adam closed forms."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mlp

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))


def test_param_counts_reproduce_paper_totals():
    for name, v in GOLDEN["param_totals"].items():
        if name.startswith("_"):
            continue
        total = v["experts"] * sum(mlp.param_count(*n) for n in v["nets"])
        assert total == v["total"], name
    # memory table: 4 experts of 512->128x3->1 and 256->64x3->1
    assert 4 * mlp.param_count(512, 128, 3, 1) == GOLDEN["memory_cost"]["nn4_voxel_params"]
    assert 4 * mlp.param_count(256, 64, 3, 1) == GOLDEN["memory_cost"]["nn4_l1_params"]


def test_param_count_matches_layer_shapes():
    for K, W, H, c in [(36, 64, 3, 1), (128, 128, 4, 1), (128, 64, 4, 3)]:
        n = sum(o * i + o for o, i in mlp.layer_shapes(K, W, H, c))
        assert n == mlp.param_count(K, W, H, c)
    assert mlp.param_count(36, 64, 3, 1) == 10753
    assert mlp.param_count(128, 128, 4, 1) == 66177
    assert mlp.param_count(128, 64, 4, 3) == 20931


def test_encoding_closed_forms():
    B = np.random.default_rng(0).standard_normal((64, 3)) * 10
    z = mlp.encode(np.zeros((2, 3)), B)
    assert np.array_equal(z, np.concatenate([np.ones((2, 64)), np.zeros((2, 64))], axis=1))
    z = mlp.encode(np.random.default_rng(1).random((5, 3)), np.zeros((8, 3)))
    assert np.array_equal(z, np.concatenate([np.ones((5, 8)), np.zeros((5, 8))], axis=1))
    # PE: cos/sin(2^k pi x_d); at x_d = 1/2: sin -> 1, 0, 0, ...; cos -> 0, -1, 1, 1, ...
    P = mlp.pe_matrix(6)
    z = mlp.encode(np.full((1, 3), 0.5), P)[0]
    cos, sin = z[:18].reshape(6, 3), z[18:].reshape(6, 3)
    assert np.allclose(sin[:, 0], [1, 0, 0, 0, 0, 0], atol=1e-12)
    assert np.allclose(cos[:, 1], [0, -1, 1, 1, 1, 1], atol=1e-12)
    x = np.array([[0.3, 0.7, 0.1]])
    z = mlp.encode(x, P)[0]
    for k in range(6):
        for d in range(3):
            assert math.isclose(z[3 * k + d], math.cos(2 ** k * math.pi * x[0, d]), abs_tol=1e-12)
            assert math.isclose(z[18 + 3 * k + d], math.sin(2 ** k * math.pi * x[0, d]), abs_tol=1e-12)


def test_forward_closed_forms():
    shapes = mlp.layer_shapes(4, 3, 2, 2)
    params = [(np.zeros(s), np.zeros(s[0])) for s in shapes]
    params[-1] = (np.zeros(shapes[-1]), np.array([0.25, -2.0]))
    y, _ = mlp.forward(params, np.random.default_rng(0).random((7, 4)))
    assert np.array_equal(y, np.tile([0.25, -2.0], (7, 1)))
    # one active ReLU path: y = 3 * relu(2 * z0 + 1) - 1 with everything else zero
    params = [(np.zeros(s), np.zeros(s[0])) for s in shapes]
    params[0][0][1, 2] = 2.0; params[0][1][1] = 1.0
    params[1][0][0, 1] = 1.0
    params[2][0][1, 0] = 3.0; params[2][1][1] = -1.0
    z0 = np.zeros((3, 4)); z0[:, 2] = [-2.0, 0.0, 0.75]
    y, _ = mlp.forward(params, z0)
    assert np.allclose(y[:, 1], 3 * np.maximum(2 * z0[:, 2] + 1, 0) - 1)
    assert np.array_equal(y[:, 0], np.zeros(3))


def test_forward_sin_special_values():
    """sin(omega z) on every hidden layer, the head linear (omega = 1.5): one active
    path y = 3 act(act(2 z0 + 1)) - 1 at inputs where the phases are known: a zero
    pre-activation, omega z = pi / 2 (activation 1), omega z = pi (activation 0,
    where cos would give -1 and an unscaled sine sin(z) would not vanish)."""
    w = 1.5
    shapes = mlp.layer_shapes(4, 3, 2, 2, omega=w)
    params = mlp.unflatten(np.zeros(mlp.param_count(4, 3, 2, 2)), shapes)
    assert params.omega == w
    params[0][0][1, 2] = 2.0; params[0][1][1] = 1.0
    params[1][0][0, 1] = 1.0
    params[2][0][1, 0] = 3.0; params[2][1][1] = -1.0
    z0 = np.zeros((3, 4))
    z0[:, 2] = [-0.5, (math.pi / (2 * w) - 1) / 2, (math.pi / w - 1) / 2]
    y, cache = mlp.forward(params, z0)
    assert np.allclose(cache[2][:, 1], [0.0, 1.0, 0.0], atol=1e-15)
    assert np.allclose(y[:, 1], [-1.0, 3 * math.sin(w * 1.0) - 1, -1.0], atol=1e-14)
    assert np.allclose(y[:, 0], 0.0)   # the other output sees only zero weights and biases
    # zero weights leave every hidden value at sin(omega b) of its bias
    params = mlp.unflatten(np.zeros(mlp.param_count(4, 3, 2, 2)), shapes)
    params[0][1][:] = [0.0, 1.0, -2.0]
    _, cache = mlp.forward(params, z0)
    assert np.allclose(cache[2][0], [0.0, math.sin(1.5), math.sin(-3.0)], atol=1e-15)


def test_loss_special_values():
    assert math.isclose(mlp.loss_bce(np.zeros(5), np.array([0, 1, 1, 0, 1])), math.log(2))
    assert math.isclose(mlp.loss_ce(np.zeros((4, 3)), np.array([0, 1, 2, 2])), math.log(3))
    t = np.array([0.5, -1.0, 0.25])
    assert math.isclose(mlp.loss_mse(np.zeros(3), t), float(np.mean(t * t)))
    # large logits stay finite and approach the hinge
    assert math.isclose(mlp.loss_bce(np.array([800.0]), np.array([0.0])), 800.0)
    assert mlp.loss_bce(np.array([-800.0]), np.array([0.0])) < 1e-300 + 1e-12


@pytest.mark.parametrize("kind,c", [("mse", 1), ("bce", 1), ("ce", 3)])
def test_output_grad_finite_differences(kind, c):
    rng = np.random.default_rng(3)
    y = rng.standard_normal((6, c))
    t = rng.standard_normal(6) if kind == "mse" else (rng.integers(0, 2, 6) if kind == "bce" else rng.integers(0, 3, 6))
    g = mlp.output_grad(kind, y, t)
    h = 1e-6
    for i in range(6):
        for j in range(c):
            yp, ym = y.copy(), y.copy()
            yp[i, j] += h; ym[i, j] -= h
            fd = (mlp.loss(kind, yp, t) - mlp.loss(kind, ym, t)) / (2 * h)
            assert abs(fd - g[i, j]) < 1e-8


def _fd_check(K, W, H, c, kind, h, seed, omega=0.0):
    rng = np.random.default_rng(seed)
    shapes = mlp.layer_shapes(K, W, H, c, omega=omega)
    theta = rng.standard_normal(mlp.param_count(K, W, H, c)) * 0.5
    z0 = rng.standard_normal((32, K))
    t = rng.standard_normal(32) if kind == "mse" else rng.integers(0, c if kind == "ce" else 2, 32)

    def f(th):
        y, _ = mlp.forward(mlp.unflatten(th, shapes), z0)
        return mlp.loss(kind, y, t)

    def pre_acts(th):
        _, cache = mlp.forward(mlp.unflatten(th, shapes), z0)
        return [cache[i] > 0 for i in range(1, len(cache), 2)]

    params = mlp.unflatten(theta, shapes)
    y, cache = mlp.forward(params, z0)
    g = mlp.flatten(mlp.backward(params, cache, mlp.output_grad(kind, y, t)))
    idx = rng.choice(len(theta), size=64, replace=False)
    errs, kinks = [], 0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h; tm[i] -= h
        if any(np.any(a != b) for a, b in zip(pre_acts(tp), pre_acts(tm))):
            kinks += 1          # a ReLU flips between theta +- h: the difference quotient is not a derivative
            continue
        fd = (f(tp) - f(tm)) / (2 * h)
        errs.append(abs(fd - g[i]) / max(abs(g[i]), 1e-8))
    return np.array(errs), kinks


@pytest.mark.parametrize("K,W,H,c,kind", [(12, 8, 3, 1, "mse"), (10, 6, 2, 1, "bce"), (9, 7, 3, 3, "ce")])
def test_backward_finite_differences(K, W, H, c, kind):
    errs, kinks = _fd_check(K, W, H, c, kind, 1e-5, 11)
    assert len(errs) >= 48
    assert np.median(errs) < 1e-7 and np.max(errs) < 1e-4
    errs, kinks = _fd_check(K, W, H, c, kind, 1e-3, 12)
    assert np.median(errs) < 1e-5


@pytest.mark.parametrize("omega", [1.5, 3.0])
def test_backward_finite_differences_sin(omega):
    """The sin activation is smooth: every sampled weight's central difference
    matches the hand-derived gradient (omega cos(omega z) per hidden layer)."""
    errs, kinks = _fd_check(12, 8, 3, 1, "mse", 1e-5, 13, omega=omega)
    assert kinks == 0 and len(errs) == 64
    assert np.median(errs) < 1e-7 and np.max(errs) < 1e-4


def test_adam_first_step_and_constant_gradient():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 1e-3)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(th[:2], [-1e-3, 1e-3], atol=1e-12)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    theta, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    expect = np.zeros(4)
    for s in range(1, 251):
        lr = mlp.lr_at(s, 1e-3)
        theta, m, v = mlp.adam_step(theta, g, m, v, s, lr)
        expect -= lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(theta, expect, rtol=1e-9, atol=1e-15)


def test_lr_staircase():
    assert mlp.lr_at(1, 1e-3) == 1e-3
    assert mlp.lr_at(100, 1e-3) == 1e-3
    assert math.isclose(mlp.lr_at(101, 1e-3), 0.975e-3)
    assert math.isclose(mlp.lr_at(2000, 1e-3), 1e-3 * 0.975 ** 19)


def test_flatten_roundtrip():
    shapes = mlp.layer_shapes(36, 64, 3, 1)
    th = np.arange(mlp.param_count(36, 64, 3, 1), dtype=np.float64)
    p = mlp.unflatten(th, shapes)
    assert p[0][0][1, 0] == 36 and p[0][1][0] == 36 * 64
    assert np.array_equal(mlp.flatten(p), th)
