"""Pins of the oracle's learned-R parts (CPU only): the feature definition and
the FP64 network reference (bf16 rounding, GELU, analytic gradient)."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.mlp as M


def test_features_of_a_constructed_grid():
    # 7 x 7 grid of unit cells over [0, 7)^2 (cell width 1); data placed at cell centres with
    # chosen multiplicities; the query sits in cell (col 3, row 2).
    mult = {(3, 2): 4, (1, 0): 2, (5, 4): 1, (6, 2): 3, (3, 4): 5, (2, 1): 1}
    xs, ys = [], []
    for (c, r), k in mult.items():
        xs += [c + 0.5] * k
        ys += [r + 0.5] * k
    xs += [0.0, 7.0 - 2 ** -20]  # corner points pin the bounds to [0, 7)
    ys += [0.0, 7.0 - 2 ** -20]
    x = np.array(xs, np.float32)
    y = np.array(ys, np.float32)
    n, ncells = x.size, 49
    f = O.features(x, y, [3.25], [2.75], 0.0, 0.0, 1.0, 7, 7)[0]
    grid = np.zeros((7, 7))  # [row, col]
    for (c, r), k in mult.items():
        grid[r, c] += k
    grid[0, 0] += 1
    grid[6, 6] += 1
    expect = np.zeros((5, 5))
    for dr in range(-2, 3):
        for dc in range(-2, 3):
            r, c = 2 + dr, 3 + dc
            expect[dr + 2, dc + 2] = grid[r, c] if 0 <= r < 7 and 0 <= c < 7 else 0
    assert np.allclose(f[:25].reshape(5, 5), expect * ncells / n, rtol=1e-7)
    # (3, 2) itself is the centre, (6, 2) is outside the window (column offset +3)
    assert f[12] == pytest.approx(4 * ncells / n, rel=1e-7)
    assert f[25] == 0.25 and f[26] == 0.75


def test_features_window_clipping_and_total():
    # a 3 x 3 grid: the window around the centre cell covers every cell, so the counts sum to n;
    # from a corner cell, the cells beyond the grid contribute 0
    rng = np.random.default_rng(3)
    x = rng.random(500).astype(np.float32) * np.float32(3)
    y = rng.random(500).astype(np.float32) * np.float32(3)
    f = O.features(x, y, [1.5, 0.2], [1.5, 0.2], 0.0, 0.0, 1.0, 3, 3)
    assert f[0, :25].sum() * 500 / 9 == pytest.approx(500, rel=1e-6)
    window = f[1, :25].reshape(5, 5)
    assert np.all(window[:2, :] == 0) and np.all(window[:, :2] == 0)
    assert f[1, 25] == pytest.approx(0.2, abs=1e-7) and f[1, 26] == pytest.approx(0.2, abs=1e-7)


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 2 ** -7, 1 + 3 * 2 ** -8, -2.5, 3.0e-3, 65504.0])
    r = M.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0            # tie -> even
    assert r[2] == 1 + 2 ** -7                    # representable
    assert r[3] == 1 + 2 ** -6                    # tie -> even (mantissa 2)
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert r[6] == 65536.0


def test_gelu():
    assert M.gelu(0.0) == 0.0
    assert M.gelu(10.0) == pytest.approx(10.0, rel=1e-12)
    assert abs(M.gelu(-10.0)) < 1e-12
    u = np.linspace(-4, 4, 81)
    h = 1e-6
    assert np.allclose(M.gelu_grad(u), (M.gelu(u + h) - M.gelu(u - h)) / (2 * h), rtol=1e-7, atol=1e-9)
    # value at 1 by hand: 0.5 (1 + tanh(sqrt(2/pi) * 1.044715))
    assert M.gelu(1.0) == pytest.approx(0.5 * (1 + math.tanh(math.sqrt(2 / math.pi) * 1.044715)), rel=1e-15)


def test_forward_closed_form():
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    d["W1"][0, 0] = 1.0
    d["W2"][0, 0] = 1.0
    d["W3"][0] = 1.0
    d["b3"][0] = 0.25
    feat = np.zeros((2, 27))
    feat[0, 0] = 1.0
    feat[1, 0] = -0.5
    y, _ = M.forward(M.pack(d), feat, rounding=False)
    assert y[0] == pytest.approx(M.gelu(M.gelu(1.0)) + 0.25, rel=1e-15)
    assert y[1] == pytest.approx(M.gelu(M.gelu(-0.5)) + 0.25, rel=1e-15)
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    d["b3"][0] = 1.5
    y, _ = M.forward(M.pack(d), feat)
    assert np.all(y == 1.5)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    params = rng.standard_normal(M.N_PARAMS) * 0.3
    feat = rng.random((5, 27)) * 2
    target = rng.random(5) * 3
    loss, g = M.loss_and_grad(params, feat, target, rounding=False)
    h = 1e-6
    fd = np.empty_like(g)
    for i in range(M.N_PARAMS):
        p1 = params.copy()
        p1[i] += h
        p2 = params.copy()
        p2[i] -= h
        l1 = np.mean((M.forward(p1, feat, False)[0] - target) ** 2)
        l2 = np.mean((M.forward(p2, feat, False)[0] - target) ** 2)
        fd[i] = (l1 - l2) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-8)
    assert loss == pytest.approx(np.mean((M.forward(params, feat, False)[0] - target) ** 2))
