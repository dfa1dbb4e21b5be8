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


# ---------------------------------------------------------------- float32 output model

def _f32_network(params, feat, order="forward", plant=None):
    """An independent float32 evaluation of the network: sequential float32 sums in the given
    input order, the GELU as u - u / (1 + 2^z) in float32, bf16 rounding of the float32 values.
    plant names a deliberate mistake (for the pins that the model has teeth)."""
    f32 = np.float32
    P = M.unpack(params)
    W1 = M.bf16(P["W1"]).astype(f32)
    W2 = M.bf16(P["W2"]).astype(f32)
    W3 = M.bf16(P["W3"]).astype(f32)
    b1, b2 = P["b1"].astype(f32), P["b2"].astype(f32)
    b3 = f32(P["b3"][0])
    if plant == "drop_b2":
        b2 = np.zeros_like(b2)
    if plant == "transpose_w2":
        W2 = np.ascontiguousarray(W2.T)
    x = M.bf16(feat).astype(f32)
    k1 = f32(2.0 * np.sqrt(2.0 / np.pi) / np.log(2.0))
    k2 = f32(2.0 * np.sqrt(2.0 / np.pi) * 0.044715 / np.log(2.0))

    def dense(inp, W, b):
        n = inp.shape[1]
        idx = {"forward": range(n), "reversed": range(n - 1, -1, -1),
               "strided": list(range(0, n, 2)) + list(range(1, n, 2))}[order]
        acc = np.broadcast_to(b, (inp.shape[0], W.shape[0])).astype(f32).copy()
        for i in idx:
            acc = (acc + (inp[:, i][:, None] * W[:, i][None, :]).astype(f32)).astype(f32)
        return acc

    def gelu32(a):
        z = (a * (k1 + k2 * (a * a).astype(f32)).astype(f32)).astype(f32)
        with np.errstate(over="ignore"):
            e = np.exp2(z).astype(f32)
        r = (f32(1.0) / (e + f32(1.0)).astype(f32)).astype(f32)
        g = (a - (a * r).astype(f32)).astype(f32)
        if plant == "gelu_sign":
            g = (a + (a * r).astype(f32)).astype(f32)
        return M.bf16(g.astype(np.float64)).astype(f32)

    h1 = gelu32(dense(x, W1, b1))
    h2 = gelu32(dense(h1, W2, b2))
    return dense(h2, W3[None, :], np.array([b3], f32))[:, 0].astype(np.float64)


def _features(seed, B, grid_offsets):
    rng = np.random.default_rng(seed)
    f = np.zeros((B, 27))
    f[:, :25] = rng.poisson(2.0, (B, 25)) * 0.5
    f[:, 25:] = rng.integers(0, 256, (B, 2)) / 256.0 if grid_offsets else rng.random((B, 2))
    return f.astype(np.float32)


@pytest.mark.parametrize("kind", ["positive", "signed", "mixed"])
@pytest.mark.parametrize("grid_offsets", [True, False])
def test_forward_candidates_hold_float32_evaluations(kind, grid_offsets):
    """Every float32 evaluation (three summation orders) lies in the model's intervals; where
    the model says the output is fixed and exact, each evaluation returns it bit for bit."""
    params = M.grid_params(17, kind).astype(np.float64)
    feat = _features(31, 1500, grid_offsets)
    cand = M.forward_candidates(params, feat)
    assert cand["resolved"].mean() > 0.998
    for order in ("forward", "reversed", "strided"):
        y32 = _f32_network(params, feat, order)
        ok = M.within(y32, cand)
        assert np.all(ok[cand["resolved"]]), (kind, order, int((~ok[cand["resolved"]]).sum()))
        ex = cand["exact"]
        assert np.all(y32[ex] == np.float32(cand["y"][ex])), (kind, order)
    if kind == "positive":
        assert cand["exact"].mean() > 0.95
    if kind == "signed":
        assert cand["exact"].mean() > 0.4
        # GELU's negative branch is exercised by the exact samples
        P = M.unpack(params)
        a1 = M.bf16(feat) @ M.bf16(P["W1"]).T + P["b1"]
        assert np.mean(a1[cand["exact"]] < -0.5) > 0.02


@pytest.mark.parametrize("plant", ["drop_b2", "transpose_w2", "gelu_sign"])
def test_forward_candidates_reject_planted_mistakes(plant):
    params = M.grid_params(18, "signed").astype(np.float64)
    feat = _features(32, 800, True)
    cand = M.forward_candidates(params, feat)
    ok = M.within(_f32_network(params, feat, "forward", plant), cand)
    assert ok.mean() < 0.05, (plant, ok.mean())


def test_forward_candidates_exact_sums_and_ambiguity():
    """Hand-checked cases: a sum of terms on the 2^-8 grid is exact (bound 0); an activation
    whose GELU value sits on a bf16 rounding boundary takes both neighbouring values."""
    X = np.array([[0.5, 0.25, 1.0 / 256]])
    W = np.array([[1.0 / 256, -0.5, 3.0]])
    c, e = M._sum_bound(X, W, np.array([0.125]), 30.0)
    assert c[0, 0] == 0.5 / 256 - 0.125 + 3.0 / 256 + 0.125 and e[0, 0] == 0.0
    c, e = M._sum_bound(np.array([[2.0 ** -30, 1.0]]), np.array([[1.0, 1.0]]), np.array([0.0]), 30.0)
    assert e[0, 0] == 30.0 * M.U32 * (1.0 + 2.0 ** -30)
    assert list(M.grid_exponent(np.array([0.75, 6.0, 2.0 ** -20, 0.0]))) == [-2.0, 1.0, -20.0, np.inf]
    # a one-path network whose layer-2 activation is gelu(a2) with a2 chosen so that gelu(a2)
    # lies within 1e-9 of the bf16 boundary 1 + 2^-8 (between 1 and 1 + 2^-7)
    from scipy.optimize import brentq
    a2 = brentq(lambda a: M.gelu(a) - (1.0 + 2.0 ** -8), 1.0, 2.0)
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    d["W1"][0, 0] = 1.0
    d["W2"][0, 0] = 0.0
    d["b2"][0] = np.float32(a2)
    d["W3"][0] = 1.0
    cand = M.forward_candidates(M.pack(d), np.zeros((1, 27)))
    iv = cand["ivals"][0]
    assert cand["ambiguous"][0] >= 1 and not cand["exact"][0]
    assert iv.shape == (1, 2) and iv[0, 0] <= 1.0 and iv[0, 1] >= 1.0 + 2.0 ** -7
