"""Pins of the FP64 oracle to what the paper and the mathematics fix (CPU only).

Every function of the oracle is checked against something other than itself:
closed forms, hand-derived worked examples (tests/golden), brute force by a
different route (full lexicographic sort instead of the oracle's insertion),
invariants and a statistical closed form.  A plausible slip (a dropped term, a
wrong sign or index, r_exp from the query count, Eq. 5's denominator, a swapped
Eq. 6 level) fails at least one test here.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_1601_05904_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- grid (Section 4.1.1 / 4.1.2, Eq. 2)

def test_bounds_cover_data_and_queries():
    x = np.array([0.25, 0.5], np.float32)
    y = np.array([0.125, 0.375], np.float32)
    qx = np.array([0.875], np.float32)
    qy = np.array([0.0625], np.float32)
    assert list(O.bounds(x, y, qx, qy)) == [0.25, 0.0625, 0.875, 0.375]


def test_grid_params_closed_form():
    # unit square, n = 64, two points per cell: A = 1, r_exp = 1/(2*sqrt(64)) = 1/16,
    # cw = sqrt(2/64) ... use occupancy 1 so that cw = 1/8 exactly, nCol = (1 + 1/8) / (1/8) = 9.
    g = O.grid_params([0.0, 0.0, 1.0, 1.0], 64, occupancy=1.0)
    assert g["area"] == 1.0 and g["r_exp"] == 1.0 / 16 and g["cw"] == 0.125
    assert g["inv_cw"] == np.float32(8.0) and g["ncol"] == 9 and g["nrow"] == 9
    # given area overrides the bounding box: r_exp = 1/(2*sqrt(64/4)) = 1/8
    g = O.grid_params([0.0, 0.0, 1.0, 1.0], 64, area=4.0, occupancy=1.0)
    assert g["r_exp"] == 0.125 and g["cw"] == 0.25
    # rectangle 2 x 0.5: nCol = (2 + 0.25)/0.25 = 9, nRow = (0.5 + 0.25)/0.25 = 3
    g = O.grid_params([0.0, 0.0, 2.0, 0.5], 16, occupancy=1.0)
    assert g["cw"] == 0.25 and g["ncol"] == 9 and g["nrow"] == 3


def test_paper_cell_width_is_r_exp():
    # Section 4.1.1 takes the cell width from Eq. 2: occupancy 1/4 reproduces cw = r_exp.
    g = O.grid_params([0.0, 0.0, 0.7, 1.3], 1000, occupancy=0.25)
    assert g["cw"] == pytest.approx(g["r_exp"], rel=1e-15)


def test_grid_degenerate_and_capacity():
    with pytest.raises(O.OracleError) as e:
        O.grid_params([0.0, 0.5, 1.0, 0.5], 10)  # collinear: zero area
    assert e.value.code == O.EDEGENERATE
    g = O.grid_params([0.0, 0.5, 1.0, 0.5], 10, area=1.0)  # a given area makes it valid
    assert g["nrow"] == 1
    with pytest.raises(O.OracleError) as e:
        O.grid_params([0.0, 0.0, 1.0, 1.0], 10, cell_width=1e-9)
    assert e.value.code == O.ECAPACITY


def test_cell_index_boundaries():
    # cw = 1/8, 9 columns: a point on a cell edge belongs to the cell on its right / above,
    # the upper bound lands in column 8; flat index = row * nCol + col (Section 4.1.2).
    x = np.array([0.0, 0.125, 0.124999, 0.5, 1.0], np.float32)
    y = np.array([0.0, 0.0, 0.25, 0.375, 1.0], np.float32)
    c = O.cell_index(x, y, 0.0, 0.0, 8.0, 9, 9)
    assert list(c) == [0, 1, 2 * 9 + 0, 3 * 9 + 4, 8 * 9 + 8]
    # indices past the last column / row are clamped into the grid
    c = O.cell_index(np.array([1.0], np.float32), np.array([1.0], np.float32), 0.0, 0.0, 8.0, 8, 8)
    assert list(c) == [7 * 8 + 7]


# ---------------------------------------------------------------- kNN (Section 2.3) and Eq. 3

def _sort_knn(x, y, qx, qy, k):
    """Brute force by a different route: full lexicographic sort of (d^2, index)."""
    idx = np.zeros((qx.size, k), np.int64)
    d2o = np.zeros((qx.size, k))
    X = x.astype(np.float64)
    Y = y.astype(np.float64)
    for j in range(qx.size):
        dx = X - np.float64(qx[j])
        dy = Y - np.float64(qy[j])
        d2 = dx * dx + dy * dy
        order = np.lexsort((np.arange(x.size), d2))[:k]
        idx[j] = order
        d2o[j] = d2[order]
    return idx, d2o


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_knn_matches_full_sort_with_ties(seed):
    rng = np.random.default_rng(seed)
    n, m, k = 150, 40, 12
    # coarse lattice (1/8 spacing) forces many equal distances and duplicate points
    x = (rng.integers(0, 8, n) / 8).astype(np.float32)
    y = (rng.integers(0, 8, n) / 8).astype(np.float32)
    qx = (rng.integers(0, 16, m) / 16).astype(np.float32)
    qy = (rng.integers(0, 16, m) / 16).astype(np.float32)
    i1, d1 = O.knn(x, y, qx, qy, k)
    i2, d2 = _sort_knn(x, y, qx, qy, k)
    assert np.array_equal(i1, i2)
    assert np.array_equal(d1, d2)


def test_knn_random_lattice_inputs():
    ds = W.make(500, 64, 10, 7)
    i1, d1 = O.knn(ds.x, ds.y, ds.qx, ds.qy, 10)
    i2, d2 = _sort_knn(ds.x, ds.y, ds.qx, ds.qy, 10)
    assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


def test_knn_k_equals_n_returns_every_point():
    ds = W.make(37, 5, 37, 3)
    idx, d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, 37)
    for j in range(5):
        assert sorted(idx[j]) == list(range(37))
        assert np.all(np.diff(d2[j]) >= 0)


def test_knn_lattice_square_closed_form():
    # 16 x 16 lattice of spacing h; a query at the centre of a lattice square has its
    # 4 nearest neighbours at distance h / sqrt(2) -> r_obs = h / sqrt(2) (Eq. 3).
    h = 1.0 / 16
    g = np.arange(16) * h
    X, Y = np.meshgrid(g, g, indexing="xy")
    x = X.ravel().astype(np.float32)
    y = Y.ravel().astype(np.float32)
    qx = np.array([5.5 * h], np.float32)
    qy = np.array([9.5 * h], np.float32)
    idx, d2 = O.knn(x, y, qx, qy, 4)
    assert sorted(idx[0]) == [9 * 16 + 5, 9 * 16 + 6, 10 * 16 + 5, 10 * 16 + 6]
    assert list(idx[0]) == sorted(idx[0])  # equal distances: ascending index
    r = O.robs(d2)
    assert r[0] == pytest.approx(h / math.sqrt(2), rel=1e-15)


def test_robs_is_mean_distance():
    d2 = np.array([[1.0, 4.0, 9.0], [0.0, 0.25, 0.25]])
    assert list(O.robs(d2)) == [2.0, 1.0 / 3.0]


@pytest.mark.parametrize("k", [1, 10])
def test_poisson_nn_statistic(k):
    # For a random (Poisson) pattern of density rho = n / A, E[d_j] sqrt(rho) = Gamma(j + 1/2) / (Gamma(j) sqrt(pi)),
    # so E[R] = E[r_obs] / r_exp = (2/k) sum_j Gamma(j + 1/2) / (Gamma(j) sqrt(pi)); k = 1 gives the classic R = 1.
    # Uses n data points and a different number m of queries (r_exp must use n), queries away from the edges.
    n, m = 1 << 16, 3000
    rng = np.random.default_rng(11)
    x = W.quantise(rng.random(n))
    y = W.quantise(rng.random(n))
    qx = W.quantise(0.15 + 0.7 * rng.random(m))
    qy = W.quantise(0.15 + 0.7 * rng.random(m))
    z = np.zeros(n, np.float32)
    res = O.aidw(x, y, z, qx, qy, k=k)
    expect = 2.0 / k * sum(math.gamma(j + 0.5) / (math.gamma(j) * math.sqrt(math.pi)) for j in range(1, k + 1))
    if k == 10:
        assert expect == pytest.approx(2.467, abs=1e-3)
    assert np.mean(res["R"]) == pytest.approx(expect, rel=0.02)


# ---------------------------------------------------------------- Eq. 4, 5, 6

def _R_for_mu(mu, r_max=2.0):
    # inverse of Eq. 5 with R_min = 0: mu = (1 - cos(pi R / R_max)) / 2
    return r_max / math.pi * math.acos(1.0 - 2.0 * mu)


def test_alpha_knots_and_midpoints():
    levels = (1.0, 10.0, 100.0, 1000.0, 10000.0)  # distinct magnitudes: a swapped level shows
    mus = [0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95]
    expect = [1, 1, 5.5, 10, 55, 100, 550, 1000, 5500, 10000, 10000]
    r_exp = 0.37
    r_obs = np.array([_R_for_mu(mu) * r_exp for mu in mus])
    R, mu, a = O.alpha(r_obs, r_exp, 0.0, 2.0, levels)
    assert np.allclose(mu, mus, rtol=1e-12, atol=1e-14)
    assert np.allclose(a, expect, rtol=1e-9)


def test_alpha_closed_form_levels_1_to_5():
    # levels 1..5, R_min = 0, R_max = 2: mu = (1 - cos(pi R / 2)) / 2 and Eq. 6 is alpha = 5 mu + 1/2
    # on [0.1, 0.9], so alpha(R) = clamp(3 - 2.5 cos(pi R / 2), 1, 5) for R <= 2 and 5 beyond.
    R = np.linspace(0.0, 3.0, 301)
    _, _, a = O.alpha(R * 0.25, 0.25, 0.0, 2.0, W.LEVELS)
    closed = np.where(R >= 2.0, 5.0, np.clip(3.0 - 2.5 * np.cos(np.pi * R / 2.0), 1.0, 5.0))
    assert np.allclose(a, closed, rtol=1e-12, atol=1e-12)
    assert a.min() >= 1.0 and a.max() <= 5.0
    # alpha is saturated below R = (2/pi) acos(0.8) and above (2/pi) acos(-0.8)
    assert (2 / math.pi) * math.acos(0.8) == pytest.approx(0.4097, abs=1e-4)


def test_statistic_R_is_ratio():
    R, mu, a = O.alpha(np.array([0.1, 0.05, 0.0]), 0.05)
    assert list(R) == [2.0, 1.0, 0.0]
    assert list(mu) == [1.0, 0.5, 0.0] or np.allclose(mu, [1.0, 0.5, 0.0], atol=1e-15)
    assert a[0] == 5.0 and a[2] == 1.0 and a[1] == pytest.approx(3.0, abs=1e-12)


def test_membership_literal_reading_with_nonzero_rmin():
    # Eq. 5 as printed divides by R_max, not by R_max - R_min (the two agree only for R_min = 0).
    # R_min = 0.5, R_max = 2, R = 1.5: literal mu = 0.5 - 0.5 cos(pi/2 * 1) = 0.5 -> alpha_3.
    R, mu, a = O.alpha(np.array([1.5, 0.4, 2.5]), 1.0, 0.5, 2.0, (1.0, 2.0, 3.0, 4.0, 5.0))
    assert mu[0] == pytest.approx(0.5, abs=1e-15) and a[0] == pytest.approx(3.0, abs=1e-12)
    assert mu[1] == 0.0 and a[1] == 1.0  # R <= R_min
    assert mu[2] == 1.0 and a[2] == 5.0  # R >= R_max


# ---------------------------------------------------------------- Eq. 1

def _golden_cases():
    with open(os.path.join(GOLDEN, "idw_worked_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_idw_worked_examples(case):
    d = np.array(case["data"], np.float64)
    zq = O.idw(d[:, 0], d[:, 1], d[:, 2], [case["query"][0]], [case["query"][1]], case["alpha"])[0]
    if "expected" in case:
        exp = float(Fraction(case["expected"]))
    else:
        exp = eval(case["expected_expr"], {"sqrt": math.sqrt})
    assert zq == pytest.approx(exp, rel=1e-14)


def test_idw_constant_field_and_hull():
    ds = W.make(300, 50, 10, 5)
    zc = np.full(300, 0.75, np.float32)
    a = np.linspace(0.5, 6.0, 50)
    assert np.allclose(O.idw(ds.x, ds.y, zc, ds.qx, ds.qy, a), 0.75, rtol=1e-14)
    zq = O.idw(ds.x, ds.y, ds.z, ds.qx, ds.qy, a)
    assert zq.min() >= ds.z.min() and zq.max() <= ds.z.max()


def test_idw_square_centre_is_mean_for_any_alpha():
    x = np.array([0, 1, 0, 1], np.float32)
    y = np.array([0, 0, 1, 1], np.float32)
    z = np.array([1.0, -2.0, 4.0, 8.5], np.float32)
    for a in (0.3, 1.0, 2.7, 5.0, 9.0):
        assert O.idw(x, y, z, [0.5], [0.5], a)[0] == pytest.approx(11.5 / 4, rel=1e-15)


def test_idw_sign_of_power():
    # nearer points must dominate: a query next to z = 1 among far z = 0 points moves toward 1 as alpha grows
    x = np.array([0.0, 10.0, -10.0], np.float32)
    y = np.array([0.0, 0.0, 0.0], np.float32)
    z = np.array([1.0, 0.0, 0.0], np.float32)
    v = [O.idw(x, y, z, [1.0], [0.0], a)[0] for a in (1.0, 2.0, 4.0)]
    assert v[0] < v[1] < v[2] < 1.0 and v[0] > 0.5


# ---------------------------------------------------------------- whole method

def test_equal_levels_reduce_to_shepard():
    ds = W.make(400, 60, 10, 9)
    res = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=10, levels=(2.0,) * 5)
    assert np.all(res["alpha"] == 2.0)
    assert np.array_equal(res["z"], O.idw(ds.x, ds.y, ds.z, ds.qx, ds.qy, 2.0))


def test_aidw_five_point_worked_example():
    # corners of [0,2]^2 with z = 1..4, a fifth point at (1, 1.5) with z = 10, query at (1, 1), k = 1.
    # A = 4 (bounding box), n = 5 -> r_exp = 1/(2 sqrt(5/4)) = 1/sqrt(5); r_obs = 0.5; R = sqrt(5)/2;
    # alpha = 3 - 2.5 cos(pi R / 2) (levels 1..5); weights (d^2)^(-alpha/2) with d^2 = 1/4 and 2.
    x = np.array([0, 2, 0, 2, 1], np.float32)
    y = np.array([0, 0, 2, 2, 1.5], np.float32)
    z = np.array([1, 2, 3, 4, 10], np.float32)
    res = O.aidw(x, y, z, np.array([1.0], np.float32), np.array([1.0], np.float32), k=1)
    R = math.sqrt(5) / 2
    a = 3 - 2.5 * math.cos(math.pi * R / 2)
    w_near, w_corner = 0.25 ** (-a / 2), 2.0 ** (-a / 2)
    zexp = (10 * w_near + 10 * w_corner) / (w_near + 4 * w_corner)
    assert res["r_exp"] == pytest.approx(1 / math.sqrt(5), rel=1e-15)
    assert res["R"][0] == pytest.approx(R, rel=1e-15)
    assert res["alpha"][0] == pytest.approx(a, rel=1e-13)
    assert res["z"][0] == pytest.approx(zexp, rel=1e-13)


def test_translation_and_scaling_invariance():
    ds = W.make(512, 64, 10, 13)
    base = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=10)
    # translation by a lattice multiple keeps every coordinate difference exact
    t = O.aidw(ds.x + np.float32(0.25), ds.y + np.float32(0.5), ds.z, ds.qx + np.float32(0.25),
               ds.qy + np.float32(0.5), k=10)
    assert np.array_equal(base["knn_idx"], t["knn_idx"])
    assert np.array_equal(base["R"], t["R"]) and np.array_equal(base["z"], t["z"])
    # scaling by 2 is exact: R and alpha unchanged, z unchanged up to rounding of the powers
    s = O.aidw(ds.x * 2, ds.y * 2, ds.z, ds.qx * 2, ds.qy * 2, k=10)
    assert np.array_equal(base["knn_idx"], s["knn_idx"])
    assert np.array_equal(base["R"], s["R"]) and np.array_equal(base["alpha"], s["alpha"])
    assert np.allclose(base["z"], s["z"], rtol=1e-13, atol=1e-15)


def test_permutation_invariance():
    ds = W.make(300, 40, 8, 21)
    base = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=8)
    p = np.random.default_rng(0).permutation(300)
    r = O.aidw(ds.x[p], ds.y[p], ds.z[p], ds.qx, ds.qy, k=8)
    assert np.array_equal(base["knn_d2"], r["knn_d2"])
    assert np.allclose(base["z"], r["z"], rtol=1e-13)
    assert np.allclose(base["r_obs"], r["r_obs"], rtol=1e-15)


def test_query_selection_uses_all_queries_for_bounds():
    ds = W.make(200, 100, 10, 4)
    full = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=10)
    sel = np.array([3, 17, 99])
    part = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=10, qsel=sel)
    assert part["area"] == full["area"]
    assert np.array_equal(part["z"], full["z"][sel]) and np.array_equal(part["knn_idx"], full["knn_idx"][sel])


def test_coincident_query_inside_whole_method():
    ds = W.make(100, 10, 5, 8)
    qx = ds.qx.copy()
    qy = ds.qy.copy()
    qx[3], qy[3] = ds.x[42], ds.y[42]
    res = O.aidw(ds.x, ds.y, ds.z, qx, qy, k=5)
    assert res["knn_d2"][3, 0] == 0.0 and res["knn_idx"][3, 0] == 42
    assert res["z"][3] == np.float64(ds.z[42])


# ------------------------------------------------------------------ the paper's "+1 level" rule

def _unit_grid_case():
    # bounds [0, 10]^2 (corner points), cell side 1 -> 11 x 11 cells, inv_cw = 1
    x = np.array([0.0, 10.0, 5.99, 3.98], np.float32)   # A, B, P (in the query's cell), R (two columns left)
    y = np.array([0.0, 10.0, 5.99, 5.5], np.float32)
    qx = np.array([5.01], np.float32)
    qy = np.array([5.5], np.float32)
    b = O.bounds(x, y, qx, qy)
    gp = O.grid_params(b, x.size, 0.0, 1.0, 2.0)
    assert (gp["ncol"], gp["nrow"], gp["inv_cw"]) == (11, 11, 1.0)
    return x, y, qx, qy, b, gp


def test_paper_rule_misses_a_nearer_point_outside_the_final_block():
    """k = 1: the query's own cell holds P, so the search stops at level 0 + 1 = 1 (cells 4..6);
    R lies in column 3, outside that block, yet nearer (1.03 against 1.096)."""
    x, y, qx, qy, b, gp = _unit_grid_case()
    idx, d2 = O.knn_paper(x, y, qx, qy, 1, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    eidx, ed2 = O.knn(x, y, qx, qy, 1)
    assert idx[0, 0] == 2 and eidx[0, 0] == 3
    assert d2[0, 0] == pytest.approx((5.99 - 5.01) ** 2 + (5.99 - 5.5) ** 2, rel=1e-6)
    assert ed2[0, 0] == pytest.approx((5.01 - 3.98) ** 2, rel=1e-6)
    # k = 2: levels 0 and 1 hold only P, level 2 (cells 3..7) holds P and R -> final level 3 -> exact
    idx2, _ = O.knn_paper(x, y, qx, qy, 2, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    eidx2, _ = O.knn(x, y, qx, qy, 2)
    assert idx2.tolist() == eidx2.tolist() == [[3, 2]]
    # the extra level matters: a point in the next column (level 1) is found although the
    # query's own cell already held one
    x3 = np.append(x, np.float32(4.9))
    y3 = np.append(y, np.float32(5.5))
    idx3, _ = O.knn_paper(x3, y3, qx, qy, 1, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    assert idx3[0, 0] == 4


def test_paper_rule_on_one_cell_is_brute_force():
    rng = np.random.default_rng(31)
    x, y = W.quantise(rng.random(300)), W.quantise(rng.random(300))
    qx, qy = W.quantise(rng.random(50)), W.quantise(rng.random(50))
    b = O.bounds(x, y, qx, qy)
    gp = O.grid_params(b, x.size, 0.0, 4.0, 2.0)  # one cell covers the unit square
    assert gp["ncol"] == gp["nrow"] == 1
    for k in (1, 7, 300):
        idx, d2 = O.knn_paper(x, y, qx, qy, k, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
        eidx, ed2 = O.knn(x, y, qx, qy, k)
        assert np.array_equal(idx, eidx) and np.array_equal(d2, ed2)


@pytest.mark.parametrize("occ", [0.25, 2.0])
def test_paper_rule_never_beats_exact_and_is_exact_when_it_must_be(occ):
    """Its k distances are those of k points, so each is >= the exact one; and a query whose
    k-th found distance is within the distance to the final block's edge has the exact set."""
    ds = W.make(4096, 1500, 10, 33)
    b = O.bounds(ds.x, ds.y, ds.qx, ds.qy)
    gp = O.grid_params(b, ds.n, 0.0, 0.0, occ)
    idx, d2 = O.knn_paper(ds.x, ds.y, ds.qx, ds.qy, 10, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    eidx, ed2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, 10)
    assert np.all(d2 >= ed2)
    same = np.all(idx == eidx, axis=1)
    assert same.mean() > 0.99  # the rule rarely fails on uniform data (the Remark's claim)
    # recompute the final level and the distance to its edge, and check exactness where it is implied
    cq = O.cell_index(ds.qx, ds.qy, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    cd = O.cell_index(ds.x, ds.y, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    dc, dr = cd % gp["ncol"], cd // gp["ncol"]
    cw = 1.0 / float(np.float32(gp["inv_cw"]))
    for j in range(0, ds.m, 7):
        c0, r0 = cq[j] % gp["ncol"], cq[j] // gp["ncol"]
        L = 0
        while np.count_nonzero((abs(dc - c0) <= L) & (abs(dr - r0) <= L)) < 10:
            L += 1
        Lf = L + 1
        edges = []
        if c0 - Lf > 0:
            edges.append(float(ds.qx[j]) - (b[0] + (c0 - Lf) * cw))
        if c0 + Lf < gp["ncol"] - 1:
            edges.append(b[0] + (c0 + Lf + 1) * cw - float(ds.qx[j]))
        if r0 - Lf > 0:
            edges.append(float(ds.qy[j]) - (b[1] + (r0 - Lf) * cw))
        if r0 + Lf < gp["nrow"] - 1:
            edges.append(b[1] + (r0 + Lf + 1) * cw - float(ds.qy[j]))
        e = min(edges) - 1e-6 if edges else np.inf
        if d2[j, -1] < e * e:
            assert same[j], j
