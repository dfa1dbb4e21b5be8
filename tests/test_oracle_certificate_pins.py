"""Pins of the count certificate of alpha saturation (oracle/certificate.py): a case
derived by hand, the bound against brute-force r_obs (Eq. 3) on generated inputs,
and certified queries having alpha = alpha_5 by Eq. 4-6."""
import numpy as np
import pytest

import oracle as O
import oracle.certificate as C
from paper_1601_05904_amd import workloads as W


def slack_for(ncol, nrow):
    # binning slack in cells: (max(ncol, nrow) + 1) * 2^-21 + 1e-9 (covers the float32 cell index)
    return (max(ncol, nrow) + 1) * 2.0 ** -21 + 1e-9


def grid_of(x, y, qx, qy, **kw):
    b = O.bounds(x, y, qx, qy)
    gp = O.grid_params(b, x.size, **kw)
    return b, gp


def bound(x, y, qx, qy, k, b, gp, slack=None):
    s = slack_for(gp["ncol"], gp["nrow"]) if slack is None else slack
    return C.robs_lower_bound_sum(x, y, qx, qy, k, b[0], b[1], gp["cw"], gp["inv_cw"], gp["ncol"], gp["nrow"], s)


def test_hand_derived_case():
    # data: the four corners of the unit square, one point in the query's cell, one in each of
    # the cells left and right of it, one two cells to the left; cell width 0.1 -> an 11 x 11
    # grid on [0, 1.1)^2
    x = np.array([0, 1, 0, 1, 0.41, 0.35, 0.55, 0.25], np.float32)
    y = np.array([0, 0, 1, 1, 0.41, 0.45, 0.45, 0.46], np.float32)
    qx = np.array([0.43], np.float32)
    qy = np.array([0.46], np.float32)
    b, gp = grid_of(x, y, qx, qy, cell_width=0.1)
    assert (gp["ncol"], gp["nrow"]) == (11, 11)
    px, py = float(qx[0]), float(qy[0])
    # query in cell (col 4, row 4) = [0.4, 0.5)^2; c_0 = 1, c_1 = 3 (3 x 3), c_2 = 4 (5 x 5)
    s = slack_for(11, 11) * 0.1
    d0 = min(px - 0.4, 0.5 - px, py - 0.4, 0.5 - py) - s           # 0.03
    d1 = min(px - 0.3, 0.6 - px, py - 0.3, 0.6 - py) - s           # 0.13
    d2 = min(px - 0.2, 0.7 - px, py - 0.2, 0.7 - py) - s           # 0.23
    near = [np.hypot(float(x[i]) - px, float(y[i]) - py) for i in (4, 5, 6)]  # 0.054, 0.081, 0.120 < D_1
    assert max(near) < d1
    # the count bound for k = 3: j = 2, 3 >= D_0
    assert C.robs_lower_bound_sum(x, y, qx, qy, 3, b[0], b[1], 0.1, gp["inv_cw"], 11, 11, slack_for(11, 11)) >= 2 * d0
    # k = 3: K = min(3, c_2) = 3 = v_cnt -> the three distances
    assert bound(x, y, qx, qy, 3, b, gp)[0] == pytest.approx(sum(near), abs=1e-12)
    # k = 4: K = 4 > v_cnt = 3 -> the three distances plus D_1
    got = bound(x, y, qx, qy, 4, b, gp)[0]
    assert got == pytest.approx(sum(near) + d1, abs=1e-12)
    assert got == pytest.approx(0.38489, abs=1e-4)
    # without the 3 x 3 route (dense_limit below c_1): the count bound, j = 2, 3 >= D_0, j = 4 >= D_1
    only_counts = C.robs_lower_bound_sum(x, y, qx, qy, 4, b[0], b[1], gp["cw"], gp["inv_cw"], 11, 11,
                                         slack_for(11, 11), dense_limit=2)[0]
    assert only_counts == pytest.approx(2 * d0 + d1, abs=1e-12)
    # k = 6: K = 4; j = 5, 6 lie beyond the 5 x 5 block
    assert bound(x, y, qx, qy, 6, b, gp)[0] == pytest.approx(sum(near) + d1 + 2 * d2, abs=1e-12)
    # k = 1: K = 1 < v_cnt = 3 -> the three distances less twice the largest (0.0139)
    assert bound(x, y, qx, qy, 1, b, gp)[0] == pytest.approx(sum(near) - 2 * max(near), abs=1e-12)
    # the bound holds: the exact sum of the k nearest distances (Eq. 3 times k)
    for k in (1, 3, 4, 6, 8):
        _, d2k = O.knn(x, y, qx, qy, k)
        assert bound(x, y, qx, qy, k, b, gp)[0] <= np.sqrt(d2k).sum() + 1e-12


def test_side_distance_skips_closed_sides():
    # query in the corner cell: the left and bottom sides have no cells beyond them
    d = C.side_distance(0.02, 0.03, 0, 0, 0, 10, 10, 0.0, 0.0, 0.1, 0.0)
    assert d == pytest.approx(min(0.1 - 0.02, 0.1 - 0.03))
    # a block covering the grid has no open side
    assert C.side_distance(0.5, 0.5, 2, 2, 2, 5, 5, 0.0, 0.0, 0.2, 0.0) == np.inf


CASES = [
    ("uniform", 3000, 800, 10, 2.0, 0.0),
    ("uniform", 3000, 800, 1, 2.0, 0.0),
    ("mixture", 6000, 800, 15, 2.0, 0.0),
    ("mixture", 6000, 800, 15, 0.25, 0.0),
    ("uniform", 40, 300, 8, 2.0, 0.0),       # 4 x 4 grid: most blocks clipped
    ("uniform", 2000, 400, 5, 0.0, 0.002),   # a fine grid: most blocks empty
    ("mixture", 3000, 600, 15, 0.0, 0.7),    # cells wider than half the square
]


@pytest.mark.parametrize("kind,n,m,k,occ,cw", CASES)
def test_bound_below_brute_force(kind, n, m, k, occ, cw):
    ds = W.make(n, m, k, 700 + n + k, kind, 8)
    kw = dict(cell_width=cw) if cw > 0 else dict(occupancy=occ)
    b, gp = grid_of(ds.x, ds.y, ds.qx, ds.qy, **kw)
    lb = bound(ds.x, ds.y, ds.qx, ds.qy, k, b, gp)
    _, d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, k)
    exact = np.sqrt(d2).sum(axis=1)
    assert np.all(lb <= exact * (1 + 1e-12)), float((lb - exact).max())  # equal, up to the summation order, when tight
    # the bound is not vacuous: it certifies something on sparse inputs
    if kind == "mixture" and occ == 2.0:
        assert np.mean(lb > 0) > 0.5


def test_bound_on_a_strip():
    ds = W.make(3000, 500, 10, 731)
    ds.x = (ds.x * np.float32(1 / 64)).astype(np.float32)
    ds.qx = (ds.qx * np.float32(1 / 64)).astype(np.float32)
    b, gp = grid_of(ds.x, ds.y, ds.qx, ds.qy, occupancy=2.0)
    lb = bound(ds.x, ds.y, ds.qx, ds.qy, 10, b, gp)
    _, d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, 10)
    assert np.all(lb <= np.sqrt(d2).sum(axis=1) * (1 + 1e-12))


def test_certified_queries_have_saturated_alpha():
    ds = W.make(20000, 2000, 15, 741, "mixture", 16)
    b, gp = grid_of(ds.x, ds.y, ds.qx, ds.qy, occupancy=2.0)
    r_sat = 0.0 + 2.0 / np.pi * np.arccos(-0.8)
    sum_min = 15 * gp["r_exp"] * min(r_sat, 2.0) * (1 + 1e-6)
    cert = C.certified(ds.x, ds.y, ds.qx, ds.qy, 15, b[0], b[1], gp["cw"], gp["inv_cw"], gp["ncol"], gp["nrow"],
                       slack_for(gp["ncol"], gp["nrow"]), sum_min)
    _, d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, 15)
    _, mu, a = O.alpha(O.robs(d2), gp["r_exp"], 0.0, 2.0, W.LEVELS)
    assert cert.mean() > 0.5
    assert np.all(mu[cert] > 0.9) and np.all(a[cert] == 5.0)
