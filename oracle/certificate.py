"""Count certificate of alpha saturation -- TEST INFRASTRUCTURE ONLY (plain FP64 numpy).

The learned-R form may skip the kNN search of a query only where its alpha is
already fixed.  By Eq. 5 and 6 alpha equals alpha_5 once mu > 0.9, i.e. once
R = r_obs / r_exp (Eq. 3, 4) exceeds a saturation point.  This module states a
lower bound of r_obs that needs only the number of data points binned into the
blocks of 1, 3 x 3 and 5 x 5 cells around the query's cell (the grid of
Section 4.1) and the query's position:

  * B_L is the block of (2L + 1)^2 cells centred on the query's cell, clipped
    to the grid; c_L is the number of data points whose cell lies in B_L.
  * D_L is the distance from the query to the nearest side of B_L beyond which
    the grid has further cells, less `slack` cell widths (the single-precision
    binning may put a point up to that far on the wrong side of a cell edge),
    and at least 0; a block with no such side holds every data point.
  * At most c_L of the query's neighbours lie in B_L, so the j-th nearest
    distance is >= D_L whenever c_L < j.  Summed over j = 1..k:
        sum_k >= sum_L D_L * (min(k, c_{L+1}) - min(k, c_L)),  c_3 = k,
    and r_obs = sum_k / k (Eq. 3).
  * Tighter, from the exact distances of the 3 x 3 block: every data point
    within D_1 of the query lies in that block; if v_cnt of them are nearer
    than D_1, with distances summing to v_sum, then the j-th nearest distance
    is >= min(s_j, D_1) (s_j the j-th smallest distance in the block) and
    >= D_2 when c_2 < j.  With K = min(k, c_2) and v_cnt < K:
        sum_k >= v_sum + (K - v_cnt) * D_1 + (k - K) * D_2,
    and with v_cnt >= K (v_max the largest of the v_cnt distances):
        sum_k >= v_sum - (v_cnt - K) * v_max + (k - K) * D_2;
    the larger of this and the count bound is the bound.  When dense_limit is
    given, the 3 x 3 route is taken only for c_1 <= dense_limit (the library
    leaves denser blocks, whose R lies far below saturation, to the exact path).
  * The query is certified when the bound exceeds sum_min (the caller passes
    k * r_exp * the saturation point of R, with any rounding margin).

Pinned in tests/test_oracle_certificate_pins.py: a hand-derived case, and the
bound against brute-force r_obs on many generated inputs.
"""
from __future__ import annotations

import numpy as np

from . import cell_index


def block_counts(cells_data, qcol, qrow, ncol, nrow):
    """c_0, c_1, c_2 [m] int64: data points binned into the 1 x 1, 3 x 3, 5 x 5 blocks."""
    grid = np.bincount(cells_data, minlength=ncol * nrow).reshape(nrow, ncol)
    out = np.zeros((3, qcol.size), np.int64)
    for j in range(qcol.size):
        r, c = int(qrow[j]), int(qcol[j])
        for L in range(3):
            out[L, j] = grid[max(r - L, 0):r + L + 1, max(c - L, 0):c + L + 1].sum()
    return out


def side_distance(px, py, col, row, L, ncol, nrow, minx, miny, cw, slack):
    """D_L of one query (float64, the operations in the order stated above)."""
    d = np.inf
    if col - L > 0:
        d = min(d, px - (minx + float(col - L) * cw))
    if col + L < ncol - 1:
        d = min(d, (minx + float(col + L + 1) * cw) - px)
    if row - L > 0:
        d = min(d, py - (miny + float(row - L) * cw))
    if row + L < nrow - 1:
        d = min(d, (miny + float(row + L + 1) * cw) - py)
    return max(d - slack * cw, 0.0)


def robs_lower_bound_sum(x, y, qx, qy, k, minx, miny, cw, inv_cw, ncol, nrow, slack, dense_limit=None):
    """Lower bound of the sum of the k nearest distances of every query -> float64 [m]."""
    cells = cell_index(x, y, minx, miny, inv_cw, ncol, nrow)
    qcell = cell_index(qx, qy, minx, miny, inv_cw, ncol, nrow)
    qcol, qrow = qcell % ncol, qcell // ncol
    cnt = block_counts(cells, qcol, qrow, ncol, nrow)
    x64 = np.asarray(x, np.float32).astype(np.float64)
    y64 = np.asarray(y, np.float32).astype(np.float64)
    qx64 = np.asarray(qx, np.float32).astype(np.float64)
    qy64 = np.asarray(qy, np.float32).astype(np.float64)
    minx, miny = float(np.float32(minx)), float(np.float32(miny))
    order = np.argsort(cells, kind="stable")
    start = np.searchsorted(cells[order], np.arange(ncol * nrow + 1))
    out = np.zeros(qx64.size)
    for j in range(qx64.size):
        col, row = int(qcol[j]), int(qrow[j])
        D = [side_distance(qx64[j], qy64[j], col, row, L, ncol, nrow, minx, miny, cw, slack) for L in range(3)]
        c = [min(int(cnt[0, j]), k), min(int(cnt[1, j]), k), min(int(cnt[2, j]), k), k]
        s = 0.0
        for L in range(3):
            mult = c[L + 1] - c[L]
            if mult > 0:
                s += float(mult) * D[L]
        if dense_limit is not None and int(cnt[1, j]) > dense_limit:
            out[j] = s
            continue
        # the 3 x 3 block's points nearer than D_1
        idx = np.concatenate([order[start[r * ncol + max(col - 1, 0)]:start[r * ncol + min(col + 1, ncol - 1) + 1]]
                              for r in range(max(row - 1, 0), min(row + 2, nrow))])
        d = np.sqrt((x64[idx] - qx64[j]) ** 2 + (y64[idx] - qy64[j]) ** 2)
        v = d[d < D[1]]
        kk = c[2]
        if v.size < kk:
            t = float(np.sum(v)) + float(kk - v.size) * D[1]
        else:
            t = float(np.sum(v)) - float(v.size - kk) * (float(v.max()) if v.size else 0.0)
        if k > kk:
            t += float(k - kk) * D[2]
        s = max(s, t)
        out[j] = s
    return out


def certified(x, y, qx, qy, k, minx, miny, cw, inv_cw, ncol, nrow, slack, sum_min, dense_limit=None):
    """True where the bound proves the sum of the k nearest distances exceeds sum_min."""
    return robs_lower_bound_sum(x, y, qx, qy, k, minx, miny, cw, inv_cw, ncol, nrow, slack, dense_limit) > sum_min
