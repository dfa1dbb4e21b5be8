"""Parity of the HIP path with the FP64 oracle, through the C ABI (needs an MI355X).

Bars: grid arrays and kNN index sets bit-exact; d1sq exact; r_obs within one
float32 ulp; alpha within 1e-6; z within 1e-5 in the normwise relative metric
e = |z - z64| / max(|z64|, sum w|z| / sum w).
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1601_05904_amd import workloads as W

pytestmark = pytest.mark.gpu

Z_TOL = 1e-5


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1601_05904_amd as aidw
    aidw.load(build_if_missing=False)
    return torch


def aidw_mod():
    import paper_1601_05904_amd as aidw
    return aidw


def dev(T, a):
    return T.from_numpy(np.ascontiguousarray(a)).to("cuda")


def upload(T, ds):
    return [dev(T, getattr(ds, k)) for k in ("x", "y", "z", "qx", "qy")]


def zerr(zg, ref):
    zg = np.asarray(zg, np.float64)
    return np.abs(zg - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])


def tiny_lattice(seed, n, m, res=8):
    rng = np.random.default_rng(seed)
    x = (rng.integers(0, res, n) / res).astype(np.float32)
    y = (rng.integers(0, res, n) / res).astype(np.float32)
    z = rng.standard_normal(n).astype(np.float32)
    qx = (rng.integers(0, 2 * res, m) / (2 * res)).astype(np.float32)
    qy = (rng.integers(0, 2 * res, m) / (2 * res)).astype(np.float32)
    return W.Dataset("lattice%d" % seed, x, y, z, qx, qy, 8, seed)


# ------------------------------------------------------------------ grid build

def _check_grid(T, ds, params, offset=0):
    aidw = aidw_mod()
    x, y, z, qx, qy = upload(T, ds)
    if offset:
        # views that start `offset` floats into their buffers: device pointers off 16-byte alignment
        x, y, qx, qy = (T.cat([T.zeros(offset, dtype=a.dtype, device=a.device), a])[offset:] for a in (x, y, qx, qy))
        assert all(a.data_ptr() % 16 != 0 for a in (x, y, qx, qy))
    g = aidw.build_grid(x, y, qx, qy, params)
    d = g.describe()
    b = O.bounds(ds.x, ds.y, ds.qx, ds.qy)
    gp = O.grid_params(b, ds.n, params.area, params.cell_width, params.occupancy)
    assert [d["min_x"], d["min_y"], d["max_x"], d["max_y"]] == list(np.float32(b))
    assert d["area"] == gp["area"] and d["r_exp"] == gp["r_exp"] and d["cell_width"] == gp["cw"]
    assert np.float32(d["inv_cell_width"]) == gp["inv_cw"]
    assert (d["ncol"], d["nrow"]) == (gp["ncol"], gp["nrow"])
    assert g.info() == {"area": gp["area"], "r_exp": gp["r_exp"], "cell_width": gp["cw"], "ncol": gp["ncol"],
                        "nrow": gp["nrow"]}
    cs, sx, sy, si = (a.cpu().numpy() for a in g.arrays())
    cells = O.cell_index(ds.x, ds.y, b[0], b[1], gp["inv_cw"], gp["ncol"], gp["nrow"])
    counts = np.bincount(cells, minlength=gp["ncol"] * gp["nrow"])
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(counts)]).astype(np.int32))
    order = np.argsort(cells, kind="stable")  # each cell's segment ordered by original index
    assert np.array_equal(si, order.astype(np.int32))
    assert np.array_equal(sx, ds.x[order]) and np.array_equal(sy, ds.y[order])
    g.close()


def dense_cells(seed, n=30000, m=3000, spots=50, dup=100):
    """Uniform points plus `spots` positions holding `dup` coincident points each: cells of more
    than 64 points, so their bands take the ballot-ranked local sort."""
    rng = np.random.default_rng(seed)
    ds = W.make(n, m, 10, seed)
    sx, sy = W.quantise(rng.random(spots)), W.quantise(rng.random(spots))
    pick = rng.permutation(n)[:spots * dup]
    ds.x[pick] = np.repeat(sx, dup)
    ds.y[pick] = np.repeat(sy, dup)
    return ds


@pytest.mark.parametrize("name", ["uniform_4k", "mixture", "ragged_rect", "unaligned", "lattice", "dense_cells",
                                  "uniform_1m", "clustered_1m"])
def test_grid_matches_oracle(T, name):
    """The grid (bounds, scalars, CSR offsets, points in cell order with each cell by index)
    bit for bit against the oracle's stable sort by cell.  uniform_1m takes the rank-ordered
    local sort in every band, dense_cells the ballot-ranked one in the bands of its crowded
    cells, clustered_1m (the 2^20 mixture) also bands too large for the LDS tile; ragged_rect
    has lengths that are not multiples of four, unaligned coordinate arrays (views) that do
    not start on a 16-byte boundary."""
    aidw = aidw_mod()
    if name == "uniform_1m":
        ds, p = W.WORKLOADS["uniform_1m"](), aidw.Params()
    elif name == "clustered_1m":
        ds, p = W.WORKLOADS["learned_1m"](), aidw.Params(k=15)
    elif name == "dense_cells":
        ds, p = dense_cells(33), aidw.Params()
    elif name == "uniform_4k":
        ds, p = W.uniform_4k(), aidw.Params()
    elif name == "mixture":
        ds, p = W.make(20000, 3000, 15, 31, "mixture"), aidw.Params(k=15)
    elif name == "ragged_rect":
        ds = W.make(1237, 999, 7, 32)
        ds.x = (ds.x * np.float32(0.25)).astype(np.float32)  # a 1/4 x 1 rectangle
        ds.qx = (ds.qx * np.float32(0.25)).astype(np.float32)
        p = aidw.Params(k=7, occupancy=3.0)
    elif name == "unaligned":
        ds, p = W.make(5003, 1201, 10, 34), aidw.Params()
        _check_grid(T, ds, p, offset=1)
        return
    else:
        ds, p = tiny_lattice(5, 300, 50), aidw.Params(k=8, occupancy=0.5)
    _check_grid(T, ds, p)


# ------------------------------------------------------------------ kNN

def _knn_case(T, ds, k, params=None):
    aidw = aidw_mod()
    params = params or aidw.Params(k=k)
    x, y, z, qx, qy = upload(T, ds)
    g = aidw.build_grid(x, y, qx, qy, params)
    r, d1, ix = aidw.knn(g, qx, qy, k, want_d1sq=True, want_idx=True)
    T.cuda.synchronize()
    ref_i, ref_d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, k)
    assert np.array_equal(ix.cpu().numpy(), ref_i), "kNN index sets differ"
    assert np.array_equal(d1.cpu().numpy(), ref_d2[:, 0].astype(np.float32))
    assert np.allclose(r.cpu().numpy(), O.robs(ref_d2), rtol=1.2e-7, atol=0)
    g.close()


@pytest.mark.parametrize("case", ["uniform_4k_k10", "mixture_k15", "ragged_k7", "k1", "k8", "k16", "k17", "k64",
                                  "k_equals_n"])
def test_knn_bit_exact(T, case):
    if case == "uniform_4k_k10":
        _knn_case(T, W.uniform_4k(), 10)
    elif case == "mixture_k15":
        _knn_case(T, W.make(20000, 3000, 15, 41, "mixture"), 15)
    elif case == "ragged_k7":
        _knn_case(T, W.make(1237, 999, 7, 42), 7)
    elif case == "k_equals_n":
        _knn_case(T, W.make(20, 33, 20, 43), 20)
    else:
        k = int(case[1:])
        _knn_case(T, W.make(3001, 517, k, 44 + k), k)


@pytest.mark.parametrize("seed", range(6))
def test_knn_ties_and_duplicates(T, seed):
    # coarse lattice: many equal distances and duplicate data points; ties go to the smaller index
    ds = tiny_lattice(seed, 150 + 37 * seed, 40 + seed)
    for k in (1, 5, 12):
        _knn_case(T, ds, k)


@pytest.mark.parametrize("mode", ["tiny", "paper_r_exp", "one_cell", "wide"])
def test_knn_independent_of_cell_width(T, mode):
    aidw = aidw_mod()
    ds = W.make(5000, 800, 10, 51, "mixture", 8)
    if mode == "tiny":
        p = aidw.Params(k=10, occupancy=0.02)
    elif mode == "paper_r_exp":
        p = aidw.Params(k=10, occupancy=0.25)  # the cell width of Eq. 2, the paper's choice
    elif mode == "one_cell":
        p = aidw.Params(k=10, cell_width=4.0)
    else:
        p = aidw.Params(k=10, occupancy=40.0)
    _knn_case(T, ds, 10, p)


# ------------------------------------------------------------------ whole method

def _run_case(T, ds, params=None, qsel=None):
    aidw = aidw_mod()
    params = params or aidw.Params(k=ds.k)
    x, y, z, qx, qy = upload(T, ds)
    qz, al, ro = aidw.run(x, y, z, qx, qy, params, want_alpha=True, want_robs=True)
    T.cuda.synchronize()
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=params.k, levels=params.levels, r_min=params.r_min,
                 r_max=params.r_max, area=params.area, cell_width=params.cell_width, occupancy=params.occupancy,
                 qsel=qsel)
    sel = slice(None) if qsel is None else qsel
    zq = qz.cpu().numpy()[sel]
    e = zerr(zq, ref)
    assert np.all(np.isfinite(zq))
    assert e.max() <= Z_TOL, "max z error %.3e" % e.max()
    assert np.allclose(ro.cpu().numpy()[sel], ref["r_obs"], rtol=1.2e-7, atol=0)
    assert np.allclose(al.cpu().numpy()[sel], ref["alpha"], rtol=0, atol=2e-6)
    return qz, e, ref


def test_run_uniform_4k(T):
    _run_case(T, W.uniform_4k())


def test_run_mixture(T):
    _run_case(T, W.make(20000, 20000, 15, 61, "mixture"))


def test_run_other_levels_and_rmin(T):
    aidw = aidw_mod()
    ds = W.make(3000, 1500, 12, 62, "mixture", 4)
    _run_case(T, ds, aidw.Params(k=12, levels=(0.5, 1.25, 2.0, 3.5, 7.0), r_min=0.3, r_max=3.0))


@pytest.mark.parametrize("q,split", [(1, 1), (2, 3), (4, 1), (4, 7), (8, 1), (8, 16)])
@pytest.mark.parametrize("intpow", [1, 0])
def test_run_launch_shapes(T, q, split, intpow):
    aidw = aidw_mod()
    ds = W.make(4099, 2053, 10, 63)  # ragged: n not a multiple of the chunk or tile, m not of the block
    aidw.set_interp_config(q, split, intpow)
    try:
        _run_case(T, ds)
    finally:
        aidw.set_interp_config(0, 0, -1)


@pytest.mark.parametrize("levels", [(1.0, 2.0, 3.0, 4.0, 5.0), (2.0, 2.5, 3.0, 3.5, 4.0), (1.5, 2.0, 2.5, 3.0, 3.5),
                                    (3.0, 4.0, 5.0, 6.0, 8.0), (0.75, 1.0, 1.5, 2.0, 7.0)])
def test_integer_power_classes(T, levels):
    # alpha saturates at alpha_1 (low R) and alpha_5 (high R); integer levels take the rsq^p kernels.
    # A clustered set gives both low-R queries (inside clusters) and high-R ones (background).
    aidw = aidw_mod()
    ds = W.make(6000, 5000, 10, 64, "mixture", 6)
    p = aidw.Params(k=10, levels=levels, r_min=0.0, r_max=2.0)
    qz_fast, e_fast, ref = _run_case(T, ds, p)
    aidw.set_interp_config(0, 0, 0)
    try:
        qz_gen, e_gen, _ = _run_case(T, ds, p)
    finally:
        aidw.set_interp_config(0, 0, -1)
    # both paths evaluate the same definition; in the error metric they agree far inside the tolerance
    d = np.abs(qz_fast.cpu().numpy().astype(np.float64) - qz_gen.cpu().numpy()) / np.maximum(np.abs(ref["z"]), ref["s"])
    assert d.max() < 2e-6


def test_run_deterministic(T):
    aidw = aidw_mod()
    ds = W.uniform_4k()
    x, y, z, qx, qy = upload(T, ds)
    a = aidw.run(x, y, z, qx, qy, aidw.Params())
    b = aidw.run(x, y, z, qx, qy, aidw.Params())
    assert T.equal(a, b)


def test_coincident_queries(T):
    ds = W.make(3000, 500, 10, 71)
    # duplicate some data points, and put queries exactly on data points (some on duplicates)
    ds.x[10], ds.y[10] = ds.x[20], ds.y[20]
    ds.x[11], ds.y[11] = ds.x[20], ds.y[20]
    for j, i in enumerate([20, 5, 1000, 2999, 10]):
        ds.qx[j], ds.qy[j] = ds.x[i], ds.y[i]
    qz, _, _ = _run_case(T, ds)
    got = qz.cpu().numpy()
    assert got[0] == np.float32((np.float64(ds.z[10]) + ds.z[11] + ds.z[20]) / 3)
    assert got[1] == ds.z[5] and got[2] == ds.z[1000] and got[3] == ds.z[2999]


def test_interpolate_without_grid(T):
    aidw = aidw_mod()
    ds = W.make(2500, 700, 10, 72)
    ds.qx[3], ds.qy[3] = ds.x[9], ds.y[9]
    x, y, z, qx, qy = upload(T, ds)
    p = aidw.Params(k=10)
    g = aidw.build_grid(x, y, qx, qy, p)
    r, d1, _ = aidw.knn(g, qx, qy, 10)
    area = g.describe()["area"]
    g.close()
    qz, al = aidw.interpolate(x, y, z, qx, qy, r, d1, aidw.Params(k=10, area=area), grid=None, want_alpha=True)
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=10)
    assert zerr(qz.cpu().numpy(), ref).max() <= Z_TOL
    assert qz.cpu().numpy()[3] == ds.z[9]


@pytest.mark.parametrize("n,m,k", [(1, 3, 1), (2, 1, 2), (3, 7, 2), (65, 1, 64), (257, 300, 3)])
def test_small_and_edge_sizes(T, n, m, k):
    ds = W.make(n, m, k, 80 + n)
    _run_case(T, ds)


@pytest.mark.parametrize("n,m,k", [((1 << 22) + 13, 300, 10), (37, (1 << 19) + 5, 7)])
def test_skewed_shapes(T, n, m, k):
    """Few queries over many data points (the data axis split as finely as the partials allow,
    256 splits with a ragged last one) and many queries over a handful of points (one chunk and
    a tail per query, the kNN over a grid of a few cells): sampled queries against the oracle."""
    ds = W.make(n, m, k, 95 + k)
    _run_case(T, ds, qsel=W.sample_queries(m, 256, ds.seed))


def test_error_paths_on_gpu(T):
    aidw = aidw_mod()
    ds = W.make(100, 20, 5, 90)
    x, y, z, qx, qy = upload(T, ds)
    bad = x.clone()
    bad[7] = float("nan")
    with pytest.raises(aidw.AidwError) as e:
        aidw.run(bad, y, z, qx, qy, aidw.Params(k=5))
    assert e.value.code == aidw.ENONFINITE
    line = T.linspace(0, 1, 50, device="cuda")
    zero = T.zeros(50, device="cuda")
    with pytest.raises(aidw.AidwError) as e:
        aidw.run(line, zero, zero, line[:5].contiguous(), zero[:5].contiguous(), aidw.Params(k=3))
    assert e.value.code == aidw.EDEGENERATE
    # collinear data with an explicit area is valid
    qz = aidw.run(line, zero, line, line[:5].contiguous(), zero[:5].contiguous(), aidw.Params(k=3, area=1.0))
    assert T.isfinite(qz).all()
    os.environ["AIDW_FAULT"] = "alloc"
    try:
        with pytest.raises(aidw.AidwError) as e:
            aidw.run(x, y, z, qx, qy, aidw.Params(k=5))
        assert e.value.code == aidw.ENOMEM
    finally:
        del os.environ["AIDW_FAULT"]
    assert T.isfinite(aidw.run(x, y, z, qx, qy, aidw.Params(k=5))).all()


# ------------------------------------------------------------------ full sizes, sampled

@pytest.mark.parametrize("name", ["uniform_1m", "clustered_256k"])
def test_full_size_sampled(T, name):
    aidw = aidw_mod()
    ds = W.WORKLOADS[name]()
    sel = W.sample_queries(ds.m, 4096, ds.seed)
    x, y, z, qx, qy = upload(T, ds)
    p = aidw.Params(k=ds.k)
    # kNN of every query (the kernels run() uses), checked on the sample
    g = aidw.build_grid(x, y, qx, qy, p)
    r, d1, ix = aidw.knn(g, qx, qy, ds.k, want_idx=True)
    g.close()
    ref_i, ref_d2 = O.knn(ds.x, ds.y, ds.qx[sel], ds.qy[sel], ds.k)
    assert np.array_equal(ix.cpu().numpy()[sel], ref_i)
    # the whole method in the launch configuration the benchmark times
    qz, al, ro = aidw.run(x, y, z, qx, qy, p, want_alpha=True, want_robs=True)
    T.cuda.synchronize()
    assert T.equal(ro, r)
    zall = qz.cpu().numpy()
    assert np.all(np.isfinite(zall)) and zall.min() >= ds.z.min() and zall.max() <= ds.z.max()
    a = al.cpu().numpy()
    assert a.min() >= 1.0 and a.max() <= 5.0
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=ds.k, qsel=sel)
    e = zerr(zall[sel], ref)
    assert e.max() <= Z_TOL, "max z error %.3e" % e.max()
    assert np.allclose(a[sel], ref["alpha"], atol=2e-6)
    # the grid built for the same cell side given explicitly (exactly sized, LSD-sorted, queries
    # binned separately) gives every query the same r_obs, alpha and z bit for bit
    g2 = aidw.build_grid(x, y, qx, qy, p)
    cw = g2.info()["cell_width"]
    g2.close()
    qz2, al2, ro2 = aidw.run(x, y, z, qx, qy, aidw.Params(k=ds.k, cell_width=cw), want_alpha=True, want_robs=True)
    T.cuda.synchronize()
    assert T.equal(ro2, ro) and T.equal(al2, al) and T.equal(qz2, qz)


@pytest.mark.parametrize("name", ["uniform_1m", "clustered_256k", "ragged_rect"])
def test_knn_lds_window_equals_cache_read(T, name):
    """The kNN with each workgroup's cells staged in LDS (aidw_set_knn_config(1)) gives every
    query the same index set, r_obs and d1^2 bit for bit as the cache-read kernel, and index sets
    equal to the oracle's brute force on sampled queries.  ragged_rect: 2^17 + 37 queries over a
    1/4 x 1 rectangle (a ragged last workgroup, windows at the grid's edges)."""
    aidw = aidw_mod()
    if name == "ragged_rect":
        ds = W.make(90001, (1 << 17) + 37, 7, 41)
        ds.x = (ds.x * np.float32(0.25)).astype(np.float32)
        ds.qx = (ds.qx * np.float32(0.25)).astype(np.float32)
    else:
        ds = W.WORKLOADS[name]()
    x, y, z, qx, qy = upload(T, ds)
    p = aidw.Params(k=ds.k)
    g = aidw.build_grid(x, y, qx, qy, p)
    out = []
    for win in (0, 1):
        aidw.set_knn_config(win)
        try:
            out.append(aidw.knn(g, qx, qy, ds.k, want_d1sq=True, want_idx=True))
            T.cuda.synchronize()
        finally:
            aidw.set_knn_config(0)
    g.close()
    for a, b in zip(out[0], out[1]):
        assert T.equal(a, b)
    sel = W.sample_queries(ds.m, 1024, ds.seed)
    ref_i, _ = O.knn(ds.x, ds.y, ds.qx[sel], ds.qy[sel], ds.k)
    assert np.array_equal(out[1][2].cpu().numpy()[sel], ref_i)


# ------------------------------------------------------------------ the paper's stop rule

@pytest.mark.parametrize("case", ["constructed_miss", "uniform_4k_cw_rexp", "mixture_cw_rexp", "uniform_occ2"])
def test_knn_paper_rule_matches_oracle(T, case):
    """aidw_knn_paper (level expansion to >= k points, one more level) against the oracle's
    reading of the same rule: index sets bit-exact; the mismatch against exact kNN printed."""
    aidw = aidw_mod()
    if case == "constructed_miss":
        x = np.array([0.0, 10.0, 5.99, 3.98, 4.9], np.float32)
        y = np.array([0.0, 10.0, 5.99, 5.5, 7.2], np.float32)
        ds = W.Dataset("miss", x, y, np.zeros(5, np.float32), np.array([5.01], np.float32),
                       np.array([5.5], np.float32), 1, 0)
        params = aidw.Params(k=1, cell_width=1.0)
    elif case == "uniform_4k_cw_rexp":
        ds, params = W.uniform_4k(), aidw.Params(k=10, occupancy=0.25)
    elif case == "mixture_cw_rexp":
        ds, params = W.make(20000, 3000, 15, 41, "mixture", 16), aidw.Params(k=15, occupancy=0.25)
    else:
        ds, params = W.make(8192, 2000, 10, 42), aidw.Params(k=10)
    x, y, z, qx, qy = upload(T, ds)
    g = aidw.build_grid(x, y, qx, qy, params)
    d = g.describe()
    r, d1, ix = aidw.knn(g, qx, qy, params.k, want_idx=True, paper_rule=True)
    re, _, ixe = aidw.knn(g, qx, qy, params.k, want_idx=True)
    g.close()
    oi, od2 = O.knn_paper(ds.x, ds.y, ds.qx, ds.qy, params.k, d["min_x"], d["min_y"], d["inv_cell_width"], d["ncol"],
                          d["nrow"])
    assert np.array_equal(ix.cpu().numpy(), oi)
    assert np.allclose(r.cpu().numpy(), O.robs(od2), rtol=1.2e-7, atol=0)
    miss = np.any(ix.cpu().numpy() != ixe.cpu().numpy(), axis=1)
    rel = np.abs(r.cpu().numpy().astype(np.float64) / re.cpu().numpy() - 1.0)
    print("%s: %d of %d queries differ from exact kNN, max r_obs rel. error %.3g" % (case, miss.sum(), ds.m,
                                                                                       rel.max()))
    if case == "constructed_miss":
        assert ix.cpu().numpy()[0, 0] == 2 and ixe.cpu().numpy()[0, 0] == 3


# ------------------------------------------------------------------ the paper's baselines

@pytest.mark.parametrize("case", ["uniform_4k", "lattice_ties", "mixture"])
def test_knn_bruteforce_matches_oracle(T, case):
    aidw = aidw_mod()
    if case == "uniform_4k":
        ds, k = W.uniform_4k(), 10
    elif case == "lattice_ties":
        ds, k = tiny_lattice(51, 300, 200), 8
    else:
        ds, k = W.make(20000, 2000, 15, 52, "mixture", 16), 15
    x, y, z, qx, qy = upload(T, ds)
    r, d1, ix = aidw.knn_bruteforce(x, y, qx, qy, k, want_idx=True)
    oi, od2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, k)
    assert np.array_equal(ix.cpu().numpy(), oi)
    assert np.allclose(r.cpu().numpy(), O.robs(od2), rtol=1.2e-7, atol=0)
    d1_ref = np.where(od2[:, 0] == 0, 0.0, np.maximum(od2[:, 0].astype(np.float32), np.finfo(np.float32).tiny))
    assert np.array_equal(d1.cpu().numpy(), d1_ref.astype(np.float32))


def test_grid_knn_equals_bruteforce_at_scale(T):
    """The grid search against the O(nm) definition on the GPU: 2^18 uniform data points,
    2^15 queries, and the same on clustered data -- index sets, r_obs and d1sq bit for bit."""
    aidw = aidw_mod()
    for ds, k in ((W.make(1 << 18, 1 << 15, 10, 53), 10), (W.make(1 << 18, 1 << 15, 15, 54, "mixture", 16), 15)):
        x, y, z, qx, qy = upload(T, ds)
        g = aidw.build_grid(x, y, qx, qy, aidw.Params(k=k))
        r, d1, ix = aidw.knn(g, qx, qy, k, want_idx=True)
        g.close()
        rb, d1b, ixb = aidw.knn_bruteforce(x, y, qx, qy, k, want_idx=True)
        assert T.equal(ix, ixb) and T.equal(r, rb) and T.equal(d1, d1b)


def test_naive_interpolation_matches(T):
    aidw = aidw_mod()
    ds = W.uniform_4k()
    x, y, z, qx, qy = upload(T, ds)
    p = aidw.Params(k=10)
    g = aidw.build_grid(x, y, qx, qy, p)
    r, d1, _ = aidw.knn(g, qx, qy, 10)
    qn, an = aidw.interpolate(x, y, z, qx, qy, r, d1, p, grid=g, want_alpha=True, naive=True)
    try:
        aidw.set_interp_config(1, 1, 0)
        qt, at = aidw.interpolate(x, y, z, qx, qy, r, d1, p, grid=g, want_alpha=True)
    finally:
        aidw.set_interp_config(0, 0, -1)
    g.close()
    T.cuda.synchronize()
    assert T.equal(qn, qt) and T.equal(an, at)
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=10)
    assert zerr(qn.cpu().numpy(), ref).max() <= Z_TOL


def test_cached_temporaries_across_streams(T):
    """Temporaries are cached between calls: runs alternating between two streams (a block
    released on one stream is reused on the other after an event wait), with the cache
    released midway, all give the first run's result."""
    aidw = aidw_mod()
    ds = W.make(30000, 20000, 10, 61, "mixture", 8)
    x, y, z, qx, qy = upload(T, ds)
    p = aidw.Params(k=10)
    ref = aidw.run(x, y, z, qx, qy, p)
    T.cuda.synchronize()
    streams = [T.cuda.Stream(), T.cuda.Stream()]
    outs = []
    for i in range(6):
        s = streams[i % 2]
        s.wait_stream(T.cuda.current_stream())
        with T.cuda.stream(s):
            outs.append(aidw.run(x, y, z, qx, qy, p, stream=s))
        if i == 3:
            T.cuda.synchronize()
            aidw.release_cached_memory()
    T.cuda.synchronize()
    for o in outs:
        assert T.equal(o, ref)
