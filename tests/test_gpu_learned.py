"""Learned-R form on the GPU through the C ABI: features bit-exact against the
oracle, network forward and gradient against the FP64 reference on the same
bf16 operands, training, checkpointing, the fallback mechanics of
aidw_run_learned, and the gain of a trained network over exact kNN."""
import os
import tempfile

import numpy as np
import pytest

import oracle as O
import oracle.mlp as OM
from paper_1601_05904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1601_05904_amd as aidw
    aidw.load(build_if_missing=False)
    return torch


def mods():
    import paper_1601_05904_amd as aidw
    import paper_1601_05904_amd.learned as L
    return aidw, L


def dev(T, a):
    return T.from_numpy(np.ascontiguousarray(a)).to("cuda")


def random_params(seed, scale=0.35):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(OM.N_PARAMS) * scale
    p[-1] = 1.5
    return p.astype(np.float32)


# ------------------------------------------------------------------ features

@pytest.mark.parametrize("case", ["uniform", "mixture", "edges"])
def test_features_match_oracle(T, case):
    aidw, L = mods()
    if case == "uniform":
        ds = W.make(8000, 3000, 15, 201)
    elif case == "mixture":
        ds = W.make(20000, 4000, 15, 202, "mixture", 16)
    else:
        ds = W.make(3000, 500, 15, 203)
        ds.qx[:4] = [0.0, 1.0 - 2 ** -20, 0.0, 1.0 - 2 ** -20]
        ds.qy[:4] = [0.0, 0.0, 1.0 - 2 ** -20, 1.0 - 2 ** -20]
        ds.qx[4], ds.qy[4] = ds.x[17], ds.y[17]  # coincident with a data point
    x, y, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "qx", "qy"))
    g = aidw.build_grid(x, y, qx, qy, aidw.Params(k=15))
    d = g.describe()
    f, d1 = L.features(g, qx, qy)
    g.close()
    ref = O.features(ds.x, ds.y, ds.qx, ds.qy, d["min_x"], d["min_y"], d["inv_cell_width"], d["ncol"], d["nrow"])
    assert np.array_equal(f.cpu().numpy(), ref)
    # d1sq: exact when the nearest point is nearer than one cell width, a lower bound otherwise
    _, kd = O.knn(ds.x, ds.y, ds.qx, ds.qy, 1)
    exact = kd[:, 0].astype(np.float32)
    got = d1.cpu().numpy()
    near = np.sqrt(kd[:, 0]) < 0.999 * d["cell_width"]
    assert np.array_equal(got[near], exact[near])
    assert np.all(got <= exact * (1 + 1e-6))
    if case == "edges":
        assert got[4] == 0.0


@pytest.mark.parametrize("case", ["mixture_k15", "uniform_k10_noclip"])
def test_nn_statistic_matches_oracle(T, case):
    """aidw_nn_statistic (the training targets): R = min(r_obs / r_exp, clip) of Eq. 3-4
    against the oracle's r_obs (brute force) and r_exp (Eq. 2), within one float32 rounding."""
    aidw, L = mods()
    if case == "mixture_k15":
        ds, k, clip = W.make(20000, 5000, 15, 205, "mixture", 16), 15, 3.0
    else:
        ds, k, clip = W.make(9000, 3000, 10, 206), 10, 0.0
    x, y, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "qx", "qy"))
    g = aidw.build_grid(x, y, qx, qy, aidw.Params(k=k))
    R = aidw.nn_statistic(g, qx, qy, k, clip).cpu().numpy().astype(np.float64)
    g.close()
    b = O.bounds(ds.x, ds.y, ds.qx, ds.qy)
    r_exp = O.grid_params(b, ds.n)["r_exp"]
    _, d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, k)
    ref = O.robs(d2) / r_exp
    if clip > 0:
        ref = np.minimum(ref, clip)
        assert np.any(ref == clip) and np.any(ref < clip)
    assert np.all(np.abs(R - ref) <= 2.5 * 2.0 ** -24 * np.abs(ref)), float(np.max(np.abs(R - ref) / ref))


# ------------------------------------------------------------------ network

def check_outputs(yk, params, feat, min_exact=0.0):
    """The network's float32 outputs yk against the FP64 reference on the same bf16 operands
    (oracle.mlp.forward_candidates): every output lies in the intervals the float32 arithmetic
    allows (a bf16 activation whose value is within the float32 error of a rounding boundary
    counts with each value it can take, each such flip bounded by its own effect); outputs the
    model proves fixed and exact are bit-exact; outputs with no ambiguous activation are within
    1e-4 of the reference element-wise.  Returns the candidate model."""
    yk = np.asarray(yk, np.float64)
    cand = OM.forward_candidates(np.asarray(params, np.float64), feat)
    res = cand["resolved"]
    assert res.mean() > 0.995, res.mean()
    ok = OM.within(yk, cand)
    assert np.all(ok[res]), "outputs outside their bound: %d of %d" % (int((~ok[res]).sum()), int(res.sum()))
    clean = res & (cand["ambiguous"] == 0)
    err = np.abs(yk - cand["y"]) / (1.0 + np.abs(cand["y"]))
    assert np.all(err[clean] <= 1e-4), float(err[clean].max())
    assert cand["exact"].mean() >= min_exact, cand["exact"].mean()
    assert np.all(yk[cand["exact"]] == np.float32(cand["y"][cand["exact"]]))
    return cand


def grid_features(seed, B):
    """Network inputs on the 2^-8 grid: counts / occupancy and in-cell offsets."""
    rng = np.random.default_rng(seed)
    f = np.zeros((B, 27))
    f[:, :25] = rng.poisson(2.0, (B, 25)) * 0.5
    f[:, 25:] = rng.integers(0, 256, (B, 2)) / 256.0
    return f.astype(np.float32)


@pytest.mark.parametrize("kind,min_exact", [("positive", 0.9), ("signed", 0.4), ("mixed", 0.0)])
def test_forward_matches_fp64_reference(T, kind, min_exact):
    """aidw_mlp_forward (matrix cores) against the FP64 network, on features of a clustered
    grid and on grid-aligned synthetic features."""
    aidw, L = mods()
    ds = W.make(20000, 6000, 15, 211, "mixture", 8)
    x, y, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "qx", "qy"))
    g = aidw.build_grid(x, y, qx, qy, aidw.Params(k=15))
    f, _ = L.features(g, qx, qy, want_d1sq=False)
    g.close()
    params = OM.grid_params(5, kind)
    mlp = L.MLP(seed=1)
    mlp.set_params(params)
    assert np.array_equal(mlp.get_params(), params)
    for feat in (f.cpu().numpy(), grid_features(212, 4000)):
        yk = mlp.forward(dev(T, feat)).cpu().numpy()
        check_outputs(yk, params, feat, min_exact)


@pytest.mark.parametrize("kind", ["positive", "signed"])
def test_gradients_match_fp64_reference(T, kind):
    """aidw_mlp_gradients against the FP64 gradient on identical bf16 operands: the batch is
    drawn from samples whose every bf16 activation the float32 error cannot move (the
    forward model proves the output fixed), so both sides differentiate the same network
    at the same points.  Each entry is within 1e-4 of the sum of the magnitudes of its
    per-sample contributions (the scale of float32 summation error; entries without
    cancellation are within 1e-4 relative of their value)."""
    aidw, L = mods()
    rng = np.random.default_rng(221)
    params = OM.grid_params(6, kind)
    pool = grid_features(222, 6000)
    cand = OM.forward_candidates(params.astype(np.float64), pool)
    fixed = np.nonzero(cand["exact"])[0]
    B = 700
    assert fixed.size >= B
    feat = pool[rng.choice(fixed, B, replace=False)]
    target = (rng.random(B) * 3).astype(np.float32)
    mlp = L.MLP()
    mlp.set_params(params)
    g, loss = mlp.gradients(dev(T, feat), dev(T, target))
    lo, go, scale = OM.loss_and_grad_abs(params.astype(np.float64), feat, target)
    gk = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss) - lo) <= 1e-5 * lo
    bad = np.abs(gk - go) > 1e-4 * scale + 1e-12
    assert not bad.any(), "%d entries, worst ratio %.3g" % (
        int(bad.sum()), float((np.abs(gk - go) / (scale + 1e-30)).max()))
    well = scale > 0
    well[well] = np.abs(go[well]) >= 0.5 * scale[well]
    assert np.all(np.abs(gk[well] - go[well]) <= 1e-4 * np.abs(go[well]))
    assert well.mean() > 0.3


def test_training_reduces_loss_and_checkpoint_roundtrip(T):
    aidw, L = mods()
    sets = [W.make(1 << 15, 6000, 15, 300 + i, "mixture", 8) for i in range(2)]
    feat, target = L.training_pairs(sets)
    mlp = L.MLP(seed=3)
    losses = mlp.train(feat, target, epochs=6, batch=512, lr=3e-3, seed=3)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    # deterministic: the same seed and data give the same network
    mlp2 = L.MLP(seed=3)
    mlp2.train(feat, target, epochs=6, batch=512, lr=3e-3, seed=3)
    assert np.array_equal(mlp.get_params(), mlp2.get_params())
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        mlp.save(path)
        back = L.MLP.load_file(path)
        assert np.array_equal(back.get_params(), mlp.get_params())
        assert T.equal(back.forward(feat[:1000]), mlp.forward(feat[:1000]))
        # resuming keeps the optimiser state: one more epoch from either gives the same network
        mlp.train(feat, target, epochs=1, batch=512, lr=3e-3, seed=9)
        back.train(feat, target, epochs=1, batch=512, lr=3e-3, seed=9)
        assert np.array_equal(back.get_params(), mlp.get_params())
        with open(path, "r+b") as fh:
            fh.write(b"XXXX")
        with pytest.raises(aidw.AidwError):
            L.MLP.load_file(path)


# ------------------------------------------------------------------ learned run

def _plain_and_learned(T, ds, mlp, rule, delta, k):
    aidw, L = mods()
    x, y, z, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "z", "qx", "qy"))
    p = aidw.Params(k=k)
    qz_p, al_p, ro_p = aidw.run(x, y, z, qx, qy, p, want_alpha=True, want_robs=True)
    qz_l, al_l, rh, nfb = L.run_learned(x, y, z, qx, qy, p, mlp, rule, delta, want_alpha=True, want_rhat=True)
    T.cuda.synchronize()
    return (qz_p.cpu().numpy(), al_p.cpu().numpy(), ro_p.cpu().numpy(), qz_l.cpu().numpy(), al_l.cpu().numpy(),
            rh.cpu().numpy(), nfb)


@pytest.mark.parametrize("kind", ["positive", "signed"])
def test_learned_run_prediction_matches_fp64_network(T, kind):
    """The learned run computes features, network and decision in one kernel (network on the
    matrix cores); its prediction R_hat matches the FP64 network on the oracle's features."""
    aidw, L = mods()
    ds = W.make(30000, 9000, 15, 241, "mixture", 16)
    params = OM.grid_params(12, kind)
    mlp = L.MLP(seed=6)
    mlp.set_params(params)
    x, y, z, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "z", "qx", "qy"))
    p = aidw.Params(k=15)
    _, _, rh, _ = L.run_learned(x, y, z, qx, qy, p, mlp, L.ALPHA_EXACT, 0.3, want_rhat=True)
    g = aidw.build_grid(x, y, qx, qy, p)
    d = g.describe()
    g.close()
    feat = O.features(ds.x, ds.y, ds.qx, ds.qy, d["min_x"], d["min_y"], d["inv_cell_width"], d["ncol"], d["nrow"])
    check_outputs(rh.cpu().numpy(), params, feat, 0.3 if kind == "signed" else 0.9)


def _strip(n, m, seed):
    """Data and queries on a thin horizontal strip: a grid of one or two rows."""
    rng = np.random.default_rng(seed)
    q = lambda a: (np.floor(np.asarray(a) * 2.0 ** 20) / 2.0 ** 20).astype(np.float32)
    x, y = q(rng.random(n)), q(0.5 + 0.001 * rng.random(n))
    qx, qy = q(rng.random(m)), q(0.5 + 0.001 * rng.random(m))
    return x, y, rng.standard_normal(n).astype(np.float32), qx, qy


@pytest.mark.parametrize("case", ["n5_m37", "n40_m16", "n200_m33", "strip"])
def test_learned_prediction_small_grids(T, case):
    """R_hat of the fused fronts on grids where most of the 5 x 5 window lies outside the
    grid (a handful of cells, a one-row strip) and with a ragged last tile of queries."""
    aidw, L = mods()
    if case == "strip":
        x, y, z, qx, qy = _strip(3000, 517, 77)
        area = 0.05  # cell width sqrt(2 A / n) ~ 1 / 170 of the strip's length
    else:
        n, m = (int(v[1:]) for v in case.split("_"))
        ds = W.make(n, m, min(15, n), 300 + n, "uniform")
        x, y, z, qx, qy = ds.x, ds.y, ds.z, ds.qx, ds.qy
        area = 0.0
    params = OM.grid_params(21, "signed")
    mlp = L.MLP(seed=7)
    mlp.set_params(params)
    p = aidw.Params(k=min(15, x.size), area=area)
    dx, dy, dz, dqx, dqy = (dev(T, a) for a in (x, y, z, qx, qy))
    _, _, rh, _ = L.run_learned(dx, dy, dz, dqx, dqy, p, mlp, L.ALPHA_EXACT, 0.3, want_rhat=True)
    g = aidw.build_grid(dx, dy, dqx, dqy, p)
    d = g.describe()
    g.close()
    if case == "strip":
        assert d["nrow"] <= 2 and d["ncol"] > 100
    feat = O.features(x, y, qx, qy, d["min_x"], d["min_y"], d["inv_cell_width"], d["ncol"], d["nrow"])
    check_outputs(rh.cpu().numpy(), params, feat)
    # the one-lane front (rule 3) runs the same network on the queries the counts leave open,
    # gathered per wavefront: its predictions there are rule 1's, bit for bit
    _, _, rh3, _ = L.run_learned(dx, dy, dz, dqx, dqy, p, mlp, L.CERTIFIED_THEN_ALPHA_EXACT, 0.3, want_rhat=True)
    rh, rh3 = rh.cpu().numpy(), rh3.cpu().numpy()
    ev = ~np.isnan(rh3)
    assert np.array_equal(rh[ev], rh3[ev])


@pytest.mark.parametrize("m", [3000, 1 << 18])
def test_all_fallback_equals_plain_path(T, m):
    """Every query takes the exact kNN (delta beyond any prediction): alpha and z equal the plain
    path's bit for bit, also with a fallback list of 2^18 queries."""
    aidw, L = mods()
    ds = W.make(6000 if m < 10000 else 1 << 16, m, 15, 231, "mixture", 8)
    mlp = L.MLP(seed=4)
    qz_p, al_p, _, qz_l, al_l, _, nfb = _plain_and_learned(T, ds, mlp, L.ALPHA_EXACT, 1e9, 15)
    assert nfb == ds.m
    assert np.array_equal(al_l, al_p) and np.array_equal(qz_l, qz_p)


@pytest.mark.parametrize("rule", ["alpha_exact", "literal"])
def test_learned_rules(T, rule):
    aidw, L = mods()
    ds = W.make(8000, 4000, 15, 232, "mixture", 8)
    ds.qx[7], ds.qy[7] = ds.x[3], ds.y[3]  # a coincident query always falls back
    mlp = L.MLP(seed=5)
    mlp.set_params(random_params(9, 0.2))
    r = L.ALPHA_EXACT if rule == "alpha_exact" else L.LITERAL
    qz_p, al_p, ro_p, qz_l, al_l, rh, nfb = _plain_and_learned(T, ds, mlp, r, 0.1, 15)
    # the decision each query took, recomputed from the predictions
    lo, hi = 2 / np.pi * np.arccos(0.8), 2 / np.pi * np.arccos(-0.8)
    rh64 = rh.astype(np.float64)
    if r == L.ALPHA_EXACT:
        skip = (rh64 >= hi + 0.1) | (rh64 <= lo - 0.1)
        expect_alpha = np.where(rh64 >= hi + 0.1, 5.0, 1.0)
    else:
        skip = ~((np.abs(rh64 - 0.0) < 0.1) | (np.abs(rh64 - 2.0) < 0.1))
        _, _, expect_alpha = O.alpha(rh64, 1.0, 0.0, 2.0, W.LEVELS)  # r_exp = 1: R = r_hat
    skip[7] = False
    assert nfb == int((~skip).sum())
    assert np.allclose(al_l[skip], expect_alpha[skip], atol=2e-6)
    # fallback queries take the exact path: same alpha, and the same z as the plain run
    fb = ~skip
    assert np.array_equal(al_l[fb], al_p[fb])
    assert np.allclose(qz_l[fb], qz_p[fb], rtol=2e-6, atol=1e-7)
    assert qz_l[7] == ds.z[3]
    # skipped queries whose alpha happens to equal the exact one agree with the plain run
    same = skip & (al_l == al_p)
    assert np.allclose(qz_l[same], qz_p[same], rtol=2e-6, atol=1e-7)
    assert np.all(np.isfinite(qz_l))


def test_trained_network_gain(T):
    """A network trained on held-out mixture datasets, credited under the network-gated
    certificate (rule 4): no loss of z accuracy -- every query's alpha equals the plain path's
    bitwise, z equals the plain run's up to float32 rounding and is within 1e-5 of the FP64
    oracle -- while the
    network sends a share (at least a fifth) of the queries whose 3 x 3 certificate would fail
    straight to the exact kNN (the scan is skipped) and loses almost no certification.  An untrained network cannot
    do both.  The network's own alpha rule (rule 1) is reported, not credited: it assigns
    alpha to a few queries in the membership's transition band."""
    aidw, L = mods()
    n, mq = 1 << 18, 50000
    train = [W.make(n, mq, 15, 400 + i, "mixture", 16) for i in range(4)]
    mlp, losses = L.train_default(train, seed=11, epochs=10, batch=1024, lr=2e-3)
    assert losses[-1] < losses[0]
    ds = W.make(n, 16000, 15, 499, "mixture", 16)
    qz_p, al_p, _, qz_g, al_g, rh, nfb_g = _plain_and_learned(T, ds, mlp, L.NETWORK_GATED_CERTIFICATE, 0.3, 15)
    assert np.array_equal(al_g, al_p)
    assert np.allclose(qz_g, qz_p, rtol=2e-6, atol=1e-7)
    sel = np.arange(0, ds.m, 16)
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=15, qsel=sel)
    e = np.abs(qz_g[sel].astype(np.float64) - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
    assert e.max() <= 1e-5
    x, y, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "qx", "qy"))
    p = aidw.Params(k=15)

    def stats(net, rule):
        r, _ = L.learned_routes(x, y, qx, qy, p, net, rule, 0.3)
        r = r.cpu().numpy()
        return {"skipped": float(np.mean(r >= 2)), "failed_scans": float(np.mean(r == 1))}

    cert = stats(mlp, L.CERTIFIED)
    gated = stats(mlp, L.NETWORK_GATED_CERTIFICATE)
    untrained = L.MLP(seed=12)
    gated_u = stats(untrained, L.NETWORK_GATED_CERTIFICATE)
    _, _, _, _, al_1, _, nfb_1 = _plain_and_learned(T, ds, mlp, L.ALPHA_EXACT, 0.3, 15)
    print("certified %s | gated (trained) %s | gated (untrained) %s | rule 1 skipped %.3f wrong alpha %.4f" % (
        cert, gated, gated_u, 1.0 - nfb_1 / ds.m, float(np.mean(al_1 != al_p))))
    assert abs(1.0 - nfb_g / ds.m - gated["skipped"]) < 1e-9
    assert cert["skipped"] > 0.85
    assert gated["skipped"] >= cert["skipped"] - 0.01
    assert gated["failed_scans"] <= 0.8 * cert["failed_scans"]
    # the untrained network either loses certifications or keeps the failing scans
    assert gated_u["skipped"] < cert["skipped"] - 0.01 or gated_u["failed_scans"] > 0.8 * cert["failed_scans"]


@pytest.mark.parametrize("case", ["mixture", "uniform_k10"])
def test_certificate_independent_of_kernel(T, case):
    """The certified rule against the oracle, with nothing taken from the kernel: every query
    (not coincident with a data point) that the certificate written from the paper's grid
    (oracle.certificate: block counts and 3 x 3 distances, no dense-block limit) certifies
    with a 1 % margin is skipped; and every skipped query has R beyond the saturation point
    and alpha = alpha_5 by Eq. 4-6 on the oracle's exact (brute-force) r_obs."""
    aidw, L = mods()
    import oracle.certificate as C
    if case == "mixture":
        ds, k = W.make(40000, 6000, 15, 271, "mixture", 16), 15
    else:
        ds, k = W.make(30000, 5000, 10, 272), 10
    x, y, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "qx", "qy"))
    route, _ = L.learned_routes(x, y, qx, qy, aidw.Params(k=k), L.MLP(seed=1), L.CERTIFIED, 0.0)
    skipped = route.cpu().numpy() >= 2
    b = O.bounds(ds.x, ds.y, ds.qx, ds.qy)
    gp = O.grid_params(b, ds.n, occupancy=2.0)
    r_sat = 2.0 / np.pi * np.arccos(-0.8)  # mu(R) = 0.9 in Eq. 5 with R_min = 0, R_max = 2
    slack = (max(gp["ncol"], gp["nrow"]) + 1) * 2.0 ** -21
    cert = C.certified(ds.x, ds.y, ds.qx, ds.qy, k, b[0], b[1], gp["cw"], gp["inv_cw"], gp["ncol"], gp["nrow"],
                       slack, 1.01 * k * gp["r_exp"] * r_sat)
    _, d2 = O.knn(ds.x, ds.y, ds.qx, ds.qy, k)
    R, _, alpha = O.alpha(O.robs(d2), gp["r_exp"])
    assert cert.mean() > 0.5
    assert np.all(skipped[cert & (d2[:, 0] > 0)])
    assert np.all(alpha[skipped] == 5.0) and np.all(R[skipped] > r_sat)


def _certificate_oracle(ds, k, margin=0.0):
    """Oracle certified set (oracle/certificate.py) on the grid the library builds for ds; the
    threshold is the library's (k r_exp R_sat (1 + 1e-6)) raised by the relative margin."""
    import oracle.certificate as C
    b = O.bounds(ds.x, ds.y, ds.qx, ds.qy)
    gp = O.grid_params(b, ds.n, occupancy=2.0)
    slack = (max(gp["ncol"], gp["nrow"]) + 1) * 2.0 ** -21 + 1e-9
    r_sat = 0.0 + 2.0 / np.pi * np.arccos(-0.8)
    sum_min = k * gp["r_exp"] * min(r_sat, 2.0) * (1 + 1e-6) * (1 + margin)
    return C.certified(ds.x, ds.y, ds.qx, ds.qy, k, b[0], b[1], gp["cw"], gp["inv_cw"], gp["ncol"], gp["nrow"],
                       slack, sum_min, dense_limit=8 * k + 16)


@pytest.mark.parametrize("case", ["mixture", "uniform_k1", "small_grid"])
def test_certified_rule_is_exact(T, case):
    """Rule 2 skips kNN where the certificate proves alpha = alpha_5: as many queries as the
    oracle's bound certifies, up to the kernel's float32 margin (the oracle's distances are
    FP64); every query's alpha equals the plain path's and z stays within the error bar of
    the FP64 oracle."""
    aidw, L = mods()
    if case == "mixture":
        ds, k = W.make(40000, 6000, 15, 251, "mixture", 16), 15
    elif case == "uniform_k1":
        ds, k = W.make(20000, 3000, 1, 252), 1
    else:
        ds, k = W.make(60, 500, 5, 253, "mixture", 4), 5
    ds.qx[5], ds.qy[5] = ds.x[2], ds.y[2]  # a coincident query always falls back
    mlp = L.MLP(seed=7)
    qz_p, al_p, _, qz_l, al_l, rh, nfb = _plain_and_learned(T, ds, mlp, L.CERTIFIED, 0.0, k)
    cert = _certificate_oracle(ds, k)
    cert_strict = _certificate_oracle(ds, k, 1e-3)
    cert[5] = cert_strict[5] = False
    assert int(cert_strict.sum()) <= ds.m - nfb <= int(cert.sum())
    if case == "mixture":
        assert cert.mean() > 0.8
    assert np.all(np.isnan(rh))  # the network is not evaluated
    assert np.array_equal(al_l, al_p)
    assert qz_l[5] == ds.z[2]
    assert np.allclose(qz_l, qz_p, rtol=2e-6, atol=1e-7)
    sel = np.arange(0, ds.m, max(1, ds.m // 400))
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=k, qsel=sel)
    e = np.abs(qz_l[sel].astype(np.float64) - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
    assert e.max() <= 1e-5


def test_certified_then_network_rule(T):
    """Rule 3 skips the union of rule 2's and rule 1's queries; certified ones keep the exact alpha.
    The network runs only where the block counts do not certify: its prediction there is rule
    1's bit for bit (the same features and network in another kernel), NaN elsewhere."""
    aidw, L = mods()
    ds = W.make(20000, 4000, 15, 254, "mixture", 8)
    mlp = L.MLP(seed=5)
    mlp.set_params(random_params(9, 0.2))
    _, al_p, _, _, al_1, rh1, nfb1 = _plain_and_learned(T, ds, mlp, L.ALPHA_EXACT, 0.1, 15)
    _, _, _, _, _, _, nfb2 = _plain_and_learned(T, ds, mlp, L.CERTIFIED, 0.1, 15)
    _, _, _, qz_3, al_3, rh3, nfb3 = _plain_and_learned(T, ds, mlp, L.CERTIFIED_THEN_ALPHA_EXACT, 0.1, 15)
    ev = ~np.isnan(rh3)
    assert 0 < ev.sum() < ds.m
    assert np.array_equal(rh1[ev], rh3[ev])
    assert np.all(al_3[~ev] == al_p[~ev])  # not evaluated: certified by the counts, the exact alpha
    cert = _certificate_oracle(ds, 15)
    cert_strict = _certificate_oracle(ds, 15, 1e-3)
    hi, lo = 2 / np.pi * np.arccos(-0.8), 2 / np.pi * np.arccos(0.8)
    rh64 = rh3.astype(np.float64)
    net_skip = (rh64 >= hi + 0.1) | (rh64 <= lo - 0.1)
    assert int((cert_strict | net_skip).sum()) <= ds.m - nfb3 <= int((cert | net_skip).sum())
    assert nfb3 <= min(nfb1, nfb2)
    assert np.all(al_3[cert_strict] == al_p[cert_strict])
    assert np.all(np.isfinite(qz_3))


@pytest.mark.parametrize("rule", ["certified", "gated"])
def test_certificate_other_levels(T, rule):
    """Rules 2 and 4 with R_min = 0.2, R_max = 1.8 and levels (0.5, 1.5, 2, 2.5, 3.7): the
    saturation point the certificate must clear moves with R_min and R_max (mu >= 0.9 from
    R = R_min + R_max acos(-0.8) / pi on, Eq. 5), and a skipped query takes alpha_5 = 3.7, a
    level that is not an integer (the general pair form).  Every query's alpha equals the plain
    path's, most queries skip the kNN search, and z stays within the bar of the FP64 oracle."""
    aidw, L = mods()
    ds = W.make(40000, 6000, 15, 271, "mixture", 16)
    kw = dict(levels=(0.5, 1.5, 2.0, 2.5, 3.7), r_min=0.2, r_max=1.8)
    p = aidw.Params(k=15, **kw)
    mlp = L.MLP(seed=9)
    x, y, z, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "z", "qx", "qy"))
    qz_p, al_p, _ = aidw.run(x, y, z, qx, qy, p, want_alpha=True)
    r = L.CERTIFIED if rule == "certified" else L.NETWORK_GATED_CERTIFICATE
    qz_l, al_l, _, nfb = L.run_learned(x, y, z, qx, qy, p, mlp, r, 0.3, want_alpha=True)
    T.cuda.synchronize()
    al_p, al_l, qz_l = al_p.cpu().numpy(), al_l.cpu().numpy(), qz_l.cpu().numpy()
    assert 0 < nfb < ds.m // 2
    assert np.array_equal(al_l, al_p)
    assert np.count_nonzero(al_l == np.float32(3.7)) > ds.m // 2
    assert np.allclose(qz_l, qz_p.cpu().numpy(), rtol=2e-6, atol=1e-7)
    sel = np.arange(0, ds.m, max(1, ds.m // 400))
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=15, qsel=sel, **kw)
    e = np.abs(qz_l[sel].astype(np.float64) - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
    assert e.max() <= 1e-5
    assert np.allclose(al_l[sel], ref["alpha"], rtol=0, atol=2e-6)


@pytest.mark.parametrize("case", ["mixture", "small_grid"])
def test_gated_rule_prediction(T, case):
    """Rule 4 evaluates the network in the one-lane front, on the queries the block counts leave
    open (gathered per wavefront into tiles), with the features and network of rule 1: where it
    ran, its prediction equals rule 1's bit for bit; where it did not, the query is certified by
    the counts (route 2) or takes the exact kNN without a scan (route 0); and every query it
    sent to the 3 x 3 scan had a prediction at or beyond r_sat_hi - delta."""
    aidw, L = mods()
    if case == "mixture":
        ds, k = W.make(30000, 9000, 15, 261, "mixture", 16), 15
    else:
        ds, k = W.make(60, 500, 5, 262, "mixture", 4), 5
    mlp = L.MLP(seed=8)
    mlp.set_params(random_params(13, 0.2))
    x, y, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "qx", "qy"))
    p = aidw.Params(k=k)
    _, rh1 = L.learned_routes(x, y, qx, qy, p, mlp, L.ALPHA_EXACT, 0.3, want_rhat=True)
    r4, rh4 = L.learned_routes(x, y, qx, qy, p, mlp, L.NETWORK_GATED_CERTIFICATE, 0.3, want_rhat=True)
    rh1, rh4, r4 = rh1.cpu().numpy(), rh4.cpu().numpy(), r4.cpu().numpy()
    ev = ~np.isnan(rh4)
    assert ev.any()
    assert np.array_equal(rh1[ev], rh4[ev])
    assert np.all(np.isin(r4[~ev], (0, 2)))
    scanned = (r4 == 1) | (r4 == 3)
    assert np.all(ev[scanned])
    assert np.all(rh4[scanned].astype(np.float64) >= 2 / np.pi * np.arccos(-0.8) - 0.3)


def test_certified_rule_full_size(T):
    """Rule 2 on the clustered 2^20 workload in the configuration the benchmark times: every
    query's alpha equals the plain path's (bitwise), most queries skip the kNN search, and z
    on sampled queries is within the error bar of the FP64 oracle."""
    aidw, L = mods()
    ds = W.learned_1m()
    mlp = L.MLP(seed=3)
    qz_p, al_p, _, qz_l, al_l, rh, nfb = _plain_and_learned(T, ds, mlp, L.CERTIFIED, 0.0, ds.k)
    assert np.array_equal(al_l, al_p)
    assert 1.0 - nfb / ds.m > 0.9
    assert np.allclose(qz_l, qz_p, rtol=2e-6, atol=1e-7)
    sel = W.sample_queries(ds.m, 4096, ds.seed)
    ref = O.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=ds.k, qsel=sel)
    e = np.abs(qz_l[sel].astype(np.float64) - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
    assert e.max() <= 1e-5


def test_learned_rule_validation(T):
    """An unknown rule or a negative delta is rejected before any work is queued."""
    aidw, L = mods()
    ds = W.make(500, 100, 5, 261)
    x, y, z, qx, qy = (dev(T, getattr(ds, a)) for a in ("x", "y", "z", "qx", "qy"))
    mlp = L.MLP(seed=2)
    for rule, delta in ((5, 0.1), (-1, 0.1), (L.CERTIFIED, -1.0)):
        with pytest.raises(aidw.AidwError) as e:
            L.run_learned(x, y, z, qx, qy, aidw.Params(k=5), mlp, rule, delta)
        assert e.value.code == -1
