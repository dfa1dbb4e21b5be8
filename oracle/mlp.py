"""FP64 reference of the learned-R network -- TEST INFRASTRUCTURE ONLY.

The network maps the 27 features of a query (oracle.features) to a prediction
of the nearest-neighbour statistic R of Eq. 4:

    x  = bf16(feat)                       27
    a1 = bf16(W1) x + b1,  h1 = bf16(gelu(a1))    64
    a2 = bf16(W2) h1 + b2, h2 = bf16(gelu(a2))    64
    y  = bf16(W3) h2 + b3                         1

with gelu(u) = u / 2 * (1 + tanh(sqrt(2 / pi) (u + 0.044715 u^3))) and the
training loss L = mean_b (y_b - t_b)^2.  Parameters are one float32 vector:
W1 (64 x 27, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (64), b3 (1).
bf16() rounds to the nearest bfloat16 (ties to even) after rounding to float32;
those are the points where the GPU kernels round their operands.  Everything
else is float64 here.  The gradient treats every rounding as the identity
(the straight-through gradient the GPU also computes).  With rounding=False
the network is smooth, which lets the tests check the analytic gradient by
finite differences.
"""
import numpy as np

N_IN, N_H = 27, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
C_GELU = np.sqrt(2.0 / np.pi)


def unpack(params):
    out, o = {}, 0
    p = np.asarray(params, np.float64)
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to float32, then to the nearest bfloat16 (ties to even); returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(u):
    return 0.5 * u * (1.0 + np.tanh(C_GELU * (u + 0.044715 * u ** 3)))


def gelu_grad(u):
    t = np.tanh(C_GELU * (u + 0.044715 * u ** 3))
    return 0.5 * (1.0 + t) + 0.5 * u * (1.0 - t * t) * C_GELU * (1.0 + 3 * 0.044715 * u * u)


def forward(params, feat, rounding=True):
    """-> (y [B], cache) for features [B, 27]."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    P = unpack(params)
    x = r(feat)
    a1 = x @ r(P["W1"]).T + P["b1"]
    h1 = r(gelu(a1))
    a2 = h1 @ r(P["W2"]).T + P["b2"]
    h2 = r(gelu(a2))
    y = h2 @ r(P["W3"]) + P["b3"][0]
    return y, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, y=y, W2=r(P["W2"]), W3=r(P["W3"]))


def loss_and_grad(params, feat, target, rounding=True):
    """Mean squared error over the batch and its gradient with respect to the parameter vector."""
    y, c = forward(params, feat, rounding)
    t = np.asarray(target, np.float64)
    B = y.shape[0]
    loss = np.mean((y - t) ** 2)
    dy = 2.0 * (y - t) / B
    g = {}
    g["W3"] = dy @ c["h2"]
    g["b3"] = np.array([dy.sum()])
    da2 = np.outer(dy, c["W3"]) * gelu_grad(c["a2"])
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ c["W2"]) * gelu_grad(c["a1"])
    g["W1"] = da1.T @ c["x"]
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


# ---------------------------------------------------------------------------
# Which outputs a float32 implementation may produce.
#
# The GPU kernels evaluate the same network with float32 accumulation (matrix-core
# or dot-product instructions, any summation order) and a float32 GELU of the
# form g = u - u / (1 + 2^z), z = u (K1 + K2 u^2) (hardware exp2 and reciprocal,
# each within one ulp).  Every product of two bf16 values is exact in float32, so
# the only differences from the float64 reference are (i) the rounding of the
# float32 sums, (ii) the float32 GELU, and (iii) the bf16 rounding of an activation
# whose value lies within the error of (i) + (ii) of a rounding boundary: there the
# two sides may take different bf16 values.  forward_candidates bounds all three:
#   * a sum is exact in float32, in any order, when its terms lie on a common
#     power-of-two grid 2^q and the sum of their magnitudes S is below 2^24 2^q;
#     otherwise its error is at most gamma u S (u = 2^-24, gamma >= number of terms);
#   * the GELU error follows the float32 operation count of the formula above;
#   * an activation whose bf16 value is not fixed by these bounds contributes every
#     bf16 value it can take: in layer 1 significant ones are enumerated (they pass
#     through the nonlinear layer 2), negligible ones are added to layer 2's error;
#     in layer 2 they widen the output interval by |W3_j| times their spread.
# The result is, per sample, a short list of intervals that must hold the output.
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24
_K1 = 2.0 * C_GELU * np.log2(np.e)
_K2 = _K1 * 0.044715


def grid_exponent(v):
    """Exponent e of the largest power of two 2^e dividing each finite value (v / 2^e is an
    odd integer); +inf for zero, which lies on every grid."""
    v = np.asarray(v, np.float64)
    m, e = np.frexp(np.abs(v))
    mi = (m * 2.0 ** 53).astype(np.int64)
    low = (mi & (-mi)).astype(np.float64)
    with np.errstate(divide="ignore"):
        tz = np.log2(np.where(low > 0, low, 1.0))
    return np.where(v == 0, np.inf, e - 53 + tz)


def _sum_bound(X, W, b, gamma, qx=None):
    """c = b + X W^T in float64 (exact: bf16 products and short sums), and the bound on the
    float32 error of that sum in any order (0 when provably exact)."""
    c = X @ W.T + b
    S = np.abs(X) @ np.abs(W).T + np.abs(b)
    qx = grid_exponent(X) if qx is None else qx
    qw = grid_exponent(W)
    qb = grid_exponent(np.asarray(b, np.float32).astype(np.float64))
    q = np.empty(c.shape)
    for s in range(0, X.shape[0], 256):
        q[s:s + 256] = np.min(qx[s:s + 256, None, :] + qw[None, :, :], axis=2)
    q = np.minimum(q, qb[None, :])
    with np.errstate(over="ignore"):
        exact = S < np.exp2(np.minimum(24.0 + q, 1000.0))
    return c, np.where(exact, 0.0, gamma * U32 * S)


def gelu_f32_bound(a, ea):
    """Bound on |GELU evaluated in float32 by the kernels' formula - gelu(a')| over every a'
    within ea of a (a' is what the float32 sum produced)."""
    a = np.asarray(a, np.float64)
    am = np.abs(a) + ea
    z = a * (_K1 + _K2 * a * a)
    with np.errstate(over="ignore"):
        ez = np.exp2(np.minimum(z, 1000.0))
        r = 1.0 / (1.0 + ez)
        t = np.where(np.isfinite(ez), ez / (1.0 + ez) ** 2, 0.0)
    g = np.abs(gelu(a)) + 1.13 * ea
    own = am * (3.0 * U32 * r + t * (2.0 * U32 + 3.0 * U32 * np.abs(z))) + U32 * g
    return 2.0 * own + 1.13 * ea


def _bf16_next_up(v):
    f = np.float32(v)
    bits = int(np.array(f, np.float32).view(np.uint32))
    if f == 0:
        bits = 0x00010000
    elif f > 0:
        bits += 0x10000
    else:
        bits -= 0x10000
    return float(np.array(bits, np.uint32).view(np.float32))


def _bf16_values(lo, hi, cap=64):
    """The bf16 values from lo to hi; more than cap of them: cap + 1 values (a marker)."""
    vals, v = [], lo
    while v <= hi and len(vals) <= cap:
        vals.append(v)
        v = _bf16_next_up(v)
    return vals


def forward_candidates(params, feat, max_combos=64, negligible=1e-7, max_values=4):
    """Per sample, the intervals [lo, hi] that hold every output a float32 implementation of
    forward() can produce (see above).  A layer-1 activation whose bf16 value is not fixed is
    enumerated (each of its at most max_values possible values) when its effect on layer 2
    exceeds `negligible`, the most significant first, while the product of the choices stays
    within max_combos; every other one widens layer 2's error by |W2[:, j]| times its spread.
    Returns a dict:
        y          float64 reference output (forward with rounding)
        ivals      list over samples of arrays [c, 2] of intervals (their union holds the output)
        ambiguous  number of activations whose bf16 value is not fixed
        exact      True where the output is fixed and exactly representable: ivals is one point
                   and a correct float32 implementation returns that value bit for bit
        resolved   always True (kept for callers that check it)"""
    P = unpack(params)
    W1, W2, W3 = bf16(P["W1"]), bf16(P["W2"]), bf16(P["W3"])
    b1 = np.asarray(P["b1"], np.float32).astype(np.float64)
    b2 = np.asarray(P["b2"], np.float32).astype(np.float64)
    b3 = float(np.float32(P["b3"][0]))
    x = bf16(feat)
    B = x.shape[0]
    y_ref, _ = forward(params, feat)
    c1, e1 = _sum_bound(x, W1, b1, 30.0)
    g1 = gelu(c1)
    eg1 = gelu_f32_bound(c1, e1)
    h1 = bf16(g1)
    lo1, hi1 = bf16(g1 - eg1), bf16(g1 + eg1)
    dev1 = np.maximum(hi1 - h1, h1 - lo1)              # largest change of an activation
    W2abs = np.abs(W2)
    effect1 = dev1 * np.max(W2abs, axis=0)[None, :]

    def layer2_to_y(h1v, absorbed_row):
        c2, e2 = _sum_bound(h1v, W2, b2, 70.0)
        e2 = e2 + absorbed_row
        g2 = gelu(c2)
        eg2 = gelu_f32_bound(c2, e2)
        lo2, hi2 = bf16(g2 - eg2), bf16(g2 + eg2)
        ylo = b3 + np.sum(np.minimum(W3 * lo2, W3 * hi2), axis=1)
        yhi = b3 + np.sum(np.maximum(W3 * lo2, W3 * hi2), axis=1)
        point = np.all(lo2 == hi2, axis=1)
        c3, e3 = _sum_bound(lo2, W3[None, :], np.array([b3]), 70.0)
        e3 = np.where(point, e3[:, 0], 70.0 * U32 * (np.abs(lo2) @ np.abs(W3) + np.abs(hi2) @ np.abs(W3) + abs(b3)))
        amb2 = np.sum(lo2 != hi2, axis=1)
        return ylo - e3, yhi + e3, point & (e3 == 0) & (e2.max(axis=1) == 0), amb2

    # base: every unfixed layer-1 activation folded into layer 2's error (always sound)
    absorbed = dev1 @ W2abs.T
    ylo, yhi, exact, amb2 = layer2_to_y(h1, absorbed)
    amb1 = np.sum(lo1 != hi1, axis=1)
    ivals = [np.array([[ylo[b], yhi[b]]]) for b in range(B)]
    exact = exact & (amb1 == 0)
    for b in np.nonzero(np.any(effect1 > negligible, axis=1))[0]:
        order = np.argsort(-effect1[b])
        enum_j, choices, combos = [], [], 1
        for j in order:
            if effect1[b, j] <= negligible:
                break
            vals = _bf16_values(lo1[b, j], hi1[b, j])
            if len(vals) > max_values or len(vals) < 2 or combos * len(vals) > max_combos:
                continue
            enum_j.append(j)
            choices.append(vals)
            combos *= len(vals)
        if not enum_j:
            continue
        rest = dev1[b].copy()
        rest[enum_j] = 0.0
        absorbed_b = rest @ W2abs.T
        rows = []
        for combo in np.ndindex(*[len(c) for c in choices]):
            hv = h1[b].copy()
            for j, ci, ch in zip(enum_j, combo, choices):
                hv[j] = ch[ci]
            rows.append(hv)
        lo_, hi_, _, a2 = layer2_to_y(np.array(rows), np.repeat(absorbed_b[None, :], len(rows), axis=0))
        ivals[b] = np.stack([lo_, hi_], axis=1)
        amb2[b] = max(amb2[b], int(a2.max()))
    return {"y": y_ref, "ivals": ivals, "ambiguous": amb1 + amb2, "exact": exact, "resolved": np.ones(B, bool)}


def within(yk, cand):
    """True for each sample whose float32 output yk lies in one of its intervals (a float32
    result may carry one rounding of the exact sum: half an ulp of slack)."""
    out = np.zeros(len(yk), bool)
    for b, (v, iv) in enumerate(zip(np.asarray(yk, np.float64), cand["ivals"])):
        if iv.shape[0] == 0:
            continue
        slack = 0.5 * U32 * 2 * np.maximum(np.abs(iv[:, 0]), np.abs(iv[:, 1]))
        if cand["exact"][b]:
            out[b] = v == float(np.float32(iv[0, 0]))
        else:
            out[b] = bool(np.any((v >= iv[:, 0] - slack) & (v <= iv[:, 1] + slack)))
    return out


def loss_and_grad_abs(params, feat, target, rounding=True):
    """loss_and_grad plus, per parameter, the sum over the batch of the magnitudes of the
    per-sample contributions (the scale of the float32 error of a summed gradient entry)."""
    y, c = forward(params, feat, rounding)
    t = np.asarray(target, np.float64)
    B = y.shape[0]
    dy = 2.0 * (y - t) / B
    da2 = np.outer(dy, c["W3"]) * gelu_grad(c["a2"])
    da1 = (da2 @ c["W2"]) * gelu_grad(c["a1"])
    A = np.abs
    g = {"W3": A(dy) @ A(c["h2"]), "b3": np.array([A(dy).sum()]), "W2": A(da2).T @ A(c["h1"]),
         "b2": A(da2).sum(axis=0), "W1": A(da1).T @ A(c["x"]), "b1": A(da1).sum(axis=0)}
    loss, grad = loss_and_grad(params, feat, target, rounding)
    return loss, grad, pack(g)


def grid_params(seed, kind="positive"):
    """Parameters whose bf16 weights lie on coarse power-of-two grids, so that the float32
    sums of a correct implementation are exact for inputs on the 2^-8 grid (see
    forward_candidates): "positive" keeps the pre-activations positive and below ~4 (every
    sum exact; GELU stays well away from the identity, whose values on the same grid would
    sit on bf16 rounding boundaries), "signed" keeps them in about [-1.5, 2.5] (both signs
    of GELU's argument, sums still exact), "mixed" spreads them over [-6, 6] (saturated
    negative activations with fine bf16 grids: inexact sums, bounded)."""
    rng = np.random.default_rng(seed)
    d = {}
    if kind == "positive":
        d["W1"] = rng.integers(-16, 17, (N_H, N_IN)) / 256.0
        d["b1"] = 2.0 + rng.integers(-128, 129, N_H) / 256.0
        d["W2"] = rng.integers(-2, 3, (N_H, N_H)) / 64.0
        d["b2"] = 1.5 + rng.integers(-128, 129, N_H) / 256.0
        d["W3"] = rng.integers(-16, 17, N_H) / 64.0
    elif kind == "signed":
        d["W1"] = rng.integers(-32, 33, (N_H, N_IN)) / 256.0
        d["b1"] = 0.5 + rng.integers(-128, 129, N_H) / 256.0
        d["W2"] = rng.integers(-4, 5, (N_H, N_H)) / 64.0
        d["b2"] = 0.5 + rng.integers(-128, 129, N_H) / 256.0
        d["W3"] = rng.integers(-32, 33, N_H) / 64.0
    else:
        d["W1"] = rng.integers(-64, 65, (N_H, N_IN)) / 256.0
        d["b1"] = rng.integers(-256, 257, N_H) / 256.0
        d["W2"] = rng.integers(-32, 33, (N_H, N_H)) / 64.0
        d["b2"] = rng.integers(-256, 257, N_H) / 256.0
        d["W3"] = rng.integers(-32, 33, N_H) / 64.0
    d["b3"] = np.array([1.5])
    return pack(d).astype(np.float32)
