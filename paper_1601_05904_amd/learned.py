"""Learned-R form: Python binding of the aidw_mlp_* / aidw_features / aidw_run_learned
calls of include/aidw.h (argument marshalling only; every step runs in the
library's kernels), and the training recipe.

Training recipe: held-out datasets drawn like the evaluation workload (mixture
data, uniform queries; seeds 100-103 unless given), targets = the exact R of
Eq. 4 from the library's exact kNN (Eq. 3), clipped at 3 (alpha is saturated
well before that: at R >= 1.59 for the default R_min, R_max), Adam on the GPU.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import Params, _VP, _check, _dev, _stream, build_grid, load, nn_statistic

N_IN = 27
N_PARAMS = 6017
LITERAL, ALPHA_EXACT, CERTIFIED, CERTIFIED_THEN_ALPHA_EXACT, NETWORK_GATED_CERTIFICATE = 0, 1, 2, 3, 4
ROUTE_KNN, ROUTE_KNN_AFTER_SCAN, ROUTE_CERT_COUNTS, ROUTE_CERT_DISTANCES, ROUTE_NETWORK = 0, 1, 2, 3, 4


class MLP:
    """An aidw_mlp handle."""

    def __init__(self, seed: int = 0, occupancy: float = 2.0, handle=None):
        if handle is None:
            h = _VP()
            _check(load().aidw_mlp_create(ctypes.c_uint64(seed), float(occupancy), ctypes.byref(h)))
            handle = h.value
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise ValueError("network is closed")
        return self._h

    @classmethod
    def load_file(cls, path: str) -> "MLP":
        h = _VP()
        _check(load().aidw_mlp_load(path.encode(), ctypes.byref(h)))
        return cls(handle=h.value)

    def save(self, path: str):
        _check(load().aidw_mlp_save(self.handle, path.encode()))

    @property
    def occupancy(self) -> float:
        return load().aidw_mlp_occupancy(self.handle)

    def get_params(self) -> np.ndarray:
        out = np.zeros(N_PARAMS, np.float32)
        _check(load().aidw_mlp_get_params(self.handle, out.ctypes.data_as(_VP)))
        return out

    def set_params(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != N_PARAMS:
            raise ValueError("need %d parameters" % N_PARAMS)
        _check(load().aidw_mlp_set_params(self.handle, a.ctypes.data_as(_VP)))

    def forward(self, feat, stream=None):
        import torch
        m = feat.shape[0]
        out = torch.empty(m, dtype=torch.float32, device=feat.device)
        _check(load().aidw_mlp_forward(self.handle, _dev(feat, "feat"), m, out.data_ptr(), _stream(stream)))
        return out

    def gradients(self, feat, target, stream=None):
        """-> (grad [N_PARAMS], loss) for one batch, no update."""
        import torch
        g = torch.empty(N_PARAMS + 1, dtype=torch.float32, device=feat.device)
        _check(load().aidw_mlp_gradients(self.handle, _dev(feat, "feat"), _dev(target, "target"), feat.shape[0],
                                         g.data_ptr(), _stream(stream)))
        return g[:N_PARAMS], g[N_PARAMS]

    def train(self, feat, target, epochs=8, batch=1024, lr=2e-3, seed=0, stream=None):
        """Adam on the GPU; returns the mean batch loss of each epoch."""
        losses = np.zeros(epochs, np.float32)
        _check(load().aidw_mlp_train(self.handle, _dev(feat, "feat"), _dev(target, "target"), feat.shape[0],
                                     int(epochs), int(batch), float(lr), ctypes.c_uint64(seed),
                                     losses.ctypes.data_as(_VP), _stream(stream)))
        return losses

    def close(self):
        if self._h:
            load().aidw_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(grid, qx, qy, want_d1sq=True, stream=None):
    """aidw_features -> (feat [m, 27], d1sq [m] or None)."""
    import torch
    m = qx.numel()
    feat = torch.empty((m, N_IN), dtype=torch.float32, device=qx.device)
    d1 = torch.empty(m, dtype=torch.float32, device=qx.device) if want_d1sq else None
    _check(load().aidw_features(grid.handle, _dev(qx, "qx"), _dev(qy, "qy"), m, feat.data_ptr(),
                                None if d1 is None else d1.data_ptr(), _stream(stream)))
    return feat, d1


def run_learned(x, y, z, qx, qy, params: Params, mlp: MLP, rule=ALPHA_EXACT, delta=0.1, want_alpha=False,
                want_rhat=False, out=None, stream=None):
    """aidw_run_learned -> (qz, alpha or None, r_hat or None, fallback_count)."""
    import torch
    p = params._c()
    m = qx.numel()
    qz = out if out is not None else torch.empty(m, dtype=torch.float32, device=qx.device)
    al = torch.empty(m, dtype=torch.float32, device=qx.device) if want_alpha else None
    rh = torch.empty(m, dtype=torch.float32, device=qx.device) if want_rhat else None
    cnt = ctypes.c_int64()
    _check(load().aidw_run_learned(_dev(x, "x"), _dev(y, "y"), _dev(z, "z"), x.numel(), _dev(qx, "qx"),
                                   _dev(qy, "qy"), m, ctypes.byref(p), mlp.handle, int(rule), float(delta),
                                   _dev(qz, "qz"), None if al is None else al.data_ptr(),
                                   None if rh is None else rh.data_ptr(), ctypes.byref(cnt), _stream(stream)))
    return qz, al, rh, int(cnt.value)


def learned_routes(x, y, qx, qy, params: Params, mlp: MLP, rule, delta, want_rhat=False, stream=None):
    """aidw_learned_routes -> (route [m] uint8, r_hat [m] or None): each query's route under the rule."""
    import torch
    p = params._c()
    m = qx.numel()
    route = torch.empty(m, dtype=torch.uint8, device=qx.device)
    rh = torch.empty(m, dtype=torch.float32, device=qx.device) if want_rhat else None
    _check(load().aidw_learned_routes(_dev(x, "x"), _dev(y, "y"), x.numel(), _dev(qx, "qx"), _dev(qy, "qy"), m,
                                      ctypes.byref(p), mlp.handle, int(rule), float(delta), route.data_ptr(),
                                      None if rh is None else rh.data_ptr(), _stream(stream)))
    return route, rh


def training_pairs(datasets, k=15, occupancy=2.0, clip=3.0):
    """(features, target) on the GPU for the queries of each dataset: target = min(R, clip),
    R = r_obs / r_exp from the exact kNN (aidw_nn_statistic)."""
    import torch
    feats, targets = [], []
    for ds in datasets:
        t = {a: torch.from_numpy(getattr(ds, a)).cuda() for a in ("x", "y", "qx", "qy")}
        g = build_grid(t["x"], t["y"], t["qx"], t["qy"], Params(k=k, occupancy=occupancy))
        f, _ = features(g, t["qx"], t["qy"], want_d1sq=False)
        targets.append(nn_statistic(g, t["qx"], t["qy"], k, clip))
        g.close()
        feats.append(f)
    return torch.cat(feats).contiguous(), torch.cat(targets).contiguous()


def train_default(datasets, seed=0, epochs=8, batch=1024, lr=2e-3, occupancy=2.0, k=15):
    """A network trained by the recipe above; returns (mlp, epoch_losses)."""
    feat, target = training_pairs(datasets, k=k, occupancy=occupancy)
    mlp = MLP(seed=seed, occupancy=occupancy)
    losses = mlp.train(feat, target, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return mlp, losses
