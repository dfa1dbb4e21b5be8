"""Batched form: many independent AIDW jobs in one pipeline (aidw_batch_* of the C ABI).

Argument marshalling and the autotuner's cache only; every step runs in the
library's kernels.

    import paper_1601_05904_amd.batch as B
    jobs = [B.Job(x, y, z, qx, qy, aidw.Params(k=10)), ...]      # device tensors
    plan = B.Plan(jobs, B.autotune(jobs), want_alpha=True)
    plan.run(stream)                 # no allocation, no host sync; graph replay if config.use_graph
    plan.qz[j], plan.alpha[j]        # outputs, one tensor per job
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import tempfile
from dataclasses import asdict, dataclass, field

from . import (AidwError, Params, _BatchConfig, _BatchDesc, _BatchTiming, _check, _dev, _Job, _stream, load)

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TUNE_FILE = os.path.join(_HERE, "batch_tune.json")


@dataclass
class Config:
    """aidw_batch_config: pair-kernel queries per lane, data points per work item
    (0 = whole job), persistent workgroups per compute unit, integer-power loops,
    HIP graph capture and replay."""
    q: int = 1
    split_points: int = 0
    workers_per_cu: int = 8
    integer_powers: int = 1
    use_graph: int = 0

    def _c(self):
        c = _BatchConfig()
        c.q, c.split_points, c.workers_per_cu = int(self.q), int(self.split_points), int(self.workers_per_cu)
        c.integer_powers, c.use_graph = int(self.integer_powers), int(self.use_graph)
        return c


@dataclass
class Job:
    """One interpolation problem: device float32 tensors x, y, z [n] and qx, qy [m]."""
    x: object
    y: object
    z: object
    qx: object
    qy: object
    params: Params = field(default_factory=Params)


def _job_array(jobs, qz, alpha, robs):
    arr = (_Job * len(jobs))()
    for j, jb in enumerate(jobs):
        n, m = int(jb.x.numel()), int(jb.qx.numel())
        if jb.y.numel() != n or jb.z.numel() != n or jb.qy.numel() != m:
            raise ValueError("job %d: x, y, z and qx, qy must have matching sizes" % j)
        a = arr[j]
        a.x, a.y, a.z = _dev(jb.x, "x"), _dev(jb.y, "y"), _dev(jb.z, "z")
        a.n, a.m = n, m
        a.qx, a.qy = _dev(jb.qx, "qx"), _dev(jb.qy, "qy")
        a.params = jb.params._c()
        a.qz = _dev(qz[j], "qz")
        a.alpha_out = _dev(alpha[j], "alpha") if alpha else None
        a.r_obs_out = _dev(robs[j], "r_obs") if robs else None
    return arr


def _outputs(jobs, want_alpha, want_robs):
    import torch
    qz = [torch.empty(int(jb.qx.numel()), dtype=torch.float32, device=jb.qx.device) for jb in jobs]
    alpha = [torch.empty_like(t) for t in qz] if want_alpha else None
    robs = [torch.empty_like(t) for t in qz] if want_robs else None
    return qz, alpha, robs


class Plan:
    """An aidw_batch plan over fixed jobs; outputs live in qz / alpha / r_obs (lists of tensors)."""

    def __init__(self, jobs, config: Config | None = None, want_alpha=False, want_robs=False):
        L = load()
        self.jobs = list(jobs)
        self.config = config or Config()
        self.qz, self.alpha, self.r_obs = _outputs(self.jobs, want_alpha, want_robs)
        self._arr = _job_array(self.jobs, self.qz, self.alpha, self.r_obs)
        h = ctypes.c_void_p()
        cfg = self.config._c()
        _check(L.aidw_batch_create(self._arr, len(self.jobs), ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if not self._h:
            raise ValueError("plan is closed")
        return self._h

    def run(self, stream=None):
        _check(load().aidw_batch_run(self.handle, _stream(stream)))

    def status(self, stream=None, raise_on_error=False):
        """Per-job aidw_status list of the last run (synchronises the stream)."""
        st = (ctypes.c_int32 * len(self.jobs))()
        r = load().aidw_batch_job_status(self.handle, st, _stream(stream))
        if raise_on_error:
            _check(r)
        return list(st)

    def describe(self) -> dict:
        d = _BatchDesc()
        _check(load().aidw_batch_describe(self.handle, ctypes.byref(d)))
        out = {f: getattr(d, f) for f, _ in _BatchDesc._fields_ if f != "config"}
        out["config"] = {f: getattr(d.config, f) for f, _ in _BatchConfig._fields_}
        return out

    def set_timing(self, enable: bool):
        _check(load().aidw_batch_set_timing(self.handle, 1 if enable else 0))

    def last_timing(self) -> dict:
        t = _BatchTiming()
        _check(load().aidw_batch_last_timing(self.handle, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in _BatchTiming._fields_}

    def close(self):
        if self._h:
            load().aidw_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batch(jobs, config: Config | None = None, want_alpha=False, want_robs=False, stream=None):
    """One-shot aidw_run_batch: returns (qz, alpha, r_obs, status) with lists of tensors and the per-job status."""
    L = load()
    qz, alpha, robs = _outputs(jobs, want_alpha, want_robs)
    arr = _job_array(jobs, qz, alpha, robs)
    st = (ctypes.c_int32 * len(jobs))()
    cfg = (config or Config())._c()
    r = L.aidw_run_batch(arr, len(jobs), ctypes.byref(cfg), st, _stream(stream))
    if r not in (0,) and not any(st):
        _check(r)  # a plan-level error (arguments, device), not a per-job status
    return qz, alpha, robs, list(st)


# ---------------------------------------------------------------- autotuner

def candidates(graph: bool = True):
    """The search space: queries per lane, data points per work item, workgroups per CU."""
    out = []
    for q in (1, 2):
        for split in (0, 16384, 4096):
            for w in (4, 8, 16):
                out.append(Config(q=q, split_points=split, workers_per_cu=w, integer_powers=1,
                                  use_graph=1 if graph else 0))
    return out


def size_class(jobs) -> str:
    """Cache key: device, job count, total queries, largest data set and total pairs, each to a power of two."""
    import torch
    dev = torch.cuda.get_device_properties(jobs[0].qx.device)
    arch = getattr(dev, "gcnArchName", dev.name).split(":")[0]
    n = [int(j.x.numel()) for j in jobs]
    m = [int(j.qx.numel()) for j in jobs]
    pairs = sum(a * b for a, b in zip(n, m))

    def lg(v):
        return int(round(math.log2(max(v, 1))))
    return "%s|jobs=2^%d|queries=2^%d|max_n=2^%d|pairs=2^%d" % (arch, lg(len(jobs)), lg(sum(m)), lg(max(n)),
                                                               lg(pairs))


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _write(path, data):
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(jobs, cands=None, reps=3, stream=None):
    """Times every candidate on these jobs (aidw_batch_tune); returns [(Config, ms per run)], fastest first."""
    L = load()
    cands = list(cands or candidates())
    qz, alpha, robs = _outputs(jobs, False, False)
    arr = _job_array(jobs, qz, alpha, robs)
    carr = (_BatchConfig * len(cands))(*[c._c() for c in cands])
    ms = (ctypes.c_float * len(cands))()
    s = stream
    if s is None:
        import torch
        s = torch.cuda.Stream()  # graph capture needs a created stream
    _check(L.aidw_batch_tune(arr, len(jobs), carr, len(cands), int(reps), ms, s.cuda_stream))
    return sorted(zip(cands, list(ms)), key=lambda t: t[1])


def autotune(jobs, cache_path=None, cands=None, reps=3, retune=False, stream=None) -> Config:
    """The tuned Config for this size class.  Looks in the cache file (default:
    $AIDW_TUNE_CACHE, else ~/.cache/aidw/batch_tune.json), then in the defaults
    shipped with the package; otherwise tunes and stores the winner in the cache."""
    key = size_class(jobs)
    path = cache_path or os.environ.get("AIDW_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "aidw", "batch_tune.json")
    if not retune:
        for src in (path, DEFAULT_TUNE_FILE):
            hit = _read(src).get(key)
            if hit:
                return Config(**hit["config"])
    ranked = tune(jobs, cands, reps, stream)
    best, ms = ranked[0]
    data = _read(path)
    data[key] = {"config": asdict(best), "ms": ms,
                 "ranking": [[asdict(c), t] for c, t in ranked]}
    try:
        _write(path, data)
    except OSError:
        pass  # a read-only cache location only costs a re-tune next time
    return best


__all__ = ["Config", "Job", "Plan", "run_batch", "candidates", "size_class", "tune", "autotune", "AidwError"]
