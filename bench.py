#!/usr/bin/env python3
"""Benchmark: interpolated points/s of the whole AIDW method on one MI355X.

A step is one aidw_run over the workload (grid build, query binning, kNN with
Eq. 3, Eq. 4-6 and the weighted mean of Eq. 1 over all data points, and the
coincident-query fix-up) with inputs already resident in HBM.  The default
workload is n = m = 2^20 uniform points, k = 10 (synthetic, seeded).

Printed: one JSON line with the metric, the pair kernel's roofline fraction
(its duration measured with HIP events on the run's stream), the plain FP64
CPU oracle timed on a bounded sample of the same workload on this host, and
the z error of the timed run on that sample.  More measurements ride on the
same line: "learned_r" (plain vs learned-R on the clustered 2^20 workload,
after training the network on held-out sets, for the network's fallback rule,
the certified rule and the two combined), "batch" (256 independent jobs as one
autotuned plan replayed as a HIP graph), "clustered" (the 2^18 mixture
workload) and "paper_rule" (the paper's kNN stop rule against exact kNN);
the plain run also reports its grid and kNN stages against
HBM ("stage_bandwidth") and a rate with host-memory copies included ("host_inclusive").

    python bench.py [--steps K] [--warmup W] [--workload uniform_1m] [--cpu-sample S] [--no-cpu-baseline]
                    [--no-learned] [--no-batch] [--no-plain] [--batch-loop] [--no-clustered]
                    [--no-host-inclusive] [--no-paper-rule]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interpolated points/s at n=m=1M (plain vs learned-R) at stated z error"

# Roofline of the pair kernels, from the chip's unit counts and clock:
#   256 CUs at 2.4 GHz; FP32 VALU issues 128 lanes / clk / CU (157.3 TFLOP/s = 256 * 2.4e9 * 128 * 2);
#   transcendentals (v_log_f32, v_exp_f32, v_rsq_f32) issue 32 lanes / clk / CU and do not overlap
#   with other VALU work.  Both rates, and the no-overlap behaviour of streams that mix them in the
#   proportions of the pair loop, are measured by `bench.py --issue-rates` (the microbenchmark
#   paper_1601_05904_amd/ubench/issue_rate.hip); the measured figures are kept in
#   profiles/valu_transcendental_issue_rates.md.
# Minimum work of one pair (query j, data point i):
#   general alpha: 7 VALU (2 sub, mul + fma for d^2, mul for the exponent, fma + add for the sums)
#                  + 2 transcendentals (log2, exp2);
#   alpha == integer p: 6 VALU (d^2 and the sums) + the multiplies of the shortest addition chain
#                  for r^p + 1 transcendental (rsq).
# The peak for a workload is the harmonic mix over its queries' classes.
CUS, CLOCK = 256, 2.4e9
VALU_PER_CLK_CU, TRANS_PER_CLK_CU = 128, 32
CHAIN_MULS = {1: 0, 2: 1, 3: 2, 4: 2, 5: 3, 6: 3, 7: 4, 8: 3}


def pair_peak(valu, trans, rates=(VALU_PER_CLK_CU, TRANS_PER_CLK_CU)):
    return CUS * CLOCK / (valu / rates[0] + trans / rates[1])


PEAK_GENERAL = pair_peak(7, 2)


def class_mix_peak(alpha, levels, rates=(VALU_PER_CLK_CU, TRANS_PER_CLK_CU)):
    """Peak pairs/s for the queries' alpha values (integer levels take the one-transcendental form)."""
    a = np.asarray(alpha, np.float64)
    inv = np.full(a.shape, 1.0 / pair_peak(7, 2, rates))
    for p in sorted(set(int(v) for v in levels if float(v).is_integer() and 1 <= v <= 8)):
        inv[a == p] = 1.0 / pair_peak(6 + CHAIN_MULS[p], 1, rates)
    return 1.0 / inv.mean(), {("alpha=%d" % p): float(np.mean(a == p)) for p in range(1, 9) if np.any(a == p)}


def measured_rates():
    """(VALU, transcendental) lanes per clock per CU that the issue-rate microbenchmark measured on
    the chip (the pair's own VALU mix; the slowest transcendental), from its committed summary."""
    path = os.path.join(ROOT, "profiles", "valu_transcendental_issue_rates.md")
    if not os.path.exists(path):
        return None
    f = profile_fields(path)
    try:
        return float(f["- valu_lanes_per_clk_cu_pair_mix"]), float(f["- trans_lanes_per_clk_cu"])
    except (KeyError, ValueError):
        return None


PAIR_SOURCES = {"k_interp": ("interp.hip", "pair_core.h", "api.hip"), "k_b_interp": ("batch.hip", "pair_core.h"),
                "grid_knn": ("grid.hip", "grid_band.hip", "grid_core.h", "knn.hip", "knn_core.h", "interp.hip",
                             "api.hip")}
HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s


def source_hash(kernel):
    """Fingerprint of the code a kernel is built from (counter summaries record it): the
    sources with their // comments and blank lines removed, so comment edits keep it."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in PAIR_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1601_05904_amd", "csrc", name)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of a pair kernel, from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel calibration); None if the kernel's sources
    have changed since the counters were taken, or no summary exists for this workload."""
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    fields = profile_fields(path)
    if fields.get("source_sha256_16") != source_hash(kernel) or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def profile_fields(path):
    """The "key: value" lines of a committed counter summary."""
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    return fields


def stage_bandwidth(grid, ds, stages):
    """The grid and kNN stages against HBM.  Algorithmic bytes (minimum traffic of the step):
    grid = 8 (n + m) bounds + 36 n (cell key and index written, sorted, gathered) + 8 nCells (CSR);
    kNN = 8 m (queries) + 12 n (sorted x, y, index) + 4 nCells (cell offsets) + 12 m (r_obs, d1^2, alpha).
    Both stages are latency-bound (sub-millisecond, dependent gathers); the measured bytes come from
    the committed FETCH_SIZE / WRITE_SIZE summary when its sources are unchanged."""
    n, m = ds.n, ds.m
    ncells = grid["ncol"] * grid["nrow"]
    alg = {"grid": 8 * (n + m) + 36 * n + 8 * ncells, "knn": 8 * m + 12 * n + 4 * ncells + 12 * m}
    ms = {"grid": stages["grid_ms"], "knn": stages["knn_ms"]}
    measured = {}
    path = os.path.join(ROOT, "profiles", "grid_knn_%s_counters.md" % ds.name)
    if os.path.exists(path):
        f = profile_fields(path)
        if f.get("source_sha256_16") == source_hash("grid_knn"):
            measured = {"grid": float(f["grid_bytes_per_call"]), "knn": float(f["knn_bytes_per_call"])}
    out = {"bound": "latency", "peak_GBps": HBM_PEAK / 1e9, "ncells": ncells,
           "note": "the knn stage is query binning + kNN + Eq. 4-6 and the class keys"}
    for st in ("grid", "knn"):
        out[st] = {"ms": ms[st], "algorithmic_bytes": alg[st], "GBps": alg[st] / (ms[st] * 1e-3) / 1e9,
                   "frac": alg[st] / (ms[st] * 1e-3) / HBM_PEAK,
                   "measured_bytes": measured.get(st),
                   "measured_GBps": measured[st] / (ms[st] * 1e-3) / 1e9 if st in measured else None}
    return out


def host_inclusive(ds, p, steps):
    """points/s with the inputs in pinned host memory: copies in, aidw_run, the output copied back."""
    import torch

    import paper_1601_05904_amd as aidw
    dev = torch.device("cuda", 0)
    host = {k: torch.from_numpy(getattr(ds, k)).pin_memory() for k in ("x", "y", "z", "qx", "qy")}
    back = torch.empty(ds.m, dtype=torch.float32).pin_memory()
    stream = torch.cuda.current_stream()

    def step():
        d = {k: v.to(dev, non_blocking=True) for k, v in host.items()}
        qz = aidw.run(d["x"], d["y"], d["z"], d["qx"], d["qy"], p, stream=stream)
        back.copy_(qz, non_blocking=True)
        torch.cuda.synchronize()
    step()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"value": ds.m / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms, "steps": steps,
            "note": "H2D of x, y, z, qx, qy and D2H of z from pinned host memory, included"}


def clustered_measurement(args):
    """The clustered workload (16-component mixture + background, uniform queries): points/s, the
    pair kernels against their roofline, and the grid / kNN stages against HBM."""
    import torch

    import paper_1601_05904_amd as aidw
    from paper_1601_05904_amd import workloads as W
    ds = W.WORKLOADS["clustered_256k"]()
    dev = torch.device("cuda", 0)
    x, y, z, qx, qy = (torch.from_numpy(getattr(ds, k)).to(dev) for k in ("x", "y", "z", "qx", "qy"))
    p = aidw.Params(k=ds.k, levels=ds.levels, r_min=ds.r_min, r_max=ds.r_max, occupancy=ds.occupancy)
    qz = torch.empty(ds.m, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    ms, stages = timed_runs(lambda: aidw.run(x, y, z, qx, qy, p, out=qz, stream=stream), args.clustered_steps, 2)
    _, alpha, _ = aidw.run(x, y, z, qx, qy, p, want_alpha=True, stream=stream)
    peak, mix = class_mix_peak(alpha.cpu().numpy(), ds.levels)
    pairs = float(ds.n) * float(ds.m)
    achieved = pairs / (stages["interp_ms"] * 1e-3)
    g = aidw.build_grid(x, y, qx, qy, p, stream=stream)
    desc = g.describe()
    g.close()
    return {"workload": "clustered_256k", "n": ds.n, "m": ds.m, "k": ds.k, "value": ds.m / (ms * 1e-3),
            "unit": "points/s", "ms_per_step": ms, "steps": args.clustered_steps, "stages_ms": stages,
            "pairs_roofline": {"bound": "alu", "kernel": "k_interp", "achieved": achieved / 1e9, "peak": peak / 1e9,
                               "unit": "Gpair/s", "frac": achieved / peak, "class_mix": mix},
            "stage_bandwidth": stage_bandwidth(desc, ds, stages)}


def paper_rule_measurement(args):
    """The paper's "+1 level" stop rule (aidw_knn_paper) against the exact kNN (aidw_knn, equal to
    brute force bit for bit) on the uniform 4096, uniform 2^20 and clustered 2^18 workloads, at the
    paper's cell width (cw = r_exp: 0.25 points per cell) and at 2 points per cell: queries whose
    neighbour set differs, the largest relative r_obs error, and both kernels' stage times."""
    import torch

    import paper_1601_05904_amd as aidw
    from paper_1601_05904_amd import workloads as W
    rows = []
    for wl in ("uniform_4k", "uniform_1m", "clustered_256k"):
        ds = W.WORKLOADS[wl]()
        x, y, qx, qy = (torch.from_numpy(getattr(ds, a)).cuda() for a in ("x", "y", "qx", "qy"))
        for occ in (0.25, 2.0):
            p = aidw.Params(k=ds.k, occupancy=occ)
            g = aidw.build_grid(x, y, qx, qy, p)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            aidw.knn(g, qx, qy, ds.k, want_idx=True)
            aidw.knn(g, qx, qy, ds.k, want_idx=True, paper_rule=True)
            ev[0].record()
            re, _, ie = aidw.knn(g, qx, qy, ds.k, want_idx=True)
            ev[1].record()
            rp, _, ip = aidw.knn(g, qx, qy, ds.k, want_idx=True, paper_rule=True)
            ev[2].record()
            torch.cuda.synchronize()
            g.close()
            differ = (ie != ip).any(dim=1)
            rel = ((rp.double() - re.double()).abs() / re.double()).max().item()
            rows.append({"workload": wl, "n": ds.n, "m": ds.m, "k": ds.k, "occupancy": occ,
                         "queries_differing": int(differ.sum().item()), "max_rel_r_obs_error": rel,
                         "exact_ms": ev[0].elapsed_time(ev[1]), "paper_rule_ms": ev[1].elapsed_time(ev[2])})
    return rows


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uniform_1m")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="queries of the CPU-baseline and z-error sample")
    ap.add_argument("--cpu-sample-1t", type=int, default=256, help="queries of the one-thread CPU-baseline run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-R comparison")
    ap.add_argument("--learned-workload", default="learned_1m")
    ap.add_argument("--learned-steps", type=int, default=5)
    ap.add_argument("--delta", type=float, default=0.3, help="fallback margin of the alpha-exact rule")
    ap.add_argument("--gate-delta", type=float, default=0.3,
                    help="margin of the network-gated certificate: the 3 x 3 certificate is tried where r_hat >= "
                         "R_sat - gate_delta")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-jobs measurement")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the headline plain run (profiling of the other legs only)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-clustered", action="store_true", help="skip the clustered 2^18 workload")
    ap.add_argument("--no-paper-rule", action="store_true", help="skip the paper's kNN stop rule against exact kNN")
    ap.add_argument("--clustered-steps", type=int, default=10)
    ap.add_argument("--no-host-inclusive", action="store_true", help="skip the host-memory-inclusive timing")
    ap.add_argument("--batch-loop", action="store_true",
                    help="also time the same jobs as one aidw_run per job (context for the batched form)")
    ap.add_argument("--sweep", action="store_true",
                    help="only the paper's size sweep (n = m = 10K..1000K): grid vs brute-force kNN, tiled vs "
                         "untiled interpolation, device stage times and host-inclusive totals")
    ap.add_argument("--sweep-sizes", default="10,50,100,500,1000", help="sizes in units of 1024 points")
    ap.add_argument("--issue-rates", action="store_true",
                    help="only the VALU / transcendental issue-rate microbenchmark behind the pair roofline")
    ap.add_argument("--knn-variants", action="store_true",
                    help="only time the two kNN kernels (cache reads; cells staged in LDS) on the 2^20 and 2^18 "
                         "workloads")
    ap.add_argument("--knn-workloads", default="uniform_1m,clustered_256k,learned_1m")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes (reference for HBM traffic counters)")
    return ap.parse_args()


ISSUE_KINDS = ["fma (v_fma_f32)", "fmac (v_fmac_f32)", "exp2", "log2", "rsq", "rsq+9fmac", "log2+exp2+7fmac",
               "pair loop alpha=5 (cached data)", "mul (v_mul_f32)", "add (v_add_f32)",
               "pair VALU mix (4 fma-type + 5 mul/add)"]


def issue_rates(args):
    """The VALU / transcendental issue-rate microbenchmark: lanes issued per clock per CU for
    streams of one float32 instruction kind (fma, fmac, mul, add, each transcendental), for the
    nine VALU operations of the integer-alpha pair without its rsq, for the two mixes of a
    transcendental with FMAs, and for the pair loop itself over cached data.  From these: the
    VALU rate of the pair's own instruction mix, the transcendental rate, whether the two
    overlap, and the ceiling they set for one alpha = 5 pair (9 VALU + 1 rsq, serial issue)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1601_05904_amd", "libaidw_ubench.so"))
    lib.aidw_ubench_issue_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    lib.aidw_ubench_counts.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    blocks = CUS * 8  # 8 wavefronts per SIMD
    rows = {}
    for kind, name in enumerate(ISSUE_KINDS):
        v, t = ctypes.c_int(), ctypes.c_int()
        lib.aidw_ubench_counts(kind, ctypes.byref(v), ctypes.byref(t))
        ms, st, rt = ctypes.c_float(), ctypes.c_uint64(), ctypes.c_uint64()
        iters = 64
        while True:
            rc = lib.aidw_ubench_issue_rate(kind, iters, blocks, ctypes.byref(ms), ctypes.byref(st), ctypes.byref(rt))
            if rc != 0:
                raise RuntimeError("issue-rate microbenchmark failed: %d" % rc)
            if ms.value >= 40.0 or iters >= 1 << 20:
                break
            iters = int(iters * max(2.0, 50.0 / max(ms.value, 0.05)))
        clk = st.value / rt.value * 100e6 if rt.value else float("nan")
        lanes = float(blocks) * 256 * iters
        sec = ms.value * 1e-3
        rows[name] = {"iters": iters, "ms": ms.value, "clock_GHz": clk / 1e9,
                      "valu_per_lane": v.value, "trans_per_lane": t.value,
                      "valu_lanes_per_clk_cu": lanes * v.value / (sec * clk * CUS),
                      "trans_lanes_per_clk_cu": lanes * t.value / (sec * clk * CUS),
                      "valu_lanes_per_clk_cu_nominal": lanes * v.value / (sec * CLOCK * CUS),
                      "trans_lanes_per_clk_cu_nominal": lanes * t.value / (sec * CLOCK * CUS)}
        print(json.dumps({"issue_rate": name, "ms": ms.value, "clock_GHz": clk / 1e9}), file=sys.stderr, flush=True)

    def best(keys, field):
        return max(rows[k][field] for k in keys)

    fma_only = best(("fma (v_fma_f32)", "fmac (v_fmac_f32)"), "valu_lanes_per_clk_cu_nominal")
    mul_add = best(("mul (v_mul_f32)", "add (v_add_f32)"), "valu_lanes_per_clk_cu_nominal")
    mix = rows["pair VALU mix (4 fma-type + 5 mul/add)"]["valu_lanes_per_clk_cu_nominal"]
    trans = min(rows[k]["trans_lanes_per_clk_cu_nominal"] for k in ("exp2", "log2", "rsq"))
    pl = rows["pair loop alpha=5 (cached data)"]
    pl["pairs_per_clk_cu"] = pl["trans_lanes_per_clk_cu"]  # one transcendental per pair
    pl["pairs_per_s_at_2.4GHz"] = pl["trans_lanes_per_clk_cu_nominal"] * CUS * CLOCK
    for name, fma_share in (("rsq+9fmac", 1.0), ("log2+exp2+7fmac", 1.0)):
        r = rows[name]
        steps = r["valu_lanes_per_clk_cu_nominal"] / r["valu_per_lane"]  # mixed steps per clk per CU
        serial = 1.0 / (r["valu_per_lane"] / fma_only + r["trans_per_lane"] / trans)
        overlap = 1.0 / max(r["valu_per_lane"] / fma_only, r["trans_per_lane"] / trans)
        r["steps_per_clk_cu_nominal"] = steps
        r["serial_model_steps_per_clk_cu"] = serial
        r["overlap_model_steps_per_clk_cu"] = overlap
        r["frac_of_serial_model"] = steps / serial
    ceiling = 1.0 / (9.0 / mix + 1.0 / trans)  # alpha = 5 pairs per clk per CU, serial issue
    return {"issue_rates": rows,
            "valu_lanes_per_clk_cu_fma_only": fma_only, "valu_lanes_per_clk_cu_mul_add": mul_add,
            "valu_lanes_per_clk_cu_pair_mix": mix, "trans_lanes_per_clk_cu": trans,
            "alpha5_pair_ceiling": {"pairs_per_clk_cu": ceiling, "pairs_per_s_at_2.4GHz": ceiling * CUS * CLOCK,
                                    "model": "9 VALU at the pair mix's rate + 1 rsq at the transcendental rate, "
                                             "no overlap"},
            "published_model": {"valu_lanes_per_clk_cu": VALU_PER_CLK_CU, "trans_lanes_per_clk_cu": TRANS_PER_CLK_CU,
                                "alpha5_pairs_per_s": pair_peak(9, 1)},
            "note": "rates per clock per CU, *_nominal at 2.4 GHz (the launch's wall time over 2.4e9 clocks); "
                    "clock_GHz is block 0's s_memtime / s_memrealtime.  A mixed stream at <= 1.0 of the serial "
                    "model means transcendentals and VALU operations do not overlap."}


def knn_variants(args):
    """aidw_knn on every query of each workload with the cache-read kernel and with each workgroup's cells
    staged in LDS (aidw_set_knn_config): device time of the call (query binning included; median of 5 after
    one warm-up) and whether the two give the same r_obs, d1^2 and index sets bit for bit."""
    import torch

    import paper_1601_05904_amd as aidw
    from paper_1601_05904_amd import workloads as W

    rows = []
    for name in args.knn_workloads.split(","):
        ds = W.WORKLOADS[name]()
        t = {a: torch.from_numpy(getattr(ds, a)).cuda() for a in ("x", "y", "qx", "qy")}
        g = aidw.build_grid(t["x"], t["y"], t["qx"], t["qy"], aidw.Params(k=ds.k))
        res, outs = {}, {}
        for win in (0, 1):
            aidw.set_knn_config(win)
            try:
                ts = []
                for rep in range(6):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    outs[win] = aidw.knn(g, t["qx"], t["qy"], ds.k, want_d1sq=True, want_idx=True)
                    e1.record()
                    torch.cuda.synchronize()
                    if rep:
                        ts.append(e0.elapsed_time(e1))
            finally:
                aidw.set_knn_config(0)
            res[win] = float(np.median(ts))
        g.close()
        same = all(torch.equal(a, b) for a, b in zip(outs[0], outs[1]))
        rows.append({"workload": name, "m": ds.m, "k": ds.k, "cache_read_ms": res[0], "lds_window_ms": res[1],
                     "bitwise_equal": same})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return rows


def copy_calibration(mb):
    """A plain elementwise kernel of known traffic: reads and writes mb MB once per launch."""
    import torch
    a = torch.ones(mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4, "launches": 3}))


def timed_runs(fn, steps, warmup):
    """Runs fn warmup + steps times with per-stage timing; returns (ms per step, mean stage times)."""
    import torch

    import paper_1601_05904_amd as aidw
    aidw.set_timing(True)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
        stages.append(aidw.last_timing())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    aidw.set_timing(False)
    mean = {k: float(np.mean([s[k] for s in stages])) for k in ("grid_ms", "knn_ms", "interp_ms", "finish_ms")}
    return (t1 - t0) * 1e3 / steps, mean


def learned_comparison(args, with_oracle):
    """Plain vs learned-R on the clustered 2^20 workload: the network is trained first on held-out
    datasets (same recipe, seeds 100-103), then both paths are timed on the evaluation set."""
    import torch

    import paper_1601_05904_amd as aidw
    import paper_1601_05904_amd.learned as L
    from paper_1601_05904_amd import workloads as W

    t0 = time.perf_counter()
    train = W.learned_training_sets()
    feat, target = L.training_pairs(train, k=15)
    del train
    t1 = time.perf_counter()
    mlp = L.MLP(seed=11)
    losses = mlp.train(feat, target, epochs=16, batch=1024, lr=2e-3, seed=11)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    npairs = int(feat.shape[0])
    del feat, target

    ds = W.WORKLOADS[args.learned_workload]()
    dev = torch.device("cuda", 0)
    x, y, z, qx, qy = (torch.from_numpy(getattr(ds, k)).to(dev) for k in ("x", "y", "z", "qx", "qy"))
    p = aidw.Params(k=ds.k, levels=ds.levels, r_min=ds.r_min, r_max=ds.r_max, occupancy=ds.occupancy)
    qz_p = torch.empty(ds.m, dtype=torch.float32, device=dev)
    ms_p, st_p = timed_runs(lambda: aidw.run(x, y, z, qx, qy, p, out=qz_p), args.learned_steps, 1)
    _, al_p, _ = aidw.run(x, y, z, qx, qy, p, want_alpha=True)
    rstage_p = st_p["grid_ms"] + st_p["knn_ms"]
    sel = ref = None
    if with_oracle:
        import oracle
        sel = W.sample_queries(ds.m, args.cpu_sample, ds.seed)
        ref = oracle.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=ds.k, levels=ds.levels, r_min=ds.r_min,
                          r_max=ds.r_max, occupancy=ds.occupancy, qsel=sel)

    def z_error(qz):
        e = np.abs(qz.cpu().numpy()[sel].astype(np.float64) - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
        return {"max": float(e.max()), "median": float(np.median(e)), "frac_within_1e-5": float(np.mean(e <= 1e-5)),
                "sample": len(sel)}

    x_, y_ = x, y

    def one_rule(rule, delta):
        qz_l = torch.empty(ds.m, dtype=torch.float32, device=dev)
        ms_l, st_l = timed_runs(lambda: L.run_learned(x, y, z, qx, qy, p, mlp, rule, delta, out=qz_l),
                                args.learned_steps, 1)
        _, al_l, _, nfb = L.run_learned(x, y, z, qx, qy, p, mlp, rule, delta, want_alpha=True)
        route, _ = L.learned_routes(x_, y_, qx, qy, p, mlp, rule, delta)
        rc = np.bincount(route.cpu().numpy(), minlength=5) / ds.m
        rstage_l = st_l["grid_ms"] + st_l["knn_ms"]
        r = {"rule": rule, "delta": delta, "learned_points_per_s": ds.m / (ms_l * 1e-3),
             "speedup_end_to_end": ms_p / ms_l, "learned_rstage_ms": rstage_l, "speedup_rstage": rstage_p / rstage_l,
             "learned_stages_ms": st_l, "skipped_knn_fraction": 1.0 - nfb / ds.m,
             "alpha_mismatch_fraction": float((al_p != al_l).float().mean().item()),
             "routes": {"exact_knn": float(rc[0]), "exact_knn_after_failed_scan": float(rc[1]),
                        "certified_by_counts": float(rc[2]), "certified_by_3x3": float(rc[3]),
                        "network_alpha": float(rc[4])}}
        if with_oracle:
            r["z_error_learned"] = z_error(qz_l)
        return r

    out = {"workload": args.learned_workload, "n": ds.n, "m": ds.m, "k": ds.k,
           "plain_points_per_s": ds.m / (ms_p * 1e-3), "plain_rstage_ms": rstage_p, "plain_stages_ms": st_p}
    if with_oracle:
        out["z_error_plain"] = z_error(qz_p)
    rules = {"network_alpha_exact": (L.ALPHA_EXACT, args.delta), "network_literal": (L.LITERAL, 0.1),
             "certified": (L.CERTIFIED, 0.0), "certified_then_network": (L.CERTIFIED_THEN_ALPHA_EXACT, args.delta),
             "network_gated_certificate": (L.NETWORK_GATED_CERTIFICATE, args.gate_delta)}
    out["rules"] = {name: one_rule(*rd) for name, rd in rules.items()}
    # equal z error: every query's alpha equals the plain path's (z is then the plain run's up to
    # the float32 rounding of the nearest-distance scale of the pair weights) and, on the oracle's
    # sample, every z is within the stated 1e-5 bar, as the plain run's
    eq = {}
    for name, r in out["rules"].items():
        ok = r["alpha_mismatch_fraction"] == 0.0
        if with_oracle:
            ok = ok and r["z_error_learned"]["max"] <= 1e-5 and out["z_error_plain"]["max"] <= 1e-5
        if ok:
            eq[name] = r
    if eq:
        best = max(eq, key=lambda k_: eq[k_]["speedup_rstage"])
        out["at_equal_z_error"] = {"rule": best, "speedup_rstage": eq[best]["speedup_rstage"],
                                   "speedup_end_to_end": eq[best]["speedup_end_to_end"],
                                   "rules_at_equal_z_error": sorted(eq),
                                   "target_2x_rstage_met": eq[best]["speedup_rstage"] >= 2.0}
    else:
        out["at_equal_z_error"] = {"rule": None, "target_2x_rstage_met": False}
    out["training"] = {"pairs": npairs, "epochs": 16, "batch": 1024, "lr": 2e-3, "final_loss": float(losses[-1]),
                       "data_s": t1 - t0, "train_s": t2 - t1}
    mlp.close()
    return out


def batch_measurement(args, with_oracle):
    """The 256-job workload (n log-uniform in [1024, 65536], m = n, k from {8, 10, 15}, half uniform, half
    8-cluster mixtures) as one plan in the autotuned launch shape, replayed as a HIP graph: aggregate
    points/s over all jobs, the persistent pair kernel against its roofline, and sampled z errors."""
    import torch

    import paper_1601_05904_amd as aidw
    import paper_1601_05904_amd.batch as B
    from paper_1601_05904_amd import workloads as W

    dss = W.batch_jobs()
    dev = torch.device("cuda", 0)
    jobs = [B.Job(*(torch.from_numpy(getattr(ds, k)).to(dev) for k in ("x", "y", "z", "qx", "qy")),
                  params=aidw.Params(k=ds.k, levels=ds.levels, r_min=ds.r_min, r_max=ds.r_max,
                                     occupancy=ds.occupancy)) for ds in dss]
    torch.cuda.synchronize()
    tt0 = time.perf_counter()
    config = B.autotune(jobs)
    tune_s = time.perf_counter() - tt0
    config.use_graph = 1
    plan = B.Plan(jobs, config, want_alpha=True)
    info = plan.describe()
    side = torch.cuda.Stream()
    for _ in range(2):
        plan.run(side)
    side.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        plan.run(side)
    side.synchronize()
    t1 = time.perf_counter()
    assert plan.status(side) == [0] * len(dss)
    ms = (t1 - t0) * 1e3 / args.batch_steps
    # stage times from timed (direct) runs of the same plan
    plan.set_timing(True)
    stages = []
    for _ in range(3):
        plan.run(side)
        stages.append(plan.last_timing())
    plan.set_timing(False)
    st = {k: float(np.mean([s_[k] for s_ in stages])) for k in stages[0]}
    # roofline of the persistent pair kernel: every query's class weighted by its job's n
    inv, pairs = 0.0, 0.0
    for ds, a in zip(dss, plan.alpha):
        al = a.cpu().numpy().astype(np.float64)
        pk = np.full(al.shape, PEAK_GENERAL)
        for p_ in sorted(set(int(v) for v in ds.levels if float(v).is_integer() and 1 <= v <= 8)):
            pk[al == p_] = pair_peak(6 + CHAIN_MULS[p_], 1)
        inv += float(ds.n) * float(np.sum(1.0 / pk))
        pairs += float(ds.n) * float(ds.m)
    peak = pairs / inv
    achieved = pairs / (st["interp_ms"] * 1e-3)
    out = {"workload": "batch_256", "jobs": len(dss), "total_queries": info["total_queries"],
           "total_data": info["total_data"], "total_pairs": pairs, "value": info["total_queries"] / (ms * 1e-3),
           "unit": "points/s", "ms_per_step": ms, "steps": args.batch_steps, "graph": True,
           "config": info["config"], "work_items": info["work_items"], "workers": info["workers"],
           "autotune_s": tune_s, "stages_ms": st,
           "roofline": {"bound": "alu", "kernel": "k_b_interp", "achieved": achieved / 1e9, "peak": peak / 1e9,
                        "unit": "Gpair/s", "frac": achieved / peak, "units_per_launch": pairs,
                        "traffic": measured_traffic("k_b_interp", "batch_256")}}
    if args.batch_loop:
        aidw.set_interp_config(0, 0, -1)
        outs = []
        torch.cuda.synchronize()
        l0 = time.perf_counter()
        for jb in jobs:
            outs.append(aidw.run(jb.x, jb.y, jb.z, jb.qx, jb.qy, jb.params))
        torch.cuda.synchronize()
        out["per_job_loop_ms"] = (time.perf_counter() - l0) * 1e3
    if with_oracle:
        import oracle
        worst, count = 0.0, 0
        for j, ds in enumerate(dss):
            sel = W.sample_queries(ds.m, 16, 9000 + j)
            ref = oracle.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, k=ds.k, levels=ds.levels, r_min=ds.r_min,
                              r_max=ds.r_max, occupancy=ds.occupancy, qsel=sel)
            zg = plan.qz[j].cpu().numpy()[sel].astype(np.float64)
            e = np.abs(zg - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
            worst, count = max(worst, float(e.max())), count + len(sel)
        out["z_error"] = {"max": worst, "sample": "%d queries (16 per job)" % count}
    plan.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(ds, args):
    """The FP64 oracle on this host's cores: all threads on the sampled queries (every data point
    each), median of 3 timings, and one thread on the first cpu_sample_1t of them, median of 3.
    The rate is per interpolated point, so the whole workload's time is extrapolated linearly in m.
    Returns (baseline dict, the oracle's results on the sample, the sample)."""
    import oracle
    from paper_1601_05904_amd import workloads as W
    sel = W.sample_queries(ds.m, args.cpu_sample, ds.seed)
    kw = dict(k=ds.k, levels=ds.levels, r_min=ds.r_min, r_max=ds.r_max, occupancy=ds.occupancy)

    def timed(q, reps):
        ts, res = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            res = oracle.aidw(ds.x, ds.y, ds.z, ds.qx, ds.qy, qsel=q, **kw)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts, res

    threads = oracle.num_threads()
    t_all, ts_all, ref = timed(sel, 3)
    sel1 = sel[:args.cpu_sample_1t]
    oracle.set_threads(1)
    try:
        t_one, ts_one, _ = timed(sel1, 3)
    finally:
        oracle.set_threads(threads)
    rate = len(sel) / t_all
    rate1 = len(sel1) / t_one
    base = {"value": rate, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the %d queries (every data point each), FP64, median of 3 runs (%s s); rate "
                      "extrapolated linearly in m" % (len(sel), ds.m, ", ".join("%.2f" % t for t in ts_all)),
            "cpu_model": cpu_model(), "timing": "median of 3", "extrapolated": True,
            "extrapolated_full_workload_s": ds.m / rate,
            "one_thread": {"value": rate1, "unit": "points/s", "cores": 1,
                           "sample": "%d queries, median of 3 runs (%s s)" % (
                               len(sel1), ", ".join("%.2f" % t for t in ts_one)),
                           "extrapolated_full_workload_s": ds.m / rate1},
            "parallel_speedup": rate / rate1}
    return base, ref, sel


def plain_measurement(args):
    """The headline: aidw_run over the workload, timed; the pair kernel's roofline; the CPU oracle baseline."""
    import torch

    import paper_1601_05904_amd as aidw
    from paper_1601_05904_amd import workloads as W

    ds = W.WORKLOADS[args.workload]()
    dev = torch.device("cuda", 0)
    x, y, z, qx, qy = (torch.from_numpy(getattr(ds, k)).to(dev) for k in ("x", "y", "z", "qx", "qy"))
    p = aidw.Params(k=ds.k, levels=ds.levels, r_min=ds.r_min, r_max=ds.r_max, occupancy=ds.occupancy)
    qz = torch.empty(ds.m, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    aidw.set_timing(True)
    for _ in range(args.warmup):
        aidw.run(x, y, z, qx, qy, p, out=qz, stream=stream)
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        aidw.run(x, y, z, qx, qy, p, out=qz, stream=stream)
        stages.append(aidw.last_timing())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    aidw.set_timing(False)

    # alpha of every query (untimed run) decides the class mix of the roofline
    _, alpha, _ = aidw.run(x, y, z, qx, qy, p, want_alpha=True, stream=stream)
    peak, mix = class_mix_peak(alpha.cpu().numpy(), ds.levels)
    rates = measured_rates()
    ceiling = class_mix_peak(alpha.cpu().numpy(), ds.levels, rates)[0] if rates else None

    ms = (t1 - t0) * 1e3 / args.steps
    value = ds.m / (ms * 1e-3)
    interp_ms = float(np.mean([s["interp_ms"] for s in stages]))
    pairs = float(ds.n) * float(ds.m)
    achieved = pairs / (interp_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; coordinates on a 2^-20 lattice, z = sin 6x cos 6y + N(0, 0.01^2))",
        "config": {"workload": args.workload, "n": ds.n, "m": ds.m, "k": ds.k, "distribution": ds.meta["kind"],
                   "levels": list(ds.levels), "r_min": ds.r_min, "r_max": ds.r_max, "occupancy": ds.occupancy,
                   "variant": "plain", "interp_q": stages[-1]["interp_q"], "interp_split": stages[-1]["interp_split"]},
        "stages_ms": {k: float(np.mean([s[k] for s in stages])) for k in ("grid_ms", "knn_ms", "interp_ms",
                                                                          "finish_ms")},
        "roofline": {"bound": "alu", "kernel": "k_interp", "achieved": achieved / 1e9, "peak": peak / 1e9,
                     "unit": "Gpair/s", "frac": achieved / peak, "traffic": measured_traffic("k_interp", args.workload),
                     "per_unit": "pair: general alpha 7 VALU + 2 transcendental; integer alpha p 6 VALU + chain(p) "
                                 "multiplies + 1 transcendental", "class_mix": mix,
                     "peak_general_form": PEAK_GENERAL / 1e9, "units_per_launch": pairs,
                     "measured_ceiling": None if ceiling is None else ceiling / 1e9,
                     "frac_of_measured_ceiling": None if ceiling is None else achieved / ceiling,
                     "measured_ceiling_note": "the same per-pair counts at the VALU and transcendental rates the "
                                              "issue-rate microbenchmark measured on the chip"},
    }

    g = aidw.build_grid(x, y, qx, qy, p, stream=stream)
    desc = g.describe()
    g.close()
    out["stage_bandwidth"] = stage_bandwidth(desc, ds, out["stages_ms"])
    if not args.no_host_inclusive:
        out["host_inclusive"] = host_inclusive(ds, p, 3)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], ref, sel = cpu_baseline(ds, args)
        zg = qz.cpu().numpy()[sel].astype(np.float64)
        e = np.abs(zg - ref["z"]) / np.maximum(np.abs(ref["z"]), ref["s"])
        out["z_error"] = {"metric": "|z - z64| / max(|z64|, sum w|z| / sum w)", "max": float(e.max()),
                          "p999": float(np.quantile(e, 0.999)), "median": float(np.median(e)),
                          "sample": len(sel)}
    return out


def sweep_measurement(args):
    """The paper's sweep shape (Section 5, Tables 1-3): n = m in {10, 50, 100, 500, 1000} x 1024 uniform points,
    k = 10, each with four versions -- kNN by the even grid ("improved") or by brute force per query
    ("original", the earlier GPU AIDW), and the interpolation by the tiled kernel or the untiled one.  Per
    version: device times of the kNN stage (grid build included) and of the interpolation stage (HIP events),
    and the host-inclusive total (inputs copied from pinned host memory, result copied back)."""
    import torch

    import paper_1601_05904_amd as aidw
    from paper_1601_05904_amd import workloads as W

    rows = []
    for kk in [int(v) for v in args.sweep_sizes.split(",")]:
        n = kk * 1024
        ds = W.make(n, n, 10, 700 + kk)
        host = {a: torch.from_numpy(getattr(ds, a)).pin_memory() for a in ("x", "y", "z", "qx", "qy")}
        p = aidw.Params(k=10)
        row = {"n": n, "m": n, "label": "%dK" % kk, "versions": {}}
        for kname in ("grid", "brute"):
            for iname in ("tiled", "untiled"):
                reps = 1 if (kname == "brute" or iname == "untiled") and n >= 500 * 1024 else 2
                ts = []
                for rep in range(reps + 1):  # the first pass warms up
                    torch.cuda.synchronize()
                    h0 = time.perf_counter()
                    dev = {a: t.to("cuda", non_blocking=True) for a, t in host.items()}
                    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                    e[0].record()
                    g = aidw.build_grid(dev["x"], dev["y"], dev["qx"], dev["qy"], p)
                    if kname == "grid":
                        r, d1, _ = aidw.knn(g, dev["qx"], dev["qy"], 10)
                    else:
                        r, d1, _ = aidw.knn_bruteforce(dev["x"], dev["y"], dev["qx"], dev["qy"], 10)
                    e[1].record()
                    qz = aidw.interpolate(dev["x"], dev["y"], dev["z"], dev["qx"], dev["qy"], r, d1, p, grid=g,
                                          naive=iname == "untiled")
                    e[2].record()
                    out = qz.to("cpu")
                    torch.cuda.synchronize()
                    h1 = time.perf_counter()
                    g.close()
                    if rep:
                        ts.append((e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), (h1 - h0) * 1e3))
                    del out
                knn_ms, interp_ms, host_ms = (float(np.mean([t[i] for t in ts])) for i in range(3))
                name = ("improved" if kname == "grid" else "original") + "_" + ("tiled" if iname == "tiled" else
                                                                                "naive")
                row["versions"][name] = {"knn_ms": knn_ms, "interp_ms": interp_ms, "total_host_ms": host_ms}
        v = row["versions"]
        row["speedup_knn_improved_vs_original"] = v["original_tiled"]["knn_ms"] / v["improved_tiled"]["knn_ms"]
        row["speedup_interp_tiled_vs_naive"] = v["improved_naive"]["interp_ms"] / v["improved_tiled"]["interp_ms"]
        row["speedup_total_improved_vs_original_tiled"] = (v["original_tiled"]["total_host_ms"] /
                                                           v["improved_tiled"]["total_host_ms"])
        rows.append(row)
        print(json.dumps({"sweep_row": row["label"], "improved_tiled_host_ms": v["improved_tiled"]["total_host_ms"]}),
              file=sys.stderr, flush=True)
    return rows


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the method is measured on a single MI355X "
              "(the query-sharded multi-GPU design is documented, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1601_05904_amd as aidw

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    aidw.load(build_if_missing=True)
    if args.issue_rates:
        print(json.dumps(issue_rates(args)))
        return
    if args.knn_variants:
        print(json.dumps({"knn_variants": knn_variants(args), "unit": "ms"}))
        return
    if args.sweep:
        print(json.dumps({"sweep": sweep_measurement(args), "unit": "ms", "dtype": "f32",
                          "data": "synthetic uniform, k = 10, levels 1-5"}))
        return
    out = {} if args.no_plain else plain_measurement(args)
    if not args.no_learned:
        out["learned_r"] = learned_comparison(args, with_oracle=not args.no_cpu_baseline)
    if not args.no_batch:
        out["batch"] = batch_measurement(args, with_oracle=not args.no_cpu_baseline)
    if not args.no_clustered:
        out["clustered"] = clustered_measurement(args)
    if not args.no_paper_rule:
        out["paper_rule"] = paper_rule_measurement(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
