"""Benchmark: 3D moments of a 512^3 uint16 CT-like volume, orders <= 6, on one MI355X.

    python bench.py [--gpus 1] [--steps 50] [--warmup 10] [--workload ct512_k6]

One step = one pass of the whole method over one volume: projection images and
per-slice power sums (one HBM pass), y-reduction to 2D moments, recombination into the
84 3D moments (35 exact int128 + all 84 as FP64), with the volume already resident in
HBM.  Three distinct volumes are rotated so repeated steps are not served from the
256 MB Infinity Cache.  Prints ONE JSON line on stdout; everything else goes to stderr.

The headline loop issues the K steps round-robin on --streams streams (default 2), each
with its own workspace, so one volume's power sums and recombination overlap the next
volume's projection; the single-stream time per volume is reported beside it
(latency_ms_single_stream).  A further pass over the same K steps
records the library's HIP events between the kernels (on the stream they run on) and
gives the stage breakdown.  The roofline figure is for the dominant kernel (the
projection, one pass over the volume): algorithmic bytes = every voxel read once
(L*M*N*elem bytes) divided by that kernel's average device time from those events.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (shape (N, M, L), dtype, K, generator)
    "ct512_k6": ((512, 512, 512), "u16", 6, "ct"),
    "ct512_k16": ((512, 512, 512), "u16", 16, "ct"),
    "mri256_k6": ((256, 256, 256), "u16", 6, "mri"),
    "u8_64_k3": ((64, 64, 64), "u8", 3, "uniform"),
    # 128 MB of 1-byte voxels at order 4: the size of one row of the paper's Table 1
    "u8_512_k4": ((512, 512, 512), "u8", 4, "uniform"),
}
GEN_DESC = {"ct": "CT-like phantom", "mri": "MRI-like phantom", "uniform": "uniform random voxels"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The sources that define, instantiate and plan the projection kernel: its measured HBM
# traffic stays valid while these are unchanged.
PROJECTION_SOURCES = ("slice_impl.h", "dpm_common.h", "kernels.h", "slice_g0_u16_fast.hip",
                      "slice_dispatch.cpp", "dpm_api.cpp")


def source_hash():
    """Hash of the projection kernel's sources: a traffic measurement is valid only for them."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2012_08099_amd", "csrc")
    for f in PROJECTION_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def make_volume(gen, shape, dt, seed):
    import numpy as np
    import synth
    if gen == "ct":
        return synth.ct_phantom(shape, seed=seed)
    if gen == "mri":
        return synth.mri_phantom(shape, seed=seed)
    return synth.uniform_volume(shape, np.uint8 if dt == "u8" else np.uint16, seed=seed)


def to_dev(V):
    import numpy as np
    import torch
    t = torch.from_numpy(V.view(np.int16) if V.dtype == np.uint16 else V)
    return t.to("cuda:0")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(V, K, target_s=4.0, runs=3):
    """The oracle on the host cores, on bounded samples of volume 0:
    - the naive direct sum (oracle/naive.c: eq. 2 per voxel, every monomial, int128,
      OpenMP over all cores): a z-slab sized for about target_s, timed `runs` times,
      the median reported (voxels/s);
    - the exact Python oracle (oracle.moments_exact: eq. 2 with hoisted powers, exact
      integers; one process): the whole of volume 0, timed once."""
    import statistics

    import oracle
    import oracle.native as onative
    onative.build(force=False)
    nz = 4
    t0 = time.perf_counter()
    onative.moments_direct(V[:nz], K)
    rate = nz / max(time.perf_counter() - t0, 1e-3)  # z-planes per second
    nz = int(min(V.shape[0], max(4, rate * target_s)))
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        onative.moments_direct(V[:nz], K)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    vox = nz * V.shape[1] * V.shape[2]
    pz = V.shape[0]
    t0 = time.perf_counter()
    oracle.moments_exact(V[:pz], K)
    py_s = time.perf_counter() - t0
    py_vox = pz * V.shape[1] * V.shape[2]
    return {"value": vox / med, "unit": "voxels/s", "cores": onative.num_threads(), "kind": "oracle",
            "sample": f"direct per-voxel sum of eq. (2), all {(K + 1) * (K + 2) * (K + 3) // 6} monomials, "
                      f"exact int128, z-slab {nz}x{V.shape[1]}x{V.shape[2]} of volume 0, median of {runs} runs",
            "runs_s": times, "cpu_model": cpu_model(),
            "python_oracle": {"value": py_vox / py_s, "unit": "voxels/s", "threads": 1, "seconds": py_s,
                              "sample": f"oracle.moments_exact (eq. 2, hoisted powers, exact integers) on all "
                                        f"{pz}x{V.shape[1]}x{V.shape[2]} of volume 0"}}


# The paper's Table 1: DPM times (ms) on an Intel Core i5 (7th generation) for 1-byte
# volumes of 1 ... 1024 MB at 3rd / 4th order -- context only, other hardware and data.
TABLE1_MB = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)
TABLE1_MS = {3: (0.30, 0.56, 1.00, 2.00, 4.03, 8.25, 17.60, 37.5, 63.5, 130.4, 273.5),
             4: (0.44, 0.90, 1.46, 2.75, 5.3, 10.95, 21.23, 41.0, 84.6, 173.8, 400.1)}
# (N, M, L) of each size: 128 x 128 x 64 (the table's 1 MB volume), then doubling one axis
TABLE1_SHAPES = ((64, 128, 128), (128, 128, 128), (128, 128, 256), (128, 256, 256), (256, 256, 256),
                 (256, 256, 512), (256, 512, 512), (512, 512, 512), (512, 512, 1024), (512, 1024, 1024),
                 (1024, 1024, 1024))


def sweep_main(a):
    """The sizes of the paper's Table 1 on one GPU: uniform random uint8 volumes of 1-1024 MB
    at orders 3 and 4; per volume the single-stream time of one dpm_moments_async call
    (HIP events over 10 calls), beside the paper's CPU times and, up to 64 MB, the naive
    direct-sum oracle on this host's cores."""
    import numpy as np
    import torch

    import paper_2012_08099_amd as dpm
    rows = []
    for mb, shape in zip(TABLE1_MB, TABLE1_SHAPES):
        V = np.random.default_rng(mb).integers(0, 256, size=shape, dtype=np.uint8)
        vol = torch.from_numpy(V).to("cuda:0")
        for K in (3, 4):
            nm, nm4 = dpm.num_moments(K), dpm.num_moments(min(K, 4))
            ws = torch.empty(dpm.workspace_bytes(shape, 1, K), dtype=torch.uint8, device="cuda:0")
            ex = torch.empty((nm4, 2), dtype=torch.int64, device="cuda:0")
            fp = torch.empty(nm, dtype=torch.float64, device="cuda:0")
            for _ in range(3):
                dpm.moments_async(vol, K, ex, fp, ws)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                dpm.moments_async(vol, K, ex, fp, ws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            row = {"mb": mb, "shape_zyx": list(shape), "K": K, "gpu_ms": ms, "gpu_voxels_per_s": V.size / (ms / 1e3),
                   "hbm_frac": V.size / (ms / 1e3) / (HBM_PEAK_GBS * 1e9), "paper_cpu_ms": TABLE1_MS[K][TABLE1_MB.index(mb)]}
            if mb <= 64 and not a.no_cpu_baseline:
                import oracle.native as onative
                onative.build(force=False)
                t0 = time.perf_counter()
                ref = onative.moments_direct(V, K)
                row["naive_cpu_ms"] = (time.perf_counter() - t0) * 1e3
                assert [int(v) for v in ref[:nm4]] == dpm._exact_from_tensor(ex)
            rows.append(row)
            log(row)
        del vol
    big = [r for r in rows if r["mb"] == 1024 and r["K"] == 4][0]
    out = {"metric": "voxels/s (1024^3 uint8, orders <= 4; the paper's Table 1 sizes)", "value": big["gpu_voxels_per_s"],
           "unit": "voxels/s", "n_gpus": 1, "steps": 10, "warmup": 3, "ms_per_step": big["gpu_ms"],
           "higher_is_better": True, "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "table1_sweep: uniform random uint8 volumes of 1-1024 MB, orders 3 and 4"},
           "cpu_cores": None, "sweep": rows}
    if not a.no_cpu_baseline:
        import oracle.native as onative
        out["cpu_cores"] = onative.num_threads()
    print(json.dumps(out), flush=True)
    return 0


def read_traffic(workload, shash):
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        t = json.load(fh)
    if t.get("source_hash") != shash:
        return None
    return t.get("bytes_per_launch")


def serve_leg(a, requests, modes=("device", "host"), ct0=None, log_prefix="serve"):
    """Served workload: a Poisson stream of mixed requests through dpm_server.

    Mix (per request): 70% uint8 sphere-mask ROIs with dims U{32..128}^3, 25% uint16
    MRI-like 256x256xZ with Z in [100, 300], 5% 512^3 uint16 CT-like; K = 6.  Volumes
    come from pools of pre-generated inputs (64 / 8 / 3 distinct).  First the capacity
    (all requests arriving at once), then Poisson arrivals at 0.5x and 0.8x of it; per
    mode: inputs resident on the device, or in pinned host memory (copied per request).
    Latency = result in the caller's buffer - scheduled arrival.  Beside them, the plain
    path: the same requests one dpm_moments_async call after another on one stream.
    """
    import numpy as np
    import threading
    import torch

    import paper_2012_08099_amd as dpm
    import synth

    rng = np.random.default_rng(a.seed)
    K = 6
    t0 = time.perf_counter()
    small = [synth.sphere_mask(tuple(int(v) for v in rng.integers(32, 129, size=3)), rng) for _ in range(64)]
    mid = [synth.mri_phantom((int(rng.integers(100, 301)), 256, 256), seed=s) for s in range(8)]
    if ct0 is None:
        ct0 = make_volume("ct", (512, 512, 512), "u16", 0)
    log(f"{log_prefix}: pools generated in {time.perf_counter() - t0:.1f} s")

    def to_t(V, dev):
        t = torch.from_numpy(V.view(np.int16) if V.dtype == np.uint16 else V)
        return t.to("cuda:0") if dev else t.pin_memory()

    results = {}
    for mode in modes:
        dev = mode == "device"
        ps = [to_t(V, dev) for V in small]
        pm = [to_t(V, dev) for V in mid]
        c0 = to_t(ct0, dev)
        pc = [c0, torch.flip(c0, dims=[2]).contiguous(), torch.roll(c0, shifts=37, dims=0).contiguous()]
        if not dev:
            pc = [t.pin_memory() if not t.is_pinned() else t for t in pc]
        torch.cuda.synchronize()  # the pools are complete before any request reads them
        kinds = rng.choice(3, size=requests, p=[0.70, 0.25, 0.05])
        vols = [ps[int(rng.integers(len(ps)))] if k == 0 else pm[int(rng.integers(len(pm)))] if k == 1
                else pc[int(rng.integers(len(pc)))] for k in kinds]
        nvox = sum(int(v.numel()) for v in vols)

        def run(rate_hz):
            srv = dpm.Server(hbm_budget=a.hbm_budget << 30, n_streams=a.server_streams,
                             batch_voxels=128 ** 3, batch_max=256, max_inflight=16)
            try:
                start = srv.now_ms() + 50.0
                if rate_hz:
                    arr = start + np.cumsum(rng.exponential(1e3 / rate_hz, size=len(vols)))
                else:
                    arr = np.full(len(vols), start)
                items = [(v, K, float(t)) for v, t in zip(vols, arr)]
                th = threading.Thread(target=lambda: srv.replay(items))
                th.start()
                done = []
                while len(done) < len(items):
                    done += srv.poll(1024, wait_ms=20)
                th.join()
                st = srv.stats()
            finally:
                srv.close()
            bad = [c for c in done if c["status"] != 0]
            if bad:
                import collections
                kinds = collections.Counter((c["status"], c["batched"]) for c in bad)
                raise RuntimeError(f"{len(bad)} of {len(done)} requests failed; (status, batched): {dict(kinds)}; "
                                   f"last device error {dpm.lib().dpm_last_device_error()}")
            lat = np.array([c["t_done_ms"] - c["t_arrival_ms"] for c in done])
            wait = np.array([c["t_start_ms"] - c["t_arrival_ms"] for c in done])
            bat = np.array([bool(c["batched"]) for c in done])
            t_first = min(c["t_arrival_ms"] for c in done)
            t_last = max(c["t_done_ms"] for c in done)
            span_s = (t_last - t_first) / 1e3
            tail = lat >= np.percentile(lat, 99)
            t_tail = np.array([c["t_arrival_ms"] for c in done])[tail] - t_first
            return {"offered_per_s": rate_hz, "served_per_s": len(done) / span_s,
                    "voxels_per_s": nvox / span_s, "p50_ms": float(np.percentile(lat, 50)),
                    "p99_ms": float(np.percentile(lat, 99)), "batched_jobs": st["batched_jobs"],
                    "single_jobs": st["single_jobs"], "arena_peak_gib": st["arena_peak_used"] / 2 ** 30,
                    # where the slowest 1% spend their time, and when they arrived
                    "tail": {"n": int(tail.sum()), "wait_ms_mean": float(wait[tail].mean()),
                             "run_ms_mean": float((lat - wait)[tail].mean()),
                             "batched_frac": float(bat[tail].mean()),
                             "arrival_s_min": float(t_tail.min() / 1e3), "arrival_s_max": float(t_tail.max() / 1e3)},
                    "p99_ms_batched": float(np.percentile(lat[bat], 99)) if bat.any() else None,
                    "p99_ms_single": float(np.percentile(lat[~bat], 99)) if (~bat).any() else None}

        cap = run(0.0)
        log(log_prefix, mode, "capacity", cap)
        r50 = run(0.5 * cap["served_per_s"])
        log(log_prefix, mode, "0.5x", r50)
        r80 = run(0.8 * cap["served_per_s"])
        log(log_prefix, mode, "0.8x", r80)
        # plain path for reference: the same requests one after another on one stream
        nplain = min(len(vols), 500)
        ws_b = max(dpm.workspace_bytes(tuple(v.shape), 2 if v.dtype == torch.int16 else 1, K) for v in vols[:nplain])
        ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda:0")
        ex = torch.empty((35, 2), dtype=torch.int64, device="cuda:0")
        fp = torch.empty(84, dtype=torch.float64, device="cuda:0")
        plain = vols[:nplain] if dev else [v.to("cuda:0", non_blocking=True) for v in vols[:nplain]]
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for v in plain:
            dpm.moments_async(v, K, ex, fp, ws)
        torch.cuda.synchronize()
        plain_s = (time.perf_counter() - tp) / len(plain)
        results[mode] = {"capacity": cap, "poisson_0.5x": r50, "poisson_0.8x": r80,
                         "plain_serial_per_s": 1.0 / plain_s, "plain_requests_timed": nplain,
                         "voxels_per_request_mean": nvox / len(vols)}
        del ps, pm, pc, vols, plain
        torch.cuda.empty_cache()
    return results


def serve_main(a):
    """The served workload on its own (both input modes, --requests per run)."""
    results = serve_leg(a, a.requests)
    out = {"metric": "served requests/s (mix 70% u8 ROI 32-128^3 / 25% u16 256x256xZ / 5% 512^3 u16, K=6)",
           "value": results["device"]["capacity"]["served_per_s"], "unit": "requests/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "requests": a.requests,
           "config": {"workload": "serve_mix", "hbm_budget_gib": a.hbm_budget, "server_streams": a.server_streams},
           "modes": results}
    print(json.dumps(out), flush=True)
    return 0


def rois_leg(n, seed, steps, warmup, tune=True):
    """Batched ROIs: n uint8 sphere-mask ROIs with dims U{8..96}^3 (sizes vary per axis),
    K = 4 (35 exact moments each), all packed in one device buffer.  One step = every
    ROI's moments by one dpm_moments_batched launch sequence; compared with the same ROIs
    as n plain dpm_moments_async calls on one stream."""
    import numpy as np
    import torch

    import paper_2012_08099_amd as dpm
    import synth

    K = 4
    t0 = time.perf_counter()
    vols = synth.roi_batch(n=n, seed=seed)
    log(f"{len(vols)} ROIs generated in {time.perf_counter() - t0:.1f} s")
    packed, rois = dpm.pack_rois(vols, "cuda:0")
    n = len(vols)
    nvox = int(sum(v.size for v in vols))
    batch_tuning = None
    if tune:
        # the batch geometry (fused or separate kernels, slices per wave), measured on this batch
        from paper_2012_08099_amd import autotune
        t0 = time.perf_counter()
        r = autotune.tune_batched(packed, rois, K, reps=10)
        default = next((c["ms"] for c in r["confirmed"] if (c["fused"], c["units"], c["max_spw"]) == (0, 0, 0)), None)
        batch_tuning = {"fused": r["best"]["fused"], "units": r["best"]["units"], "max_spw": r["best"]["max_spw"],
                        "ms_best": r["best"]["ms"], "ms_planner_default": default,
                        "candidates": len(r["candidates"]), "seconds": time.perf_counter() - t0}
    ws = torch.empty(dpm.batched_workspace_bytes(rois, K), dtype=torch.uint8, device="cuda:0")
    ex = torch.empty((n, dpm.num_moments(K), 2), dtype=torch.int64, device="cuda:0")
    fp = torch.empty((n, dpm.num_moments(K)), dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    batched = lambda: dpm.moments_batched(packed, rois, K, ex, fp, ws)  # noqa: E731
    for _ in range(warmup):
        batched()
    ms_b = timed(batched, steps)
    dpm.profile_collect()
    dpm.profile_enable(True)
    for _ in range(steps):
        batched()
    torch.cuda.synchronize()
    dpm.profile_enable(False)
    prof = dpm.profile_collect()
    stages = {k: prof["ms_" + k] / max(prof["calls"], 1) for k in ("project", "power", "combine")}

    singles = [torch.from_numpy(v).to("cuda:0") for v in vols]
    wsb = max(dpm.workspace_bytes(tuple(v.shape), 1, K) for v in vols)
    ws1 = torch.empty(wsb, dtype=torch.uint8, device="cuda:0")
    ex1 = torch.empty((dpm.num_moments(K), 2), dtype=torch.int64, device="cuda:0")
    fp1 = torch.empty(dpm.num_moments(K), dtype=torch.float64, device="cuda:0")

    def plain():
        for v in singles:
            dpm.moments_async(v, K, ex1, fp1, ws1)
    plain()
    ms_p = timed(plain, max(1, steps // 10))
    # the batched results equal single calls (spot check a few ROIs)
    for i in (0, n // 2, n - 1):
        r = dpm.moments(singles[i], K)
        assert r.exact == [dpm.i128_to_int(int(lo) & (2 ** 64 - 1), int(hi)) for lo, hi in ex[i].tolist()]
    return {"rois": n, "voxels": nvox, "ms_per_batch": ms_b, "rois_per_s": n / (ms_b / 1e3),
            "voxels_per_s": nvox / (ms_b / 1e3), "hbm_frac_algorithmic": nvox / (ms_b / 1e3) / (HBM_PEAK_GBS * 1e9),
            "plain_launches_ms": ms_p, "speedup_vs_plain": ms_p / ms_b, "stages_ms": stages,
            "workspace_bytes": int(ws.numel()), "batch_tuning": batch_tuning}


def rois_main(a):
    r = rois_leg(a.requests, a.seed, a.steps, a.warmup, tune=not a.no_tune)
    n, nvox, ms_b = r["rois"], r["voxels"], r["ms_per_batch"]
    out = {"metric": "ROIs/s (1000 u8 ROIs U{8..96}^3, orders <= 4)", "value": n / (ms_b / 1e3), "unit": "ROIs/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_b, "higher_is_better": True,
           "dtype": "u8", "data": "synthetic",
           "config": {"workload": f"rois{n}: {n} uint8 sphere-mask ROIs, dims U{{8..96}}^3, {nvox} voxels, K=4"},
           "voxels_per_s": r["voxels_per_s"], "plain_launches_ms": r["plain_launches_ms"],
           "speedup_vs_plain": r["speedup_vs_plain"], "stages_ms": r["stages_ms"], "batch_tuning": r["batch_tuning"]}
    print(json.dumps(out), flush=True)
    return 0


def paper_leg(vols, shape, code, K=4, reps=10):
    """The paper's own route (five images incl. ZX with partial images summed in a fixed
    order, 1D integrals, eqs. 10-16) and the 1D-integral route for the default images,
    timed per call (HIP events, one stream, volumes rotated) beside the default path at
    the same order; with the paper route's extra bytes (partial images written and read
    back) from its workspace layout."""
    import torch

    import paper_2012_08099_amd as dpm
    nm = dpm.num_moments(K)
    ex = torch.empty((nm, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.empty(nm, dtype=torch.float64, device="cuda:0")
    ws_p = torch.empty(dpm.paper_workspace_bytes(shape, code, K), dtype=torch.uint8, device="cuda:0")
    ws_d = torch.empty(dpm.drt_workspace_bytes(shape, code, K), dtype=torch.uint8, device="cuda:0")
    ws_f = torch.empty(dpm.workspace_bytes(shape, code, K), dtype=torch.uint8, device="cuda:0")
    calls = {"default": lambda v: dpm.moments_async(v, K, ex, fp, ws_f),
             "paper": lambda v: dpm.moments_paper_async(v, K, ex, fp, ws_p),
             "drt": lambda v: dpm.moments_drt_async(v, K, ex, fp, ws_d)}
    res = {}
    ref = None
    for name, fn in calls.items():
        for i in range(3):
            fn(vols[i % len(vols)])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(reps):
            fn(vols[i % len(vols)])
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = e0.elapsed_time(e1) / reps
        got = dpm._exact_from_tensor(ex)
        if ref is None:
            ref = got
        assert got == ref, f"{name} route differs from the default path"
    N, M, L = shape
    elem = 1 if code == 1 else 2
    PP_BY, PP_BZ, PP_XT, PP_DW = 16, 64, 512, 512 + 64 - 1
    nyb, nzb, nxt = -(-M // PP_BY), -(-N // PP_BZ), -(-L // PP_XT)
    ndiag = (K >= 3) + (K >= 4)  # X+Z from order 3, X-Z at order 4
    part = 4 * (nzb * M * L + ndiag * nzb * nxt * M * PP_DW + nyb * N * L + nxt * N * M)
    res.update({"order": K, "volume_bytes": N * M * L * elem, "paper_partial_bytes_written": part,
                "paper_extra_traffic_frac": 2 * part / (N * M * L * elem),
                "paper_vs_default": res["paper_ms"] / res["default_ms"],
                "drt_vs_default": res["drt_ms"] / res["default_ms"]})
    return res


def paper_main(a):
    """The paper's own route and the 1D-integral route at order 4 on the 512^3 uint16
    CT-like volume (three rotated copies), beside the default path."""
    import torch
    V0 = make_volume("ct", (512, 512, 512), "u16", 0)
    v0 = to_dev(V0)
    vols = [v0, torch.flip(v0, dims=[2]).contiguous(), torch.roll(v0, shifts=37, dims=0).contiguous()]
    r = paper_leg(vols, (512, 512, 512), 2, K=4, reps=a.steps)
    out = {"metric": "ms per 512^3 uint16 volume, orders <= 4, the paper's own route", "value": r["paper_ms"],
           "unit": "ms", "n_gpus": 1, "steps": a.steps, "higher_is_better": False, "dtype": "u16",
           "data": "synthetic", "config": {"workload": "paper_route: 512x512x512 u16 CT-like phantom, K=4"}, **r}
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ct512_k6",
                    choices=sorted(WORKLOADS) + ["serve_mix", "rois1000", "table1_sweep", "paper_route"])
    ap.add_argument("--requests", type=int, default=10000, help="serve_mix: requests per run; rois1000: ROIs")
    ap.add_argument("--hbm-budget", type=int, default=16, help="serve_mix: server arena, GiB")
    ap.add_argument("--server-streams", type=int, default=4, help="serve_mix: server streams")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, 3 plain device copies of MIB MiB (calibrates HBM byte counters)")
    ap.add_argument("--nvol", type=int, default=3, help="distinct volumes rotated between steps")
    ap.add_argument("--streams", type=int, default=2,
                    help="volumes in flight (one stream and workspace each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the short batched / served / paper-route legs of the default run")
    ap.add_argument("--serve-requests", type=int, default=3000, help="requests per run of the served leg")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (planner defaults for the work split)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); the moments of one volume "
              "need no collective, and this benchmark measures one GPU", file=sys.stderr)
        return 2

    if a.workload == "serve_mix":
        return serve_main(a)
    if a.workload == "table1_sweep":
        return sweep_main(a)
    if a.workload == "paper_route":
        return paper_main(a)
    if a.workload == "rois1000":
        if a.requests == 10000:
            a.requests = 1000
        return rois_main(a)

    import numpy as np
    import torch

    import paper_2012_08099_amd as dpm

    shape, dt, K, gen = WORKLOADS[a.workload]
    N, M, L = shape
    elem = 1 if dt == "u8" else 2
    t0 = time.perf_counter()
    V0 = make_volume(gen, shape, dt, seed=0)
    log(f"generated {shape} {dt} in {time.perf_counter() - t0:.1f} s")
    vols = [to_dev(V0)]
    for i in range(1, a.nvol):  # distinct buffers and data: flipped / rolled copies
        v = torch.flip(vols[0], dims=[2]) if i % 2 else torch.roll(vols[0], shifts=37 * i, dims=0)
        vols.append(v.contiguous())
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(min(K, 4))
    code = 1 if dt == "u8" else 2
    tuning = None
    if not a.no_tune:
        # the work split (z-splits, power-tile chunk) measured for this shape; every
        # candidate must give the default plan's moments bit for bit
        from paper_2012_08099_amd import autotune
        t0 = time.perf_counter()
        r = autotune.tune(vols[0], K, reps=20, warmup=3, objective="throughput")
        default = [c for c in r["confirmed"] if c["z_splits"] == 0 and c["power_chunk"] == 0 and c["waves"] == 0][0]
        tuning = {"z_splits": r["best"]["z_splits"], "power_chunk": r["best"]["power_chunk"], "waves": r["best"]["waves"],
                  "ms_best": r["best"]["ms"], "ms_planner_default": default["ms"],
                  "candidates": len(r["candidates"]), "objective": r["objective"], "seconds": time.perf_counter() - t0}
        log("tuning", tuning)
    # object features (Section 4) of volume 0: blocking calls (moments + features kernel +
    # copies), timed on the host; before the warmup so the timed phases are undisturbed
    dpm.features(vols[0], K)
    t0 = time.perf_counter()
    for _ in range(5):
        feats = dpm.features(vols[0], K)
    features_ms = (time.perf_counter() - t0) / 5 * 1e3
    # moments from supplied projection images (the volume's own, projected once)
    flat = torch.cat([im.reshape(-1) for im in dpm.project_images(vols[0], K)]).contiguous()
    fi = dpm.moments_from_images(flat, shape, code, K)
    assert fi.exact == dpm.moments(vols[0], K).exact
    t0 = time.perf_counter()
    for _ in range(5):
        dpm.moments_from_images(flat, shape, code, K)
    from_images_ms = (time.perf_counter() - t0) / 5 * 1e3
    del flat
    depth = max(1, a.streams)
    wsb = dpm.workspace_bytes(shape, code, K)
    ws = [torch.empty(wsb, dtype=torch.uint8, device="cuda:0") for _ in range(depth)]
    ex = [torch.empty((nm4, 2), dtype=torch.int64, device="cuda:0") for _ in range(depth)]
    fp = [torch.empty(nm, dtype=torch.float64, device="cuda:0") for _ in range(depth)]
    streams = [torch.cuda.Stream(device="cuda:0") for _ in range(depth)]  # default priority
    plan = dpm.plan(shape, code, K)
    log("plan", plan)

    def run(n, nstreams):
        """n steps, step i on stream i % nstreams with that stream's workspace/outputs."""
        main = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(main)
        for s in streams[:nstreams]:
            s.wait_event(e0)
        for i in range(n):
            j = i % nstreams
            dpm.moments_async(vols[i % a.nvol], K, ex[j], fp[j], ws[j], stream=streams[j])
        for s in streams[:nstreams]:
            main.wait_stream(s)
        e1.record(main)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run(a.warmup, depth)
    # headline: K steps, consecutive volumes on `depth` streams so that one volume's
    # power sums and recombination overlap the next volume's projection
    ms = run(a.steps, depth)
    ms_step = ms / a.steps
    voxels = N * M * L
    value = voxels * a.steps / (ms / 1e3)
    # latency of one volume alone: the same K steps on a single stream
    ms_serial = run(a.steps, 1) / a.steps

    # stage breakdown: the same K steps again on one stream with the library's HIP
    # events recorded between the kernels (the events themselves add small gaps, which
    # is why the timed loops run without them)
    dpm.profile_collect()
    dpm.profile_enable(True)
    for i in range(a.steps):
        dpm.moments_async(vols[i % a.nvol], K, ex[0], fp[0], ws[0], stream=streams[0])
    torch.cuda.synchronize()
    dpm.profile_enable(False)
    prof = dpm.profile_collect()

    proj_ms = prof["ms_project"] / max(prof["calls"], 1)
    proj_kernel = ("slice_kernel (projection, one pass over the volume)" if plan["n_groups"] == 1 else
                   "slice_groups_kernel (projection, one pass over the volume, all direction groups)")
    bytes_launch = voxels * elem
    achieved = bytes_launch / (proj_ms / 1e3) / 1e9
    shash = source_hash()
    traffic = read_traffic(a.workload, shash)

    # sanity: the last result equals a fresh blocking call on the same volume
    res = dpm.moments(vols[(a.steps - 1) % a.nvol], K)
    assert res.exact == dpm._exact_from_tensor(ex[0])

    out = {
        "metric": "voxels/s (512^3 uint16, orders <= 6)" if a.workload == "ct512_k6" else f"voxels/s ({a.workload})",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "latency_ms_single_stream": ms_serial,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16" if elem == 2 else "u8",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {L}x{M}x{N} {dt} {GEN_DESC[gen]}, max_order {K} "
                               f"({nm} moments; orders<=4 exact int128, all FP64)", "volumes_rotated": a.nvol,
                   "streams": depth},
        "hbm_gbs_algorithmic": voxels * elem / (ms_step / 1e3) / 1e9,
        "stages_ms": {"project": proj_ms, "power": prof["ms_power"] / max(prof["calls"], 1),
                      "combine": prof["ms_combine"] / max(prof["calls"], 1),
                      "total_with_events": prof["ms_total"] / max(prof["calls"], 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": proj_kernel,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     # the whole kernel sequence of a step (projection, power sums,
                     # recombination) against the same bytes: per step of the headline
                     # (2 streams) and per volume on one stream
                     "sequence_frac": bytes_launch / (ms_step / 1e3) / (HBM_PEAK_GBS * 1e9),
                     "sequence_frac_single_stream": bytes_launch / (ms_serial / 1e3) / (HBM_PEAK_GBS * 1e9)},
        "source_hash": shash,
        "tuning": tuning,
        "features": {"call_ms_blocking": features_ms, "centroid": [float(c) for c in feats["centroid"]]},
        "from_images": {"call_ms_blocking": from_images_ms},
        "plan": {k: plan[k] for k in ("z_splits", "n_items", "power_tiles", "power_chunk", "proj_waves")},
    }
    if not a.no_legs:
        # the other workloads, short: batched ROIs, the served mix (device inputs), and
        # the paper's own route / the 1D-integral route at order 4 on this volume
        if K <= 6:
            out["paper_route"] = paper_leg(vols, shape, code, K=4)
            log("paper_route", out["paper_route"])
        out["rois1000"] = rois_leg(1000, a.seed, 20, 5, tune=not a.no_tune)
        log("rois1000", out["rois1000"])
        out["serve_mix"] = serve_leg(a, a.serve_requests, modes=("device",),
                                     ct0=V0 if (gen == "ct" and shape == (512, 512, 512)) else None)["device"]
        out["serve_mix"]["requests"] = a.serve_requests
        log("serve_mix", out["serve_mix"])
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(V0, K)
    print(json.dumps(out), flush=True)
    if a.copy_probe:
        src = torch.empty(a.copy_probe << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
