"""Autotuner for the planner's work split, through the C ABI.

Three planner choices change how one volume's work is divided, never its result:

* ``z_splits``: projection work items per y-slice (each workgroup projects a z range of
  one slice; more splits mean more workgroups and more image rows to sum);
* ``power_chunk``: steps of 64 coordinates per power-sum tile on the matrix cores (smaller
  chunks mean more, shorter workgroups and more tile partials to combine);
* ``waves``: waves per projection workgroup (first direction group, whole-row loads): 8
  by default, which keeps more loads in flight per CU; 4 halves the LDS per workgroup.

``tune`` times every candidate triple with ``dpm_moments_async`` (HIP events around ``reps``
calls: on one stream for the "latency" objective, alternating over two streams with a
workspace each for the "throughput" objective, where one volume's power sums overlap the
next one's projection), requires each candidate's moments to be bit-identical to the
planner's default, installs the fastest with ``dpm_tune_set`` and returns the timings.
Results can be kept in a JSON file (``save`` / ``load``) keyed by shape, dtype and order,
and installed again in a later process without re-measuring.

``tune_batched`` does the same for the batched call's geometry (``dpm_batch_tune_set``: fused
or separate kernels, and how many slices one wave of the fused kernel projects together),
per order, on a batch the caller supplies.
"""
from __future__ import annotations

import ctypes
import json
import os

from . import _lib
from . import (_dims_of_shape, _dtype_code, batched_workspace_bytes, check, lib, moments_async, moments_batched,
               num_moments, workspace_bytes)

Z_SPLITS = (0, 1, 2, 4, 8)        # 0: the planner's choice
POWER_CHUNKS = (0, 4, 8, 16, -1)  # 0: the planner's choice, -1: whole rows
WAVES = (0, 4)                    # 0: the planner's choice (8 where whole rows are loaded)


def set_tuning(shape, dtype_code, K, z_splits=0, power_chunk=0, waves=0):
    """Install an override for volumes of numpy shape (N, M, L), dtype code and order K."""
    t = _lib.Tuning(int(z_splits), int(power_chunk), int(waves))
    check(lib().dpm_tune_set(_dims_of_shape(shape), int(dtype_code), int(K), ctypes.byref(t)), "dpm_tune_set")


def unset_tuning(shape, dtype_code, K):
    check(lib().dpm_tune_set(_dims_of_shape(shape), int(dtype_code), int(K), None), "dpm_tune_set")


def clear():
    check(lib().dpm_tune_clear(), "dpm_tune_clear")


def _key(shape, dtype_code, K):
    N, M, L = (int(s) for s in shape)
    return f"{L}x{M}x{N}:{int(dtype_code)}:{int(K)}"


def tune(vol, K, reps=10, warmup=2, z_splits=Z_SPLITS, power_chunks=POWER_CHUNKS, waves=WAVES, stream=None,
         objective="latency", finalists=3, confirm_rounds=3, margin=0.02):
    """Measure every (z_splits, power_chunk, waves) candidate on the device volume ``vol``
    ((N, M, L) uint8, or uint16 carried as int16) and install the fastest.

    One sweep of short timings is noisy, so the ``finalists`` fastest candidates and the
    planner's default (0, 0, 0) are timed again, ``confirm_rounds`` times each in turn with
    twice the repetitions, and the one with the lowest median is installed -- unless it beats
    the default by less than ``margin`` (a fraction of the default's time): then the
    default stays, so that differences inside the timing noise do not flip the choice
    from run to run.

    Returns {"best": {...}, "candidates": [{"z_splits", "power_chunk", "waves", "ms"}, ...],
    "confirmed": [{..., "ms": median of the confirmation rounds}, ...]}."""
    import torch
    code = _dtype_code(vol)
    shape = tuple(vol.shape)
    dev = vol.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    nm = num_moments(K)
    nm4 = num_moments(min(K, 4))

    if objective not in ("latency", "throughput"):
        raise ValueError("objective must be 'latency' or 'throughput'")
    depth = 2 if objective == "throughput" else 1
    streams = [st] + [torch.cuda.Stream(device=dev) for _ in range(depth - 1)]  # default priority

    def run(cand, reps=reps):
        if cand is None:
            unset_tuning(shape, code, K)
        else:
            set_tuning(shape, code, K, *cand)
        nb = workspace_bytes(shape, code, K)
        ws = [torch.empty(nb, dtype=torch.uint8, device=dev) for _ in range(depth)]
        ex = [torch.empty((nm4, 2), dtype=torch.int64, device=dev) for _ in range(depth)]
        fp = [torch.empty(nm, dtype=torch.float64, device=dev) for _ in range(depth)]
        for i in range(warmup * depth):
            moments_async(vol, K, ex[i % depth], fp[i % depth], ws[i % depth], stream=streams[i % depth])
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        t0.record(st)
        for s in streams[1:]:
            s.wait_event(t0)
        for i in range(reps):
            moments_async(vol, K, ex[i % depth], fp[i % depth], ws[i % depth], stream=streams[i % depth])
        for s in streams[1:]:
            st.wait_stream(s)
        t1.record(st)
        t1.synchronize()
        return t0.elapsed_time(t1) / reps, ex[0].cpu(), fp[0].cpu()

    _, ref_ex, ref_fp = run(None)
    results = []
    for zs in z_splits:
        for pc in power_chunks:
            for w in waves:
                ms, ex, fp = run((zs, pc, w))
                if not (torch.equal(ex, ref_ex) and torch.equal(fp.view(torch.int64), ref_fp.view(torch.int64))):
                    raise RuntimeError(f"tuning candidate z_splits={zs} power_chunk={pc} waves={w} changed the result")
                results.append({"z_splits": zs, "power_chunk": pc, "waves": w, "ms": ms})
    trip = lambda r: (r["z_splits"], r["power_chunk"], r["waves"])
    final = [trip(r) for r in sorted(results, key=lambda r: r["ms"])[:max(1, finalists)]]
    if (0, 0, 0) not in final and any(trip(r) == (0, 0, 0) for r in results):
        final.append((0, 0, 0))
    times = {c: [] for c in final}
    for _ in range(max(1, confirm_rounds)):
        for c in final:
            times[c].append(run(c, 2 * reps)[0])
    confirmed = [{"z_splits": c[0], "power_chunk": c[1], "waves": c[2], "ms": sorted(t)[len(t) // 2]}
                 for c, t in times.items()]
    best = min(confirmed, key=lambda r: r["ms"])
    default = next((r for r in confirmed if trip(r) == (0, 0, 0)), None)
    if default is not None and best["ms"] > default["ms"] * (1.0 - margin):
        best = default
    set_tuning(shape, code, K, best["z_splits"], best["power_chunk"], best["waves"])
    return {"key": _key(shape, code, K), "best": best, "candidates": results, "confirmed": confirmed,
            "objective": objective}


BATCH_FUSED = (0, -1)    # 0: the planner's routing, -1: separate kernels for every ROI
BATCH_UNITS = (0, 1, 4)  # 0: the planner's choice (2 units per sub-row)
BATCH_SPW = (0, 1, 2)    # 0: the planner's choice (at most 4 slices per wave)


def set_batch_tuning(K, fused=0, units=0, max_spw=0):
    """Install a geometry override for batched calls of order K (see dpm_batch_tune_set)."""
    t = _lib.BatchTuning(int(fused), int(units), int(max_spw))
    check(lib().dpm_batch_tune_set(int(K), ctypes.byref(t)), "dpm_batch_tune_set")


def unset_batch_tuning(K):
    check(lib().dpm_batch_tune_set(int(K), None), "dpm_batch_tune_set")


def tune_batched(packed, rois, K, reps=10, warmup=3, fused=BATCH_FUSED, units=BATCH_UNITS, max_spw=BATCH_SPW,
                 stream=None, finalists=3, confirm_rounds=3, margin=0.02):
    """Measure every (fused, units, max_spw) candidate on one batch (``packed`` and ``rois``
    from ``pack_rois``) and install the fastest for order K.

    Each candidate is timed as a repeated call (graph replays after its first two calls),
    must give moments bit-identical to the planner's default, and wins only by beating the
    default by ``margin``, after the same confirmation rounds as ``tune``.  With fused = -1
    the other two knobs do not apply, so that candidate is timed once.

    Returns {"best": {...}, "candidates": [{"fused", "units", "max_spw", "ms"}, ...],
    "confirmed": [...]}."""
    import torch
    dev = packed.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    n = len(rois)
    nm, nm4 = num_moments(K), num_moments(min(K, 4))

    def run(cand, reps=reps):
        if cand is None:
            unset_batch_tuning(K)
        else:
            set_batch_tuning(K, *cand)
        ws = torch.empty(max(batched_workspace_bytes(rois, K), 1), dtype=torch.uint8, device=dev)
        ex = torch.zeros((n * nm4, 2), dtype=torch.int64, device=dev)
        fp = torch.zeros(n * nm, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            moments_batched(packed, rois, K, ex, fp, ws, stream=st)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(st)
        for _ in range(reps):
            moments_batched(packed, rois, K, ex, fp, ws, stream=st)
        t1.record(st)
        t1.synchronize()
        return t0.elapsed_time(t1) / reps, ex.cpu(), fp.cpu()

    try:
        _, ref_ex, ref_fp = run(None)
        cands = []
        for f in fused:
            for u in (units if f == 0 else (0,)):
                for s in (max_spw if f == 0 else (0,)):
                    cands.append((f, u, s))
        results = []
        for c in cands:
            ms, ex, fp = run(c)
            if not (torch.equal(ex, ref_ex) and torch.equal(fp.view(torch.int64), ref_fp.view(torch.int64))):
                raise RuntimeError(f"batch tuning candidate fused={c[0]} units={c[1]} max_spw={c[2]} changed the result")
            results.append({"fused": c[0], "units": c[1], "max_spw": c[2], "ms": ms})
        trip = lambda r: (r["fused"], r["units"], r["max_spw"])
        final = [trip(r) for r in sorted(results, key=lambda r: r["ms"])[:max(1, finalists)]]
        if (0, 0, 0) not in final and (0, 0, 0) in cands:
            final.append((0, 0, 0))
        times = {c: [] for c in final}
        for _ in range(max(1, confirm_rounds)):
            for c in final:
                times[c].append(run(c, 2 * reps)[0])
        confirmed = [{"fused": c[0], "units": c[1], "max_spw": c[2], "ms": sorted(t)[len(t) // 2]}
                     for c, t in times.items()]
        best = min(confirmed, key=lambda r: r["ms"])
        default = next((r for r in confirmed if trip(r) == (0, 0, 0)), None)
        if default is not None and best["ms"] > default["ms"] * (1.0 - margin):
            best = default
    except BaseException:
        unset_batch_tuning(K)
        raise
    set_batch_tuning(K, best["fused"], best["units"], best["max_spw"])
    return {"best": best, "candidates": results, "confirmed": confirmed}


def save(results, path):
    """Merge tuning results ({"key", "best"} dicts from ``tune``) into a JSON file."""
    table = {}
    if os.path.exists(path):
        with open(path) as fh:
            table = json.load(fh)
    for r in results:
        table[r["key"]] = {"z_splits": r["best"]["z_splits"], "power_chunk": r["best"]["power_chunk"],
                           "waves": r["best"].get("waves", 0), "ms": r["best"]["ms"]}
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


def load(path):
    """Install every override stored in a JSON file written by ``save``; returns the count."""
    with open(path) as fh:
        table = json.load(fh)
    for key, v in table.items():
        dims, code, K = key.split(":")
        L, M, N = (int(x) for x in dims.split("x"))
        set_tuning((N, M, L), int(code), int(K), v["z_splits"], v["power_chunk"], v.get("waves", 0))
    return len(table)
