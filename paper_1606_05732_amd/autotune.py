"""Autotuner for the batched planner's tuning table.

The batched launch (cg_sketch_batched) takes two tile shapes per class of d
(c = ceil(log2 d)): the rows of X per S X work item and the columns of G per
contraction wavefront.  autotune_batched() times the whole batch on the GPU
for candidate values -- one class and one parameter at a time, the others
held at their current best (coordinate descent) -- and leaves the fastest
table installed.  Timing uses HIP events on the current stream around
`reps` runs after `warmup` runs; each trial plans the batch afresh.
"""
import time

import torch

from . import api


def d_class(d):
    c = 0
    while c < 10 and (1 << c) < d:
        c += 1
    return c


def time_batch(items, reps=3, warmup=1):
    """Milliseconds per run of the batch under the current tuning table."""
    plan = api.BatchedSketch(items)
    for _ in range(warmup):
        plan.run()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        plan.run()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def autotune_batched(items, rows_candidates=(4096, 8192, 16384, 32768),
                     kc_candidates=(128, 256, 512, 1024, 2048), reps=3, warmup=1, passes=1,
                     log=None):
    """Tune the table for this batch; returns a dict with the chosen
    rows_per_item / kc_per_item (all classes), the per-run time before and
    after, and every trial.  The chosen table stays installed."""
    t0 = time.perf_counter()
    classes = sorted({d_class(api._as_csr(it[0]).d) for it in items})
    rows, kc = api.get_tuning()
    api.set_tuning(rows, kc)
    base = best = time_batch(items, reps, warmup)
    trials = [{"class": None, "rows": None, "kc": None, "ms": base}]
    for _ in range(passes):
        for c in classes:
            for name, cands in (("rows", rows_candidates), ("kc", kc_candidates)):
                for v in cands:
                    cur = rows if name == "rows" else kc
                    if cur[c] == v:
                        continue
                    old = cur[c]
                    cur[c] = v
                    api.set_tuning(rows, kc)
                    ms = time_batch(items, reps, warmup)
                    trials.append({"class": c, "rows": rows[c], "kc": kc[c], "ms": ms})
                    if log:
                        log(f"autotune class {c}: rows {rows[c]} kc {kc[c]} -> {ms:.3f} ms")
                    if ms < best:
                        best = ms
                    else:
                        cur[c] = old
                api.set_tuning(rows, kc)
    return {"classes": classes, "rows_per_item": rows, "kc_per_item": kc, "ms_before": base,
            "ms_after": best, "trials": trials, "seconds": time.perf_counter() - t0}


def choose_algo(X, m, B, seed, precision="native", candidates=("binned", "atomic", "rows", "fused",
                                                                 "sorted"),
                reps=3, warmup=1, row_offset=0):
    """Measured choice of the S X algorithm for one call shape: each
    candidate the library accepts for these inputs is planned and timed
    (whole forward calls, HIP events on the current stream, `reps` runs
    after `warmup`), and the fastest is returned with every timing:
    {"algo": name, "ms": {name: ms per call}, "rejected": {name: reason}}.
    AUTO's static cost model picks without timing; this is the measured
    alternative for callers that sketch one shape many times."""
    from ._lib import CountGaussError
    ms, rejected = {}, {}
    for algo in candidates:
        try:
            plan = api.SketchPlan(X, m, B, seed, precision=precision, algo=algo,
                                  row_offset=row_offset)
            for _ in range(warmup):
                plan.run()
        except CountGaussError as e:
            rejected[algo] = str(e)
            continue
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            plan.run()
        stop.record()
        stop.synchronize()
        ms[algo] = start.elapsed_time(stop) / reps
        del plan
    if not ms:
        raise RuntimeError(f"no S X algorithm accepted these inputs: {rejected}")
    return {"algo": min(ms, key=ms.get), "ms": ms, "rejected": rejected}
