#!/usr/bin/env python
"""Benchmark of the CountGauss transform T.X = G.(S.X) on one MI355X.

Default workload: CSR X with n = 2^24 rows, d = 32 columns, density 5%
(about 26.8M stored entries, values |N(0,1)|, FP32), m = 64, B = 65536 --
the FP32-at-scale workload.  One step is one whole T.X call on inputs
already resident in HBM: S X (binned: count, scan, scatter, reduce), the
split MFMA contraction with in-register G, and its fixed-order reduction.

Prints ONE JSON line on stdout (everything else goes to stderr):
  value        nnz(X) / wall time per step (nnz/s)
  roofline     the S X stage (the dominant one; its four kernels run back to
               back): algorithmic bytes per launch / its average duration
               from HIP events recorded by the library on the launch stream,
               against the 8 TB/s HBM peak; `traffic` is the stage's HBM
               bytes per launch from committed rocprofv3 FETCH_SIZE /
               WRITE_SIZE counters scaled by a plain-copy calibration, or
               null if the kernel sources changed since they were taken, and
               `traffic_gbs` those bytes over the stage's time
  cpu_baseline the FP64 oracle on the host cores, same workload
  ladder       the G.(S X) precision ladder on the dense spiky workload
               (n = 2^22, d = 64, m = 64, B = 262144): time per step and
               error against the FP64 oracle for FP32, BF16 and FP8 inputs
  batched      512 uneven CSR instances: 512 sequential calls against one
               batch (built-in tuning table, then autotuned)
  adjoint      dX = T^T dY at the gradient workload's shape (n = 2^22,
               d = 64, m = 128, B = 2^19): time per call and its roofline
  adjoint_csr  the gradient with respect to the stored values of the CSR
               workload's X: time per call and its roofline
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_FP32_TFLOPS = 157.3
METRIC = "T·X nnz/sec and % HBM roofline at 1 GPU; fused BF16/FP8 vs FP32 at stated error"
COUNTERS = os.path.join(ROOT, "profiles", "sx_stage_csr_n16777216_d32_counters.json")
SX_SOURCES = [os.path.join(ROOT, "paper_1606_05732_amd", "csrc", f)
              for f in ("cg_sx_binned.hip", "cg_rng.hpp", "cg_internal.hpp")]


def sx_source_digest():
    h = hashlib.sha256()
    for f in SX_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime torch already loaded."""

    def __init__(self):
        import torch  # noqa: F401  (loads the runtime)
        self.rt = None
        for name in ("libamdhip64.so.7", "libamdhip64.so"):
            try:
                self.rt = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self.rt is None:
            raise RuntimeError("HIP runtime not found")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, k):
        out = []
        for _ in range(k):
            h = ctypes.c_void_p()
            if self.rt.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            out.append(h.value)
        return out

    def ms(self, a, b):
        f = ctypes.c_float()
        if self.rt.hipEventElapsedTime(ctypes.byref(f), ctypes.c_void_p(a), ctypes.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return f.value

    def destroy(self, hs):
        for h in hs:
            self.rt.hipEventDestroy(ctypes.c_void_p(h))


def timed_steps(plan, steps, warmup, ev):
    """Run warmup steps, then three timed passes of `steps` steps each:
      1. no stage events: wall ms/step (every recorded event leaves the GPU
         idle for about 6 us between the kernels it separates, so the
         step time is taken without them);
      2. events at the S X stage's two ends only: the stage's time per
         launch, with nothing recorded inside it;
      3. events at all five boundaries: the per-stage breakdown (each stage
         then also carries an event's idle time).
    Returns (wall ms/step, per-stage ms, total ms of pass 3, S X stage ms)."""
    import torch
    for _ in range(warmup):
        plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps

    def event_pass(mask):
        sets = [ev.create(5) for _ in range(steps)]
        for i in range(steps):
            plan.set_stage_events([h if keep else None for h, keep in zip(sets[i], mask)])
            plan.run()
        torch.cuda.synchronize()
        plan.set_stage_events(None)
        return sets

    sets = event_pass([True, False, True, False, False])
    sx_stage = sum(ev.ms(s[0], s[2]) for s in sets) / steps
    for s in sets:
        ev.destroy(s)
    sets = event_pass([True] * 5)
    # stage events: [0, 1) the S X prologue (binned: count and scan; atomic:
    # zero fill), [1, 2) the rest of S X, [2, 3) G (S X), [3, 4) the split reduction
    names = ["sx_prologue", "sx", "gsx", "reduce"]
    stage = {k: 0.0 for k in names}
    total = 0.0
    for s in sets:
        for j, k in enumerate(names):
            stage[k] += ev.ms(s[j], s[j + 1]) / steps
        total += ev.ms(s[0], s[4]) / steps
    for s in sets:
        ev.destroy(s)
    return wall, stage, total, sx_stage


def counters_traffic(kernel_launches_bytes):
    """HBM bytes per launch of the S X kernel from committed rocprofv3
    counter summaries, if they were taken on the current kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as f:
        c = json.load(f)
    if c.get("kernel_source_sha256") != sx_source_digest():
        return None
    return c.get("traffic_bytes_per_launch")


def cpu_baseline(w):
    import numpy as np  # noqa: F401
    import oracle as O
    c = w.csr
    runs = []
    cpu = []
    for _ in range(2):
        t0, c0 = time.perf_counter(), os.times()
        O.sketch_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.m, w.B, w.seed)
        c1 = os.times()
        runs.append(time.perf_counter() - t0)
        cpu.append((c1.user - c0.user) + (c1.system - c0.system))
    t = sorted(runs)[0]
    cores = max(1, round(sum(cpu) / sum(runs)))
    return {"value": c.nnz / t, "unit": "nnz/s", "cores": cores, "kind": "oracle",
            "sample": f"whole workload ({c.nnz} stored entries), best of 2 runs, "
                      f"{t:.2f} s per run, numpy FP64; host has {os.cpu_count()} logical CPUs"}


def ladder(steps, warmup, ev):
    import numpy as np  # noqa: F401
    import torch

    import oracle as O
    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    w = W.workload3()
    log("ladder: oracle FP64 reference ...")
    ref = O.sketch_dense(w.dense, w.m, w.B, w.seed)
    X = torch.from_numpy(w.dense).to("cuda")
    out = {"workload": w.name, "nnz": int(w.nnz)}
    for prec in ("native", "bf16", "fp8"):
        plan = cg.SketchPlan(X, w.m, w.B, w.seed, precision=prec)
        wall, stage, total, _ = timed_steps(plan, steps, warmup, ev)
        err = O.rel_frobenius(plan.Y.cpu().numpy(), ref)
        flops = 2.0 * w.m * w.B * w.d
        out["fp32" if prec == "native" else prec] = {
            "ms_per_step": round(wall, 4), "gsx_us": round(stage["gsx"] * 1e3, 2),
            "sx_us": round((stage["sx_prologue"] + stage["sx"]) * 1e3, 2),
            "gsx_tflops": round(flops / (stage["gsx"] * 1e-3) / 1e12, 2),
            "rel_fro_err_vs_fp64": float(f"{err:.3e}")}
        log(f"ladder {prec}: {wall:.3f} ms/step, gsx {stage['gsx']*1e3:.1f} us, err {err:.2e}")
        del plan
    del X
    torch.cuda.empty_cache()
    return out


def batched(log_fn):
    """The batched workload (512 uneven CSR instances, m = 32): 512
    sequential single-instance calls against one batch, with the built-in
    tuning table and after the autotuner."""
    import torch

    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import autotune
    from paper_1606_05732_amd import workloads as W
    log_fn("batched: generating 512 instances ...")
    ws = W.workload5()
    items = [(cg.CsrMatrix(torch.from_numpy(w.csr.row_ptr).cuda(),
                           torch.from_numpy(w.csr.col_idx).cuda(),
                           torch.from_numpy(w.csr.vals).cuda(), w.csr.n, w.csr.d),
              w.m, w.B, w.seed) for w in ws]
    nnz = sum(w.csr.nnz for w in ws)
    plans = [cg.SketchPlan(X, m, B, seed) for (X, m, B, seed) in items]
    for p in plans:
        p.run()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    start.record()
    for _ in range(reps):
        for p in plans:
            p.run()
    stop.record()
    stop.synchronize()
    seq_ms = start.elapsed_time(stop) / reps
    del plans
    torch.cuda.empty_cache()
    cg.set_tuning()
    default_ms = autotune.time_batch(items, reps=5, warmup=2)
    res = autotune.autotune_batched(items, reps=3, warmup=1)
    tuned_ms = autotune.time_batch(items, reps=10, warmup=2)
    log_fn(f"batched: sequential {seq_ms:.2f} ms, batch {default_ms:.2f} ms (built-in table), "
           f"{tuned_ms:.2f} ms (autotuned in {res['seconds']:.1f} s)")
    cls = res["classes"]
    plan = cg.BatchedSketch(items)
    rows_route = sum(plan.plan_fields(i)["route"] for i in range(len(items)))
    del plan
    return {"workload": "512 CSR instances, n log-uniform [1e4, 1e6], d in {8,16,32,64}, "
                        "density log-uniform [0.1%, 10%], m = 32, B = min(32 d^2, n/4)",
            "instances": len(items), "nnz": nnz, "rows_route_instances": rows_route,
            "sequential_ms": round(seq_ms, 3), "batched_builtin_ms": round(default_ms, 3),
            "batched_tuned_ms": round(tuned_ms, 3),
            "speedup_vs_sequential": round(seq_ms / tuned_ms, 2),
            "batched_nnz_per_s": nnz / (tuned_ms * 1e-3),
            "tuning": {f"d<=2^{c}": {"rows_per_item": res["rows_per_item"][c],
                                     "kc": res["kc_per_item"][c]} for c in cls},
            "autotune_trials": len(res["trials"]), "autotune_seconds": round(res["seconds"], 2)}


def adjoint(steps, warmup):
    """The adjoint dX = T^T dY = S^T (G^T dY) at the gradient workload's
    shape (dense dX: n = 2^22, d = 64; m = 128, B = 2^19): Z = G^T dY on
    MFMA (B x d, G generated in registers), then the signed row gather
    dX[r] = sigma(r) Z[h(r)].  Timed with events on the launch stream; the
    roofline counts the bytes the gather must move (dX written, Z read)."""
    import numpy as np
    import torch

    import paper_1606_05732_amd as cg
    n, d, m, B, seed = 1 << 22, 64, 128, 1 << 19, 2004
    dY = torch.from_numpy(np.random.default_rng(1004).standard_normal((m, d)).astype(np.float32)).cuda()
    dX = torch.empty((n, d), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        cg.sketch_adjoint(dY, n, m, B, seed, out=dX)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        cg.sketch_adjoint(dY, n, m, B, seed, out=dX)
    stop.record()
    stop.synchronize()
    t = start.elapsed_time(stop) / steps * 1e-3
    nbytes = 4 * n * d + 4 * B * d
    achieved = nbytes / t / 1e9
    log(f"adjoint: {t * 1e3:.3f} ms per call")
    return {"workload": f"dense_grad_n{n}_d{d}_m{m}_B{B}", "ms_per_call": round(t * 1e3, 4),
            "flops_gt_dy": 2.0 * m * B * d, "normals": m * B,
            "roofline": {"bound": "hbm", "kernel": "adjoint (G^T dY, then the dX gather)",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes_per_launch": nbytes}}


def algos(steps, warmup, ev, X2, w2):
    """Every S X algorithm on the FP32 CSR workload (X2, already on the GPU),
    and the FP64 CSR workload (n = 10^6, d = 10, 1% density, m = 20,
    B = 2000) with its automatic choice (atomic: FP64) and the sorted
    path: ms per step and the S X stage's time against its algorithmic
    bytes."""
    import torch

    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    out = {}

    def one(X, w, c, algo, elem):
        plan = cg.SketchPlan(X, w.m, w.B, w.seed, algo=algo)
        wall, stage, total, sx_stage = timed_steps(plan, steps, warmup, ev)
        sx_bytes = (4 + elem) * c.nnz + 4 * (c.n + 1) + elem * w.B * c.d
        ach = sx_bytes / (max(sx_stage, 1e-6) * 1e-3) / 1e9
        log(f"algos: {w.name} {algo}: {wall:.4f} ms/step, S X stage {sx_stage * 1e3:.1f} us")
        r = {"ms_per_step": round(wall, 4), "nnz_per_s": c.nnz / (wall * 1e-3)}
        if algo != "rows":   # the rows route forms no S X: no stage of its own
            r.update({"sx_stage_us": round(sx_stage * 1e3, 2), "sx_gbs": round(ach, 1),
                      "sx_frac_hbm": round(ach / HBM_PEAK_GBS, 4)})
        return r

    c2 = w2.csr
    out[w2.name] = {a: one(X2, w2, c2, a, 4) for a in ("binned", "atomic", "sorted", "rows")}
    w1 = W.workload1()
    c1 = w1.csr
    X1 = cg.CsrMatrix(torch.from_numpy(c1.row_ptr).cuda(), torch.from_numpy(c1.col_idx).cuda(),
                      torch.from_numpy(c1.vals).cuda(), c1.n, c1.d)
    out[w1.name + "_fp64"] = {a: one(X1, w1, c1, a, 8) for a in ("auto", "sorted")}
    return out


def adjoint_csr(steps, warmup, X, w):
    """The CSR adjoint (the gradient with respect to the stored values,
    dvals[k] = sigma(r) Z[h(r)][col_k]) on the FP32 CSR workload's matrix
    and sketch: Z = G^T dY, then one gather per stored entry.  The
    roofline counts the entries' reads (col_idx, row_ptr), the dvals
    writes and one read of Z."""
    import numpy as np
    import torch

    import paper_1606_05732_amd as cg
    c = w.csr
    dY = torch.from_numpy(np.random.default_rng(1002).standard_normal((w.m, c.d)).astype(np.float32)).cuda()
    for _ in range(warmup):
        cg.sketch_adjoint_csr(X, dY, w.m, w.B, w.seed)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        cg.sketch_adjoint_csr(X, dY, w.m, w.B, w.seed)
    stop.record()
    stop.synchronize()
    t = start.elapsed_time(stop) / steps * 1e-3
    nbytes = 8 * c.nnz + 4 * (c.n + 1) + 4 * w.B * c.d
    achieved = nbytes / t / 1e9
    log(f"adjoint csr: {t * 1e3:.3f} ms per call")
    return {"workload": w.name, "ms_per_call": round(t * 1e3, 4),
            "roofline": {"bound": "hbm", "kernel": "CSR adjoint (G^T dY, then the per-entry gather)",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes_per_launch": nbytes}}


def copy_calibration(mib=512, reps=3):
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters: run it under the same rocprofv3 --pmc pass as the
    kernels, then bytes_true / counter_reading is the scale factor."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.randn(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4,
                                           "launches": reps}}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--algo", default="auto", choices=["auto", "binned", "atomic", "sorted"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ladder", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--algos", action="store_true",
                    help="also time every S X algorithm (and the FP64 CSR workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the transform shards by rows with one m x d all-reduce; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        copy_calibration()
        return
    ev = HipEvents()
    log("generating workload ...")
    w = W.workload2()
    c = w.csr
    X = cg.CsrMatrix(torch.from_numpy(c.row_ptr).cuda(), torch.from_numpy(c.col_idx).cuda(),
                     torch.from_numpy(c.vals).cuda(), c.n, c.d)
    plan = cg.SketchPlan(X, w.m, w.B, w.seed, algo=args.algo)
    log(f"workload {w.name}: nnz {c.nnz}, workspace {plan.workspace_bytes/2**20:.1f} MiB")
    wall, stage, total, sx_stage = timed_steps(plan, args.steps, args.warmup, ev)
    nnz = c.nnz
    sx_bytes = 8 * nnz + 4 * (c.n + 1) + 4 * w.B * c.d
    # the whole S X stage (count, scan, scatter, reduce; timed with events at
    # its two ends only) against its algorithmic bytes
    sx_s = sx_stage * 1e-3
    achieved = sx_bytes / sx_s / 1e9
    traffic = counters_traffic(sx_bytes)
    gsx_flops = 2.0 * w.m * w.B * c.d
    log(f"wall {wall:.4f} ms/step; S X stage {sx_stage*1e3:.1f} us; "
        f"with all stage events: sx prologue {stage['sx_prologue']*1e3:.1f} us, "
        f"sx {stage['sx']*1e3:.1f} us, gsx {stage['gsx']*1e3:.1f} us, "
        f"reduce {stage['reduce']*1e3:.1f} us, total {total*1e3:.1f} us")
    result = {
        "metric": METRIC,
        "value": nnz / (wall * 1e-3),
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": c.n, "d": c.d, "density": 0.05, "nnz": nnz,
                   "m": w.m, "B": w.B, "values": "|N(0,1)| float32", "sx_algo": args.algo,
                   "precision": "fp32", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm",
                     "kernel": f"S.X stage ({args.algo}: bin_count, bin_scan, bin_scatter, bin_reduce)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # the counted bytes over the same time: how close the stage
                     # runs to the memory system, whatever it has to move
                     "traffic_gbs": round(traffic / sx_s / 1e9, 1) if traffic else None,
                     "algorithmic_bytes_per_launch": sx_bytes,
                     "avg_launch_us": round(sx_s * 1e6, 2)},
        # per-stage breakdown from a pass with an event at every stage
        # boundary (each stage then carries one event's idle time)
        "stages_us": {k: round(v * 1e3, 2) for k, v in stage.items()},
        "gsx": {"avg_launch_us": round(stage["gsx"] * 1e3, 2),
                "tflops": round(gsx_flops / (stage["gsx"] * 1e-3) / 1e12, 3),
                "frac_fp32_mfma_peak": round(gsx_flops / (stage["gsx"] * 1e-3) / 1e12
                                             / MFMA_FP32_TFLOPS, 4),
                "normals_per_launch": w.m * w.B},
    }
    if args.algos:
        result["algos"] = algos(max(5, args.steps // 2), 2, ev, X, w)
    if not args.no_adjoint:
        result["adjoint_csr"] = adjoint_csr(max(5, args.steps // 2), 2, X, w)
    del plan, X
    torch.cuda.empty_cache()
    if not args.no_ladder:
        result["ladder"] = ladder(max(5, args.steps // 2), 2, ev)
    if not args.no_batched:
        result["batched"] = batched(log)
    if not args.no_adjoint:
        result["adjoint"] = adjoint(max(5, args.steps // 2), 2)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
