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
  dense_gaussian  the dense Gaussian projection G~ X (the product T X
               stands in for) against T X on the same inputs: the CSR
               workload and the dense n = 2^22 workloads (d = 32 and 64)
  nmf_recovery Algorithm 1's anchor recovery rate on the separable
               generator of the paper's Section 6, CountGauss against the
               Gaussian baseline
  lemma_lb     the lower-bound lemma's sweep over B on its block matrix:
               distinguishing rate of T U against G~ U, unique-collision
               rate, ||I - M||_F^2, KL and Pinsker bound given S
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
# dense MFMA peaks of MI355X per input type (TFLOP/s), without sparsity
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
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


def graph_steps(plan, steps, warmup):
    """ms per step when the step is captured once in a HIP graph and
    replayed (SketchPlan.capture): the same kernels, one launch per step.
    Timed like pass 1 of timed_steps (host clock around synchronised
    replays)."""
    import torch
    graph = plan.capture()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    del graph
    return ms


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


_CPU_JOB = {}   # the workload and S X, inherited by the forked workers


def _oracle_sx_rows(block):
    """S X of one row block of the CSR workload, by the oracle's sx_csr with
    the block's global row offset (S X is linear in the rows, so the
    blocks' results add up to the whole)."""
    import oracle as O
    w, (a, b) = _CPU_JOB["w"], block
    c = w.csr
    k0, k1 = int(c.row_ptr[a]), int(c.row_ptr[b])
    return O.sx_csr(c.row_ptr[a:b + 1] - k0, c.col_idx[k0:k1], c.vals[k0:k1], b - a, c.d, w.seed,
                    w.B, row_offset=a)


def _oracle_g_cols(block):
    """G[:, a:b] (S X)[a:b] by the oracle's gaussian_block: one column block
    of the product G (S X)."""
    import oracle as O
    w, SX, (a, b) = _CPU_JOB["w"], _CPU_JOB["SX"], block
    return O.gaussian_block(w.seed, w.m, a, b - a) @ SX[a:b]


def cpu_baseline_all_cores(w, procs):
    """The oracle on all host cores: S X of `procs` row blocks in parallel
    processes, summed, then G (S X) as `procs` column blocks of G in
    parallel, summed -- the oracle's own functions on blocks (the inputs
    reach the workers by fork, not by copies)."""
    import multiprocessing as mp

    import numpy as np
    import oracle as O
    c = w.csr
    rb = np.linspace(0, c.n, procs + 1).astype(np.int64)
    cb = np.linspace(0, w.B, procs + 1).astype(np.int64)
    ctx = mp.get_context("fork")
    _CPU_JOB["w"] = w
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        SX = sum(pool.map(_oracle_sx_rows, [(int(a), int(b)) for a, b in zip(rb[:-1], rb[1:])]))
    _CPU_JOB["SX"] = SX
    with ctx.Pool(procs) as pool:
        Y = sum(pool.map(_oracle_g_cols, [(int(a), int(b)) for a, b in zip(cb[:-1], cb[1:])]))
    t = time.perf_counter() - t0
    _CPU_JOB.clear()
    ref = O.sketch_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.m, w.B, w.seed)
    assert O.rel_frobenius(Y, ref) < 1e-12
    return {"value": c.nnz / t, "unit": "nnz/s", "cores": procs, "kind": "oracle",
            "sample": f"whole workload: S X over {procs} row blocks, then G (S X) over {procs} "
                      f"column blocks of G, in {procs} forked processes (fork time included), "
                      f"{t:.2f} s"}


def normals_ceiling(m, B, seed, reps=20):
    """The generator's own ceiling: time for the library to draw the m x B
    normals of G and nothing else (cg_debug_normals, the contractions'
    counters and FP32 Box-Muller), with events around `reps` launches."""
    import torch

    from paper_1606_05732_amd import _lib as L
    lib = L.load()
    sink = torch.empty(L.CG_NORMALS_SINK, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call():
        L.check(lib.cg_debug_normals(seed, m, B, ctypes.c_void_p(sink.data_ptr()), stream),
                "cg_debug_normals")
    ms = event_time_ms(call, reps, 3)
    del sink
    return ms * 1e3


def ladder(steps, warmup, ev, read_gbs):
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
    # every rung draws the same m B normals: the generator's ceiling bounds
    # the contraction from below whatever the MFMA type
    rng_us = normals_ceiling(w.m, w.B, w.seed)
    out["rng_bound_us"] = round(rng_us, 2)
    out["rng_normals_per_s"] = float(f"{w.m * w.B / (rng_us * 1e-6):.4g}")
    log(f"ladder: drawing the {w.m} x {w.B} normals alone takes {rng_us:.1f} us")
    # every rung reads the FP32 S X once, at best at the measured read rate
    sx_read_us = 4.0 * w.B * w.d / (read_gbs * 1e9) * 1e6
    out["sx_read_bound_us"] = round(sx_read_us, 2)
    for prec in ("native", "bf16", "fp8"):
        plan = cg.SketchPlan(X, w.m, w.B, w.seed, precision=prec)
        wall, stage, total, _ = timed_steps(plan, steps, warmup, ev)
        err = O.rel_frobenius(plan.Y.cpu().numpy(), ref)
        flops = 2.0 * w.m * w.B * w.d
        rung = "fp32" if prec == "native" else prec
        tflops = flops / (stage["gsx"] * 1e-3) / 1e12
        out[rung] = {
            "ms_per_step": round(wall, 4), "gsx_us": round(stage["gsx"] * 1e3, 2),
            "sx_us": round((stage["sx_prologue"] + stage["sx"]) * 1e3, 2),
            "gsx_tflops": round(tflops, 2),
            "mfma_peak_tflops": MFMA_PEAK_TFLOPS[rung],
            "frac_of_mfma_peak": round(tflops / MFMA_PEAK_TFLOPS[rung], 4),
            "frac_of_rng_bound": round(rng_us / (stage["gsx"] * 1e3), 3),
            "rel_fro_err_vs_fp64": float(f"{err:.3e}")}
        # the rung's floor: its S X read, or its normals plus its MFMA time
        # at the dtype's peak (added: a SIMD never issues vector ALU and
        # MFMA instructions in the same cycle on this part -- the
        # co-execution counter stays at zero), whichever is longer
        mfma_us = flops / (MFMA_PEAK_TFLOPS[rung] * 1e12) * 1e6
        floor_us = max(sx_read_us, rng_us + mfma_us)
        out[rung]["floor_us"] = round(floor_us, 2)
        out[rung]["frac_of_floor"] = round(floor_us / (stage["gsx"] * 1e3), 3)
        log(f"ladder {prec}: {wall:.3f} ms/step, gsx {stage['gsx']*1e3:.1f} us "
            f"({rng_us / (stage['gsx'] * 1e3):.2f} of the generator's ceiling), err {err:.2e}")
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
    seq_Y = [p.Y.clone() for p in plans]
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
    # accuracy of the (autotuned) batch: every instance against its own
    # single call, and a sample against the FP64 oracle
    import oracle as O
    Ys = cg.sketch_batched(items)
    torch.cuda.synchronize()
    vs_seq = max(O.rel_frobenius(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(Ys, seq_Y))
    picks = list(range(0, len(ws), 16))
    vs_oracle = max(O.rel_frobenius(Ys[k].cpu().numpy(),
                                    O.sketch_csr(ws[k].csr.row_ptr, ws[k].csr.col_idx,
                                                 ws[k].csr.vals, ws[k].csr.n, ws[k].csr.d,
                                                 ws[k].m, ws[k].B, ws[k].seed)) for k in picks)
    log(f"batched: max error vs FP64 oracle {vs_oracle:.2e} ({len(picks)} instances), "
        f"max difference vs single calls {vs_seq:.2e} (all)")
    return {"workload": "512 CSR instances, n log-uniform [1e4, 1e6], d in {8,16,32,64}, "
                        "density log-uniform [0.1%, 10%], m = 32, B = min(32 d^2, n/4)",
            "instances": len(items), "nnz": nnz, "rows_route_instances": rows_route,
            "sequential_ms": round(seq_ms, 3), "batched_builtin_ms": round(default_ms, 3),
            "batched_tuned_ms": round(tuned_ms, 3),
            "speedup_vs_sequential": round(seq_ms / tuned_ms, 2),
            "batched_nnz_per_s": nnz / (tuned_ms * 1e-3),
            "tuning": {f"d<=2^{c}": {"rows_per_item": res["rows_per_item"][c],
                                     "kc": res["kc_per_item"][c]} for c in cls},
            "autotune_trials": len(res["trials"]), "autotune_seconds": round(res["seconds"], 2),
            "max_rel_fro_err_vs_fp64": float(f"{vs_oracle:.3e}"), "err_sample": len(picks),
            "max_rel_diff_vs_single_calls": float(f"{vs_seq:.3e}")}


def other_configs(steps, warmup, ev):
    """The other configurations in the headline list, one line each: the
    dense n = 2^22, d = 32 input of the FP32-at-scale workload (m = 64,
    B = 65536) and the FP64 CSR workload (n = 10^6, d = 10, 1% density,
    m = 20, B = 2000), each as a whole T X step (nnz/s) and its S X stage
    against that stage's algorithmic bytes, with the error against the FP64
    oracle."""
    import torch

    import oracle as O
    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    out = {}
    w = W.workload2_dense()
    X = torch.from_numpy(w.dense).cuda()
    plan = cg.SketchPlan(X, w.m, w.B, w.seed)
    wall, stage, total, sx_stage = timed_steps(plan, steps, warmup, ev)
    nbytes = 4 * w.n * w.d + 4 * w.B * w.d   # read X, write S X
    ach = nbytes / (sx_stage * 1e-3) / 1e9
    err = O.rel_frobenius(plan.Y.cpu().numpy(), O.sketch_dense(w.dense, w.m, w.B, w.seed))
    out["dense"] = {"workload": w.name, "dtype": "f32", "ms_per_step": round(wall, 4),
                    "value": w.n * w.d / (wall * 1e-3), "unit": "nnz/s",
                    "rel_fro_err_vs_fp64": float(f"{err:.3e}"),
                    "roofline": {"bound": "hbm", "kernel": "S.X stage (binned, dense)",
                                 "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(ach / HBM_PEAK_GBS, 4),
                                 "algorithmic_bytes_per_launch": nbytes,
                                 "avg_launch_us": round(sx_stage * 1e3, 2)}}
    log(f"dense d=32: {wall:.4f} ms/step, S X stage {sx_stage*1e3:.1f} us, err {err:.2e}")
    del plan, X
    torch.cuda.empty_cache()
    w = W.workload1()
    c = w.csr
    X = cg.CsrMatrix(torch.from_numpy(c.row_ptr).cuda(), torch.from_numpy(c.col_idx).cuda(),
                     torch.from_numpy(c.vals).cuda(), c.n, c.d)
    plan = cg.SketchPlan(X, w.m, w.B, w.seed)
    wall, stage, total, sx_stage = timed_steps(plan, steps, warmup, ev)
    nbytes = 12 * c.nnz + 4 * (c.n + 1) + 8 * w.B * c.d
    ach = nbytes / (max(sx_stage, 1e-6) * 1e-3) / 1e9
    err = O.rel_frobenius(plan.Y.cpu().numpy(),
                          O.sketch_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.m, w.B, w.seed))
    out["fp64_csr"] = {"workload": w.name, "dtype": "f64", "ms_per_step": round(wall, 4),
                       "value": c.nnz / (wall * 1e-3), "unit": "nnz/s", "nnz": c.nnz,
                       "rel_fro_err_vs_fp64": float(f"{err:.3e}"),
                       "roofline": {"bound": "hbm", "kernel": "S.X stage (auto: atomic, FP64)",
                                    "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(ach / HBM_PEAK_GBS, 4),
                                    "algorithmic_bytes_per_launch": nbytes,
                                    "avg_launch_us": round(sx_stage * 1e3, 2)}}
    log(f"fp64 csr: {wall:.4f} ms/step, S X stage {sx_stage*1e3:.1f} us, err {err:.2e}")
    return out


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
        if algo not in ("rows", "fused"):   # no S X stage of its own there
            r.update({"sx_stage_us": round(sx_stage * 1e3, 2), "sx_gbs": round(ach, 1),
                      "sx_frac_hbm": round(ach / HBM_PEAK_GBS, 4)})
        return r

    c2 = w2.csr
    out[w2.name] = {a: one(X2, w2, c2, a, 4) for a in ("binned", "atomic", "sorted", "rows", "fused")}
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


def event_time_ms(fn, steps, warmup):
    """Mean ms per call of fn() over `steps` calls after `warmup`, with
    events on torch's current stream (where the library queues its work)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / steps


def dense_gaussian(steps, warmup, X2, w2):
    """The dense Gaussian projection G~ X that T X stands in for (the
    paper's comparison, Section 1.1 "Our Results"), against T X on the same
    inputs: the FP32 CSR workload (X2, already on the GPU), and the dense
    n = 2^22 workloads with d = 32 (m = 64, B = 65536) and d = 64 (m = 64,
    B = 262144).  G~ X draws m normals per (nonempty) row of X and does
    2 m nnz flops on MFMA; T X draws m normals per bucket."""
    import torch

    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    out = {}

    def one(name, X, nnz, rows, d, m, B, seed):
        plan = cg.SketchPlan(X, m, B, seed)
        t_tx = event_time_ms(plan.run, steps, warmup)
        del plan
        t_g = event_time_ms(lambda: cg.gaussian(X, m, seed), steps, warmup)
        flops = 2.0 * m * nnz
        normals = m * rows
        log(f"dense gaussian {name}: G~X {t_g:.3f} ms, TX {t_tx:.3f} ms")
        out[name] = {"gx_ms": round(t_g, 4), "tx_ms": round(t_tx, 4),
                     "tx_speedup_over_gx": round(t_g / t_tx, 2),
                     "gx_nnz_per_s": nnz / (t_g * 1e-3), "tx_nnz_per_s": nnz / (t_tx * 1e-3),
                     "gx_tflops": round(flops / (t_g * 1e-3) / 1e12, 2),
                     "gx_frac_fp32_mfma_peak": round(flops / (t_g * 1e-3) / 1e12 / MFMA_FP32_TFLOPS, 4),
                     "gx_normals_per_s": normals / (t_g * 1e-3),
                     "gx_normals": normals}

    c = w2.csr
    nonempty = int((c.row_ptr[1:] > c.row_ptr[:-1]).sum())
    one(w2.name, X2, c.nnz, nonempty, c.d, w2.m, w2.B, w2.seed)
    for w in (W.workload2_dense(), W.workload3()):
        Xd = torch.from_numpy(w.dense).cuda()
        one(w.name, Xd, w.n * w.d, w.n, w.d, w.m, w.B, w.seed)
        del Xd
        torch.cuda.empty_cache()
    return out


def nmf_recovery(trials):
    """The exact-recovery experiment of Section 6 on its synthetic separable
    generator: for a grid of (k, m), `trials` datasets of 1000 x 500 (features
    x points) with nonnegative rank k; the fraction of datasets whose anchors
    all appear among Algorithm 1's row extrema, with Z = T X (CountGauss,
    B = 5 m as in the paper's experiments) and with Z = G~ X (the Gaussian
    baseline, "GP").  FP32 on the GPU."""
    import numpy as np
    import torch

    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    grid = []
    for k in (5, 10, 20, 40):
        mk = int(np.ceil(k * np.log(k)))
        grid += [(k, m) for m in sorted({k, mk, 2 * mk})]
    rng = np.random.Generator(np.random.PCG64(1006))
    out = {"features": 1000, "points": 500, "trials": trials, "B": "5 m", "grid": []}
    t0 = time.perf_counter()
    for k, m in grid:
        hit_cg = hit_gp = 0
        for t in range(trials):
            X, anchors = W.separable_nmf(rng, 1000, 500, k, dtype=np.float32)
            Xg = torch.from_numpy(X).cuda()
            seed = 6_000_000 + 1000 * k + t
            a = set(anchors.tolist())
            for proj in ("countgauss", "gaussian"):
                imax, imin = cg.anchors(Xg, m, 5 * m, seed, proj)
                found = set(imax.cpu().tolist()) | set(imin.cpu().tolist())
                if a <= found:
                    if proj == "countgauss":
                        hit_cg += 1
                    else:
                        hit_gp += 1
        out["grid"].append({"k": k, "m": m, "countgauss": hit_cg / trials, "gaussian": hit_gp / trials})
        log(f"nmf recovery k={k} m={m}: countgauss {hit_cg / trials:.3f}, gaussian {hit_gp / trials:.3f}")
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def lemma_sweep(seeds):
    """The lower-bound lemma of Section 7 on its block matrix U (d = 16
    columns of L = ceil(sqrt(B) / d) rows each, orthonormal), FP64, m = 64:
    for B from d^2 m / 64 up to d^2 m, `seeds` draws of T U and of G~ U.
    Reported per B: the pair statistic's rate above the 95th percentile of
    its G~ U values (so the difference of the two rates is an empirical
    lower bound on the total variation between T U and G~ U), how often M
    has exactly one nonzero off-diagonal pair (the lemma's unique
    collision), and the means of ||I - M||_F^2 (against its closed form
    (d^2 + d - 2 d / L) / B), of KL(N(0, I) || N(0, M)) and of Pinsker's
    bound on the total variation given S (the proof of Theorem 1)."""
    import numpy as np
    import torch

    import paper_1606_05732_amd as cg
    from paper_1606_05732_amd import workloads as W
    d, m = 16, 64
    out = {"d": d, "m": m, "seeds": seeds, "precision": "fp64", "sweep": []}
    t0 = time.perf_counter()
    for B in [d * d * m // f for f in (64, 32, 16, 8, 4, 2, 1)]:
        L = int(np.ceil(np.sqrt(B) / d))
        rp, ci, v, n = W.block_orthonormal(d, L)
        X = cg.CsrMatrix(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                         torch.from_numpy(v).cuda(), n, d)
        Ud = torch.from_numpy(np.ascontiguousarray(
            np.kron(np.eye(d), np.ones((L, 1))) / np.sqrt(L))).cuda()
        SU = torch.empty((B, d), dtype=torch.float64, device="cuda")
        st_t, st_g = [], []
        for s in range(seeds):
            seed = 7_000_000 + 1000 * B + s
            Y = cg.sketch(X, m, B, seed, algo="atomic", sx_out=SU)
            st_t.append(cg.lemma_stats(Y, SU))
            st_g.append(cg.lemma_stats(cg.gaussian(Ud, m, seed)))
        T = torch.stack(st_t).cpu().numpy()
        G = torch.stack(st_g).cpu().numpy()
        tau = float(np.quantile(G[:, 0], 0.95))
        p_t, p_g = float(np.mean(T[:, 0] > tau)), float(np.mean(G[:, 0] > tau))
        row = {"B": B, "L": L, "B_over_d2m": B / (d * d * m), "threshold": round(tau, 2),
               "rate_TU": p_t, "rate_GU": p_g, "tv_lower_estimate": round(p_t - p_g, 3),
               "unique_collision_rate": float(np.mean(T[:, 4] == 1)),
               "frobenius_gap_mean": float(np.mean(T[:, 1])),
               "frobenius_gap_expected": (d * d + d - 2.0 * d / L) / B,
               "kl_mean": float(np.mean(T[np.isfinite(T[:, 2]), 2])) if np.any(np.isfinite(T[:, 2])) else None,
               "singular_rate": float(np.mean(T[:, 5] == 0)),
               "tv_pinsker_bound_mean": float(np.mean(T[:, 3]))}
        out["sweep"].append(row)
        log(f"lemma B={B} L={L}: T U above threshold {p_t:.3f}, G~ U {p_g:.3f}, "
            f"unique collision {row['unique_collision_rate']:.3f}, "
            f"E||I-M||^2 {row['frobenius_gap_mean']:.4f} (closed form {row['frobenius_gap_expected']:.4f}), "
            f"Pinsker {row['tv_pinsker_bound_mean']:.3f}")
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def memory_ceilings(mib=1024, reps=10):
    """Measured ceilings of this GPU's memory system (cg_debug_stream, 16-byte
    accesses): a device copy, a read and a write of `mib` MiB, in GB/s of
    bytes moved (the copy counts its reads and its writes)."""
    import torch

    from paper_1606_05732_amd import _lib as L
    lib = L.load()
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(1 << 14, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {"bytes": nbytes}
    for name, kinds, a, b, moved in (("copy", (L.CG_STREAM_COPY, L.CG_STREAM_COPY_NT), src, dst, 2 * nbytes),
                                     ("read", (L.CG_STREAM_READ, L.CG_STREAM_READ_NT), src, sink, nbytes),
                                     ("write", (L.CG_STREAM_WRITE, L.CG_STREAM_WRITE_NT), None, dst,
                                      nbytes)):
        best = 0.0
        for kind in kinds:   # plain and non-temporal accesses: the faster is the ceiling
            def call():
                L.check(lib.cg_debug_stream(kind, ctypes.c_void_p(a.data_ptr()) if a is not None
                                            else None, ctypes.c_void_p(b.data_ptr()), nbytes, stream),
                        "cg_debug_stream")
            ms = event_time_ms(call, reps, 2)
            best = max(best, moved / (ms * 1e-3) / 1e9)
        out[name + "_gbs"] = round(best, 1)
    log(f"memory ceilings: copy {out['copy_gbs']} GB/s, read {out['read_gbs']} GB/s, "
        f"write {out['write_gbs']} GB/s")
    del src, dst
    torch.cuda.empty_cache()
    return out


def copy_calibration(mib=512, reps=3):
    """A plain device copy of known size (the library's 16-byte copy kernel,
    cg_debug_stream), for scaling the HBM byte counters: run it under the
    same rocprofv3 --pmc pass as the kernels, then bytes_true /
    counter_reading is the scale factor."""
    import torch

    from paper_1606_05732_amd import _lib as L
    lib = L.load()
    nbytes = mib << 20
    src = torch.randn(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for _ in range(reps):
        L.check(lib.cg_debug_stream(L.CG_STREAM_COPY, ctypes.c_void_p(src.data_ptr()),
                                    ctypes.c_void_p(dst.data_ptr()), nbytes, stream),
                "cg_debug_stream")
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"kernel": "stream_copy_kernel", "bytes_read": nbytes,
                                           "bytes_written": nbytes, "launches": reps}}), flush=True)


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
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the dense d = 32 and FP64 CSR lines")
    ap.add_argument("--no-gaussian", action="store_true",
                    help="skip the dense Gaussian G~ X comparison")
    ap.add_argument("--nmf-trials", type=int, default=100,
                    help="datasets per (k, m) in the anchor recovery experiment (0: skip)")
    ap.add_argument("--lemma-seeds", type=int, default=200,
                    help="seeds per B in the lower-bound lemma sweep (0: skip)")
    ap.add_argument("--algos", action="store_true",
                    help="also time every S X algorithm (and the FP64 CSR workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the transform shards by rows with one m x d all-reduce per call)",
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
    graph_ms = graph_steps(plan, args.steps, args.warmup)
    log(f"the same step replayed from a HIP graph: {graph_ms:.4f} ms/step")
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
        # the same step replayed from a HIP graph (one launch per step)
        "graph": {"ms_per_step": round(graph_ms, 5), "nnz_per_s": nnz / (graph_ms * 1e-3)},
        "gsx": {"avg_launch_us": round(stage["gsx"] * 1e3, 2),
                "tflops": round(gsx_flops / (stage["gsx"] * 1e-3) / 1e12, 3),
                "frac_fp32_mfma_peak": round(gsx_flops / (stage["gsx"] * 1e-3) / 1e12
                                             / MFMA_FP32_TFLOPS, 4),
                "normals_per_launch": w.m * w.B},
    }
    ceil = memory_ceilings()
    result["memory_ceilings"] = ceil
    # the S X stage's algorithmic bytes over its time, against the measured
    # copy rate (a copy reads and writes, like the stage)
    result["roofline"]["frac_of_copy_ceiling"] = round(achieved / ceil["copy_gbs"], 4)
    if args.algos:
        result["algos"] = algos(max(5, args.steps // 2), 2, ev, X, w)
    if not args.no_adjoint:
        result["adjoint_csr"] = adjoint_csr(max(5, args.steps // 2), 2, X, w)
    del plan
    if not args.no_gaussian:
        result["dense_gaussian"] = dense_gaussian(max(5, args.steps // 2), 2, X, w)
    del X
    torch.cuda.empty_cache()
    if not args.no_other_configs:
        result["other_configs"] = other_configs(max(5, args.steps // 2), 2, ev)
    if not args.no_ladder:
        result["ladder"] = ladder(max(5, args.steps // 2), 2, ev, ceil["read_gbs"])
    if not args.no_batched:
        result["batched"] = batched(log)
    if not args.no_adjoint:
        result["adjoint"] = adjoint(max(5, args.steps // 2), 2)
    if args.nmf_trials > 0:
        result["nmf_recovery"] = nmf_recovery(args.nmf_trials)
    if args.lemma_seeds > 0:
        result["lemma_lb"] = lemma_sweep(args.lemma_seeds)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w)
        procs = min(16, os.cpu_count() or 1)
        if procs > 1:
            log(f"cpu baseline (oracle, {procs} processes) ...")
            result["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w, procs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
