"""Benchmark of the FP64 tiled QR on one MI355X.

A step is one tiled QR factorisation (tqr_factor: column-major -> tiles, the
persistent task-graph launch, tiles -> column-major) of an 8192 x 8192 N(0,1)
matrix with tile_b = 256, inner_ib = 16; every timed step factors its own
pristine copy of the input, resident in HBM before the timed region starts.
`value` is the rate on the standard Householder count 2n^2(m - n/3); the
tiled method's executed count and the (4mn^2 - 4n^3/3) convention are
reported beside it.  The tall-skinny 65536 x 1024 U[-1,1] factorisation
(same tiling) is reported beside it too.  Prints one JSON line.
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

FP64_MFMA_PEAK_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_factor_8192_b256.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0707_3548_amd", "csrc", f)
                  for f in ("tqr.hip", "tqr_inst.hip", "tqr_batched.hip", "tqr_impl.h", "tqr_device.h", "tqr_graph.h",
                            "tqr_narrow.h", "tqr_offsets.h")] + \
    [os.path.join(ROOT, "paper_0707_3548_amd", "build.py")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--tile-b", type=int, default=256)
    ap.add_argument("--inner-ib", type=int, default=16)
    ap.add_argument("--policy", choices=["default", "paper", "lookahead", "column"], default="default",
                    help="default: the plain tqr_factor call (no options)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the oracle's CPU sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tall", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--batch-count", type=int, default=20000)
    return ap.parse_args()


def time_factor(tqr, torch, A_host, b, ib, steps, warmup, policy):
    """Factor `warmup + steps` device copies of A through the plain boundary
    call tqr_factor (no options; with --policy other than "default" through
    tqr_factor_ex with that policy); returns (wall ms/step over the timed
    steps, the per-step scheduler-launch times from HIP events recorded by the
    library around the launch in a second pass of the same call with options,
    the last factored matrix, its workspace)."""
    m, n = A_host.shape
    src = tqr.fortran(torch.from_numpy(A_host).cuda())
    copies = [src.clone() for _ in range(warmup + steps)]  # clone keeps the column-major strides
    ws = tqr.Workspace(m, n, 0, b, ib)
    pol = {"paper": tqr.POLICY_PAPER, "lookahead": tqr.POLICY_LOOKAHEAD, "column": tqr.POLICY_COLUMN,
           "default": tqr.POLICY_COLUMN}[policy]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def run(X, events=None):
        if policy == "default" and events is None:
            tqr.factor_plain(X, b, ib, ws)
        else:
            tqr.factor(X, b, ib, ws, policy=pol, status=status, events=events)

    for w in range(warmup):
        run(copies[w])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        run(copies[warmup + s])
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    out = copies[-1].clone()
    # the scheduler launch alone, from HIP events on the launch stream
    ev = tqr.HipEvents()
    evs = [(ev.create(), ev.create()) for _ in range(steps)]
    for s in range(steps):
        copies[s].copy_(src)
    for s in range(steps):
        run(copies[s], events=evs[s])
    torch.cuda.synchronize()
    kern_ms = [ev.elapsed_ms(a, e) for a, e in evs]
    if int(status.item()) != 0:
        raise RuntimeError(f"scheduler reported status {int(status.item())}")
    for a, e in evs:
        ev.destroy(a)
        ev.destroy(e)
    del copies, src
    return wall_ms, kern_ms, out, ws


def cond2_estimate(torch, R, iters=60):
    """kappa_2 of the input from its R factor (on the device): power
    iteration on R^T R for sigma_max, inverse iteration through two
    triangular solves for sigma_min."""
    g = torch.Generator(device=R.device)
    g.manual_seed(0)
    n = R.shape[0]
    x = torch.randn(n, 1, dtype=torch.float64, device=R.device, generator=g)
    for _ in range(iters):
        x = R.T @ (R @ x)
        x /= torch.linalg.norm(x)
    smax = float(torch.linalg.norm(R.T @ (R @ x))) ** 0.5
    y = torch.randn(n, 1, dtype=torch.float64, device=R.device, generator=g)
    for _ in range(iters):
        y = torch.linalg.solve_triangular(R, torch.linalg.solve_triangular(R.T, y, upper=False), upper=True)
        y /= torch.linalg.norm(y)
    z = torch.linalg.solve_triangular(R, torch.linalg.solve_triangular(R.T, y, upper=False), upper=True)
    smin = 1.0 / float(torch.linalg.norm(z)) ** 0.5
    return smax / smin


def spot_check(torch, A_host, F, n_check=256):
    """Properties that hold at any size, checked on the GPU result:
    column norms of R equal those of A (Q is orthogonal), and the leading
    n_check x n_check block of R equals the R of A[:, :n_check] (computed by
    LAPACK through numpy here -- a sanity check, the parity tests use the
    oracle)."""
    import numpy as np
    m, n = A_host.shape
    R = torch.triu(F[:n, :])
    cn_r = torch.linalg.vector_norm(R, dim=0).cpu().numpy()
    cn_a = np.linalg.norm(A_host, axis=0)
    col_err = float(np.max(np.abs(cn_r - cn_a) / cn_a))
    _, R0 = np.linalg.qr(A_host[:, :n_check])
    d = np.sign(np.diag(R0)); d[d == 0] = 1
    R0 = d[:, None] * R0
    Rg = R[:n_check, :n_check].cpu().numpy()
    dg = np.sign(np.diag(Rg)); dg[dg == 0] = 1
    Rg = dg[:, None] * Rg
    lead_err = float(np.linalg.norm(Rg - R0) / np.linalg.norm(R0))
    return {"column_norm_rel_err": col_err, "leading_block_rel_err": lead_err}


def cpu_baseline(A_host, seconds):
    """The oracle (plain FP64 Householder QR, C, OpenMP over the trailing
    columns) on the leading columns of the same matrix: a 512-column run sets
    the rate, then the widest power-of-two column count whose predicted time
    stays within `seconds` is timed."""
    import numpy as np
    import oracle

    m = A_host.shape[0]
    threads = oracle.num_threads(omp=True)

    def run(cols, omp=True):
        sample = np.asfortranarray(A_host[:, :cols])
        t0 = time.perf_counter()
        oracle.geqr2(sample, omp=omp)
        return time.perf_counter() - t0

    def std(cols):
        return 2.0 * cols * cols * (m - cols / 3.0)

    def widest(first, budget, omp):
        rate = std(first) / run(first, omp)
        cols = first
        while cols * 2 <= A_host.shape[1] and std(cols * 2) / rate <= budget:
            cols *= 2
        return cols, run(cols, omp)

    cols, dt = widest(512, seconds, True)
    # the single-threaded build of the same oracle, on a sample half as long
    cols1, dt1 = widest(128, seconds / 2, False)
    return {"value": round(std(cols) / dt / 1e9, 3), "unit": "Gflop/s", "cores": threads, "kind": "oracle",
            "sample": f"unblocked Householder QR (OpenMP over the trailing columns) of the leading {m}x{cols} "
                      f"columns of the same 8192x8192 input, standard count 2n^2(m-n/3); {dt:.1f} s",
            "single_thread": {"value": round(std(cols1) / dt1 / 1e9, 3), "unit": "Gflop/s", "cores": 1,
                              "sample": f"the same oracle built without OpenMP, leading {m}x{cols1} columns; "
                                        f"{dt1:.1f} s"}}


def serving_leg(count: int, pool_size: int = 96):
    """The serving loop on the least-squares request stream (m log-uniform in
    [256, 8192], n uniform in [m/8, m], 1-4 right-hand sides, cond
    log-uniform in [1e1, 1e6], Poisson arrivals), answered by the mixed
    solver (FP32-update factor + FP64 CGLS): `count` requests at the target
    rate 2000 req/s, which saturates one GPU (throughput and queueing
    latency), and a third as many at 100 req/s (below saturation); the FP64
    solver on the 2000 req/s stream beside it.  The requests' matrices come
    from a pool of `pool_size` generated requests (arrival i carries pool
    entry i mod pool_size), so that a thousand requests need neither a
    thousand host generations nor their pinned memory.  Host data pinned
    before the clock starts; copies in and out timed."""
    from paper_0707_3548_amd import serving, workloads

    out = {"workload": f"least-squares requests, m log-uniform [256, 8192], n uniform [m/8, m], 1-4 RHS, "
                       f"cond log-uniform [1e1, 1e6], Poisson arrivals, matrices from a pool of {pool_size}; "
                       "FP64 answers from the mixed solver (FP32-update factor + FP64 CGLS, accepted at a "
                       "backward-error estimate <= 1e-14) or the FP64 solver, 8 streams, admission by HBM footprint"}
    pool_spec = workloads.arrivals(rate=1.0, count=pool_size, seed=5)
    pool = [workloads.ls_request(r["m"], r["n"], r["nrhs"], r["cond"], r["seed"])[:2] for r in pool_spec]
    for name, solver, rate, cnt, seed in (("mixed_offered_2000_per_s", "mixed", 2000.0, count, 3),
                                          ("mixed_offered_100_per_s", "mixed", 100.0, max(1, count // 3), 4),
                                          ("fp64_offered_2000_per_s", "fp64", 2000.0, count, 3)):
        arr = workloads.arrivals(rate=rate, count=cnt, seed=seed)
        ex = serving.GpuExecutor(slots=8, solver=solver)
        prepared = {}
        reqs = []
        for i, r in enumerate(arr):
            k = i % pool_size
            A, b = pool[k]
            if k not in prepared:
                prepared[k] = ex.prepare(serving.Request(-1, 0.0, A.shape[0], A.shape[1], b.shape[1]), A, b)
            proto = prepared[k]
            reqs.append(serving.Request(i, r["t"], proto.m, proto.n, proto.nrhs, proto.footprint,
                                        ex.payload_copy(proto.payload)))
        sch = serving.Scheduler(8, 64 << 30, ex.launch, ex.poll)
        done = sch.run(reqs)
        st = serving.latency_stats(done)
        span = max(c.t_done for c in done) - min(c.t_arrive for c in done)
        st["gflop_per_s"] = sum(2.0 * r.n * r.n * (r.m - r.n / 3.0) for r in reqs) / span / 1e9
        bad = sum(not c.result["ok"] for c in done)
        row = {k: round(v, 3) for k, v in st.items()} | {"offered_per_s": rate, "peak_in_flight": sch.peak_inflight,
                                                        "peak_hbm_gb": round(sch.peak_bytes / 1e9, 3), "failed": bad}
        if solver == "mixed":
            its = [r["iterations"] for c in done for r in (c.result["refine"] or [])]
            row["cgls_iterations_mean"] = round(float(sum(its)) / max(1, len(its)), 2)
            row["cgls_iterations_max"] = max(its) if its else 0
        out[name] = row
        print(f"bench: serving {solver} {cnt} requests at {rate:g} req/s: p50 {st['p50_ms']:.1f} ms, "
              f"p99 {st['p99_ms']:.1f} ms, {st['solves_per_s']:.1f} solves/s, {bad} failed", file=sys.stderr,
              flush=True)
    return out


def mixed_legs(A_host, b: int, ib: int, fp64_ms: float, steps: int = 5):
    """The FP32 precision tier: (1) the same 8192x8192 factorisation with the
    trailing updates on the FP32 matrix cores (FP64 panels), timed like the
    headline, and with BF16 operands; (2) least squares 16384x4096 at cond
    1e2, 1e5 and 1e8, solved in FP64 and mixed (FP32-, BF16- or FP64-update
    factor + FP64 CGLS),
    inputs in HBM: times, iterations, the device's backward-error estimate,
    and the relative difference from the FP64 solution."""
    import numpy as np
    import torch
    from paper_0707_3548_amd import tqr, workloads

    out = {}
    m, n = A_host.shape
    src = tqr.fortran(torch.from_numpy(A_host).cuda())
    ws = tqr.Workspace(m, n, 0, b, ib)
    copies = [src.clone() for _ in range(2)]
    fl = 2.0 * n * n * (m - n / 3.0)
    for name, prec, what in (("fp32_updates_factor", tqr.PRECISION_FP32_UPDATES, "on FP32 MFMA"),
                             ("bf16_updates_factor", tqr.PRECISION_BF16_UPDATES, "on BF16 MFMA with FP32 accumulation")):
        ts = []
        for s in range(steps + 2):
            dA = copies[s % 2]
            dA.copy_(src)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            tqr.factor(dA, b, ib, ws, precision=prec, policy=tqr.POLICY_COLUMN)
            e1.record()
            torch.cuda.synchronize()
            if s >= 2:
                ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[len(ts) // 2]
        out[name] = {"workload": f"{m}x{n} N(0,1), tile_b={b}, inner_ib={ib}, LARFB/SSRFB {what}, "
                                 "GEQRT/TSQRT in FP64", "ms_per_step": round(ms, 3),
                     "gflops_standard": round(fl / ms / 1e6, 1), "speedup_vs_fp64": round(fp64_ms / ms, 3)}
    ms = out["fp32_updates_factor"]["ms_per_step"]
    del copies, ws, src
    torch.cuda.empty_cache()

    # least squares 16384 x 4096 (A = U diag(s) V^T, U and V from QR of
    # Gaussians, s log-spaced; b = A x + 1e-6 N(0,1)) per condition number:
    # the FP64 solve (factor, Q^T b, back substitution) against the mixed
    # solve (FP32-update factor + FP64 CGLS on A R^{-1}, stopping on the
    # device), and the mixed solve with the FP64 factor where cond exceeds
    # 1 / u32 (the FP32 factor stalls there and says so in its statistics)
    lm, ln = 16384, 4096
    work = torch.empty(int(tqr.lib().tqr_ls_mixed_workspace_bytes(lm, ln, 1, 256)), dtype=torch.uint8, device="cuda")
    ws64 = tqr.Workspace(lm, ln, 1, 256, 16)

    def time_it(fn, reps=3):
        t = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            fn(e0, e1)
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return sorted(t[1:])[len(t[1:]) // 2]

    ls = {"workload": f"{lm}x{ln} least squares, A = U diag(s) V^T (U, V from QR of Gaussians, s log-spaced), "
                      "one right-hand side b = A x + 1e-6 N(0,1); FP64 solve vs FP32-, BF16- or FP64-update factor "
                      "+ FP64 CGLS (at most 20 iterations, device stopping test)"}
    for cond in (1e2, 1e5, 1e8):
        Ah, Bh, _ = workloads.ls_problem(lm, ln, cond, seed=41, nrhs=1)
        dA0 = tqr.fortran(torch.from_numpy(Ah).cuda())
        dB0 = tqr.fortran(torch.from_numpy(Bh).cuda())
        del Ah

        def run64(e0, e1):
            dA, dB = dA0.clone(), dB0.clone()
            e0.record()
            tqr.solve_ls(dA, dB, 256, 16, ws64)
            e1.record()
            run64.X = dB

        def runmx(e0, e1, prec):
            e0.record()
            X, _, info, stats = tqr.solve_ls_mixed(dA0, dB0, 256, iterations=20, work=work, precision=prec)
            e1.record()
            runmx.X, runmx.info, runmx.stats = X, info, stats

        t64 = time_it(run64)
        x64 = run64.X[:ln].cpu().numpy()
        row = {"fp64_ms": round(t64, 3)}
        for name, prec in (("fp32_factor", tqr.PRECISION_FP32_UPDATES), ("bf16_factor", tqr.PRECISION_BF16_UPDATES),
                           ("fp64_factor", tqr.PRECISION_FP64)):
            tmx = time_it(lambda e0, e1: runmx(e0, e1, prec))
            st = tqr.refine_stats(runmx.stats)[0]
            xmx = runmx.X.cpu().numpy()
            row[name] = {"ms": round(tmx, 3), "speedup_vs_fp64": round(t64 / tmx, 3), "iterations": st["iterations"],
                         "stop": {1: "converged", 2: "stagnated", 3: "iteration limit", 4: "breakdown"}.get(st["stop"], st["stop"]),
                         "eta_estimate": st["eta"],
                         "rel_diff_vs_fp64_solution": float(np.linalg.norm(xmx - x64) / np.linalg.norm(x64)),
                         "info": int(runmx.info.item())}
        ls[f"cond_{cond:g}"] = row
        print(f"bench: LS cond {cond:g}: fp64 {t64:.2f} ms, mixed fp32 {row['fp32_factor']['ms']:.2f} ms "
              f"({row['fp32_factor']['iterations']} it, {row['fp32_factor']['stop']}, eta {row['fp32_factor']['eta_estimate']:.2e}), "
              f"mixed fp64-factor {row['fp64_factor']['ms']:.2f} ms", file=sys.stderr, flush=True)
        del dA0, dB0
        torch.cuda.empty_cache()
    out["least_squares"] = ls
    print(f"bench: mixed tier: factor {ms:.2f} ms (fp64 {fp64_ms:.2f})", file=sys.stderr, flush=True)
    return out


def batched_leg(count: int, steps: int = 5):
    """The batched factorisation: ``count`` independent N(0,1) problems, m
    log-uniform in [16, 512], n uniform in [8, m], one launch per batch
    ((tile_b, inner_ib) per problem from the tuned size-bucket table), FP64
    and FP32-update variants, inputs already in HBM; timed eagerly (HIP
    events around the launch, the inputs restored by a device copy outside)
    and as a replayed graph."""
    import torch
    from paper_0707_3548_amd import autotune, tqr, workloads

    shapes = workloads.batch_shapes(count, seed=11)
    flops = sum(2.0 * n * n * (m - n / 3.0) for m, n in shapes)
    out = {"workload": f"{count} independent N(0,1) QRs, m log-uniform [16, 512], n uniform [8, m], one launch, "
                       "one workgroup per problem, (tile_b, inner_ib) per bucket of n from the autotuner",
           "problems": count, "gflop_standard": round(flops / 1e9, 2)}
    for name, prec in (("fp64", tqr.PRECISION_FP64), ("fp32_updates", tqr.PRECISION_FP32_UPDATES)):
        table = autotune.current_table("fp64" if name == "fp64" else "fp32")
        tilings = [autotune.tiling_for(n, table) for _, n in shapes]
        bt = tqr.Batch(shapes, [t[0] for t in tilings], [t[1] for t in tilings], precision=prec)
        workloads.fill_normal_device(bt.A, 12)
        pristine = bt.A.clone()

        def timed(run):
            ts = []
            for s in range(steps + 1):
                bt.A.copy_(pristine)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                run()
                e1.record()
                torch.cuda.synchronize()
                if s > 0:
                    ts.append(e0.elapsed_time(e1))
            return sorted(ts)[len(ts) // 2]

        eager_ms = timed(bt.factor)
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        bt.A.copy_(pristine)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=st):
            bt.factor()
        graph_ms = timed(g.replay)
        ok = int(bt.status.item()) == 0
        out[name] = {"tile_table": [list(e) for e in table], "ms_per_batch": round(eager_ms, 3),
                     "ms_per_batch_graph": round(graph_ms, 3), "problems_per_s": round(count / (eager_ms / 1e3), 1),
                     "gflops_standard": round(flops / eager_ms / 1e6, 1), "status_ok": ok}
        print(f"bench: batched {name} {count} problems: {eager_ms:.2f} ms eager, {graph_ms:.2f} ms graph",
              file=sys.stderr, flush=True)
        del bt, pristine, g
        torch.cuda.empty_cache()
    return out


def traffic_from_profile(per_launch_flops):
    """HBM bytes per launch of the scheduler kernel, from the committed
    rocprofv3 counter summary, if it was taken on the current kernel sources."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_hash") != kernel_source_hash():
        return None
    return prof.get("hbm_bytes_per_launch")


def counters_from_profile():
    """The matrix-core counters of the committed rocprofv3 summary, if it was
    taken on the current kernel sources."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_hash") != kernel_source_hash() or "mfma_busy_fraction" not in prof:
        return None
    return {"mfma_busy_fraction": round(prof["mfma_busy_fraction"], 4),
            "mfma_f64_flops_per_launch": prof["mfma_f64_flops_per_launch"],
            "source": "rocprofv3 SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCD x 1024 SIMDs); "
                      "SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 (profiles/factor_8192_b256.md)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the tiled QR here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0707_3548_amd import flops, tqr, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    tqr.lib()  # fail loudly when the HIP library is missing
    n, b, ib = args.n, args.tile_b, args.inner_ib
    print(f"bench: generating {n}x{n} N(0,1)", file=sys.stderr, flush=True)
    A = workloads.gaussian(n, n, seed=0)
    print("bench: timing the 8192^2 factorisation", file=sys.stderr, flush=True)
    wall_ms, kern_list, F, ws = time_factor(tqr, torch, A, b, ib, args.steps, args.warmup, args.policy)
    kern_ms = sum(kern_list) / len(kern_list)
    std = flops.standard(n, n)
    exe = flops.tiled(n, n, b, ib)
    value = std / (wall_ms * 1e-3) / 1e9
    achieved_tf = exe / (kern_ms * 1e-3) / 1e12
    print("bench: spot check", file=sys.stderr, flush=True)
    check = spot_check(torch, A, F)
    check["kappa2_input"] = round(cond2_estimate(torch, torch.triu(F[:n, :])), 1)
    del F, ws
    torch.cuda.empty_cache()

    tall = None
    if not args.no_tall:
        print("bench: tall-skinny 65536x1024", file=sys.stderr, flush=True)
        At = workloads.uniform(65536, 1024, seed=1)
        t_wall, t_kl, Ft, wst = time_factor(tqr, torch, At, b, ib, max(2, args.steps // 4), 1, args.policy)
        t_kern = sum(t_kl) / len(t_kl)
        tall = {"workload": f"tiled QR 65536x1024 U[-1,1], tile_b={b}, inner_ib={ib}",
                "ms_per_step": round(t_wall, 3), "gflops_standard": round(flops.standard(65536, 1024) / t_wall / 1e6, 1),
                "gflops_tiled_executed": round(flops.tiled(65536, 1024, b, ib) / t_kern / 1e6, 1)}
        print(f"bench: tall-skinny {t_wall:.1f} ms/step", file=sys.stderr, flush=True)
        del Ft, wst
        torch.cuda.empty_cache()

    mixed_out = None
    if not args.no_mixed:
        print("bench: mixed-precision tier", file=sys.stderr, flush=True)
        mixed_out = mixed_legs(A, b, ib, wall_ms)

    batched_out = None
    if not args.no_batched:
        print("bench: batched", file=sys.stderr, flush=True)
        batched_out = batched_leg(args.batch_count)

    serving_out = None
    if not args.no_serving:
        print("bench: serving loop", file=sys.stderr, flush=True)
        serving_out = serving_leg(args.serving_requests)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        print(f"bench: oracle on the host (about {args.cpu_seconds:.0f} s)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(A, args.cpu_seconds)

    traffic = traffic_from_profile(exe)
    line = {
        "metric": "QR Gflop/s (FP64 vs FP32/BF16+refine) at N=8192; p99 LS-solve latency",
        "value": round(value, 2),
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 tiled QR of one {n}x{n} N(0,1) matrix, tile_b={b}, inner_ib={ib}, "
                               + ("the plain tqr_factor call (persistent task-graph scheduler, default priorities: "
                                  "GEQRT > TSQRT > updates by their column's distance from the current panel, "
                                  "one worker in four serving the farthest columns first)"
                                  if args.policy == "default" else
                                  f"tqr_factor_ex with the {args.policy} priority policy"),
                   "m": n, "n": n, "tile_b": b, "inner_ib": ib},
        "rates": {"gflops_standard_2n2(m-n/3)": round(value, 2),
                  "gflops_tiled_executed": round(exe / (wall_ms * 1e-3) / 1e9, 2),
                  "gflops_4mn2-4n3/3": round(flops.bj_formula(n, n) / (wall_ms * 1e-3) / 1e9, 2),
                  "scheduler_kernel_ms": round(kern_ms, 3),
                  "scheduler_kernel_ms_median": round(sorted(kern_list)[len(kern_list) // 2], 3),
                  "scheduler_kernel_ms_min": round(min(kern_list), 3)},
        "roofline": {"bound": "mfma", "achieved": round(achieved_tf, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tf / FP64_MFMA_PEAK_TFLOPS, 4),
                     "traffic": traffic},
        "counters": counters_from_profile(),
        "cpu_baseline": cpu,
        "check": check,
        "tall_skinny": tall,
        "mixed_precision": mixed_out,
        "batched": batched_out,
        "serving": serving_out,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
