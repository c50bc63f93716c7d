#!/usr/bin/env python3
"""Benchmark of the over-decomposed Jacobi sweep on one MI355X.

Workload (one "step" = one whole solve, every step of the hot path):
  2D 5-point Poisson Jacobi, 8192^2 interior, FP32 state and source, FP64
  residual; source = sum of 16 Gaussians (seeded); zero Dirichlet ring; u_0 = 0;
  over-decomposed into 16 x 16 blocks of 512^2 with one-cell halos;
  1000 sweeps with the residual taken every 50 sweeps (and at 0).
  Per step: scale the source into the blocks, scatter the initial state into
  the blocks, 1000 sweeps (halo reads fused into the pass kernel, an explicit
  halo exchange after each 50-sweep interval), 21 FP64 residuals, gather the
  final state.  Inputs are resident in HBM before timing starts.

Output: one JSON line (see the fields below).  `value` is GLUP/s (10^9 interior
cell updates per second) of the whole step.  `roofline` describes the dominant
kernel (the sweep pass kernel), timed live with HIP events on its own stream;
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Jacobi GLUP/s + HBM GB/s (% peak); adjoint/batched vs plain at 1e-5 rel err"
N = 8192
BLOCKS = (16, 16)
SWEEPS = 1000
CHECK_EVERY = 50
HBM_PEAK_GBS = 8000.0
# FP32 vector ALU peak without packed or fused instructions:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T ops/s
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
FLOPS_PER_UPDATE = 5  # (W+E), (S+N), their sum, +b: 4 adds; *w: 1 mul
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep2d_march_poisson8192.json")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2303_02543_amd", "csrc", "k_march2d.hip")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--depth", type=int, default=0,
                    help="temporal depth (0 = the library's default schedule)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the autotuner's schedule instead of the library default")
    ap.add_argument("--rows", type=int, default=0, help="rows per tile (with --depth)")
    ap.add_argument("--flags", type=int, default=0,
                    help="schedule flags with --depth (2 = non-temporal stores)")
    ap.add_argument("--explicit-halo", action="store_true",
                    help="exchange halos and sweep block-locally every sweep (depth 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--cpu-full-seconds", type=float, default=45.0,
                    help="run the whole workload on the oracle (and report the GPU result's "
                         "error against it) when it is estimated to take at most this long")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and adjoint measurements")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB mebibytes (a "
                         "known-size kernel for calibrating HBM byte counters) and exit")
    return ap.parse_args()


def copy_probe(mib):
    """Five plain copies of `mib` MiB (torch's copy kernel): each reads and
    writes exactly mib MiB, the reference for FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "bytes_read_per_copy": n * 4,
                      "bytes_written_per_copy": n * 4, "copies": 5}), flush=True)


def bench_batched(plain_glups):
    """64 independent 2D Poisson grids, sides uniform on [257, 4097]
    (default_rng(4)), per-grid 16-Gaussian sources (default_rng(4000+g)), FP32
    with FP64 residual, stop at relative residual 1e-6 or 5000 sweeps, residual
    every 50; one launch per pass over all active grids, check intervals
    replayed as hipGraphs, autotuned depth and tile height."""
    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic
    dev = torch.device("cuda:0")
    sizes = [int(n) for n in synthetic.batched_sizes()]
    srcs = [torch.from_numpy(synthetic.batched_source(n, g).astype(np.float32)).to(dev)
            for g, n in enumerate(sizes)]
    zeros = [torch.zeros((n + 2, n + 2), dtype=torch.float32, device=dev) for n in sizes]
    B = jb.Batch([(n, n) for n in sizes], torch.float32, block=512, device=dev)
    try:
        depth, rows = B.autotune(50)
        B.set_tuning(depth, rows, True)

        def solve():
            for g, n in enumerate(sizes):
                B.set_grid(g, zeros[g], srcs[g], synthetic.spacing2(n))
            return B.solve(1e-6, 5000, 50)

        solve()  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sw, rl, st = solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        B.close()
    updates = float(sum(n * n * k for n, k in zip(sizes, sw)))
    glups = updates / dt / 1e9
    counts = {}
    for v in st:
        counts[jb.STATUS_NAMES[v]] = counts.get(jb.STATUS_NAMES[v], 0) + 1
    return {
        "workload": "64 independent 2D 5-point Poisson grids, sides U{257..4097}, FP32, FP64 "
                    "residual every 50, stop at rel 1e-6 or 5000 sweeps",
        "grids": len(sizes), "sum_n2": int(sum(n * n for n in sizes)),
        "cell_updates": updates, "seconds": round(dt, 4), "glups": round(glups, 3),
        "ratio_vs_plain": round(glups / plain_glups, 4), "t_depth": depth, "rows": rows,
        "graph": True, "status_counts": counts,
        "rel_min": min(rl), "rel_max": max(rl),
    }


def bench_adjoint(plain_glups):
    """Adjoint: L = 1/2 ||u_K - t||^2 on 4096^2 FP32 2D Poisson, K = 500,
    checkpoint interval C = 50, gradients w.r.t. the source and the boundary
    values through JacobiK (forward sweeps, then the hand-written adjoint
    passes with FP64 accumulation)."""
    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic
    from paper_2303_02543_amd.autograd import JacobiK
    dev = torch.device("cuda:0")
    n, K, C = 4096, 500, 50
    U0, f, t = synthetic.adjoint_gaussians(n)
    h2 = synthetic.spacing2(n)
    U0d = torch.from_numpy(U0.astype(np.float32)).to(dev)
    fd = torch.from_numpy(f.astype(np.float32)).to(dev)
    td = torch.from_numpy(t.astype(np.float32)).to(dev)
    s = jb.Solver((n, n), (8, 8), torch.float32, device=dev)
    try:
        def run():
            fT = fd.clone().requires_grad_(True)
            UT = U0d.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uK = JacobiK.apply(fT, UT, s, K, h2, C)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss = 0.5 * ((uK[1:-1, 1:-1] - td) ** 2).sum()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            return t1 - t0, t2 - t1, float(loss)
        run()
        fwd, bwd, L = run()
    finally:
        s.close()
    cells = float(n) * n
    return {
        "workload": "adjoint of 1/2||u_K - t||^2, 4096^2 FP32 2D Poisson, K=500, C=50",
        "forward_ms": round(fwd * 1e3, 3), "backward_ms": round(bwd * 1e3, 3),
        "fwd_plus_bwd_over_fwd": round((fwd + bwd) / fwd, 4),
        "forward_glups": round(cells * K / fwd / 1e9, 3),
        "adjoint_glups": round(cells * K / bwd / 1e9, 3),
        "adjoint_ratio_vs_plain": round(cells * K / bwd / 1e9 / plain_glups, 4),
        "loss": L,
    }


def bench_poisson3d(plain_glups):
    """3D 7-point Poisson 512^3, f ~ U[-1,1) (default_rng(3)), zero ring, u_0 = 0,
    8x8x8 blocks of 64^3, 200 sweeps, residual every 20; FP32 and FP64."""
    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic
    dev = torch.device("cuda:0")
    n, K, R = 512, 200, 20
    U0, f = synthetic.poisson3d_uniform(n)
    h2 = synthetic.spacing2(n)
    out = {"workload": "3D 7-point Poisson 512^3, 8x8x8 blocks of 64^3, 200 sweeps, residual "
                       "every 20"}
    for name, np_dt, t_dt in (("f32", np.float32, torch.float32), ("f64", np.float64, torch.float64)):
        fd = torch.from_numpy(f.astype(np_dt)).to(dev)
        Ud = torch.from_numpy(U0.astype(np_dt)).to(dev)
        s = jb.Solver((n, n, n), (8, 8, 8), t_dt, device=dev)
        try:
            s.autotune(R, with_source=True)
            res = torch.empty(jb.residual_count(K, R), dtype=torch.float64, device=dev)

            def step():
                s.set_source(fd, h2)
                s.set_state(Ud)
                s.solve(K, R, res)
            step()
            torch.cuda.synchronize()
            s.profile(True)
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            p = s.profile_read(0)
            s.profile(False)
            tuning = s.get_tuning()
        finally:
            s.close()
        es = 4 if name == "f32" else 8
        kms = p["ms"] / max(p["launches"], 1)
        d3, z3, f3 = tuning
        out[name] = {"glups": round(float(n) ** 3 * K / dt / 1e9, 3),
                     "zseg": z3, "flags": f3,
                     "pass_kernel_avg_ms": round(kms, 5),
                     "pass_kernel_hbm_gbs_alg": round(3 * es * float(n) ** 3 / (kms * 1e-3) / 1e9, 1),
                     "ratio_vs_plain_2d": round(float(n) ** 3 * K / dt / 1e9 / plain_glups, 4)}
        del fd, Ud
    return out


def bench_plain2d():
    """Plain sweeps (one sweep per kernel) of the 8192^2 Poisson grid in 16x16
    blocks: the block-local sweep after an explicit halo exchange (the step
    order of the paper's proxy) and the fused pass at depth 1 (halo cells read
    from their owning blocks), FP32 and FP64.  HBM figures are algorithmic
    bytes (state read + source read + state write per cell) over the sweep
    kernel's own time (HIP events on the solver's stream)."""
    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic
    dev = torch.device("cuda:0")
    n, K = N, 50
    f64 = synthetic.gaussian_sum(n, 2, 2)
    h2 = synthetic.spacing2(n)
    out = {"workload": "2D 5-point Poisson %dx%d, 16x16 blocks, %d plain sweeps" % (n, n, K)}
    for name, np_dt, t_dt in (("f32", np.float32, torch.float32), ("f64", np.float64, torch.float64)):
        es = 4 if name == "f32" else 8
        s = jb.Solver((n, n), BLOCKS, t_dt, device=dev)
        try:
            s.set_source(torch.from_numpy(f64.astype(np_dt)).to(dev), h2)
            s.set_state(torch.zeros((n + 2, n + 2), dtype=t_dt, device=dev))
            rec = {}
            for form, flags in (("explicit_halo", jb.JACOBI_FLAG_EXPLICIT_HALO), ("fused", 0)):
                s.set_tuning(1, 0, flags)
                s.sweep(K)
                torch.cuda.synchronize()
                s.profile(True)
                t0 = time.perf_counter()
                s.sweep(K)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                p = s.profile_read(0)
                s.profile(False)
                kms = p["ms"] / max(p["launches"], 1)
                gbs = 3 * es * float(n) ** 2 / (kms * 1e-3) / 1e9
                rec[form] = {"glups": round(float(n) ** 2 * K / dt / 1e9, 3),
                             "sweep_kernel_avg_ms": round(kms, 5),
                             "sweep_kernel_hbm_gbs_alg": round(gbs, 1),
                             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
            out[name] = rec
        finally:
            s.close()
    return out


def bench_overdecomposition():
    """The paper's over-decomposition analogue on one GPU: explicit-halo
    sweeps (exchange, then block-local update) of the 8192^2 FP32 Poisson
    grid in 4x4 ... 64x64 blocks, without and with the overlap of each slab's
    face sends with the next slab's sweep (JACOBI_FLAG_OVERLAP).  Whole-sweep
    GLUP/s, exchange included."""
    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic
    dev = torch.device("cuda:0")
    n, K = N, 50
    f = torch.from_numpy(synthetic.gaussian_sum(n, 2, 2).astype(np.float32)).to(dev)
    rows = []
    for nb in (4, 8, 16, 32, 64):
        s = jb.Solver((n, n), (nb, nb), torch.float32, device=dev)
        try:
            s.set_source(f, synthetic.spacing2(n))
            s.set_state(torch.zeros((n + 2, n + 2), dtype=torch.float32, device=dev))
            rec = {"blocks": [nb, nb]}
            for name, fl in (("explicit_halo", jb.JACOBI_FLAG_EXPLICIT_HALO),
                             ("overlapped", jb.JACOBI_FLAG_EXPLICIT_HALO | jb.JACOBI_FLAG_OVERLAP)):
                s.set_tuning(1, 0, fl)
                s.sweep(5)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.sweep(K)
                torch.cuda.synchronize()
                rec[name + "_glups"] = round(float(n) ** 2 * K / (time.perf_counter() - t0) / 1e9, 2)
            rows.append(rec)
        finally:
            s.close()
    return {"workload": "2D 5-point Poisson %dx%d FP32, %d explicit-halo sweeps per point" % (n, n, K),
            "points": rows}


def bench_paper_domain():
    """The paper's Jacobi3D domain (Section 4.3), 1024 x 1024 x 768, 7-point
    Poisson in 16 x 16 x 12 blocks of 64^3, a fixed number of sweeps as in the
    paper (no residual), FP32 and FP64, autotuned 3D schedule."""
    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic
    dev = torch.device("cuda:0")
    nx, ny, nz, K = 1024, 1024, 768, 40
    out = {"workload": "3D 7-point Poisson %dx%dx%d (the paper's Jacobi3D domain), 16x16x12 "
                       "blocks of 64^3, %d sweeps" % (nx, ny, nz, K)}
    tile = synthetic.uniform((48, 64, 64), 13, -1.0, 1.0)
    for name, np_dt, t_dt in (("f32", np.float32, torch.float32), ("f64", np.float64, torch.float64)):
        s = jb.Solver((nx, ny, nz), (16, 16, 12), t_dt, device=dev)
        try:
            s.autotune(10, with_source=True)
            s.set_source(torch.from_numpy(np.tile(tile.astype(np_dt), (16, 16, 16))).to(dev),
                         synthetic.spacing2(nx))
            s.set_state(torch.zeros((nz + 2, ny + 2, nx + 2), dtype=t_dt, device=dev))
            s.sweep(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.sweep(K)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            es = 4 if name == "f32" else 8
            glups = float(nx) * ny * nz * K / dt / 1e9
            d3, z3, f3 = s.get_tuning()
            out[name] = {"glups": round(glups, 2), "hbm_gbs_alg": round(glups * 3 * es, 1),
                         "zseg": z3, "flags": f3}
        finally:
            s.close()
    return out


def source_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_for(kernel_name, launches_alg_bytes):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    they are missing or were taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_hash(SWEEP_SOURCE):
        return None
    k = rec.get("kernels", {}).get(kernel_name)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(U0_np, f_np, h2, target_seconds, full_max_seconds, gpu_final):
    """Time the FP64 oracle on the host's cores.  When the whole workload
    (SWEEPS sweeps, a residual every CHECK_EVERY) is estimated to fit in
    full_max_seconds it is run in full and the GPU's final FP32 state is
    compared with it (max-abs error and max-abs error / max-abs value over the
    interior); otherwise a bounded sample of sweeps on the full grid is timed."""
    import numpy as np
    import oracle
    U = U0_np.astype(np.float64)
    b = oracle.scale_source(f_np.astype(np.float64), h2, np.float64)
    oracle.sweep(U, b, 1)  # untimed: thread start-up, first touch of the arrays
    # per-sweep time from two run lengths (each call also copies the grid)
    t0 = time.perf_counter()
    oracle.sweep(U, b, 2)
    t2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.sweep(U, b, 12)
    per_sweep = max((time.perf_counter() - t0 - t2) / 10, 1e-6)
    cells = float(N) * N
    out = {"unit": "GLUP/s", "cores": oracle.num_threads(), "kind": "oracle"}
    if per_sweep * SWEEPS <= full_max_seconds:
        t0 = time.perf_counter()
        res = [oracle.residual(U, b)]
        k = 0
        while k < SWEEPS:
            step = min(CHECK_EVERY, SWEEPS - k)
            U = oracle.sweep(U, b, step)
            k += step
            res.append(oracle.residual(U, b))
        dt = time.perf_counter() - t0
        out["value"] = round(cells * SWEEPS / dt / 1e9, 4)
        out["sample"] = ("the whole workload: FP64 oracle, %dx%d, %d sweeps + %d residuals "
                         "(%.1f s)" % (N, N, SWEEPS, len(res), dt))
        gi = np.asarray(gpu_final, dtype=np.float64)[1:-1, 1:-1]
        oi = U[1:-1, 1:-1]
        err = float(np.max(np.abs(gi - oi)))
        out["error_vs_fp64_oracle"] = {
            "max_abs": err, "rel": err / float(np.max(np.abs(oi))), "bound": 1e-5,
            "oracle_final_residual": res[-1]}
        return out
    k = int(max(2, min(200, target_seconds / max(per_sweep, 1e-6))))
    t0 = time.perf_counter()
    U = oracle.sweep(U, b, k)
    r = oracle.residual(U, b)
    dt = time.perf_counter() - t0
    out["value"] = round(cells * k / dt / 1e9, 4)
    out["sample"] = ("FP64 oracle on the full %dx%d grid: %d sweeps + 1 residual (%.1f s)"
                     % (N, N, k, dt))
    out["residual_check"] = r if math.isfinite(r) else None
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the Jacobi library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2303_02543_amd as jb
    import synthetic

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")

    # inputs: drawn in FP64, rounded once to FP32, resident in HBM
    f64 = synthetic.gaussian_sum(N, 2, 2)
    f32 = f64.astype(np.float32)
    U0_np = np.zeros((N + 2, N + 2), dtype=np.float32)
    h2 = synthetic.spacing2(N)
    f_dev = torch.from_numpy(f32).to(dev)
    U0_dev = torch.from_numpy(U0_np).to(dev)
    U_out = torch.empty_like(U0_dev)
    nres = jb.residual_count(SWEEPS, CHECK_EVERY)
    res = torch.empty(nres, dtype=torch.float64, device=dev)

    s = jb.Solver((N, N), BLOCKS, torch.float32, device=dev)
    if args.explicit_halo:
        s.set_tuning(1, 0, jb.JACOBI_FLAG_EXPLICIT_HALO)
    elif args.depth > 0:
        s.set_tuning(args.depth, args.rows, args.flags)
    elif args.autotune:
        s.autotune(CHECK_EVERY, with_source=True)
    # else: the library's default schedule (measured fastest for this
    # workload; the autotuner lands within a few percent of it)
    schedule = ("explicit" if args.explicit_halo else "fixed" if args.depth > 0 else
                "autotuned" if args.autotune else "library default")
    depth, rows, flags = s.get_tuning()

    def step():
        s.set_source(f_dev, h2)            # scaled source into the blocks
        s.set_state(U0_dev)                # scatter + halo fill
        s.solve(SWEEPS, CHECK_EVERY, res)  # sweeps, halo exchange, residuals
        s.get_state(U_out)                 # gather

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    cells = float(N) * N
    glups = cells * SWEEPS / (ms_per_step * 1e-3) / 1e9

    # dominant kernel: the pass depth with the most kernel time
    tot = s.profile_read(0)
    best = None
    for d in range(1, 17):
        p = s.profile_read(d)
        if p["launches"] and (best is None or p["ms"] > best[1]["ms"]):
            best = (d, p)
    d_dom, p = best
    avg_ms = p["ms"] / p["launches"]
    bytes_per_launch = p["alg_bytes"] / p["launches"]
    flops_per_launch = FLOPS_PER_UPDATE * p["cell_updates"] / p["launches"]
    hbm_gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    alu_tops = flops_per_launch / (avg_ms * 1e-3) / 1e12
    if flags & jb.JACOBI_FLAG_EXPLICIT_HALO:
        kname = "k_sweep_local<float, true>"
    else:
        # Poisson pass kernel of depth d_dom and its prefetch distance; the
        # traffic record aggregates its two residual variants
        kname = "k_march2d<float, %d, %d, 1>" % (
            d_dom, 3 if flags & jb.JACOBI_FLAG_DEEP_PREFETCH else 1)
    traffic = traffic_for(kname, bytes_per_launch)
    hbm_frac = hbm_gbs / HBM_PEAK_GBS
    alu_frac = alu_tops / ALU_PEAK_TOPS
    if hbm_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_frac, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(alu_tops, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
    roof["traffic"] = traffic
    roof.update({
        "kernel": kname,
        "avg_launch_ms": round(avg_ms, 5),
        "launches": p["launches"],
        "alg_bytes_per_launch": bytes_per_launch,
        "alg_flops_per_launch": flops_per_launch,
        "hbm_gbs_alg": round(hbm_gbs, 1),
        "alu_tops_alg": round(alu_tops, 3),
        "kernel_share_of_step": round(tot["ms"] / (ms_per_step * args.steps), 4),
    })

    out = {
        "metric": METRIC,
        "value": round(glups, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "2D 5-point Poisson Jacobi %dx%d FP32 (FP64 residual), 16-Gaussian "
                        "source, %dx%d blocks of %dx%d, %d sweeps, residual every %d"
                        % (N, N, BLOCKS[0], BLOCKS[1], N // BLOCKS[0], N // BLOCKS[1], SWEEPS,
                           CHECK_EVERY),
            "grid": [N, N], "blocks": list(BLOCKS), "sweeps": SWEEPS,
            "check_every": CHECK_EVERY, "schedule": schedule, "t_depth": depth, "rows": rows,
            "explicit_halo": bool(flags & jb.JACOBI_FLAG_EXPLICIT_HALO),
            "nt_stores": bool(flags & jb.JACOBI_FLAG_NT_STORES),
            "deep_prefetch": bool(flags & jb.JACOBI_FLAG_DEEP_PREFETCH), "flags": flags,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "final_residual": float(res[-1].item()),
        "residual_ratio": float(res[-1].item() / res[0].item()),
    }
    s.close()
    if not args.no_forms:
        out["batched"] = bench_batched(glups)
        out["adjoint"] = bench_adjoint(glups)
        out["poisson3d"] = bench_poisson3d(glups)
        out["plain2d"] = bench_plain2d()
        out["overdecomposition"] = bench_overdecomposition()
        out["paper_domain_3d"] = bench_paper_domain()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(U0_np, f32, h2, args.cpu_seconds,
                                           args.cpu_full_seconds, U_out.cpu().numpy())
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
