#!/usr/bin/env python3
"""Throughput of batched mixed-precision RB-PCG on one MI355X.

Workload (synthetic, seeded): 3D 7-point diffusion on a 127^3 interior grid
(N = 2,048,383), kappa constant on 2x2x2 octants with mu log-uniform in [0.1, 10]
(P = Q = 8), f = 1; reduced basis n = 40 from the GPU adaptive greedy (Alg. 4, residual
indicator) over 256 training parameters; 256 test parameters per call.  A step is
one rb_solve_batch of the 256 queries to relative residual 1e-10 (RBCG of Alg. 3,
FP32 preconditioner with six red-black Gauss-Seidel sweeps per application, FP64 CG),
its kernels timed one by one with HIP events.  value = converged mu-solves per second.
Also: the same solves replayed from a captured HIP graph (two iterations per launch, no
per-kernel events) as `graph_replay`.

Also reported: the plain path (same library and smoother, FP64 everywhere, one query per
call), the roofline of the dominant kernel (pass B of the iteration: x += alpha p,
r -= alpha A p) and of the whole solve, the differences from the FP64 oracle per
precision, and the CPU oracle on a bounded sample.
Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of the dominant kernel's code (the stencil passes and their device helpers): a
# traffic figure measured on other sources is stale
KERNEL_SOURCES = ("paper_1804_06363_amd/csrc/stencil.hip", "paper_1804_06363_amd/csrc/common.h")
TRAFFIC_FILE = "profiles/pass_b_zmarch_3d127_B256_fp32.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec, B, kernel):
    """HBM bytes per launch of pass B's kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the calibration kernels; one line per profiled tile
    choice), or None when the summary is for another configuration or kernel, or the
    kernel's sources changed since."""
    import re
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if workload != "3d127" or prec != "fp32" or B != 256 or not os.path.exists(path):
        return None
    with open(path) as f:
        lines = re.findall(r"^traffic_bytes_per_launch: (\d+) sources_sha256: ([0-9a-f]+) "
                           r"kernel: (.+)$", f.read(), re.M)
    for value, digest, name in lines:
        if digest == kernel_source_hash() and name.strip() == kernel:
            return int(value)
    return None


def pass_b_kernel(cache_path, dim, N, B, n, prec, paired=True):
    """Name of the kernel that ran pass B, from the tile choice the autotuner wrote to
    its cache file: {"arch|d<dim>|N<log2 N>|B<log2 B>|n<ceil(n/16)>|p<prec>|s<smoother>":
    [qpb_a, qpb_b, qpb_gs, proj_target, kind_a, kind_b, kind_gs, kind_pro, zn_a, zn_b,
    np_gs, nb_b], ...}; the marching pass B takes four nodes per thread (zn_b = 4) with at
    most two queries per block, else two, and stages nb_b plane buffers.  The template
    argument after the nodes per thread is the update of x: 0 every iteration; with paired
    updates 1 (none, even iterations) and 2 (two updates, odd iterations) alternate, and the
    name gives both."""
    suffix = (f"|d{dim}|N{int(N).bit_length() - 1}|B{int(B).bit_length() - 1}"
              f"|n{(n + 15) // 16}|p{ {'fp64': 0, 'fp32': 1, 'bf16': 2}[prec] }|s0")
    try:
        with open(cache_path) as f:
            tiles = [v for k, v in json.load(f).items() if k.endswith(suffix)]
    except (OSError, ValueError):
        tiles = []
    if len(tiles) != 1 or len(tiles[0]) < 6:
        return "pass B (tiles unknown)"
    t = tiles[0]
    qpb_b, kind_b = t[1], t[5]
    if dim == 3 and kind_b == 2:
        zn = 4 if len(t) >= 10 and t[9] == 4 and qpb_b <= 2 else 2
        if len(t) < 12 or t[11] not in (1, 2):
            return "pass B (tiles unknown)"
        stem, tail = f"k_zmarch<{qpb_b}, 1, double, {zn}, ", f", {t[11]}>"
    else:
        stem, tail = f"k_pass_b<{dim}, {qpb_b}, ", ">"
    return f"{stem}1{tail} / {stem}2{tail}" if paired else f"{stem}0{tail}"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="3d127")
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--B", type=int, default=0, help="queries per call (default: workload's)")
    ap.add_argument("--flexible", type=int, default=0)
    ap.add_argument("--sweeps", type=int, default=6,
                    help="red-black Gauss-Seidel sweeps per preconditioner application (the "
                         "smoother study on this workload: 1 -> 130.2, 2 -> 160.0, 3 -> 182.9, "
                         "4 -> 190.6, 5 -> 194.0, 6 -> 195.4, 8 -> 194.1 mu-solves/s)")
    ap.add_argument("--residual-copy", type=int, default=1,
                    help="keep an FP32 copy of r for the projection and the sweeps without dot "
                         "products (FP32 / BF16 preconditioner; same results, fewer bytes)")
    ap.add_argument("--paired-x", type=int, default=1,
                    help="pass B updates x every second iteration, for two iterations (same "
                         "results, fewer bytes)")
    ap.add_argument("--uneven-sweeps", type=int, default=8,
                    help="Gauss-Seidel sweeps per preconditioner application in the uneven batch "
                         "(4 -> 90.7, 6 -> 111.0, 8 -> 113.2, 10 -> 113.9 mu-solves/s)")
    ap.add_argument("--graph", type=int, default=0,
                    help="time the main steps with the iterations replayed from a captured HIP "
                         "graph (the per-kernel events then see no launches: roofline null)")
    ap.add_argument("--graph-leg", type=int, default=1,
                    help="also time the same solves replayed from a captured HIP graph")
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--greedy", default="residual", choices=["l1", "residual"])
    ap.add_argument("--snapshot-sweeps", type=int, default=1,
                    help="Gauss-Seidel sweeps per preconditioner application in the greedy's "
                         "snapshot solves")
    ap.add_argument("--uneven", type=int, default=0,
                    help="also time the uneven batch (1024 queries over four grids)")
    ap.add_argument("--uneven-only", type=int, default=0,
                    help="time only the uneven batch and print its record (for profiling)")
    ap.add_argument("--learned", type=int, default=0,
                    help="also compare the surrogate-ranked greedy with the plain greedy")
    ap.add_argument("--basis", default="",
                    help="load the basis from this file if it exists, else build and save it")
    ap.add_argument("--fem", type=int, default=0,
                    help="also run the paper's two P1 cases (Table 1) through the sparse path")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also fill and sum a buffer of this many MiB (profiler calibration)")
    ap.add_argument("--cpu-sample", type=int, default=2,
                    help="test queries the CPU oracle solves (timed, and compared with the GPU)")
    ap.add_argument("--mixed-error", type=int, default=1,
                    help="also solve the batch with the BF16 preconditioner and report every "
                         "precision's difference from the oracle on the CPU sample")
    ap.add_argument("--smoother-study", default="",
                    help="also time the batch with each smoother variant of this list "
                         "(e.g. rbgs:1,rbgs:2,rbgs_sym:1,jacobi:1; 'all' for a default set)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (the "
              "queries are independent and would be split across GPUs).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1804_06363_amd import rb
    from workloads import WORKLOADS

    if args.uneven_only:
        print(json.dumps({"uneven_batch": uneven_leg(rb, torch, args.uneven_sweeps)}), flush=True)
        return

    if args.copy_calib > 0:
        # a plain copy of known size: the profiler's byte counters are scaled by what
        # they read for this kernel
        # a fill kernel writes exactly this many bytes and a sum kernel reads them
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        s_ = float(a.sum())
        torch.cuda.synchronize()
        log(f"counter calibration: fill writes and sum reads {args.copy_calib} MiB ({s_:.0f})")
        del a
    w = WORKLOADS[args.workload]
    B = args.B or w.B
    N, Q = w.N, w.Q
    log(f"workload {w.name}: N={N} Q={Q} n={w.n} B={B} prec={args.prec}")
    # the autotuner's tile choice goes to this file, read back to name pass B's kernel
    tune_cache = os.environ.get("RB_AUTOTUNE_CACHE")
    if not tune_cache:
        import tempfile
        tune_cache = os.path.join(tempfile.mkdtemp(prefix="rb_tiles_"), "tiles.json")
        os.environ["RB_AUTOTUNE_CACHE"] = tune_cache
    ctx = rb.Context(0)
    prob = rb.Problem(ctx, w.dims, w.blocks)
    train = w.train_mu()
    t0 = time.time()
    if args.basis and os.path.exists(args.basis):
        basis = rb.Basis.load(ctx, prob, args.basis)
        log(f"basis n={basis.n} loaded from {args.basis}")
    else:
        basis, rep = rb.offline_build(ctx, prob, train, mu=train, n_max=w.n,
                                      indicator=args.greedy,
                                      snapshot_sweeps=args.snapshot_sweeps)
        log(f"offline greedy ({args.snapshot_sweeps} sweeps per snapshot preconditioner): "
            f"n={basis.n} in {time.time() - t0:.1f}s, snapshot iters "
            f"{rep['snapshot_iters'][:5]}..{rep['snapshot_iters'][-3:]}")
        if args.basis:
            basis.save(args.basis)
    test = w.test_mu(B)
    x = torch.empty((B, N), dtype=torch.float64, device="cuda:0")
    opts = rb.solve_opts(prec=args.prec, flexible=bool(args.flexible), graph=bool(args.graph),
                         sweeps=args.sweeps, residual_copy=bool(args.residual_copy),
                         paired_x=bool(args.paired_x))

    # warm-up solves autotune the batched kernels' tiles (kept in the context)
    wopts = rb.solve_opts(prec=args.prec, flexible=bool(args.flexible), graph=bool(args.graph),
                          autotune=True, sweeps=args.sweeps,
                          residual_copy=bool(args.residual_copy), paired_x=bool(args.paired_x))
    for i in range(args.warmup):
        _, st = rb.solve_batch(ctx, prob, basis, test, x=x, opts=wopts)
        log(f"warmup {i}: iters mean {st.iters.mean():.1f} max {st.iters.max()} "
            f"max rel res {st.rel_res_true.max():.2e} status {np.bincount(st.status)}")
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    iters_total = 0
    odd_total = 0  # odd iterations (k = 1, 3, ...) summed over the queries
    conv = 0
    stats = []
    step_s = []
    for i in range(args.steps):
        ts = time.perf_counter()
        _, st = rb.solve_batch(ctx, prob, basis, test, x=x, opts=opts)  # returns synchronised
        step_s.append(time.perf_counter() - ts)
        stats.append(st)
        conv += int(((st.status == rb.RB_OK) & (st.rel_res_true <= 1e-10)).sum())
        iters_total += int(st.iters.sum())
        odd_total += int((st.iters // 2).sum())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ctx.profile(False)
    prof = ctx.profile_totals()
    value = conv / elapsed
    st = stats[-1]
    log(f"timed: {args.steps} steps in {elapsed:.3f}s -> {value:.1f} mu-solves/s; "
        f"iters mean {st.iters.mean():.1f} max rel res {st.rel_res_true.max():.2e}")
    for k, (ms, n) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        log(f"  {k:14s} {ms:9.2f} ms  {n:6d} launches  {ms / max(n, 1) * 1e3:9.1f} us/launch")

    # roofline of the dominant kernel: pass B reads p, r and writes r (FP64) for every
    # active query, and the FP32 copy of r with an FP32 / BF16 preconditioner: 24 (28)
    # algorithmic bytes per DOF per active query-iteration; the update of x reads and
    # writes x, 16 more in every iteration, or with paired updates 24 more (x and the
    # previous direction read, x written) in odd iterations only: 40 (44), or 36 (40) on
    # average
    copy = bool(args.residual_copy) and args.prec != "fp64"
    paired = bool(args.paired_x)
    ms_b, n_b = prof.get("pass_b", (0.0, 0))
    bytes_b = (28.0 if copy else 24.0) * N * iters_total + \
        (24.0 * N * odd_total if paired else 16.0 * N * iters_total)
    kernel_b = pass_b_kernel(tune_cache, len(w.dims), N, B, basis.n, args.prec, paired)
    if args.graph:  # graph replays record no per-kernel events
        roofline = {"kernel": kernel_b, "bound": "hbm", "achieved": None,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}
    else:
        achieved = bytes_b / (ms_b * 1e-3) / 1e9 if ms_b > 0 else 0.0
        roofline = {"kernel": kernel_b, "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(args.workload, args.prec, B, kernel_b),
                    "bytes_per_launch": round(bytes_b / max(n_b, 1)),
                    "avg_launch_us": round(ms_b / max(n_b, 1) * 1e3, 1)}

    # whole solve against the HBM roofline: the fused three-pass model of the iteration,
    # N (64 + 2 s_y + 1.5 s_W n / B) bytes per query-iteration (x, r, p in FP64, y in
    # s_y bytes, W in s_W bytes shared by the B queries), plus 24 N per query for the
    # start and the final true residual, over the wall time of a step
    s_y = 8 if args.prec == "fp64" else 4
    s_w = {"fp64": 8, "fp32": 4, "bf16": 2}[args.prec]
    # each sweep beyond the first reads r (its FP32 copy if kept) and y and writes y:
    # N (s_r + 2 s_y) more
    s_r = 4 if copy else 8
    per_it = 64 + 2 * s_y + 1.5 * s_w * basis.n / B + (args.sweeps - 1) * (s_r + 2 * s_y)
    path_bytes = sum(float(N) * per_it * float(ss.iters.sum()) + 24.0 * N * B for ss in stats)
    path_gbs = path_bytes / elapsed / 1e9
    roofline["path_model_bytes_per_step"] = round(path_bytes / args.steps)
    roofline["path_achieved"] = round(path_gbs, 1)
    roofline["path_frac"] = round(path_gbs / HBM_PEAK_GBS, 4)
    log(f"whole solve: {path_bytes / args.steps / 1e9:.1f} GB of model traffic per step, "
        f"{path_gbs:.0f} GB/s = {path_gbs / HBM_PEAK_GBS:.3f} of the HBM peak")

    # the same solves with the iterations replayed from a captured HIP graph
    graph_leg = None
    if args.graph_leg and not args.graph:
        gopts = rb.solve_opts(prec=args.prec, flexible=bool(args.flexible), graph=True,
                              sweeps=args.sweeps, residual_copy=bool(args.residual_copy),
                              paired_x=bool(args.paired_x))
        rb.solve_batch(ctx, prob, basis, test, x=x, opts=gopts)  # capture
        torch.cuda.synchronize()
        tg = time.perf_counter()
        gconv = 0
        for i in range(args.steps):
            _, gs = rb.solve_batch(ctx, prob, basis, test, x=x, opts=gopts)
            gconv += int(((gs.status == rb.RB_OK) & (gs.rel_res_true <= 1e-10)).sum())
        torch.cuda.synchronize()
        gel = time.perf_counter() - tg
        graph_leg = {"value": round(gconv / gel, 2), "unit": "mu-solves/s",
                     "ms_per_step": round(gel / args.steps * 1e3, 2),
                     "iters_mean": round(float(gs.iters.mean()), 2)}
        log(f"graph replay: {args.steps} steps in {gel:.3f}s -> {gconv / gel:.1f} mu-solves/s")

    # plain path: FP64 everywhere, one query per call, sequential
    plain = None
    x_plain = {}
    if args.plain_sample > 0:
        S = min(args.plain_sample, B)
        popts = rb.solve_opts(prec="fp64", sweeps=args.sweeps)
        xs = torch.empty((1, N), dtype=torch.float64, device="cuda:0")
        rb.solve_batch(ctx, prob, basis, test[:1], x=xs, opts=popts)  # warm-up
        torch.cuda.synchronize()
        tp = time.perf_counter()
        pc = 0
        pit = []
        x_plain = {}
        for b in range(S):
            _, ps = rb.solve_batch(ctx, prob, basis, test[b:b + 1], x=xs, opts=popts)
            pc += int(((ps.status == rb.RB_OK) & (ps.rel_res_true <= 1e-10)).sum())
            pit.append(int(ps.iters[0]))
            if b < args.cpu_sample:
                x_plain[b] = xs[0].clone()
        torch.cuda.synchronize()
        pe = time.perf_counter() - tp
        plain = {"value": round(pc / pe, 2), "sample": S, "iters_mean": float(np.mean(pit))}
        log(f"plain FP64 B=1: {plain['value']} mu-solves/s over {S} queries, iters {np.mean(pit):.1f}")

    cpu = None
    oracle_error = None
    if args.cpu_baseline:
        S = min(args.cpu_sample, B)
        cpu, x_orc = cpu_baseline(basis, w, test[:S], args.sweeps)
        # difference of each precision's solutions from the oracle's FP64 RBCG on the same
        # basis: ||x - x_oracle|| / ||x_oracle|| for the sampled queries
        def errs(xg):
            return [float(np.linalg.norm(xg[b] - x_orc[b]) / np.linalg.norm(x_orc[b]))
                    for b in range(S)]
        oracle_error = {"sample": f"the first {S} test queries", args.prec: errs(x.cpu().numpy())}
        if x_plain:
            oracle_error["fp64_plain"] = errs({b: v.cpu().numpy() for b, v in x_plain.items()})
        if args.mixed_error and args.prec == "fp32":
            xb = torch.empty_like(x)
            _, sb = rb.solve_batch(ctx, prob, basis, test, x=xb,
                                   opts=rb.solve_opts(prec="bf16", flexible=bool(args.flexible),
                                                      sweeps=args.sweeps))
            oracle_error["bf16"] = errs(xb.cpu().numpy())
            oracle_error["bf16_iters_mean"] = round(float(sb.iters.mean()), 2)
            del xb
        log(f"difference from the oracle: {oracle_error}")

    extra = {}
    if args.smoother_study:
        extra["smoother_study"] = smoother_study(rb, ctx, prob, basis, test, x, args)
    for flag, name, fn in ((args.uneven, "uneven_batch",
                            lambda: uneven_leg(rb, torch, args.uneven_sweeps)),
                           (args.learned, "learned_greedy", lambda: learned_leg(rb)),
                           (args.fem, "fem_cases", lambda: fem_leg(rb, torch))):
        if flag:
            try:
                extra[name] = fn()
            except Exception as exc:  # a failed extra leg is reported, not fatal
                log(f"{name} failed: {exc}")
                extra[name] = {"error": str(exc)}

    out = {
        "metric": "mu-solves/sec to rel. residual 1e-10 (batched mixed RB-PCG)",
        "value": round(value, 2), "unit": "mu-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+" + args.prec, "data": "synthetic",
        "config": {"workload": f"{len(w.dims)}D {2 * len(w.dims) + 1}-pt diffusion "
                               f"{'x'.join(map(str, w.dims))} (N={N}), "
                               f"{'x'.join(map(str, w.blocks))} kappa blocks, "
                               f"n={basis.n}, B={B}, {args.prec} preconditioner",
                   "N": N, "B": B, "n": basis.n, "Q": Q, "prec": args.prec,
                   "beta": "flexible" if args.flexible else "literal",
                   "smoother": f"red-black Gauss-Seidel x{args.sweeps}",
                   "residual_copy": copy, "paired_x_update": paired,
                   "graph": bool(args.graph), "parallelism": "single-gpu"},
        "step_ms": [round(v * 1e3, 2) for v in step_s],
        "median_step_ms": round(float(np.median(step_s)) * 1e3, 2),
        "iters_mean": round(float(st.iters.mean()), 2), "iters_max": int(st.iters.max()),
        "max_rel_res": float(st.rel_res_true.max()), "converged": conv,
        "plain_fp64_b1": plain,
        "speedup_vs_plain": round(value / plain["value"], 2) if plain and plain["value"] else None,
        "roofline": roofline, "cpu_baseline": cpu, "oracle_error": oracle_error,
        "graph_replay": graph_leg,
        "kernel_ms": {k: round(v[0], 3) for k, v in prof.items()},
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


def uneven_leg(rb, torch, sweeps=8):
    """1024 queries mixing 2D 63^2, 255^2, 1023^2 (4x4 kappa blocks) and 3D 63^3 (2x2x2),
    mu log-uniform in [0.01, 100], per-query basis sizes n in {10, 20, 40, 60} (leading
    columns of one n = 60 basis per grid), FP32 preconditioner, one rb_solve_multi call.
    Target true relative residual 1e-10, 1e-9 on 1023^2 (the FP64 rounding floor of that
    grid's residual is about 1e-10)."""
    from workloads import UNEVEN_GRIDS, uneven_batch
    ctx = rb.Context(0)
    probs, bases = [], []
    t0 = time.time()
    for wk in UNEVEN_GRIDS:
        pr = rb.Problem(ctx, wk.dims, wk.blocks)
        tr = wk.train_mu()
        # the first snapshot is smoother-only PCG (W_0 empty): on 1023^2 with a kappa
        # contrast of 1e4 it needs far more than the default 5000 iterations
        b, _ = rb.offline_build(ctx, pr, tr, mu=tr, n_max=60, indicator="l1",
                                snapshot_maxit=100000, snapshot_rtol=wk.rtol)
        probs.append(pr)
        bases.append(b)
    log(f"uneven: four bases in {time.time() - t0:.1f}s")
    qs = uneven_batch()
    xs = [torch.empty(UNEVEN_GRIDS[g].N, dtype=torch.float64, device="cuda:0") for g, _, _ in qs]
    queries = [(g, nu, mu, None, x, UNEVEN_GRIDS[g].rtol) for (g, nu, mu), x in zip(qs, xs)]
    tol = np.array([UNEVEN_GRIDS[g].rtol for g, _, _ in qs])
    # small bases on the 1023^2 grid need up to ~7500 iterations; a query whose FP64
    # rounding level lies above its tolerance is accepted there (at_floor, counted apart)
    opts = rb.solve_opts(prec="fp32", flexible=True, graph=True, maxit=10000, floor_factor=16.0,
                         sweeps=sweeps)
    rb.solve_multi(ctx, probs, bases, queries, opts=opts)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = rb.solve_multi(ctx, probs, bases, queries, opts=opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    # a query counts only if its true residual meets its tolerance; queries the rounding-
    # level test accepted above it are reported apart, not counted
    good = (st.status == rb.RB_OK) & (st.rel_res_true <= tol)
    ok = int(good.sum())
    at_floor = int(((st.status == rb.RB_OK) & (st.rel_res_true > tol)).sum())
    gidx = np.array([g for g, _, _ in qs])
    nidx = np.array([nu for _, nu, _ in qs])
    groups = {}
    for g, wk in enumerate(UNEVEN_GRIDS):
        for nu in sorted(set(nidx.tolist())):
            m = (gidx == g) & (nidx == nu)
            if m.any():
                groups[f"{wk.name}/n{nu}"] = {"queries": int(m.sum()), "converged": int(good[m].sum()),
                                             "iters_mean": round(float(st.iters[m].mean()), 1),
                                             "iters_max": int(st.iters[m].max())}
                log(f"uneven {wk.name} n={nu}: {int(m.sum())} queries, {int(good[m].sum())} "
                    f"converged, iters mean {st.iters[m].mean():.1f} max {st.iters[m].max()}, "
                    f"status {np.bincount(st.status[m], minlength=6).tolist()}")
    log(f"uneven: {len(qs)} queries in {el:.3f}s -> {ok / el:.1f} mu-solves/s "
        f"({at_floor} accepted at the FP64 rounding level above their tolerance, not "
        f"counted), iters mean {st.iters.mean():.1f}, max rel res {st.rel_res_true.max():.2e}")
    return {"value": round(ok / el, 2), "unit": "mu-solves/s", "queries": len(qs),
            "sweeps": sweeps,
            "converged": ok, "accepted_above_tolerance": at_floor, "seconds": round(el, 4),
            "iters_mean": round(float(st.iters.mean()), 2),
            "max_rel_res_over_rtol": float((st.rel_res_true / tol).max()), "groups": groups}


def learned_leg(rb):
    """Adaptive greedy on 3D 63^3 (P = 8, M = 1e4 training parameters log-uniform in
    [0.1, 10]) to n = 60 with the plain residual sweep vs the MLP-ranked sweep; the
    final bases are compared on 1000 held-out parameters by the largest residual
    indicator, computed with the library's own FP64 path (one RBCG-free evaluation:
    x_hat = W a(mu), residual by rb_apply_batch)."""
    import torch
    from workloads import WORKLOADS
    w = WORKLOADS["3d63"]
    ctx = rb.Context(0)
    prob = rb.Problem(ctx, w.dims, w.blocks)
    train = w.train_mu()
    held = w.test_mu(1000)
    res = {}
    for name, kw in (("plain", {}), ("surrogate", dict(use_surrogate=1, topk=256, explore=64,
                                                      warmup_full_sweeps=4, full_sweep_every=10,
                                                      train_steps=50, lr=1e-3, mu_lo=0.1,
                                                      mu_hi=10.0, seed=1004))):
        basis, rep = rb.offline_build(ctx, prob, train, mu=train, n_max=w.n,
                                      indicator="residual", **kw)
        Wn, AN, fN = basis.info()
        worst = held_out_eta(rb, ctx, prob, Wn, AN, fN, held, torch)
        res[name] = {"seconds": round(rep["seconds"], 3), "true_evals": rep["true_evals"],
                     "full_sweeps": rep["full_sweeps"], "fallbacks": rep["surrogate_fallbacks"],
                     "held_out_max_eta": worst}
        log(f"learned greedy [{name}]: {rep['seconds']:.2f}s, {rep['true_evals']} true "
            f"evaluations, held-out max eta {worst:.3e}")
    return res


def fem_leg(rb, torch, n=63):
    """The paper's P1 cases on the unit cube (n^3 interior nodes): 100 random parameters
    solved by RBCG with greedy bases of the sizes of its Sec. 5.1 (1 and 5 for case 1,
    2 and 20 for case 2) and by plain CG, all to relative residual 1e-10 in one batch."""
    from workloads import fem
    ctx = rb.Context(0)
    out = {}
    for case, sizes in ((1, (1, 5)), (2, (2, 20))):
        s = fem.build(case, n, 3)
        rp, c, v = fem.csr_arrays(s)
        prob = rb.Problem.from_csr(ctx, rp, c, v)
        prob.set_rhs(s.b_r)
        train = s.draw_mu(1000 + case, 256)
        t0 = time.time()
        basis, rep = rb.offline_build(ctx, prob, s.theta(train), phi=s.phi(train),
                                      n_max=max(sizes), indicator="l1")
        tg = time.time() - t0
        test = s.draw_mu(2000 + case, 100)
        th, ph = s.theta(test), s.phi(test)
        res = {"N": s.N, "greedy_seconds": round(tg, 2)}
        for nb in sizes:
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st = rb.solve_batch(ctx, prob, basis, th, phi=ph, n_use=np.full(100, nb, np.int32),
                                   flexible=True, maxit=20000)
            el = time.perf_counter() - t
            ok = int(((st.status == rb.RB_OK) & (st.rel_res_true <= 1e-10)).sum())
            res[f"rbcg_n{nb}"] = {"iters_min": int(st.iters.min()), "iters_max": int(st.iters.max()),
                                  "iters_mean": round(float(st.iters.mean()), 1),
                                  "converged": ok, "mu_solves_per_s": round(ok / el, 1)}
            log(f"fem case {case} N={s.N} RBCG n={nb}: iters {st.iters.min()}..{st.iters.max()} "
                f"(mean {st.iters.mean():.1f}), {ok}/100 converged, {ok / el:.1f} mu-solves/s")
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = rb.solve_batch(ctx, prob, None, th, phi=ph, solver="cg", maxit=20000)
        el = time.perf_counter() - t
        ok = int(((st.status == rb.RB_OK) & (st.rel_res_true <= 1e-10)).sum())
        res["cg"] = {"iters_min": int(st.iters.min()), "iters_max": int(st.iters.max()),
                     "iters_mean": round(float(st.iters.mean()), 1), "converged": ok,
                     "mu_solves_per_s": round(ok / el, 1)}
        log(f"fem case {case} plain CG: iters {st.iters.min()}..{st.iters.max()}, {ok}/100 "
            f"converged, {ok / el:.1f} mu-solves/s")
        out[f"case{case}"] = res
    return out


def held_out_eta(rb, ctx, prob, Wn, AN, fN, held, torch):
    """max over held-out mu of ||f - A(mu) W a(mu)|| / ||f|| (a by a dense FP64 solve of
    the n x n reduced system on the host, A(mu) applied by the library)."""
    worst = 0.0
    f = torch.ones(prob.N, dtype=torch.float64, device="cuda:0")
    Wt = torch.from_numpy(np.ascontiguousarray(Wn)).cuda()
    for i in range(0, len(held), 100):
        th = held[i:i + 100]
        a = np.stack([np.linalg.solve(np.tensordot(t, AN, axes=1), fN[0]) for t in th])
        xh = (torch.from_numpy(a).cuda() @ Wt).contiguous()
        Ax = rb.apply_batch(ctx, prob, th, xh)
        eta = torch.linalg.norm(f[None, :] - Ax, dim=1) / torch.linalg.norm(f)
        worst = max(worst, float(eta.max()))
    return worst


def smoother_study(rb, ctx, prob, basis, test, x, args):
    """The same batch with each smoother of the preconditioner (Sec. 3.3 leaves the choice
    open): forward red-black Gauss-Seidel with several sweeps per application, the
    symmetric sweep (forward then backward), damped Jacobi; mean iterations and converged
    mu-solves per second (median of three timed solves after a warm-up that autotunes)."""
    import torch
    spec = args.smoother_study
    if spec == "all":
        spec = "rbgs:1,rbgs:2,rbgs:3,rbgs:4,rbgs:6,rbgs_sym:1,rbgs_sym:2,jacobi:1"
    out = {}
    for item in spec.split(","):
        kind, m = item.split(":")
        name = f"{kind}_x{m}"
        kw = dict(smoother=kind, sweeps=int(m))
        o = rb.solve_opts(prec=args.prec, flexible=bool(args.flexible), **kw)
        ow = rb.solve_opts(prec=args.prec, flexible=bool(args.flexible), autotune=True, **kw)
        _, st = rb.solve_batch(ctx, prob, basis, test, x=x, opts=ow)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st = rb.solve_batch(ctx, prob, basis, test, x=x, opts=o)
            times.append(time.perf_counter() - t)
        ok = int(((st.status == rb.RB_OK) & (st.rel_res_true <= 1e-10)).sum())
        el = float(np.median(times))
        out[name] = {"iters_mean": round(float(st.iters.mean()), 2), "iters_max": int(st.iters.max()),
                     "converged": ok, "mu_solves_per_s": round(ok / el, 2),
                     "ms_per_solve": round(el * 1e3, 2)}
        log(f"smoother {name}: iters mean {st.iters.mean():.1f}, {ok} converged, "
            f"{ok / el:.1f} mu-solves/s")
    return out


def cpu_baseline(basis, w, thetas, sweeps=1):
    """The oracle's RBCG (NumPy/SciPy FP64) on a few queries of the same workload."""
    from oracle import rb as orb
    from oracle.operator import BlockDiffusion
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = 1
    log("cpu baseline: building the oracle operator and its reduced operators")
    op = BlockDiffusion(w.dims, w.blocks)
    Wn, _, _ = basis.info()
    W = np.ascontiguousarray(Wn.T)
    del Wn
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)   # offline: not timed
    t = time.perf_counter()
    its, ok, xs = [], 0, []
    for th in thetas:
        res = orb.solve_rbcg(op, th, W, AN, rtol=1e-10, sweeps=sweeps)
        its.append(res.iters)
        xs.append(res.x)
        ok += int(res.converged and res.rel_res_true <= 1e-10)
    el = time.perf_counter() - t
    log(f"cpu baseline: {len(thetas)} solves in {el:.1f}s, iters {its}")
    # the same oracle on one core (BLAS limited to one thread), first query only
    one = None
    try:
        from threadpoolctl import threadpool_limits
        # the whole sample when the grid is small, else the first query
        n1 = len(thetas) if w.N < 100000 else 1
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            ok1 = 0
            for th in thetas[:n1]:
                r1 = orb.solve_rbcg(op, th, W, AN, rtol=1e-10, sweeps=sweeps)
                ok1 += int(r1.converged and r1.rel_res_true <= 1e-10)
            el1 = time.perf_counter() - t1
        one = {"value": round(ok1 / el1, 5), "cores": 1,
               "sample": f"the first {n1} test queries"}
        log(f"cpu baseline, one core: {n1} solves in {el1:.1f}s")
    except ImportError:
        pass
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(ok / el, 5), "unit": "mu-solves/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model, "host_cpus": os.cpu_count(),
            "sample": f"the first {len(thetas)} test queries of the same workload and basis "
                      "(operator setup excluded; reduced assembly, Cholesky, RBCG iterations "
                      "and true residual timed)",
            "iters": its, "one_core": one}, xs


if __name__ == "__main__":
    main()
