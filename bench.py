"""Benchmark: APPGA solve-iterations per second on one MI355X.

Workload (default): 64 independent 128 x 128 reconstructions sharing one
200-bin x 168-angle Siddon system matrix stored in BF16 (FP32 accumulation,
FP32 iterates), per-sinogram total counts log-uniform in [1e5, 1e7] and
uniform background 5-20%, lambda1 = lambda2 = 0.02, eps = 1e-3, omega = 0.5.
One step = one APPGA iteration (forward projection + ratio, back projection +
SHOITV stencil + EM-preconditioned prox + momentum) of all 64 solves.

Printed JSON line: value = solve-iterations/s of the batched path; beside it
the plain path (the same solves run one at a time through the FP32
single-solve path), the roofline of the dominant kernel (algorithmic bytes per
launch / mean launch time from HIP events recorded by the library on the
launch stream), and the FP64 CPU oracle timed on the host cores on a bounded
sample.  Inputs are resident in device memory before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("APPGA iters/s at 128²×batch64 vs plain; projector HBM GB/s; "
          "p50/p99 recon latency")
HBM_PEAK_GBS = 8000.0
# LDS read rate of 16-byte reads per lane, conflict-free, all CUs: 209 B/clk/CU x 256 CUs x
# 2.4 GHz, as measured on MI355X (the on-chip bound of the tile projections)
LDS_PEAK_BPS = 128.4e12
KERNELS_SRC = os.path.join(ROOT, "paper_2409_13344_amd", "csrc", "kernels.hip")

# HBM traffic per launch from two rocprofv3 passes (FETCH_SIZE, then WRITE_SIZE; KiB per
# dispatch, median) of `bench.py --profile --calibrate-copy 1024` on the default workload,
# scaled by what the same counters read for a 1 GiB device copy (reads x2.00, writes
# x1.00).  The step kernel's figures are those of the APPGA leg's own launches (two
# partial sums of A^T e in), not the autotuner's.  Valid only for the kernel source it
# was taken on (sha256 prefix below).
MEASURED_TRAFFIC = {
    "kernels_sha256_16": "acf877096b0a63b4",
    "storage": "bf16",
    "read_scale": 2.0,
    "write_scale": 1.0,
    "fwd_tiles": {"fetch_kib": 46034.6, "write_kib": 8577.7},
    "back_tiles": {"fetch_kib": 28266.5, "write_kib": 8192.0},
    "step_batch": {"fetch_kib": 8610.2, "write_kib": 9216.0},
    "afppa_primal": {"fetch_kib": 21589.4, "write_kib": 13568.0},
    "afppa_dual": {"fetch_kib": 27163.6, "write_kib": 49160.0},
}


def measured_traffic(kernel: str, storage: str):
    """HBM bytes per launch of `kernel`, or None when the counters do not apply."""
    import hashlib
    with open(KERNELS_SRC, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    t = MEASURED_TRAFFIC
    if sha != t["kernels_sha256_16"] or storage != t["storage"] or kernel not in t:
        return None
    k = t[kernel]
    return int(round(1024 * (k["fetch_kib"] * t["read_scale"] + k["write_kib"] * t["write_scale"])))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="bf16", choices=["f32", "bf16", "f16", "fp8"])
    ap.add_argument("--plain-steps", type=int, default=200)
    ap.add_argument("--afppa-steps", type=int, default=200,
                    help="timed AFPPA-GN steps on the same workload (0 = skip the leg)")
    ap.add_argument("--afppa-cpu-iters", type=int, default=100)
    ap.add_argument("--c4-steps", type=int, default=50,
                    help="timed batched steps at 256^2 x 47 with the FP32 matrix (0 = skip)")
    ap.add_argument("--factored-steps", type=int, default=100,
                    help="timed APPGA steps with the factored model (PSF, attenuation, scatter/randoms)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2000)
    ap.add_argument("--profile", action="store_true",
                    help="short run for profilers: no CPU baseline, no plain path")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="serving leg: requests per rate (0 = skip)")
    ap.add_argument("--serve-rate", type=float, nargs="+", default=[200.0],
                    help="serving leg: mean Poisson arrival rates, requests/s (several = a sweep)")
    ap.add_argument("--no-projector", action="store_true",
                    help="skip the single-solve projector leg on the 256^2 geometry")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also launch a plain device copy of MIB MiB (5 times) so that a "
                         "profiler's FETCH_SIZE/WRITE_SIZE can be scaled by a known size")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def timed_pass(ap, torch, ctx, fn):
    """Kernel times of the launches inside fn() alone: the library's timers are cumulative
    per context, so the totals before the pass are subtracted."""
    before = ap.appga_kernel_times(ctx)
    ap.appga_set_kernel_timing(ctx, True)
    fn()
    torch.cuda.synchronize()
    after = ap.appga_kernel_times(ctx)
    ap.appga_set_kernel_timing(ctx, False)
    out = {}
    for k, v in after.items():
        b = before.get(k, {"total_ms": 0.0, "count": 0})
        if v["count"] > b["count"]:
            out[k] = dict(total_ms=v["total_ms"] - b["total_ms"], count=v["count"] - b["count"])
    return out


def kernel_bytes(kind: str, nnz: int, m: int, d: int, B: int, s_val: int, s_idx: int) -> int:
    """Algorithmic HBM bytes of one launch: each stored entry read once (value + index),
    row pointers once, every vector read or written once."""
    if kind == "forward":
        # matrix + row_ptr + x (d x B) + g (m x B) + e (m x B, written); scalar background
        return nnz * (s_val + s_idx) + (m + 1) * 4 + 4 * B * (d + 2 * m)
    if kind == "back":
        # transpose entries (value + slot index) + e (m x B) + A^T e (d x B, written)
        return nnz * (s_val + s_idx) + 4 * B * (m + d)
    if kind == "update":
        # A^T e + ft + f read/write + ft_next (each d x B) + Lambda
        return 4 * B * 5 * d + 4 * d
    if kind == "afppa_primal":
        # A^T e + f read/write + ft + ft_next + w (each d x B), the 6 extrapolated dual
        # components (6 d x B) read, Lambda
        return 4 * B * 12 * d + 4 * d
    if kind == "afppa_dual":
        # w (d x B) read; duals and their extrapolation (6 d x B each) read and written
        return 4 * B * 25 * d
    # fused step: transpose + row_ptr + e (m x B) + ft (d x B) + f read/write + ft_next + Lambda
    return nnz * (s_val + s_idx) + (d + 1) * 4 + 4 * B * (m + 4 * d) + 4 * d


def afppa_leg(ap, torch, ctx, mat, pr, g_t, stream, args, s_val, s_idx):
    """AFPPA-GN (Section 4.3, nonsmooth HOITV model) on the same 64 sinograms: the
    same projections plus the primal and dual kernels per step."""
    B, geom = len(pr.seeds), pr.geom
    m, d, nnz = geom.m, geom.d, pr.A.nnz
    params = [ap.make_params(lam=0.02, omega=0.5, iterations=300, momentum=ap.APPGA_MOMENTUM_GN,
                             gamma_scalar=float(pr.gamma[b][0])) for b in range(B)]
    sess = ap.appga_afppa_begin(ctx, mat, g_t, None, params, None, stream)
    for _ in range(args.warmup):
        ap.appga_solve_step(sess, 1)
    torch.cuda.synchronize()
    log("timing %d AFPPA-GN steps" % args.afppa_steps)
    t0 = time.perf_counter()
    for _ in range(args.afppa_steps):
        ap.appga_solve_step(sess, 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = timed_pass(ap, torch, ctx,
                       lambda: [ap.appga_solve_step(sess, 1) for _ in range(max(10, min(args.afppa_steps, 100)))])
    out_t = torch.empty((B, d), dtype=torch.float32, device=g_t.device)
    stats = ap.appga_solve_end(sess, out_t, B)
    kernels = {}
    for name, kind in (("fwd_tiles", "forward"), ("back_tiles", "back"), ("afppa_primal", "afppa_primal"),
                       ("afppa_dual", "afppa_dual")):
        t = times.get(name)
        if not t or t["count"] == 0:
            continue
        avg_ms = t["total_ms"] / t["count"]
        nbytes = kernel_bytes(kind, nnz, m, d, B, s_val, s_idx)
        gbs = nbytes / (avg_ms * 1e-3) / 1e9
        kernels[name] = dict(avg_us=round(1e3 * avg_ms, 2), bytes=nbytes, gbs=round(gbs, 1),
                             hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                             traffic=measured_traffic(name, args.storage))
    return dict(value=round(B * args.afppa_steps / dt, 1), unit="solve-iterations/s",
                ms_per_step=round(1e3 * dt / args.afppa_steps, 4), steps=args.afppa_steps,
                method="AFPPA-GN, omega = 1/2, beta = 1, EM preconditioner, lambda1 = lambda2 = 0.02",
                kernels=kernels, objective_lane0=stats[0]["objective"])


def factored_leg(ap, torch, ctx, args, stream):
    """APPGA on Section 4.1's physics: 64 sinograms of the 128^2 geometry (the paper's 300 mm
    field of view at half its resolution) with a Gaussian PSF of 6.59 mm (2.81 pixels), water
    attenuation and 25% scatter / 25% randoms as a per-bin background; A = diag(n) G H."""
    from paper_2409_13344_amd import synth
    geom = synth.Geometry(128, 200, 168)
    log("building the factored-model workload")
    pp = synth.make_physics_problem(geom, list(range(4000, 4064)), tc=1e6, fov_mm=300.0,
                                    G=synth.cached_matrix(geom))
    B, d, m = len(pp.seeds), geom.d, geom.m
    G = pp.G
    mat = ap.appga_load_system_matrix_factored(ctx, geom.n, geom.n_angles, geom.n_bins, G.row_ptr, G.col, G.val,
                                               args.storage, row_factors=pp.att, psf_fwhm_px=pp.fwhm_px)
    psf_R = ap.appga_matrix_psf(mat)[1]
    try:
        dev = torch.device("cuda:0")
        g_t = torch.as_tensor(pp.g).to(dev)
        gam_t = torch.as_tensor(pp.gamma).to(dev)
        params = [ap.make_params(lam=0.02, eps=1e-3, omega=0.5, iterations=300) for _ in range(B)]
        sess = ap.appga_solve_begin(ctx, mat, g_t, gam_t, params, None, stream)
        for _ in range(args.warmup):
            ap.appga_solve_step(sess, 1)
        torch.cuda.synchronize()
        log("timing %d factored-model steps" % args.factored_steps)
        t0 = time.perf_counter()
        for _ in range(args.factored_steps):
            ap.appga_solve_step(sess, 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times = timed_pass(ap, torch, ctx,
                           lambda: [ap.appga_solve_step(sess, 1) for _ in range(max(10, min(args.factored_steps, 100)))])
        out_t = torch.empty((B, d), dtype=torch.float32, device=dev)
        stats = ap.appga_solve_end(sess, out_t, B)
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    kernels = {}
    split = 2
    for name in ("psf_fwd", "fwd_tiles", "back_tiles", "psf_back", "step_batch"):
        t = times.get(name)
        if not t or t["count"] == 0:
            continue
        avg_ms = t["total_ms"] / t["count"]
        k = dict(avg_us=round(1e3 * avg_ms, 2))
        if name.startswith("psf"):
            # the blur reads its input (psf_back: the two partial back projections) and writes
            # H of it, d x B floats each
            nbytes = 4 * B * d * ((split if name == "psf_back" else 1) + 1)
            k.update(bytes=nbytes, gbs=round(nbytes / (avg_ms * 1e-3) / 1e9, 1))
        kernels[name] = k
    return dict(value=round(B * args.factored_steps / dt, 1), unit="solve-iterations/s",
                ms_per_step=round(1e3 * dt / args.factored_steps, 4), steps=args.factored_steps,
                model="A = diag(att) G H: PSF FWHM %.2f px (R = %d), water attenuation, per-bin "
                      "scatter + randoms background" % (pp.fwhm_px, psf_R),
                kernels=kernels, objective_lane0=stats[0]["objective"])


def c4_leg(ap, torch, ctx, pr, mat, steps: int):
    """Batched APPGA at C4 size: 47 lanes of the 256 x 256 / 256 bins x 252 angles geometry with
    the FP32 matrix (about 320 MB for A and its transpose, above the 256 MB Infinity Cache).  The
    lanes reuse the leg's 8 sinograms in turn (timing does not depend on the data values)."""
    geom = pr.geom
    B = 47
    idx = [b % len(pr.seeds) for b in range(B)]
    g_t = torch.as_tensor(np.ascontiguousarray(pr.g[idx])).cuda()
    params = [ap.make_params(lam=0.01, eps=1e-3, omega=1.0, iterations=1000,
                             gamma_scalar=float(pr.gamma[i][0])) for i in idx]
    s = ap.appga_solve_begin(ctx, mat, g_t, None, params, None, torch.cuda.current_stream().cuda_stream)
    for _ in range(5):
        ap.appga_solve_step(s, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ap.appga_solve_step(s, 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = timed_pass(ap, torch, ctx, lambda: [ap.appga_solve_step(s, 1) for _ in range(max(10, steps // 2))])
    ap.appga_solve_end(s, torch.empty((B, geom.d), dtype=torch.float32, device="cuda"), B)
    nnz, m, d = pr.A.nnz, geom.m, geom.d
    kernels = {}
    for name, kind in (("fwd_tiles", "forward"), ("back_tiles", "back"), ("step_batch", "update")):
        t = times.get(name)
        if not t or t["count"] == 0:
            continue
        avg_ms = t["total_ms"] / t["count"]
        nb = kernel_bytes(kind, nnz, m, d, B, 4, 2)
        gbs = nb / (avg_ms * 1e-3) / 1e9
        kernels[name] = dict(avg_us=round(1e3 * avg_ms, 2), bytes=nb, gbs=round(gbs, 1),
                             frac=round(gbs / HBM_PEAK_GBS, 4))
    return dict(value=round(B * steps / dt, 1), unit="solve-iterations/s", ms_per_step=round(1e3 * dt / steps, 4),
                steps=steps, solves=B, matrix="FP32, nnz %d" % nnz, kernels=kernels)


def cpu_baseline_afppa(pr, n_iters: int):
    """FP64 AFPPA oracle on the host cores (context for the AFPPA leg)."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16, len(pr.seeds)))
    oracle.load()

    def run(i):
        oracle.afppa(pr.A, pr.geom.n, pr.geom.n_angles, pr.g[i], pr.gamma[i], 0.02, 0.02, 0.5, n_iters)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(cores)]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    dt = time.perf_counter() - t0
    return dict(value=round(cores * n_iters / dt, 1), unit="solve-iterations/s", cores=cores,
                kind="oracle", sample="%d of the 64 sinograms x %d AFPPA-GN iterations, one solve per "
                                      "thread, FP64, %.1f s wall" % (cores, n_iters, dt))


def cpu_baseline(pr, n_iters: int):
    """FP64 oracle on the host cores: one solve per thread, the first `cores` sinograms."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16, len(pr.seeds)))
    oracle.load()
    results = [None] * cores

    def run(i):
        results[i] = oracle.appga(pr.A, pr.geom.n, pr.geom.n_angles, pr.g[i], pr.gamma[i], 0.02,
                                  0.02, 1e-3, 0.5, n_iters)["f"]

    threads = [threading.Thread(target=run, args=(i,)) for i in range(cores)]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    dt = time.perf_counter() - t0
    return dict(value=cores * n_iters / dt, unit="solve-iterations/s", cores=cores,
                kind="oracle",
                sample="%d of the 64 sinograms x %d iterations, one solve per thread, FP64, "
                       "%.1f s wall" % (cores, n_iters, dt))


def serve_leg(ap, ctx, mats, n_req: int, rate: float, seed: int):
    """Continuous batching: Poisson arrivals of requests whose sizes are uniform over the
    loaded geometries, total counts log-uniform in [1e5, 1e7] (the problems' own sinograms),
    lambda ~ U[0.005, 0.1], omega in {0.3, 0.6, 1.0}, iteration budgets ~ U{50..300}.
    Latency = completion - submission, measured by the server."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_req):
        name = sorted(mats)[int(rng.integers(0, len(mats)))]
        pr, mat = mats[name]
        b = int(rng.integers(0, len(pr.seeds)))
        p = ap.make_params(lam=float(rng.uniform(0.005, 0.1)), eps=1e-3,
                           omega=float(rng.choice([0.3, 0.6, 1.0])),
                           iterations=int(rng.integers(50, 301)))
        reqs.append((pr, mat, b, p, float(rng.exponential(1.0 / rate))))
    srv = ap.appga_server_start(ctx, 16 << 30, 64)
    tickets = []
    t0 = time.perf_counter()
    t_next = t0
    for pr, mat, b, p, gap in reqs:
        t_next += gap
        while time.perf_counter() < t_next:
            pass
        tickets.append((ap.appga_submit(srv, mat, pr.g[b], pr.gamma[b], p), pr.geom.d, p.iterations))
    lat, iters = [], 0
    for t, d, k in tickets:
        _, st = ap.appga_wait(srv, t, d, 300000)
        lat.append(st["seconds"])
        iters += k
    dt = time.perf_counter() - t0
    ap.appga_server_stop(srv)
    lat = np.asarray(lat) * 1e3
    return dict(requests=n_req, offered_rate=rate, throughput_req_s=round(n_req / dt, 1),
                solve_iterations_per_s=round(iters / dt, 1),
                p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3),
                mean_iterations=round(iters / n_req, 1))


def projector_leg(ap, torch, ctx, pr, mat, steps: int):
    """Single-solve projectors (B = 1) on the 256 x 256 / 256 bins x 252 angles geometry with
    an FP32 matrix: the matrix-streaming regime (19.7 M entries in A and in its transpose,
    FP32 values + uint16 indices, about 118 MB per operator)."""
    geom = pr.geom
    g1 = torch.as_tensor(pr.g[0]).cuda()
    gm1 = torch.as_tensor(pr.gamma[0]).cuda()
    p = [ap.make_params(lam=0.01, eps=1e-3, omega=1.0, iterations=1000)]
    s = ap.appga_solve_begin(ctx, mat, g1, gm1, p, None, torch.cuda.current_stream().cuda_stream)
    for _ in range(5):
        ap.appga_solve_step(s, 1)
    torch.cuda.synchronize()
    times = timed_pass(ap, torch, ctx, lambda: [ap.appga_solve_step(s, 1) for _ in range(steps)])
    ap.appga_solve_end(s, torch.empty((1, geom.d), dtype=torch.float32, device="cuda"), 1)
    nnz, m, d = pr.A.nnz, geom.m, geom.d
    out = {}
    for name, kind in (("forward_single", "forward"), ("step_single", "step")):
        t = times.get(name)
        if not t or t["count"] == 0:
            continue
        avg_ms = t["total_ms"] / t["count"]
        nb = kernel_bytes(kind, nnz, m, d, 1, 4, 2)
        gbs = nb / (avg_ms * 1e-3) / 1e9
        out[name] = dict(avg_us=round(1e3 * avg_ms, 2), bytes=nb, gbs=round(gbs, 1),
                         frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (independent solves "
              "would shard across GPUs with no communication); run with --gpus 1", flush=True)
        sys.exit(2)
    import torch

    from paper_2409_13344_amd import appga as ap
    from paper_2409_13344_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.init()
    dev = torch.device("cuda:0")

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 copies of %d MiB" % args.calibrate_copy)
        del src, dst

    log("building the 64-sinogram workload")
    pr = synth.config_problem("c3_128x64")
    geom, A = pr.geom, pr.A
    B = len(pr.seeds)
    m, d, nnz = geom.m, geom.d, A.nnz
    ctx = ap.appga_create(0)
    mat = ap.load_matrix(ctx, A, geom, args.storage)
    info = ap.appga_matrix_info(mat)
    tuning = ap.appga_tune(ctx, mat)   # the choice the load made (re-timed)
    gam_scalar = [float(pr.gamma[b][0]) for b in range(B)]
    params = [ap.make_params(lam=0.02, eps=1e-3, omega=0.5, iterations=300,
                             gamma_scalar=gam_scalar[b]) for b in range(B)]
    g_t = torch.as_tensor(pr.g).to(dev)
    stream = torch.cuda.current_stream().cuda_stream

    # ---------------------------------------------------------- batched ---
    sess = ap.appga_solve_begin(ctx, mat, g_t, None, params, None, stream)
    for _ in range(args.warmup):
        ap.appga_solve_step(sess, 1)
    torch.cuda.synchronize()
    log("timing %d batched steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ap.appga_solve_step(sess, 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = B * args.steps / dt
    ms_per_step = 1e3 * dt / args.steps

    # kernel durations from HIP events on the launch stream (separate pass)
    n_prof = max(10, min(args.steps, 100))
    times = timed_pass(ap, torch, ctx, lambda: [ap.appga_solve_step(sess, 1) for _ in range(n_prof)])
    out_t = torch.empty((B, d), dtype=torch.float32, device=dev)
    stats = ap.appga_solve_end(sess, out_t, B)
    s_val = {"f32": 4, "bf16": 2, "f16": 2, "fp8": 1}[args.storage]
    s_idx = 2 if max(m, d) <= 65536 else 4
    kernels = {}
    tiles = "back_tiles" in times
    tinfo = {"fwd_tiles": ap.appga_matrix_tiles(mat, ap.APPGA_TILES_FORWARD),
             "back_tiles": ap.appga_matrix_tiles(mat, ap.APPGA_TILES_BACK)}
    for name, kind in (("forward_batch", "forward"), ("fwd_tiles", "forward"), ("back_tiles", "back"),
                       ("step_batch", "update" if tiles else "step")):
        t = times.get(name)
        if not t or t["count"] == 0:
            continue
        avg_ms = t["total_ms"] / t["count"]
        nbytes = kernel_bytes(kind, nnz, m, d, B, s_val, s_idx)
        kernels[name] = dict(avg_us=1e3 * avg_ms, bytes=nbytes, gbs=nbytes / (avg_ms * 1e-3) / 1e9)
        if name in tinfo:
            # on-chip side of a tile kernel: every stored entry (quad padding
            # included) reads its input's 256-byte record of 64 solves from LDS
            ti = tinfo[name]
            lds = ti["entries"] * 256 * (B // 64)
            kernels[name].update(lds_bytes=lds, lds_tbs=lds / (avg_ms * 1e-3) / 1e12,
                                 lds_frac=lds / (avg_ms * 1e-3) / LDS_PEAK_BPS,
                                 staged_records=ti["records"], windows=ti["windows"], tiles=ti["tiles"],
                                 split=ti["split"])
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
    roof = dict(bound="hbm", achieved=round(kernels[dom]["gbs"], 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(kernels[dom]["gbs"] / HBM_PEAK_GBS, 4),
                traffic=measured_traffic(dom, args.storage),
                kernel=dom, avg_us=round(kernels[dom]["avg_us"], 2),
                bytes_per_launch=kernels[dom]["bytes"])

    # ------------------------------------------- AFPPA on the same workload ---
    afppa = None
    if args.afppa_steps > 0:
        afppa = afppa_leg(ap, torch, ctx, mat, pr, g_t, stream, args, s_val, s_idx)
        if not args.no_cpu_baseline and not args.profile:
            log("timing the FP64 AFPPA oracle on the host cores")
            afppa["cpu_oracle"] = cpu_baseline_afppa(pr, args.afppa_cpu_iters)

    # ------------------------------------- factored model (Section 4.1) ---
    factored = None
    if args.factored_steps > 0:
        factored = factored_leg(ap, torch, ctx, args, stream)

    # ----------------------------------------------------- plain (B = 1) ---
    plain = None
    if not args.profile:
        mat32 = ap.load_matrix(ctx, A, geom, "f32")
        g1 = torch.as_tensor(pr.g[0]).to(dev)
        s1 = ap.appga_solve_begin(ctx, mat32, g1, None, params[:1], None, stream)
        for _ in range(args.warmup):
            ap.appga_solve_step(s1, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            ap.appga_solve_step(s1, 1)
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t0
        out1 = torch.empty((1, d), dtype=torch.float32, device=dev)
        ap.appga_solve_end(s1, out1, 1)
        ap.appga_free_system_matrix(ctx, mat32)
        plain = dict(value=round(args.plain_steps / dt1, 1), unit="solve-iterations/s",
                     ms_per_iter=round(1e3 * dt1 / args.plain_steps, 4),
                     path="single-solve FP32 matrix, the 64 solves one after another")

    # ------------------------------------ 256^2 geometry: projectors, serving ---
    projector = None
    pr256 = mat256 = None
    need256 = not args.no_projector or (args.serve_requests > 0 and not args.profile)
    if need256:
        log("building the 256^2 / 256 x 252 geometry")
        pr256 = synth.make_problem(synth.Geometry(256, 256, 252), list(range(3000, 3008)),
                                   tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
        mat256 = ap.load_matrix(ctx, pr256.A, pr256.geom, "f32")
    if not args.no_projector:
        log("single-solve projector leg (256^2, FP32 matrix)")
        projector = projector_leg(ap, torch, ctx, pr256, mat256, max(20, min(args.steps, 100)))
        t256 = ap.appga_tune(ctx, mat256, ap.APPGA_TUNE_SINGLE)
        projector["lanes_per_row"] = {"forward": t256["group_fwd"], "back": t256["group_back"]}
    c4 = None
    if not args.no_projector and args.c4_steps > 0:
        log("batched C4 leg (256^2 x 47, FP32 matrix)")
        c4 = c4_leg(ap, torch, ctx, pr256, mat256, args.c4_steps)

    serving = None
    if args.serve_requests > 0 and not args.profile:
        geom64 = synth.Geometry(64, 96, 90)
        pr64 = synth.make_problem(geom64, list(range(500, 516)), tc_range=(1e5, 1e7),
                                  rf_range=(0.05, 0.2))
        mat64 = ap.load_matrix(ctx, pr64.A, geom64, "f32")
        mats = {"064": (pr64, mat64), "128": (pr, mat), "256": (pr256, mat256)}
        serving = []
        for i, rate in enumerate(args.serve_rate):
            log("serving leg: %d requests at %.0f/s" % (args.serve_requests, rate))
            serving.append(serve_leg(ap, ctx, mats, args.serve_requests, rate, 2024 + i))
        ap.appga_free_system_matrix(ctx, mat64)
        serving = dict(
            mix="sizes uniform over 64x64 (96x90, FP32 matrix), 128x128 (200x168, the bench "
                "matrix) and 256x256 (256x252, FP32 matrix); lambda U[0.005,0.1], omega "
                "{0.3,0.6,1.0}, iterations U{50..300}, Poisson arrivals",
            runs=serving)
    if mat256 is not None:
        ap.appga_free_system_matrix(ctx, mat256)

    cpu = None
    if not args.no_cpu_baseline and not args.profile:
        log("timing the FP64 oracle on the host cores")
        cpu = cpu_baseline(pr, args.cpu_iters)

    ap.appga_free_system_matrix(ctx, mat)
    ap.appga_destroy(ctx)
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "solve-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched 2D PET: 64 sinograms sharing a 128x128 / 200 bins x 168 "
                               "angles Siddon matrix, one APPGA iteration of all 64 per step",
                   "global_batch": B, "image": [geom.n, geom.n], "bins": geom.n_bins,
                   "angles": geom.n_angles, "nnz": nnz, "matrix_storage": args.storage,
                   "lambda": 0.02, "eps": 1e-3, "omega": 0.5},
        "plain": plain,
        "speedup_vs_plain": round(value / plain["value"], 2) if plain else None,
        "kernels": {k: {kk: round(vv, 2) if isinstance(vv, float) else vv
                        for kk, vv in v.items()} for k, v in kernels.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "afppa": afppa,
        "factored": factored,
        "serving": serving,
        "projector_single_256": projector,
        "batched_c4_256x47": c4,
        "matrix_bytes": info,
        "tile_forms": tinfo,
        "tuning": {k: (round(v, 2) if isinstance(v, float) else v) for k, v in tuning.items()},
        "objective_lane0": stats[0]["objective"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
