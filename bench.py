"""Benchmark of the AR-OAM hot path on one MI355X: LSQR-Tikhonov reconstructions of the
200x200-position workload (voxels 200x200x128 at 10 um, Nt 512, cone footprint up to 41x41
offsets, 50 iterations).  One step = one full reconstruction (50 iterations = 50 A + 50 A^T
applies plus the initial A^T, with the fused FP64 vector work).  Prints one JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--dtype fp32|bf16|fp8]
                       [--workload vessels200|vessels400] [--no-cpu-baseline]
                       [--cpu-detail]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "A+Aᵀ applies/s (TMAC/s, % MFMA peak); recon p50/p99 latency vs plain FP32"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "fp64": 78.6}
# peak of the MFMA each apply dtype issues: the e4m3 table is decoded to BF16 in registers
ISSUE_PEAK = {"fp32": 157.3, "bf16": 2500.0, "fp8": 2500.0, "fp64": 78.6}
DTYPE_TAG = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8", "fp64": "f64"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_times(model, dtype, x, s, reps):
    """Average duration (ms) of one forward and one adjoint launch on dense Gaussian vectors
    (like the solver's Krylov vectors; x and s give the shapes), timed with HIP events on the
    stream the library launches on (torch's current stream)."""
    import torch
    st = torch.cuda.current_stream()
    gen = torch.Generator(device=x.device)
    gen.manual_seed(1234)
    x = torch.randn(x.shape, generator=gen, device=x.device, dtype=x.dtype)
    s = torch.randn(s.shape, generator=gen, device=s.device, dtype=s.dtype)
    out = {}
    for name, fn, arg in (("forward", model.forward, x), ("adjoint", model.adjoint, s)):
        fn(arg, dtype)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(reps):
            fn(arg, dtype)
        e1.record(st)
        e1.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


# Sources that decide what the apply kernels do and launch (kernels, layouts, launch plan).
KERNEL_SOURCES = ("apply.hip", "table.hip", "plan.h", "internal.h")


def kernel_code_digest():
    """SHA-256 of the apply kernels' sources with comments and layout whitespace removed, so
    that a counter summary stays valid across comment edits and no longer once code changes."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2009_10173_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update((name + "\0" + " ".join(text.split()) + "\0").encode())
    return h.hexdigest()


def profiled_traffic(workload, dtype, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the counters were taken on another workload or the kernels' code has changed since."""
    path = os.path.join(ROOT, "profiles", "apply_counters.json")
    try:
        prof = json.load(open(path))
        digest = kernel_code_digest()
    except (OSError, ValueError):
        return None
    if prof.get("kernel_code_digest") != digest or prof.get("workload") != workload:
        return None
    k = prof.get("kernels", {}).get(f"apply {dtype} {kernel}")
    return None if k is None else k["bytes"]


def _sample_work(H, g):
    """Band entries and algorithmic MACs of a depth-slab table H[dy, dx, slab, n]: per column
    the window from its first to its last nonzero sample, times the scan positions that see
    the column's offset."""
    import numpy as np
    nzr = H != 0
    present = nzr.any(axis=-1)
    first = np.argmax(nzr, axis=-1)
    last = g["nt"] - 1 - np.argmax(nzr[..., ::-1], axis=-1)
    length = np.where(present, last - first + 1, 0)
    K = g["k_half"]
    d = np.abs(np.arange(-K, K + 1))
    pairs = (g["ny"] - d)[:, None] * (g["nx"] - d)[None, :]
    return int(length.sum()), int(np.sum(pairs[:, :, None] * length))


def cpu_baseline(cfg, mac_full, depth_fracs=(0.31, 0.32, 0.67, 0.68)):
    """The FP64 oracle's A + A^T pair on a bounded sample of the same workload: the full scan
    grid and footprint restricted to a few depth slabs (at the given fractions of the depth
    range), scaled to full-workload pairs/s by the ratio of algorithmic MACs."""
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle import model as omodel
    from oracle import operators as oops
    g = cfg["grid"]
    ks = [int(f * g["nz"]) for f in depth_fracs]
    t0 = time.time()
    H = omodel.build_depth_slabs(cfg["sensor"], g, ks)
    t_table = time.time() - t0
    log(f"oracle table for depth slabs {ks}: {t_table:.1f} s")
    _, mac_sample = _sample_work(H, g)
    rng = W.rng(99)
    x = rng.standard_normal((g["ny"], g["nx"], len(ks)))
    y = rng.standard_normal((g["ny"], g["nx"], g["nt"]))
    times = []
    for _ in range(2):
        t0 = time.time()
        oops.forward(H, x)
        oops.adjoint(H, y)
        times.append(time.time() - t0)
        log(f"oracle A+A^T pair on the sample: {times[-1]:.1f} s")
    t_pair = min(times)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()
                   if d.get("user_api") == "blas"] or [1])
    frac = mac_sample / mac_full
    return dict(value=frac / t_pair, unit="A+A^T pairs/s", cores=int(threads), kind="oracle",
                sample=(f"FP64 oracle A+A^T pair on depth slabs {ks} of the full "
                        f"{g['nx']}x{g['ny']} scan "
                        f"({100 * frac:.2f}% of the algorithmic MACs), {t_pair:.2f} s per sample "
                        f"pair, scaled by the MAC ratio; table build for the slabs "
                        f"{t_table:.1f} s not included"))


def cpu_detail(cfg, nnz_full, mac_full, iters, depth_fracs=(0.31, 0.32, 0.67, 0.68)):
    """Detail of the CPU baseline: the FP64 oracle's table build, A + A^T pair and LSQR
    reconstruction, each timed with one core and with all cores.  The table with all cores is the full build, timed; every other
    figure is timed on the depth-slab sample of `cpu_baseline` and scaled to the full workload:
    the table by the ratio of band entries, the pair by the ratio of algorithmic MACs, and the
    reconstruction by the MAC ratio from the initial A^T and `iters` times one iteration (one
    timed LSQR iteration with its set-up, less the initial A^T)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import workloads as W
    from oracle import model as omodel
    from oracle import operators as oops
    from oracle import solvers as osolv
    g = cfg["grid"]
    ks = [int(f * g["nz"]) for f in depth_fracs]
    all_cores = min(os.cpu_count() or 1, 16)
    t0 = time.time()
    H_full = omodel.build_table(cfg["sensor"], g, workers=all_cores)
    t_full = time.time() - t0
    nnz_oracle = int(np.count_nonzero(H_full))
    del H_full
    log(f"oracle full table with {all_cores} workers: {t_full:.1f} s")
    rng = W.rng(99)
    x = rng.standard_normal((g["ny"], g["nx"], len(ks)))
    y = rng.standard_normal((g["ny"], g["nx"], g["nt"]))
    out = {}
    for label, workers, blas in (("1", 1, 1), ("all", all_cores, None)):
        t0 = time.time()
        H = omodel.build_depth_slabs(cfg["sensor"], g, ks, workers=workers)
        t_table = time.time() - t0
        nnz_sample, mac_sample = _sample_work(H, g)
        frac_mac = mac_sample / mac_full
        frac_nnz = nnz_sample / nnz_full
        with threadpool_limits(limits=blas):
            threads = max([p.get("num_threads", 1) for p in threadpool_info()
                           if p.get("user_api") == "blas"] or [1])
            t0 = time.time()
            oops.forward(H, x)
            t_fwd = time.time() - t0
            t0 = time.time()
            oops.adjoint(H, y)
            t_adj = time.time() - t0
            t_pair = t_fwd + t_adj
            t0 = time.time()
            osolv.lsqr(lambda v: oops.forward(H, v.reshape(x.shape)).ravel(),
                       lambda v: oops.adjoint(H, v.reshape(y.shape)).ravel(), y, damp=1.0,
                       iters=1)
            t_it = time.time() - t0
        log(f"oracle, {label} core(s): slab table {t_table:.1f} s, forward {t_fwd:.1f} s, "
            f"adjoint {t_adj:.1f} s, LSQR set-up and one iteration {t_it:.1f} s")
        # LSQR = one A^T to start, then per iteration one pair and the vector work
        recon = t_adj + iters * (t_it - t_adj)
        out[label] = {"workers": workers, "blas_threads": int(threads),
                      "table_build_s": t_table / frac_nnz,
                      "pair_s": t_pair / frac_mac,
                      "recon_s": recon / frac_mac,
                      "sample_s": {"table": t_table, "forward": t_fwd, "adjoint": t_adj,
                                   "lsqr_1_iteration": t_it}}
    # all cores: the measured full build (a slab sample has fewer slabs than workers)
    out["all"]["table_build_s"] = t_full
    out["table_band_entries"] = {"oracle": nnz_oracle, "model": int(nnz_full)}
    out["sample"] = (f"depth slabs {ks} of the full {g['nx']}x{g['ny']} scan "
                     f"({100 * frac_mac:.2f}% of the algorithmic MACs, {100 * frac_nnz:.2f}% of "
                     f"the table's band entries); the all-core table time is the full build, "
                     f"the others are scaled from the sample (table by band entries, pair by "
                     f"MACs, reconstruction of {iters} LSQR iterations as the initial A^T plus "
                     f"{iters} times one timed iteration, by MACs)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="vessels200")
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-detail", action="store_true",
                    help="in the CPU baseline, also time the oracle's table build, pair and "
                         "reconstruction with one core and with all cores (about two more "
                         "minutes)")
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="requests in the serving leg (0 skips it)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2009_10173_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    cfg = W.config(args.workload)
    g = cfg["grid"]
    iters = cfg["solver"]["iters"]
    log(f"building model {args.workload}")
    torch.cuda.synchronize()
    t0 = time.time()
    # inner precisions of the refined legs: BF16 and FP8 for the FP32 bench, else its own
    lows = ["bf16", "fp8"] if args.dtype == "fp32" else [args.dtype]
    model = P.Model(cfg["sensor"], g, dtypes=tuple(sorted({"fp32", args.dtype, *lows})))
    torch.cuda.synchronize()
    t_build = time.time() - t0
    info = model.info()
    log(f"model built in {t_build:.2f} s: nnz {info['nnz']}, MAC_alg {info['mac_alg']:.3e}")

    x0 = torch.from_numpy(W.make_phantom(cfg, 0).astype(np.float32)).to(dev)
    clean = model.forward(x0, "fp32")
    sigma = clean.abs().max().item() * 10 ** (-cfg["snr_db"] / 20)
    s = clean + sigma * torch.from_numpy(W.unit_noise(cfg, 0).astype(np.float32)).to(dev)
    torch.cuda.synchronize()

    def step():
        return model.solve_lsqr(s, lam=-1.0, iters=iters, inner=args.dtype)

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        x, sinfo = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
        log(f"step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms")
    elapsed = time.perf_counter() - t_start
    pairs_per_step = iters + 0.5          # 50 A + 50 A^T + the initial A^T
    pairs_s = args.steps * pairs_per_step / elapsed

    kt = kernel_times(model, args.dtype, x0, s, args.kernel_reps)
    dom = max(kt, key=kt.get)
    di = P.DTYPES[args.dtype]
    mac_exec = info["mac_exec"][di] if dom == "forward" else info["mac_exec_adj"][di]
    flops = 2.0 * info["mac_alg"]
    achieved = flops / (kt[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.dtype]
    mfma_issued = 2.0 * mac_exec / (kt[dom] * 1e-3) / 1e12 / ISSUE_PEAK[args.dtype]
    result = {
        "metric": METRIC,
        "value": pairs_s,
        "unit": "A+A^T pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_TAG[args.dtype],
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: LSQR-Tikhonov {iters} its, scan "
                                f"{g['nx']}x{g['ny']} at {g['step_m'] * 1e6:g} um, voxels "
                                f"{g['nx']}x{g['ny']}x{g['nz']}, Nt {g['nt']}, cone footprint "
                                f"K={g['k_half']}, {cfg['phantom']['n']} curved-tube phantom, "
                                f"{cfg['snr_db']:g} dB"),
                   "solver": "lsqr", "iters": iters},
        "tmac_s": 2.0 * info["mac_alg"] * pairs_s / 1e12,
        "recon_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "recon_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "kernel_ms": kt,
        "fill": {"forward": info["mac_alg"] / info["mac_exec"][di],
                 "adjoint": info["mac_alg"] / info["mac_exec_adj"][di]},
        "table_build_s": t_build,
        # workgroup rows of each staged launch: output row tiles, and pieces where the launch
        # plan cuts heavy tiles
        "launch": {dt: {"forward": {"tiles": info["row_tiles"][P.DTYPES[dt]],
                                    "pieces": info["pieces"][P.DTYPES[dt]]},
                        "adjoint": {"tiles": info["row_tiles_adj"][P.DTYPES[dt]],
                                    "pieces": info["pieces_adj"][P.DTYPES[dt]]}}
                   for dt in sorted({"fp32", args.dtype, *lows})},
        "lambda": sinfo["lam"],
        "roofline": {"bound": "mfma", "kernel": (f"{dom} (e4m3 table, bf16 MFMA)" if args.dtype == "fp8"
                                else f"{dom} ({args.dtype} MFMA)"),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "issued_frac": mfma_issued,
                     "traffic": profiled_traffic(args.workload, args.dtype, dom)},
    }
    # reduced precision with refinement on the same workload: BF16 / FP8 applies, FP32
    # residuals, two sweeps
    x32 = x if args.dtype == "fp32" else model.solve_lsqr(s, lam=-1.0, iters=iters)[0]
    for lo in lows:
        log(f"{lo}-refined reconstruction (2 sweeps)")
        model.solve_lsqr(s, lam=-1.0, iters=iters, inner=lo, outer="fp32", refine_sweeps=2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xr, rinfo = model.solve_lsqr(s, lam=-1.0, iters=iters, inner=lo, outer="fp32",
                                     refine_sweeps=2)
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t1
        diff = ((xr - x32).norm() / x32.norm()).item()
        kt_lo = kernel_times(model, lo, x0, s, args.kernel_reps)
        li = P.DTYPES[lo]
        result[f"{lo}_refined"] = {
            "recon_ms": t_ref * 1e3, "sweeps": 2,
            "pairs_per_s": ((iters + 0.5) * 3 + 2 + 0.5) / t_ref,
            "rel_diff_vs_fp32_recon": diff,
            "kernel_ms": kt_lo,
            f"issued_frac_{lo}": {k: 2.0 * (info["mac_exec"][li] if k == "forward" else
                                            info["mac_exec_adj"][li]) / (v * 1e-3) / 1e12
                                  / ISSUE_PEAK[lo] for k, v in kt_lo.items()},
        }
    if args.serve_requests > 0:
        log(f"serving leg: {args.serve_requests} mixed requests")
        model.close()
        model = None
        from paper_2009_10173_amd import serve as S
        res = S.main(["--requests", str(args.serve_requests), "--sides", "64,96,128,192",
                      "--nz", "64,128"], quiet=True)
        result["serving"] = {k: res[k] for k in ("rate_per_s", "fifo_fp32", "served_fp32",
                                                  "served_bf16r")}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(cfg, info["mac_alg"])
        if args.cpu_detail:
            log("timing the CPU oracle's table, pair and reconstruction on one and all cores")
            result["cpu_baseline"]["detail"] = cpu_detail(cfg, info["nnz"], info["mac_alg"],
                                                          iters)
    if model is not None:
        model.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
