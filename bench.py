"""Benchmark of the AR-OAM hot path on one MI355X.

Headline workload: the 400x400-position scan at 5 um (voxels 400x400x256 at 5 um, Nt 1024,
cone footprint up to 81x81 offsets), FP32 applies.  One step = one LSQR-Tikhonov iteration:
one A and one A^T apply with the fused FP64 vector work.  The timed region is one solve of
exactly `--steps` iterations (its set-up adds the initial A^T u, half a pair); `value` is A+A^T
pairs per second, (steps + 0.5) / elapsed.  Beside it, in the same JSON line: the full
50-iteration FP32 reconstruction, the FP8- and BF16-refined reconstructions (2 sweeps) with
their difference to it, the 200x200 workload as a secondary leg, the serving leg (a Poisson
trace over the whole request mix), the roofline of the dominant kernel, and the CPU oracle on
a bounded sample.  Prints one JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--dtype fp32|bf16|fp8]
                       [--workload vessels400|vessels200] [--secondary vessels200|none]
                       [--serve-requests N] [--no-cpu-baseline] [--cpu-detail]
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
# peak of the MFMA each apply dtype issues (FP8: the block-scaled FP8 MFMA)
ISSUE_PEAK = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "fp64": 78.6}
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


def cpu_baseline(cfg, mac_full, depth_fracs=(0.31, 0.32, 0.67, 0.68), side=None):
    """The FP64 oracle's A + A^T pair on a bounded sample of the same workload: the footprint
    and time axis of the full problem restricted to a few depth slabs (at the given fractions
    of the depth range) and, with `side`, to a side x side scan; scaled to full-workload
    pairs/s by the ratio of algorithmic MACs."""
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle import model as omodel
    from oracle import operators as oops
    g = cfg["grid"]
    ks = [int(f * g["nz"]) for f in depth_fracs]
    t0 = time.time()
    H = omodel.build_depth_slabs(cfg["sensor"], g, ks, workers=min(os.cpu_count() or 1, 16))
    t_table = time.time() - t0
    log(f"oracle table for depth slabs {ks}: {t_table:.1f} s")
    gs = dict(g) if side is None else dict(g, nx=side, ny=side)
    _, mac_sample = _sample_work(H, gs)
    rng = W.rng(99)
    x = rng.standard_normal((gs["ny"], gs["nx"], len(ks)))
    y = rng.standard_normal((gs["ny"], gs["nx"], g["nt"]))
    t0 = time.time()
    oops.forward(H, x)
    oops.adjoint(H, y)
    t_pair = time.time() - t0
    log(f"oracle A+A^T pair on the sample: {t_pair:.1f} s")
    threads = max([d.get("num_threads", 1) for d in threadpool_info()
                   if d.get("user_api") == "blas"] or [1])
    frac = mac_sample / mac_full
    scan = f"{gs['nx']}x{gs['ny']} scan" + ("" if side is None else
                                               f" (of the {g['nx']}x{g['ny']} workload)")
    return dict(value=frac / t_pair, unit="A+A^T pairs/s", cores=int(threads), kind="oracle",
                sample=(f"FP64 oracle A+A^T pair on depth slabs {ks} of a {scan} with the "
                        f"workload's footprint and time axis ({100 * frac:.3f}% of the "
                        f"algorithmic MACs), {t_pair:.2f} s per sample pair, scaled by the MAC "
                        f"ratio; table build for the slabs {t_table:.1f} s not included"))


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


def roofline(info, dtype, kt, workload):
    """Roofline of the dominant (slower) apply kernel from its event-timed average launch."""
    import paper_2009_10173_amd as P
    dom = max(kt, key=kt.get)
    di = P.DTYPES[dtype]
    mac_exec = info["mac_exec"][di] if dom == "forward" else info["mac_exec_adj"][di]
    achieved = 2.0 * info["mac_alg"] / (kt[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    return {"bound": "mfma",
            "kernel": (f"{dom} (e4m3 table and operand, block-scaled fp8 MFMA)" if dtype == "fp8"
                       else f"{dom} ({dtype} MFMA)"),
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "issued_frac": 2.0 * mac_exec / (kt[dom] * 1e-3) / 1e12 / ISSUE_PEAK[dtype],
            "kernel_ms": kt[dom],
            "traffic": profiled_traffic(workload, dtype, dom)}


def signals(model, cfg, dev):
    """Seeded phantom -> FP32 forward -> peak-SNR Gaussian noise, all resident in HBM."""
    import numpy as np
    import torch

    import workloads as W
    x0 = torch.from_numpy(W.make_phantom(cfg, 0).astype(np.float32)).to(dev)
    clean = model.forward(x0, "fp32")
    sigma = clean.abs().max().item() * 10 ** (-cfg["snr_db"] / 20)
    s = clean + sigma * torch.from_numpy(W.unit_noise(cfg, 0).astype(np.float32)).to(dev)
    torch.cuda.synchronize()
    return x0, s


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def secondary_leg(name, dev, reps=3):
    """Plain FP32 LSQR reconstructions of another workload: pairs/s and kernel times."""
    import paper_2009_10173_amd as P
    import workloads as W
    cfg = W.config(name)
    iters = cfg["solver"]["iters"]
    with P.Model(cfg["sensor"], cfg["grid"], dtypes=("fp32",)) as model:
        info = model.info()
        x0, s = signals(model, cfg, dev)
        model.solve_lsqr(s, lam=-1.0, iters=iters)
        lat = [timed(lambda: model.solve_lsqr(s, lam=-1.0, iters=iters))[1] for _ in range(reps)]
        kt = kernel_times(model, "fp32", x0, s, 10)
    t = sorted(lat)[len(lat) // 2]
    return {"workload": name, "iters": iters, "recon_ms": t * 1e3,
            "pairs_per_s": (iters + 0.5) / t,
            "tmac_s": 2.0 * info["mac_alg"] * (iters + 0.5) / t / 1e12,
            "kernel_ms": kt, "roofline": roofline(info, "fp32", kt, name)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="vessels400")
    ap.add_argument("--secondary", default="vessels200")
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-detail", action="store_true",
                    help="in the CPU baseline, also time the oracle's table build, pair and "
                         "reconstruction with one core and with all cores (minutes more)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests in the serving leg (0 skips it)")
    ap.add_argument("--no-recon", action="store_true",
                    help="skip the full and refined reconstructions (for profiler passes)")
    ap.add_argument("--serve-modes", default="fifo_fp32,served_bf16r")
    ap.add_argument("--serve-budget-gb", type=float, default=6.0,
                    help="device-memory budget of the scheduler's admission (GiB; small enough "
                         "that two of the mix's largest requests are not resident together)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2009_10173_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    cfg = W.config(args.workload)
    g = cfg["grid"]
    iters = cfg["solver"]["iters"]
    log(f"building model {args.workload}")
    lows = ["fp8", "bf16"] if args.dtype == "fp32" else [args.dtype]
    dtypes = tuple(sorted({"fp32", args.dtype, *lows}))
    (model, t_build) = timed(lambda: P.Model(cfg["sensor"], g, dtypes=dtypes))
    info = model.info()
    log(f"model built in {t_build:.2f} s: nnz {info['nnz']}, MAC_alg {info['mac_alg']:.3e}")
    x0, s = signals(model, cfg, dev)

    # headline: LSQR iterations, `warmup` untimed, then one solve of exactly `steps`
    if args.warmup > 0:
        timed(lambda: model.solve_lsqr(s, lam=-1.0, iters=args.warmup, inner=args.dtype))
        log(f"warmup: {args.warmup} LSQR iterations done")
    (xk, sinfo), elapsed = timed(lambda: model.solve_lsqr(s, lam=-1.0, iters=args.steps,
                                                          inner=args.dtype))
    log(f"timed: {args.steps} LSQR iterations in {elapsed:.2f} s")
    pairs_s = (args.steps + 0.5) / elapsed

    kt = kernel_times(model, args.dtype, x0, s, args.kernel_reps)
    log(f"kernel times {args.dtype}: {kt}")
    di = P.DTYPES[args.dtype]
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
        "config": {"workload": (f"{args.workload}: scan {g['nx']}x{g['ny']} at "
                                f"{g['step_m'] * 1e6:g} um, voxels {g['nx']}x{g['ny']}x{g['nz']} "
                                f"at {g['dz_m'] * 1e6:g} um, Nt {g['nt']}, cone footprint "
                                f"K={g['k_half']}, {cfg['phantom']['n']} curved-tube phantom, "
                                f"{cfg['snr_db']:g} dB; step = one LSQR-Tikhonov iteration "
                                f"(A + A^T + FP64 vector work)"),
                   "solver": "lsqr", "step": "lsqr_iteration"},
        "tmac_s": 2.0 * info["mac_alg"] * pairs_s / 1e12,
        "kernel_ms": kt,
        "fill": {"forward": info["mac_alg"] / info["mac_exec"][di],
                 "adjoint": info["mac_alg"] / info["mac_exec_adj"][di]},
        "mac_alg": info["mac_alg"],
        "table_build_s": t_build,
        "launch": {dt: {"forward": {"tiles": info["row_tiles"][P.DTYPES[dt]],
                                    "pieces": info["pieces"][P.DTYPES[dt]]},
                        "adjoint": {"tiles": info["row_tiles_adj"][P.DTYPES[dt]],
                                    "pieces": info["pieces_adj"][P.DTYPES[dt]]}}
                   for dt in dtypes},
        "lambda": sinfo["lam"],
        "roofline": roofline(info, args.dtype, kt, args.workload),
    }
    # the full reconstruction in the plain precision, then reduced precision with two FP32
    # residual-correction sweeps
    x32 = None
    if not args.no_recon:
        (x32, _), t_rec = timed(lambda: model.solve_lsqr(s, lam=-1.0, iters=iters,
                                                         inner=args.dtype))
        log(f"{args.dtype} reconstruction ({iters} iterations): {t_rec:.2f} s")
        result["recon"] = {"iters": iters, "dtype": args.dtype, "recon_ms": t_rec * 1e3,
                           "pairs_per_s": (iters + 0.5) / t_rec}
    for lo in lows:
        if lo == args.dtype:
            continue
        kt_lo = kernel_times(model, lo, x0, s, args.kernel_reps)
        log(f"kernel times {lo}: {kt_lo}")
        if args.no_recon:
            result[f"{lo}_kernel_ms"] = kt_lo
            continue
        (xr, rinfo), t_ref = timed(lambda: model.solve_lsqr(
            s, lam=-1.0, iters=iters, inner=lo, outer=args.dtype, refine_sweeps=2))
        diff = ((xr - x32).norm() / x32.norm()).item()
        log(f"{lo}-refined reconstruction (2 sweeps): {t_ref:.2f} s, diff {diff:.2e}")
        li = P.DTYPES[lo]
        result[f"{lo}_refined"] = {
            "recon_ms": t_ref * 1e3, "sweeps": 2,
            "speedup_vs_plain": t_rec / t_ref,
            "pairs_per_s": ((iters + 0.5) * 3 + 2 + 0.5) / t_ref,
            "rel_diff_vs_plain_recon": diff,
            "kernel_ms": kt_lo,
            "roofline": roofline(info, lo, kt_lo, args.workload),
            "issued_frac": {k: 2.0 * (info["mac_exec"][li] if k == "forward" else
                                      info["mac_exec_adj"][li]) / (v * 1e-3) / 1e12
                            / ISSUE_PEAK[lo] for k, v in kt_lo.items()},
        }
    model.close()
    del x0, s, xk, x32
    torch.cuda.empty_cache()
    if args.secondary != "none":
        log(f"secondary leg: {args.secondary}")
        result["secondary"] = secondary_leg(args.secondary, dev)
        log(f"secondary: {result['secondary']['pairs_per_s']:.1f} pairs/s")
    if args.serve_requests > 0:
        log(f"serving leg: {args.serve_requests} mixed requests")
        from paper_2009_10173_amd import serve as S
        # the large-request policy stays off here, so that the leg shows the admission budget
        # binding (profiles/serving_mixed40.md measures the policy)
        res = S.main(["--requests", str(args.serve_requests), "--calibrate", "predict",
                      "--modes", args.serve_modes, "--budget-gb", str(args.serve_budget_gb),
                      "--large-s", "0"], quiet=True)
        result["serving"] = res
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        side = 128 if g["nx"] > 200 else None
        fracs = (0.31, 0.32, 0.67, 0.68)
        result["cpu_baseline"] = cpu_baseline(cfg, info["mac_alg"], fracs, side)
        if args.cpu_detail:
            log("timing the CPU oracle's table, pair and reconstruction on one and all cores")
            result["cpu_baseline"]["detail"] = cpu_detail(cfg, info["nnz"], info["mac_alg"],
                                                          iters)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
