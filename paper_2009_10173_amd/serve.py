"""Serving driver: a Poisson trace of mixed reconstruction requests through the native
continuous-batching scheduler (`aroam_server_*`), and the plain-FP32 one-at-a-time baseline.

Requests mix scan sizes, depth counts, both sensors and both solvers (see
`workloads.serve_trace`).  Model tables are built once per distinct geometry and stay
resident on the device; each request's signals and result vector are device tensors.

    python -m paper_2009_10173_amd.serve --requests 24 --seed 0
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _workloads():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads
    return workloads


MODES = {
    # plain FP32 solves
    "fp32": dict(inner=B.AROAM_FP32, outer=B.AROAM_FP32, refine=False),
    # BF16 applies with FP32 residual-correction refinement (LSQR sweeps / FISTA anchors)
    "bf16r": dict(inner=B.AROAM_BF16, outer=B.AROAM_FP32, refine=True),
}


def solver_opts(req, mode):
    """Solver kind (0 LSQR, 1 FISTA) and options for one request in one mode."""
    md = MODES[mode]
    if req["kind"] == "lsqr":
        return 0, dict(lam=-1.0, iters=50, inner=md["inner"], outer=md["outer"],
                       refine_sweeps=2 if md["refine"] else 0)
    return 1, dict(lam=-1.0, iters=200, inner=md["inner"], outer=md["outer"], power_iters=50,
                   anchor_period=5, anchor_warmup=-1)


def work_macs(r, mode):
    """The scheduler's size measure of a prepared request: MACs of the whole solve (A + A^T
    pairs as the library counts them, times the model's algorithmic MACs per apply)."""
    kind, o = solver_opts(r["req"], mode)
    pairs = ((o["iters"] + 1.0) * (1 + o["refine_sweeps"]) if kind == 0
             else o["power_iters"] + o["iters"] + 1.0)
    return 2.0 * pairs * r["model"].info()["mac_alg"]


def fp32_mac_rate(reqs, reps=3):
    """FP32 multiply-accumulates per second of one forward + adjoint pair, on the largest model
    of the trace (HIP events)."""
    import torch
    r = max(reqs, key=lambda r: r["model"].info()["mac_alg"])
    m = r["model"]
    x = torch.zeros(m.image_shape, device=r["s"].device)
    m.adjoint(m.forward(x, "fp32"), "fp32", out=x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        m.adjoint(m.forward(x, "fp32"), "fp32", out=x)
    e1.record()
    e1.synchronize()
    return 2.0 * m.info()["mac_alg"] * reps / (e0.elapsed_time(e1) * 1e-3)


def pairs_of(req, mode):
    """A+A^T pairs (any precision) one request performs."""
    kind, o = solver_opts(req, mode)
    if kind == 0:
        sweeps = o["refine_sweeps"]
        rule = 0.5 if (o["lam"] < 0 and (sweeps > 0 or o["inner"] != o["outer"])) else 0.0
        return (o["iters"] + 0.5) * (1 + sweeps) + sweeps + rule
    return o["power_iters"] + o["iters"] + 0.5


class ModelCache:
    """Device-resident models keyed by geometry."""

    def __init__(self, dtypes=("fp32", "bf16")):
        self.dtypes = dtypes
        self.models = {}

    def get(self, cfg):
        key = json.dumps([cfg["sensor"], cfg["grid"]], sort_keys=True)
        if key not in self.models:
            self.models[key] = B.Model(cfg["sensor"], cfg["grid"], dtypes=self.dtypes)
        return self.models[key]

    def close(self):
        for m in self.models.values():
            m.close()
        self.models.clear()


def prepare(trace, cache, device="cuda:0", verbose=False):
    """Inputs of every request: phantom -> FP32 forward -> peak-SNR Gaussian noise (seeded
    GPU generator), plus a result tensor."""
    import torch
    W = _workloads()
    reqs = []
    for req in trace:
        cfg = W.serve_config(req)
        model = cache.get(cfg)
        x0 = torch.from_numpy(W.make_phantom(cfg, req["seed"] % 1000).astype(np.float32)).to(device)
        clean = model.forward(x0, "fp32")
        gen = torch.Generator(device=device)
        gen.manual_seed(int(req["seed"]))
        noise = torch.randn(clean.shape, generator=gen, device=device, dtype=torch.float32)
        sigma = clean.abs().max().item() * 10 ** (-req["snr_db"] / 20)
        s = clean + sigma * noise
        reqs.append(dict(req=req, model=model, s=s, x=torch.zeros(model.image_shape,
                                                                   device=device)))
        _progress(verbose, f"prepared {len(reqs)}/{len(trace)}: side {req['side']}, "
                           f"nz {req['nz']}, {req['sensor']}, {req['kind']}")
    torch.cuda.synchronize()
    return reqs


def _progress(verbose, msg):
    if verbose:
        print(f"[serve] {msg}", file=sys.stderr, flush=True)


def run_served(reqs, mode, budget_bytes, slots=8, tick=2, time_scale=1.0, verbose=False,
               large_macs=0.0, large_alone=False):
    """Replay the arrival times through the scheduler; returns per-request records and the
    scheduler's counts of polls after which a request waited although a slot was free,
    because of the device-memory budget or of the one-large-request policy (`large_macs` >
    0)."""
    import torch
    torch.cuda.synchronize()
    srv = B.aroam_server_create(budget_bytes, slots, tick)
    try:
        if large_macs > 0:
            B.aroam_server_set_large(srv, large_macs, large_alone)
        order = sorted(range(len(reqs)), key=lambda i: reqs[i]["req"]["arrival_s"])
        by_id, rec = {}, {}
        t0 = time.perf_counter()
        nxt, max_res = 0, 0
        while len(rec) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(order) and reqs[order[nxt]]["req"]["arrival_s"] * time_scale <= now:
                r = reqs[order[nxt]]
                kind, o = solver_opts(r["req"], mode)
                rid = B.aroam_server_submit(srv, r["model"].handle, kind, r["s"], r["x"], **o)
                by_id[rid] = order[nxt]
                nxt += 1
            nres, nq = B.aroam_server_poll(srv)
            max_res = max(max_res, nres)
            done = B.aroam_server_collect(srv)
            tnow = time.perf_counter() - t0
            for rid, info in done:
                i = by_id[rid]
                rec[i] = dict(latency=tnow - reqs[i]["req"]["arrival_s"] * time_scale,
                              done_at=tnow, status=info["status"], info=info)
                _progress(verbose, f"{mode} served {len(rec)}/{len(reqs)} at {tnow:.1f} s")
            if not done and nres == 0 and nq == 0 and nxt < len(order):
                wait = reqs[order[nxt]]["req"]["arrival_s"] * time_scale - now
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif not done:
                time.sleep(0.0002)
        wall = max(r["done_at"] for r in rec.values())
        held_budget, held_large = B.aroam_server_held(srv)
    finally:
        B.aroam_server_destroy(srv)
    n_large = sum(1 for r in reqs if large_macs > 0 and work_macs(r, mode) >= large_macs)
    return _summary(reqs, rec, mode, wall, extra=dict(max_resident=max_res, slots=slots,
                                                      tick=tick, budget_bytes=budget_bytes,
                                                      polls_held_by_budget=held_budget,
                                                      polls_held_by_large_policy=held_large,
                                                      large_macs=large_macs,
                                                      large_alone=large_alone,
                                                      large_requests=n_large))


def run_fifo(reqs, mode, time_scale=1.0, verbose=False):
    """One request at a time in arrival order with the blocking solver entry points."""
    import torch
    torch.cuda.synchronize()
    order = sorted(range(len(reqs)), key=lambda i: reqs[i]["req"]["arrival_s"])
    rec = {}
    t0 = time.perf_counter()
    for i in order:
        r = reqs[i]
        arr = r["req"]["arrival_s"] * time_scale
        now = time.perf_counter() - t0
        if arr > now:
            time.sleep(arr - now)
        kind, o = solver_opts(r["req"], mode)
        fn = B.aroam_solve_lsqr if kind == 0 else B.aroam_solve_l1
        info = fn(r["model"].handle, r["s"], r["x"], **o)
        tnow = time.perf_counter() - t0
        rec[i] = dict(latency=tnow - arr, done_at=tnow, status=info["status"], info=info)
        _progress(verbose, f"{mode} fifo {len(rec)}/{len(reqs)} at {tnow:.1f} s")
    wall = max(r["done_at"] for r in rec.values())
    return _summary(reqs, rec, mode, wall)


def _summary(reqs, rec, mode, wall, extra=None):
    lat = np.array([rec[i]["latency"] for i in range(len(reqs))])
    pairs = sum(pairs_of(r["req"], mode) for r in reqs)
    out = dict(mode=mode, n=len(reqs), wall_s=wall, p50_s=float(np.percentile(lat, 50)),
               p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
               recons_per_s=len(reqs) / wall, pairs_per_s=pairs / wall,
               failed=int(sum(1 for r in rec.values() if r["status"] != 0)))
    if extra:
        out.update(extra)
    return out


def predicted_service(reqs, reps=3):
    """FP32 one-at-a-time service time of each request, predicted from its pair count and the
    measured time of one FP32 forward + adjoint pair of its model (HIP events, per distinct
    model), instead of running the whole trace once to calibrate the arrival rate."""
    import torch
    pair_ms = {}
    out = []
    for r in reqs:
        m = r["model"]
        key = id(m)
        if key not in pair_ms:
            x = torch.zeros(m.image_shape, device=r["s"].device)
            m.forward(x, "fp32")
            m.adjoint(r["s"], "fp32", out=x)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                m.adjoint(m.forward(x, "fp32"), "fp32", out=x)
            e1.record()
            e1.synchronize()
            pair_ms[key] = e0.elapsed_time(e1) / reps
        out.append(pair_ms[key] * 1e-3 * pairs_of(r["req"], "fp32"))
    return out


def main(argv=None, quiet=False):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--load", type=float, default=0.8,
                    help="arrival rate as a fraction of the FP32 FIFO service rate")
    ap.add_argument("--sides", default="64,96,128,192,256,320,400")
    ap.add_argument("--nz", default="64,128,256")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--tick", type=int, default=2)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--rate", type=float, default=0.0,
                    help="arrival rate (requests/s); 0 calibrates it from the FIFO FP32 run")
    ap.add_argument("--calibrate", default="run", choices=["run", "predict"],
                    help="FP32 service time for the arrival rate: run the trace once one at a "
                         "time, or predict it from each model's measured pair time")
    ap.add_argument("--modes", default="fifo_fp32,served_fp32,served_bf16r",
                    help="legs to run (comma-separated)")
    ap.add_argument("--large-s", type=float, default=1.0,
                    help="one-large-request policy of the scheduler: requests whose solve "
                         "takes at least this many seconds of FP32 applies (at the measured "
                         "FP32 MAC rate) are large, and at most one is resident; 0 = off")
    ap.add_argument("--large-alone", action="store_true",
                    help="with --large-s: admit nothing while a large request is resident")
    ap.add_argument("--verbose", action="store_true", help="print every completion")
    args = ap.parse_args(argv)
    W = _workloads()
    sides = tuple(int(v) for v in args.sides.split(","))
    nzs = tuple(int(v) for v in args.nz.split(","))
    # calibration: FP32 FIFO service time of the requests (all arriving at t = 0)
    trace = W.serve_trace(args.requests, 1.0, args.seed, sides=sides, nzs=nzs)
    cache = ModelCache()
    t = time.time()
    reqs = prepare(trace, cache, verbose=args.verbose)
    print(f"[serve] prepared {len(reqs)} requests, {len(cache.models)} models in "
          f"{time.time() - t:.1f} s", file=sys.stderr, flush=True)
    v = args.verbose
    if args.rate > 0:
        rate = args.rate
        service = args.load / rate
    elif args.calibrate == "predict":
        service = float(np.mean(predicted_service(reqs)))
        rate = args.load / service
    else:
        for r in reqs:
            r["req"]["arrival_s"] = 0.0
        base0 = run_fifo(reqs, "fp32", verbose=v)
        service = base0["wall_s"] / len(reqs)
        rate = args.load / service
    timed = W.serve_trace(args.requests, rate, args.seed, sides=sides, nzs=nzs)
    for r, tr in zip(reqs, timed):
        r["req"]["arrival_s"] = tr["arrival_s"]
    print(f"[serve] FP32 service time {service:.3f} s/request -> Poisson rate {rate:.2f}/s",
          file=sys.stderr, flush=True)
    res = dict(rate_per_s=rate, fp32_service_s=service, calibrate=args.calibrate,
               sides=list(sides), nz=list(nzs), load=args.load)
    modes = args.modes.split(",")
    budget = int(args.budget_gb * 2 ** 30)
    large_macs = 0.0
    if args.large_s > 0:
        large_macs = args.large_s * fp32_mac_rate(reqs)
        res["large_s"] = args.large_s
        res["large_macs"] = large_macs
    for leg in modes:
        if leg == "fifo_fp32":
            res[leg] = run_fifo(reqs, "fp32", verbose=v)
        elif leg in ("served_fp32", "served_bf16r"):
            res[leg] = run_served(reqs, leg.split("_")[1], budget, args.slots, args.tick,
                                  verbose=v, large_macs=large_macs,
                                  large_alone=args.large_alone)
        else:
            raise ValueError(f"unknown serving leg {leg}")
        print(f"[serve] {leg} done: p50 {res[leg]['p50_s']:.2f} s, p99 {res[leg]['p99_s']:.2f} s",
              file=sys.stderr, flush=True)
    cache.close()
    torch.cuda.synchronize()
    if not quiet:
        print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
