"""Super-resolution evaluation on synthetic absorber pairs (Results, second simulation; Fig. 2a-b).

Two 20 um absorbers in the focal plane, 60 um apart (resolvable by every method) and 40 um
apart (beyond the acoustic diffraction limit of the band-pass filtered system, 61 um for
0.5-80 MHz at NA 0.43).  Signals and model are filtered by the same band-pass; the signals
are normalised to their largest magnitude, without noise.  Both reconstructions run on the
device: MB-L2 (Tikhonov LSQR) and MB-L1 (FISTA with soft-thresholding).

The figures of merit are read, as in Fig. 2b, from the lateral profile through both
absorbers of the maximum-intensity projection along depth:
* FWHM of each peak (linear interpolation between samples at half the peak value);
* separation: the pair counts as resolved when the profile between the two peaks falls at
  least 20 % below the smaller peak (reading of "separation for points > 20 % of the
  minimum").

    python -m paper_2009_10173_amd.superres            # prints one JSON line per case
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def mip(x):
    """Maximum-intensity projection along depth of an image [ny][nx][nz]."""
    return np.asarray(x).max(axis=-1)


def fwhm(profile, peak, step):
    """Full width at half maximum of the peak at index `peak` (same units as step), with the
    half-maximum crossings located by linear interpolation; None if a side never drops."""
    p = np.asarray(profile, dtype=np.float64)
    half = 0.5 * p[peak]
    left = right = None
    for i in range(peak, 0, -1):
        if p[i - 1] < half <= p[i]:
            left = (i - 1) + (half - p[i - 1]) / (p[i] - p[i - 1])
            break
    for i in range(peak, len(p) - 1):
        if p[i + 1] < half <= p[i]:
            right = i + (p[i] - half) / (p[i] - p[i + 1])
            break
    if left is None or right is None:
        return None
    return (right - left) * step


def pair_peaks(profile, i1, i2, reach):
    """Indices of the largest samples within `reach` of the expected positions i1 < i2."""
    p = np.asarray(profile)
    a = max(0, i1 - reach) + int(np.argmax(p[max(0, i1 - reach):i1 + reach + 1]))
    b = max(0, i2 - reach) + int(np.argmax(p[max(0, i2 - reach):i2 + reach + 1]))
    return a, b


def dip(profile, a, b):
    """1 - min(profile between the peaks a < b) / min(peak values): the relative depth of the
    valley between two peaks (0 when there is no valley)."""
    p = np.asarray(profile, dtype=np.float64)
    lo, hi = min(a, b), max(a, b)
    top = min(p[lo], p[hi])
    if top <= 0 or hi - lo < 2:
        return 0.0
    return float(max(0.0, 1.0 - p[lo + 1:hi].min() / top))


def evaluate(x, cfg, dip_threshold=0.2):
    """Figures of merit of a reconstruction of a ball-pair phantom."""
    g, ph = cfg["grid"], cfg["phantom"]
    step_um = g["step_m"] * 1e6
    row = g["ny"] // 2
    prof = mip(x)[row]
    c = g["nx"] // 2
    h = int(round(0.5 * ph["sep_um"] / step_um))
    a, b = pair_peaks(prof, c - h, c + h, max(1, h // 2))
    d = dip(prof, a, b)
    widths = [fwhm(prof, a, step_um), fwhm(prof, b, step_um)]
    return dict(peaks_um=[a * step_um, b * step_um], separation_um=(b - a) * step_um,
                dip=d, resolved=bool(d >= dip_threshold), fwhm_um=widths,
                profile=[float(v) for v in prof])


def fine_config(cfg, factor=2):
    """The same field of view, sensor, filter and phantom on a grid `factor` times finer in
    every direction (the scan positions of the coarse grid are every factor-th fine one)."""
    import copy
    f = copy.deepcopy(cfg)
    g = f["grid"]
    g.update(nx=g["nx"] * factor, ny=g["ny"] * factor, nz=g["nz"] * factor,
             step_m=g["step_m"] / factor, dz_m=g["dz_m"] / factor, k_half=g["k_half"] * factor)
    return f


def signals(cfg, factor=2, device="cuda:0"):
    """Filtered, peak-normalised signals of the phantom (no noise), on the device.

    The paper simulates these signals analytically, independently of the reconstruction's
    discretisation.  Here they come from the same kind of model on a grid `factor` times finer
    (voxels and scan), sampled at the coarse scan positions, so that the reconstruction does
    not invert exactly the model that made its data."""
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads as W

    from .binding import Model
    fcfg = fine_config(cfg, factor)
    with Model(fcfg["sensor"], fcfg["grid"], dtypes=("fp32",), filter=fcfg["band"]) as fm:
        x0 = torch.from_numpy(W.make_phantom(fcfg, 0).astype(np.float32)).to(device)
        s = fm.forward(x0, "fp32")[::factor, ::factor].contiguous()
    return s / s.abs().max()


def run_case(name, iters_l2=None, iters_l1=None, model=None):
    """MB-L2 and MB-L1 reconstructions of one ball-pair workload and their figures of merit."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads as W

    from .binding import Model
    cfg = W.config(name)
    so = cfg["solver"]
    own = model is None
    if own:
        model = Model(cfg["sensor"], cfg["grid"], dtypes=("fp32",), filter=cfg["band"])
    try:
        s = signals(cfg)
        x2, i2 = model.solve_lsqr(s, lam=-1.0, iters=iters_l2 or so["iters_l2"], inner="fp32")
        x1, i1 = model.solve_l1(s, lam=-1.0, iters=iters_l1 or so["iters_l1"], inner="fp32")
        out = dict(case=name, sep_um=cfg["phantom"]["sep_um"],
                   mb_l2=evaluate(x2.cpu().numpy(), cfg), mb_l1=evaluate(x1.cpu().numpy(), cfg),
                   lam_l2=i2["lam"], lam_l1=i1["lam"])
    finally:
        if own:
            model.close()
    return out


def main():
    for name in ("superres60", "superres40"):
        r = run_case(name)
        for k in ("mb_l2", "mb_l1"):
            r[k].pop("profile")
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
