"""GPU parity of the band-pass filtering (Results; Methods, in vivo imaging): the filtered
model F A built on the device, the signal filter F s, and reconstructions of the filtered
problem, against the oracle's FIR (oracle.filters) on the same inputs."""
import numpy as np
import pytest

import workloads as W
from oracle import filters as ofil
from oracle import operators as oops
from oracle import solvers as osol
from tests.helpers import oracle_supports, oracle_table, rel_l2, rel_max

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_10173_amd as P  # noqa: E402

BAND = dict(f_lo_hz=0.5e6, f_hi_hz=80e6, half_taps=16)


def t64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _taps(g, f):
    return ofil.bandpass_taps(f["f_lo_hz"], f["f_hi_hz"], g["fs_hz"], f["half_taps"])


@pytest.mark.parametrize("name", ["mid", "mid7"])
def test_filtered_table_matches_oracle(name):
    cfg = W.config(name)
    g = cfg["grid"]
    h = _taps(g, BAND)
    Hf = ofil.filtered_table(oracle_table(name), h)
    lo, hi = oracle_supports(name)
    flo, fhi = ofil.filtered_supports(lo, hi, BAND["half_taps"], g["nt"])
    with P.Model(cfg["sensor"], g, dtypes=("fp64", "fp32"), filter=BAND) as m:
        H, glo, ghi = m.export_table()
        info = m.info()
    assert np.array_equal(glo, flo) and np.array_equal(ghi, fhi)
    assert rel_max(H, Hf) <= 1e-12
    assert info["mac_alg"] == oops.mac_alg(g, flo, fhi)


@pytest.mark.parametrize("nt,f", [(200, BAND), (1300, BAND), (1300, dict(BAND, half_taps=0)),
                                  (96, dict(f_lo_hz=1e6, f_hi_hz=120e6, half_taps=40))])
def test_signal_filter_matches_oracle(nt, f):
    """Ragged record lengths, one and several 1024-sample tiles, L = 0 and a long filter."""
    cfg = W.config("tiny")
    g = W.grid(5, 10e-6, 4, 10e-6, nt, 1, 0, ny=3)
    h = _taps(g, f)
    y = W.rng(40).standard_normal((g["ny"], g["nx"], nt))
    ref = ofil.filter_time(y, h)
    with P.Model(cfg["sensor"], g, dtypes=("fp64", "fp32"), filter=f) as m:
        y64 = m.filter_signals(t64(y)).cpu().numpy()
        y32 = m.filter_signals(t32(y)).cpu().numpy()
    assert rel_max(y64, ref) <= 1e-13
    assert rel_l2(y32, ref) <= 1e-6


def test_unfiltered_model_rejects_signal_filtering():
    cfg = W.config("tiny")
    with P.Model(cfg["sensor"], cfg["grid"], dtypes=("fp32",)) as m:
        y = torch.zeros(m.signal_shape, device="cuda")
        with pytest.raises(P.AroamError):
            m.filter_signals(y)


@pytest.mark.parametrize("inner,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_filtered_lsqr_matches_oracle(inner, tol):
    """Tikhonov LSQR on the filtered problem min ||F s - F A x||^2 + lam ||x||^2."""
    name = "mid"
    cfg = W.config(name)
    g = cfg["grid"]
    h = _taps(g, BAND)
    Hf = ofil.filtered_table(oracle_table(name), h)
    x0 = W.make_phantom(cfg, 0)
    clean = oops.forward(oracle_table(name), x0)
    s = clean + np.max(np.abs(clean)) * 10 ** (-cfg["snr_db"] / 20) * W.unit_noise(cfg, 0)
    sf = ofil.filter_time(s, h)
    shp_x, shp_s = x0.shape, s.shape
    A = lambda v: oops.forward(Hf, v.reshape(shp_x)).ravel()
    AT = lambda u: oops.adjoint(Hf, u.reshape(shp_s)).ravel()
    lam = osol.lam_l2(AT(sf.ravel()))
    x_ref, _ = osol.lsqr(A, AT, sf.ravel(), damp=np.sqrt(lam), iters=30)
    conv = t64 if inner == "fp64" else t32
    with P.Model(cfg["sensor"], g, dtypes=("fp64", "fp32"), filter=BAND) as m:
        sf_gpu = m.filter_signals(conv(s))
        x, info = m.solve_lsqr(sf_gpu, lam=-1.0, iters=30, inner=inner)
    assert abs(info["lam"] - lam) <= (1e-12 if inner == "fp64" else 1e-5) * lam
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
