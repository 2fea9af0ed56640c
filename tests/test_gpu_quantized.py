"""GPU parity of the reduced-precision applies against the oracle's quantised arithmetic
(oracle/quantize.py): the packed tables bit for bit, and the BF16 / FP8 applies element by
element against an FP64 apply of the quantised table and operand.

The quantised value of a table entry is decided from its FP64 value, which the HIP path's
table matches to about 1e-12 of the largest entry.  Entries that close to a rounding boundary
(`oracle.quantize.quantize_table`, delta = 1e-11 of the largest entry) may round either way:
they are checked to hold one of their two valid values, and their possible effect on an
output (one quantisation step times the operand) widens that output's bound.  Every other
entry must match exactly.

Element-wise bound of the applies: 1e-5 of the largest output entry (the FP32 accumulation of
exact products, as for the FP32 apply) plus the ambiguity term.  The FP8 apply runs on the
block-scaled FP8 MFMA, which adds up each 128-term product with less than FP32 precision:
measured on gfx950 over 768 random dot products of normal e4m3 codes, its error stays below
8.7e-5 of the sum of the absolute products.  Its bound therefore adds 2^-13 (1.2e-4) times
the output's sum of absolute products, |Hq| |xq| (every MFMA's error is bounded by its share
of that sum, and the FP32 accumulation of the MFMA results adds to them).  The error of each
apply against the unquantised FP64 oracle is reported beside it (the figures the precision
discussion uses); the bounds of those reports stay in tests/test_gpu_parity.py."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import model as omodel
from oracle import operators as oops
from oracle import quantize as Q
from tests.helpers import oracle_table, rel_l2, window_apply

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_10173_amd as P  # noqa: E402

SMALL = ["tiny", "mid", "mid7"]
# operand quantisation of each reduced-precision apply
OPERAND = {"bf16": "bf16", "fp8": "fp8-operand"}
TOL = 1e-5
FP8_MFMA_SUM = 2.0 ** -13  # relative accuracy of the FP8 MFMA's sums (see the docstring)

_MODELS = {}


def gpu_model(name, dtypes=("fp32", "bf16", "fp8")):
    key = (name, tuple(dtypes))
    if key not in _MODELS:
        cfg = W.config(name)
        print(f"[build model {name} {dtypes}]", flush=True)
        _MODELS[key] = P.Model(cfg["sensor"], cfg["grid"], dtypes=dtypes)
    return _MODELS[key]


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


@functools.lru_cache(maxsize=None)
def oracle_quantized(name, dtype):
    H = oracle_table(name)
    return Q.quantize_table(H, dtype, delta=1e-11 * np.max(np.abs(H)))


# Largest share of the nonzero entries that may lie within delta of a rounding boundary.  An
# entry far below the table's largest has an FP64 value known only to delta, which spans many
# of its FP32 steps (about a third of the FP32 entries) or, below ~1e-6 of the largest, a BF16
# step (about 1 %); e4m3 steps are relative to the block's scale, so almost none are.
AMBIGUOUS_SHARE = {"fp32": 0.5, "bf16": 0.02, "fp8": 1e-3}


def check_export(Hg, Hq, lo, hi, amb, label, dtype):
    n_amb = int(amb.sum())
    n_nz = max(1, np.count_nonzero(Hq))
    bad = int(np.count_nonzero(Hg[~amb] != Hq[~amb]))
    print(f"[{label}] {n_amb} of {n_nz} nonzero entries near a rounding boundary; "
          f"{bad} of the others differ", flush=True)
    assert bad == 0, label
    assert np.all((Hg[amb] >= lo[amb]) & (Hg[amb] <= hi[amb])), label
    assert n_amb <= AMBIGUOUS_SHARE[dtype] * n_nz


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_packed_table_matches_oracle_quantisation(name, dtype, adjoint):
    """The values each pack holds equal the oracle's rounding of the oracle's FP64 table: FP32
    and BF16 nearest-even, e4m3 codes nearest-even after the power-of-two scale of the entry's
    (offset, 16-depth block); the FP8 scales themselves equal the oracle's."""
    m = gpu_model(name)
    Hg, sc = m.export_quantized(dtype, adjoint)
    Hq, lo, hi, amb = oracle_quantized(name, dtype)
    check_export(Hg, Hq, lo, hi, amb, f"{name} {dtype} {'adjoint' if adjoint else 'forward'}",
                 dtype)
    if dtype == "fp8":
        H = oracle_table(name)
        sc_ref = Q.block_scales(H)
        blk_amb = np.stack([amb[:, :, 16 * b:16 * (b + 1)].any(axis=(2, 3))
                            for b in range(sc_ref.shape[2])], axis=2)
        assert np.array_equal(sc[~blk_amb], sc_ref[~blk_amb].astype(np.float32))


def _bound(op, lo, hi, v, dtype, Hq):
    """Largest change of op(Hq, v) that the ambiguous entries can make, plus, for FP8, the
    accuracy of the FP8 MFMA's sums times the output's sum of absolute products."""
    d = hi - lo
    b = op(d, np.abs(v)) if np.any(d) else 0.0
    if dtype == "fp8":
        b = b + FP8_MFMA_SUM * op(np.abs(Hq), np.abs(v))
    return b


def check_apply(got, ref, bound, label, oracle_err):
    scale = np.max(np.abs(ref))
    err = np.abs(got - ref)
    worst = float(np.max(err - bound) / scale)
    print(f"[{label}] max |gpu - quantised reference| - ambiguity = {worst:.2e} of the largest "
          f"entry; rel L2 vs the unquantised FP64 oracle {oracle_err:.2e}", flush=True)
    assert np.all(err <= TOL * scale + bound), label


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_quantized_applies_match_reference_elementwise(name, dtype):
    cfg = W.config(name)
    m = gpu_model(name)
    H = oracle_table(name)
    Hq, lo, hi, amb = oracle_quantized(name, dtype)
    x = W.random_image(cfg, 31).astype(np.float32)
    y = W.random_signal(cfg, 31).astype(np.float32)
    xq = Q.quantize_operand(x, OPERAND[dtype])
    yq = Q.quantize_operand(y, OPERAND[dtype])
    s = m.forward(t32(x), dtype).cpu().numpy()
    xa = m.adjoint(t32(y), dtype).cpu().numpy()
    s_ref = oops.forward(Hq, xq)
    xa_ref = oops.adjoint(Hq, yq)
    check_apply(s, s_ref, _bound(oops.forward, lo, hi, xq, dtype, Hq),
                f"{name} {dtype} forward", rel_l2(s, oops.forward(H, x)))
    check_apply(xa, xa_ref, _bound(oops.adjoint, lo, hi, yq, dtype, Hq),
                f"{name} {dtype} adjoint", rel_l2(xa, oops.adjoint(H, y)))


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_quantized_elementwise_cases_include_cut_layouts(dtype):
    """The element-wise cases above cover the kernels' partial-slot path: on these grids the
    launch planner cuts some reduced-precision tiles into pieces (the split BF16 / FP8 kernels
    then write partial sums that the slot-sum kernel adds), so a mistake in that path fails
    the element-wise comparison."""
    d = P.DTYPES[dtype]
    cut = []
    for name in SMALL:
        info = gpu_model(name).info()
        for kind, tiles in (("pieces", "row_tiles"), ("pieces_adj", "row_tiles_adj")):
            if info[kind][d] > info[tiles][d]:
                cut.append(f"{name} {kind} {info[kind][d]}/{info[tiles][d]}")
    print(f"[{dtype}] cut layouts: {cut}", flush=True)
    assert cut, f"no {dtype} layout of {SMALL} is cut"


@functools.lru_cache(maxsize=None)
def window400_blocks():
    """Oracle table of the 400x400 / 5 um / K = 40 workload at two whole 16-depth blocks (one
    capped by the 81 x 81 box, one at the focus), the depths the FP8 block scales need."""
    cfg = W.config("vessels400")
    ks = list(range(16, 32)) + list(range(128, 144))
    return ks, omodel.build_depth_slabs(cfg["sensor"], cfg["grid"], ks)


def _window_bound(op, lo, hi, Hq, v, dtype, y0, x0):
    """`_bound` of a 64 x 64 window of the full grid (the operators reach K offsets)."""
    b = window_apply(op, hi - lo, np.abs(v), y0, x0, 64)
    if dtype == "fp8":
        b = b + FP8_MFMA_SUM * window_apply(op, np.abs(Hq), np.abs(v), y0, x0, 64)
    return b


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_full_size_fine_step_windows_quantized(dtype):
    """Full-size 400x400 scan at 5 um, 256 depths, Nt 1024, cone capped at 81x81 offsets, in the
    launch configuration the bench times: an image nonzero at depths 30 and 128 (the forward)
    and a dense signal (the adjoint at those depths), compared element by element with the
    quantised reference on 64x64 windows (interior and corner)."""
    cfg = W.config("vessels400")
    g = cfg["grid"]
    m = gpu_model("vessels400", ("fp32", "bf16", "fp8"))
    ks_all, Hs = window400_blocks()
    Hq, lo, hi, amb = Q.quantize_table(Hs, dtype, delta=1e-11 * np.max(np.abs(Hs)))
    print(f"[window400 {dtype}] {int(amb.sum())} ambiguous entries", flush=True)
    pick = [ks_all.index(k) for k in (30, 128)]
    rng = W.rng(402)
    x = np.zeros((g["ny"], g["nx"], g["nz"]), dtype=np.float32)
    x[:, :, [30, 128]] = rng.standard_normal((g["ny"], g["nx"], 2))
    y = rng.standard_normal((g["ny"], g["nx"], g["nt"])).astype(np.float32)
    s = m.forward(t32(x), dtype).cpu().numpy()
    xa = m.adjoint(t32(y), dtype).cpu().numpy()
    # operands quantised over the whole vectors, as the apply does
    xq = Q.quantize_operand(x, OPERAND[dtype])[:, :, [30, 128]]
    yq = Q.quantize_operand(y, OPERAND[dtype])
    Hq2, lo2, hi2 = Hq[:, :, pick], lo[:, :, pick], hi[:, :, pick]
    for y0, x0 in ((170, 203), (0, 336)):
        s_ref = window_apply(oops.forward, Hq2, xq, y0, x0, 64)
        b_f = _window_bound(oops.forward, lo2, hi2, Hq2, xq, dtype, y0, x0)
        xa_ref = window_apply(oops.adjoint, Hq2, yq, y0, x0, 64)
        b_a = _window_bound(oops.adjoint, lo2, hi2, Hq2, yq, dtype, y0, x0)
        check_apply(s[y0:y0 + 64, x0:x0 + 64], s_ref, b_f, f"window400 {dtype} forward ({y0},{x0})",
                    rel_l2(s[y0:y0 + 64, x0:x0 + 64],
                           window_apply(oops.forward, Hs[:, :, pick], x[:, :, [30, 128]].astype(
                               np.float64), y0, x0, 64)))
        check_apply(xa[y0:y0 + 64, x0:x0 + 64][:, :, [30, 128]], xa_ref, b_a,
                    f"window400 {dtype} adjoint ({y0},{x0})",
                    rel_l2(xa[y0:y0 + 64, x0:x0 + 64][:, :, [30, 128]],
                           window_apply(oops.adjoint, Hs[:, :, pick], y.astype(np.float64), y0, x0,
                                        64)))
