"""Pins of the oracle's reduced-precision definitions (oracle/quantize.py) against the formats
themselves: the OCP e4m3 code table's fixed points, nearest rounding with ties to even checked
by brute force over all codes (e4m3) or both neighbours (BF16), the power-of-two block scale's
defining inequalities, and the ambiguity marking at planted rounding boundaries."""
import numpy as np
import pytest

from oracle import quantize as Q


def test_e4m3_code_table_fixed_points():
    """OCP e4m3 (the 'fn' variant without infinities): 0x38 = 1, 0x7e = 448 the largest finite,
    0x7f NaN, 0x08 = 2^-6 the smallest normal, 0x01 = 2^-9 the smallest subnormal, 0x80 = -0,
    sign in bit 7; the positive finite codes are strictly increasing, 126 of them."""
    v = Q.e4m3_value(np.arange(256, dtype=np.uint8))
    assert v[0x38] == 1.0 and v[0x7E] == 448.0 and np.isnan(v[0x7F]) and np.isnan(v[0xFF])
    assert v[0x08] == 2.0 ** -6 and v[0x01] == 2.0 ** -9 and v[0x00] == 0.0
    assert v[0x80] == 0.0 and np.signbit(v[0x80])
    pos = v[1:0x7F]
    assert len(pos) == 126 and np.all(np.diff(pos) > 0)
    assert np.array_equal(v[0x81:0xFF], -v[0x01:0x7F])
    # normals: 8 mantissa steps per binade, binade [2^(e-7), 2^(e-6)) for exponent field e
    for e in range(1, 16):
        for mnt in range(8):
            c = (e << 3) | mnt
            if c < 0x7F:
                assert v[c] == 2.0 ** (e - 7) * (1 + mnt / 8)


def _nearest_even(x, grid_vals, grid_codes):
    """Brute force: the representable value nearest to x, ties to the code with an even
    mantissa bit."""
    d = np.abs(grid_vals - x)
    best = np.flatnonzero(d == d.min())
    if len(best) == 1:
        return grid_vals[best[0]]
    even = [i for i in best if grid_codes[i] % 2 == 0]
    assert len(even) == 1
    return grid_vals[even[0]]


def test_e4m3_rounding_is_nearest_ties_to_even():
    codes = np.concatenate([np.arange(0, 0x7F), np.arange(0x81, 0xFF)]).astype(np.uint8)
    vals = Q.e4m3_value(codes)
    rng = np.random.default_rng(0)
    mags = np.exp(rng.uniform(np.log(2.0 ** -12), np.log(448.0), 3000))
    xs = np.concatenate([mags, -mags[:500]])
    # every midpoint between neighbours, and points just beside them
    pos = np.sort(vals[vals > 0])
    mids = 0.5 * (pos[1:] + pos[:-1])
    xs = np.concatenate([xs, mids, np.nextafter(mids.astype(np.float32), 0).astype(float),
                         np.nextafter(mids.astype(np.float32), 1e9).astype(float), [2.0 ** -10]])
    xs = xs.astype(np.float32).astype(np.float64)
    got = Q.e4m3(xs)
    for x, g in zip(xs, got):
        assert g == _nearest_even(x, vals, codes), x


def test_bf16_rounding_is_nearest_ties_to_even():
    """Against both BF16 neighbours of each FP32 value (the value with its low 16 bits
    cleared, and the next BF16 above it in magnitude)."""
    rng = np.random.default_rng(1)
    x32 = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    bits = x32.view(np.uint32)
    ties = ((bits & 0xFFFF0000) | 0x8000).view(np.float32)          # exact midpoints
    x32 = np.concatenate([x32, ties])
    bits = x32.view(np.uint32)
    down = (bits & 0xFFFF0000).view(np.float32).astype(np.float64)
    up = ((bits & 0xFFFF0000) + 0x10000).view(np.float32).astype(np.float64)
    x = x32.astype(np.float64)
    got = Q.bf16(x)
    dd, du = np.abs(x - down), np.abs(up - x)
    want = np.where(dd < du, down, np.where(du < dd, up,
                    np.where(((bits >> 16) & 1) == 0, down, up)))
    assert np.array_equal(got, want)


def test_fp32_then_bf16_is_the_table_rounding():
    """The BF16 table is the FP32 table rounded once more: a value just above a BF16 midpoint
    in FP64 that rounds to the midpoint in FP32 then goes to the even neighbour."""
    mid = 1.0 + 2.0 ** -8                       # midpoint between BF16 1 and 1 + 2^-7
    v = mid + 2.0 ** -40                        # above the midpoint, but FP32 rounds it onto it
    assert Q.fp32(v) == mid
    assert Q.bf16(v) == 1.0


def test_block_scale_inequalities():
    rng = np.random.default_rng(2)
    amax = np.exp(rng.uniform(-40, 10, 500))
    amax[:5] = 448.0 * 2.0 ** np.arange(-2, 3)     # exact powers of two times 448
    sc = Q.pow2_scale(amax)
    m, e = np.frexp(sc)
    assert np.all(m == 0.5)                           # powers of two
    assert np.all(sc >= amax / 448.0) and np.all(sc / 2 < amax / 448.0)
    assert np.array_equal(sc[:5], 2.0 ** np.arange(-2, 3))
    assert Q.pow2_scale(np.array([0.0]))[0] == 0.0


def test_fp8_table_codes_span_the_format():
    """Each block's largest entry lands in the top binade of e4m3 (224 .. 448 after scaling),
    and every entry is within half an e4m3 step of its value (relative 2^-4 for normals)."""
    rng = np.random.default_rng(3)
    H = rng.standard_normal((3, 3, 40, 30)) * np.exp(rng.uniform(-8, 8, (3, 3, 40, 1)))
    H[1, 1, 20:, :] = 0.0
    sc = Q.block_scales(H)
    Hq = Q.quantize_table_values(H, "fp8")
    s = Q._expand(sc, H.shape[2])
    with np.errstate(invalid="ignore", divide="ignore"):
        scaled = np.abs(np.where(s > 0, Hq / np.where(s > 0, s, 1), 0))
    top = np.stack([scaled[:, :, 16 * b:16 * (b + 1)].max(axis=(2, 3)) for b in range(3)], axis=2)
    assert sc[1, 1, 2] == 0.0 and np.all(Hq[1, 1, 32:] == 0.0)
    nonzero = sc > 0
    assert np.all((top[nonzero] >= 224.0) & (top[nonzero] <= 448.0))
    q = H / np.where(s > 0, s, 1)
    err = np.abs(Hq / np.where(s > 0, s, 1) - q)
    normal = np.abs(q) >= 2.0 ** -6
    assert np.all(err[normal] <= np.abs(q[normal]) * 2.0 ** -4 + 1e-300)
    assert np.all(err[~normal] <= 2.0 ** -10)


def test_ambiguity_marks_planted_bf16_boundary():
    """A table entry decides its BF16 value through its FP32 rounding: an entry on the FP32
    midpoint just above the BF16 midpoint 1 + 2^-8 rounds (ties to even) onto that BF16
    midpoint and then down to 1, while any larger entry rounds up to 1 + 2^-7, so it is
    ambiguous with both values valid.  An entry a quarter BF16 step above 1 is not, and neither
    are zeros."""
    rng = np.random.default_rng(4)
    H = np.zeros((1, 1, 16, 8))
    H[0, 0, :, :4] = rng.uniform(1.0, 2.0, (16, 4))
    H[0, 0, 0, 0] = 1.0 + 2.0 ** -8 + 2.0 ** -24
    H[0, 0, 0, 1] = 1.0 + 2.0 ** -10
    Hq, lo, hi, amb = Q.quantize_table(H, "bf16", delta=1e-12)
    assert Hq[0, 0, 0, 0] == 1.0
    assert amb[0, 0, 0, 0] and lo[0, 0, 0, 0] == 1.0 and hi[0, 0, 0, 0] == 1.0 + 2.0 ** -7
    assert not amb[0, 0, 0, 1] and Hq[0, 0, 0, 1] == 1.0
    assert np.all((lo <= Hq) & (Hq <= hi))
    assert not np.any(amb[H == 0.0])


def test_ambiguity_marks_planted_fp8_scale_boundary():
    """A block whose amax is exactly 448 (scale 1, but 2 for a slightly larger amax) is
    undecided as a whole: its entries may take the values of either scale, and those that
    differ are marked; a block with amax 300 keeps its unique values."""
    rng = np.random.default_rng(5)
    H = np.zeros((1, 2, 16, 8))
    H[0, :, :, :4] = rng.uniform(0.001, 0.05, (2, 16, 4))  # subnormal at scale 2 below 0.03125
    H[0, 0, 0, 0] = 448.0
    H[0, 1, 0, 0] = 300.0
    Hq, lo, hi, amb = Q.quantize_table(H, "fp8", delta=1e-12)
    q1 = Q.quantize_table_values(H[:, :1], "fp8", np.ones((1, 1, 1)))
    q2 = Q.quantize_table_values(H[:, :1], "fp8", 2 * np.ones((1, 1, 1)))
    assert np.array_equal(lo[:, :1], np.minimum(q1, q2)) and np.array_equal(hi[:, :1], np.maximum(q1, q2))
    assert np.any(amb[0, 0]) and np.array_equal(amb[0, 0], (q1 != q2)[0, 0])
    assert not np.any(amb[0, 1])
    assert np.all((lo <= Hq) & (Hq <= hi))


def test_fp8_operand_scales_per_block_of_the_fast_axis():
    rng = np.random.default_rng(5)
    v = rng.standard_normal((3, 4, 150)).astype(np.float32)
    v[..., 64:128] *= 1e-3
    v[..., 128:] = 0.0
    sc = Q.operand_scales(v, 150)
    assert sc.shape == (3,) and sc[2] == 0.0
    for b in range(2):
        amax = np.max(np.abs(v[..., 64 * b:64 * (b + 1)]))
        assert sc[b] >= amax / 448 > sc[b] / 2
    q = Q.quantize_operand(v, "fp8-operand")
    s = np.repeat(sc, 64)[:150]
    assert np.all(q[..., 128:] == 0.0)
    s1 = np.where(s > 0, s, 1.0)
    assert np.all(np.abs(q - v) / s1 <= 16.0)        # half a step of the top binade [256, 448]
    assert np.all(np.abs(q - v) <= np.abs(v) * 2.0 ** -4 + s * 2.0 ** -10)
    # codes of the scaled values are e4m3 codes: decoding q / s gives back exactly q / s
    assert np.array_equal(Q.e4m3(q / s1), q / s1)
