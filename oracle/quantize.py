"""Reduced-precision tables and operands: what the BF16 and FP8 applies multiply.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper's model is FP64 (it gives
no precision); the reduced-precision applies are this implementation's, and this module
states their arithmetic as plain definitions, with PyTorch's format conversions as the
library primitive for rounding:

* BF16 table: every entry of the FP64 table rounded to FP32, then to BF16 (nearest, ties to
  even).  BF16 operand: the FP32 vector rounded to BF16 the same way.
* FP8 table (OCP e4m3: 4 exponent bits of bias 7, 3 mantissa bits, largest finite 448): one
  scale per (lateral offset, block of 16 depths), the smallest power of two at or above
  amax / 448 with amax the largest |entry| of the FP64 table in the block; each entry is
  e4m3(fp32(v / scale)) * scale, rounded to nearest with ties to even.
* FP8 operand: e4m3 codes of the FP32 vector divided by a power-of-two scale per block of 64
  along its fast axis (depth of an image, time of a signal), chosen like the table's from the
  block's amax over all scan positions (see `operand_scales`); products are formed from the
  decoded values and accumulated in at least FP32.

A quantised value is decided by comparing the FP64 table entry with rounding boundaries.  The
table of the HIP path agrees with the oracle's table only to about 1e-12 of its largest
entry, so an entry lying that close to a boundary may round either way on the two sides:
`quantize_table` marks such entries as ambiguous and gives the two values they may take, so
that tests compare the unique decisions exactly and check the rest for validity.
"""
from __future__ import annotations

import math

import numpy as np
import torch

E4M3_MAX = 448.0
BLOCK = 16          # depths per scale block of the FP8 table
OPERAND_BLOCK = 64  # entries of the fast axis per scale block of the FP8 operand


def fp32(a):
    """FP64 values rounded to FP32 (nearest, ties to even), returned as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16(a):
    """Values rounded to FP32 and then to BF16 (nearest, ties to even), as float64."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32)))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def e4m3_codes(a):
    """e4m3 codes (uint8) of FP32-representable values |a| <= 448, nearest with ties to even."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32)))
    return t.to(torch.float8_e4m3fn).view(torch.uint8).numpy()


def e4m3_value(codes):
    """Values (float64) of e4m3 codes (uint8 array)."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(codes, dtype=np.uint8)))
    return t.view(torch.float8_e4m3fn).to(torch.float64).numpy()


def e4m3(a):
    """FP32-representable values rounded to e4m3, as float64."""
    return e4m3_value(e4m3_codes(a))


def pow2_scale(amax):
    """Smallest power of two >= amax / 448 (elementwise; 0 where amax is 0)."""
    amax = np.asarray(amax, dtype=np.float64)
    out = np.zeros_like(amax)
    for idx, a in np.ndenumerate(amax):
        if a > 0:
            m, e = math.frexp(a / E4M3_MAX)     # a / 448 = m 2^e, 0.5 <= m < 1
            out[idx] = math.ldexp(1.0, e - 1 if m == 0.5 else e)
    return out


def block_scales(H):
    """Scale of each (offset, 16-depth block) of a table H[dy][dx][k][n]: [W][W][ceil(nz/16)]."""
    W1, W2, nz, _ = H.shape
    nblk = -(-nz // BLOCK)
    amax = np.zeros((W1, W2, nblk))
    for b in range(nblk):
        amax[:, :, b] = np.max(np.abs(H[:, :, BLOCK * b:BLOCK * (b + 1), :]), axis=(2, 3))
    return pow2_scale(amax)


def _expand(scales, nz):
    """Block scales [W][W][nblk] broadcast to [W][W][nz][1]."""
    return np.repeat(scales, BLOCK, axis=2)[:, :, :nz, None]


def quantize_table_values(H, dtype, scales=None):
    """The table the dtype's apply multiplies (float64, same layout as H)."""
    if dtype == "fp32":
        return fp32(H)
    if dtype == "bf16":
        return bf16(H)
    if dtype == "fp8":
        sc = block_scales(H) if scales is None else scales
        s = _expand(sc, H.shape[2])
        with np.errstate(invalid="ignore", divide="ignore"):
            v = np.where(s > 0, H / np.where(s > 0, s, 1.0), 0.0)
        return e4m3(fp32(v)) * s
    raise ValueError(dtype)


def quantize_table(H, dtype, delta):
    """Quantised table plus the entries whose rounding another table within `delta` (absolute)
    of H could decide differently.

    Returns (Hq, lo, hi, amb): Hq quantises H itself; lo and hi quantise H - delta and
    H + delta (the quantisers are monotone, so any table within delta of H quantises each entry
    into [min(lo, hi), max(lo, hi)]); amb marks entries where lo != hi.  Entries that are zero
    (outside the band or the footprint) are exactly zero in both tables and are not perturbed.
    For FP8, a block whose scale could differ (amax / 448 within delta / 448 of a power of two)
    is ambiguous as a whole, and its entries may take the values of either scale."""
    Hq = quantize_table_values(H, dtype)
    d = np.where(H != 0.0, delta, 0.0)  # entries outside the band are zero on both sides
    if dtype != "fp8":
        lo = quantize_table_values(H - d, dtype)
        hi = quantize_table_values(H + d, dtype)
    else:
        sc = block_scales(H)
        lo = quantize_table_values(H - d, dtype, sc)
        hi = quantize_table_values(H + d, dtype, sc)
        W1, W2, nz, _ = H.shape
        nblk = sc.shape[2]
        amax = np.zeros((W1, W2, nblk))
        for b in range(nblk):
            amax[:, :, b] = np.max(np.abs(H[:, :, BLOCK * b:BLOCK * (b + 1), :]), axis=(2, 3))
        s_lo = pow2_scale(np.maximum(amax - delta, 0.0))
        s_hi = pow2_scale(amax + delta)
        bad = (s_lo != sc) | (s_hi != sc)
        if np.any(bad):
            for sc2 in (s_lo, s_hi):
                alt = quantize_table_values(H, dtype, np.where(bad, sc2, sc))
                lo = np.minimum(lo, alt)
                hi = np.maximum(hi, alt)
    lo, hi = np.minimum(lo, hi), np.maximum(lo, hi)
    return Hq, lo, hi, lo != hi


def operand_scales(v, axis_len, block=OPERAND_BLOCK):
    """Power-of-two scale per block of `block` entries along the fast axis of a vector
    [ny][nx][L]: the smallest power of two >= amax / 448 of the block over all scan positions
    (0 for a block of zeros)."""
    v = np.asarray(v, dtype=np.float64).reshape(-1, axis_len)
    nblk = -(-axis_len // block)
    amax = np.array([np.max(np.abs(v[:, block * b:block * (b + 1)])) for b in range(nblk)])
    return pow2_scale(amax)


def quantize_operand(v, dtype):
    """The vector operand the dtype's apply multiplies (float64, same shape as v).  v holds
    FP32 values (the caller's vectors are FP32)."""
    v = np.asarray(v, dtype=np.float32).astype(np.float64)
    if dtype == "fp32":
        return v
    if dtype == "bf16":
        return bf16(v)
    if dtype == "fp8-operand":
        L = v.shape[-1]
        sc = np.repeat(operand_scales(v, L), OPERAND_BLOCK)[:L]
        with np.errstate(invalid="ignore", divide="ignore"):
            q = np.where(sc > 0, v / np.where(sc > 0, sc, 1.0), 0.0)
        return e4m3(fp32(q)) * sc
    raise ValueError(dtype)
