"""Algorithmic work models of the kernels (for roofline fractions).

Peaks are MI355X's published figures; the VALU issue peak follows from the unit
counts: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions/s.
Expressed as FP32-FMA-equivalent FLOP (2 per lane-instruction) that is the
78.6 TFLOP/s non-packed vector rate, which equals the published FP64 vector
peak; packed FP32 is not used (disabled at build time).

Work per (query, critical point) pair is counted in VALU issue slots of the
minimal arithmetic the method needs on this path.  Every instruction takes one
issue slot; a quarter-rate transcendental (sin, cos, exp2, rcp, rsq) also takes
one, since its extra cycles run beside the following independent instructions
(a three-axis Fourier-plus-Laplace pass measured above the issue rate when they
were priced at four slots).  The projection u = <xi, x> costs 2n-1 (one mul,
n-1 fmas) and is shared by every kernel of a fused pass; then per kernel:

  Fourier   phase u*s/(2 pi) 1, reduction to [0,1) 2 (floor, sub), cvt 1,
            sin 1, cos 1, two (cvt + fma) 4                          -> 10
  Laplace   exponent fma 1, shift test 1, split 2 (floor, sub), cvt 1,
            exp2 1, cvt 1, cvt-to-int 1, ldexp 1, fma 1               -> 10
  Bessel    |z| < 8: z 1, v 2, degree-9 FP64 Horner 10, scale 1, cvt 2,
            sign 1, fma 1                                             -> 18
            |z| >= 8: z 1, cvt 1, rcp 1, w 2, two degree-5 Horner 12,
            phase reduction 4, cvt 1, sin 1, cos 1, rsq 1, combine 5,
            sign 1, cvt + fma 2                                       -> 33
  Fourier backward: phase and reduction 3, cvt 1, sin 1, cos 1, cvt 2,
            cotangent combine 3, n fmas                               -> 11 + n
  Laplace backward: the forward term without its shift test and with a
            mul for its fma 9, n fmas                                 -> 9 + n
  ECT       projection 2n-1, bin guess 6 (sub, mul, ceil, max, min, cvt),
            fix-up compares 2, LDS add 1                              -> 2n + 8
  Radon     as ECT plus one equality compare (the point or open-ray
            bin), over classical and ordinary points                  -> 2n + 9
Precompute is bounded by HBM: bytes = pixels read once + each list entry
written once (8 B: the packed vertex index and the int32 value) + list
offsets.  The exact representations are priced against HBM with the bytes the
operation cannot avoid: 8 B per critical point read (the stored list entry)
and 12 B per output entry (T and E) written.
"""
from __future__ import annotations

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 78.6          # 256 CU * 64 lanes * 2 FLOP * 2.4 GHz
VALU_SLOT_RATE = 256 * 64 * 2.4e9  # lane-instruction slots per second


def slots_per_pair(kind: str, n: int, small_fraction: float = 1.0) -> float:
    """kind: 'fourier', 'laplace', 'bessel', '+'-joined fused kernels, 'fourier_bwd', 'laplace_bwd',
    'ect' or 'radon'."""
    if kind == "ect":
        return 2 * n + 8
    if kind == "radon":
        return 2 * n + 9
    if kind == "fourier_bwd":
        return (2 * n - 1) + 11 + n
    if kind == "laplace_bwd":
        return (2 * n - 1) + 9 + n
    per = {"fourier": 10.0, "laplace": 10.0,
           "bessel": small_fraction * 18.0 + (1.0 - small_fraction) * 33.0}
    parts = kind.split("+")
    if any(p not in per for p in parts):
        raise ValueError(kind)
    return (2 * n - 1) + sum(per[p] for p in parts)


def alu_roofline(kind: str, n: int, pairs: float, seconds: float, small_fraction: float = 1.0) -> dict:
    flop = 2.0 * slots_per_pair(kind, n, small_fraction) * pairs
    achieved = flop / seconds / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / VALU_PEAK_TFLOPS}


def alu_roofline_parts(parts, seconds: float) -> dict:
    """One launch doing several kinds of work: parts = [(kind, n, pairs, small_fraction), ...]."""
    flop = sum(2.0 * slots_per_pair(k, n, sf) * pairs for k, n, pairs, sf in parts)
    achieved = flop / seconds / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / VALU_PEAK_TFLOPS}


def hbm_roofline(nbytes: float, seconds: float) -> dict:
    achieved = nbytes / seconds / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS}
