"""Independent numpy restatements used to pin the oracle (tests only).

Written separately from the oracle's C code, vectorised instead of per-point,
from the definitions in Section IV-A (1) of the paper.
"""
from fractions import Fraction

import numpy as np

R, MIN, SAD, MAX = 0, 1, 2, 3


def _shift(f, ax, step):
    """Value of the neighbour at offset `step` along axis `ax` and whether it
    exists (edge cells have no neighbour beyond the boundary)."""
    n = f.shape[ax]
    g = np.zeros_like(f)
    ok = np.zeros(f.shape, dtype=bool)
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if step < 0:
        src[ax] = slice(0, n - 1)
        dst[ax] = slice(1, n)
    else:
        src[ax] = slice(1, n)
        dst[ax] = slice(0, n - 1)
    g[tuple(dst)] = f[tuple(src)]
    ok[tuple(dst)] = True
    return g, ok


def classify_np(f: np.ndarray) -> np.ndarray:
    f = np.asarray(f, dtype=np.float32)
    all_gt = np.ones(f.shape, bool)
    all_lt = np.ones(f.shape, bool)
    navail = np.zeros(f.shape, np.int32)
    pair_ok = np.ones(f.shape, bool)
    any_up = np.zeros(f.shape, bool)
    any_dn = np.zeros(f.shape, bool)
    for ax in range(f.ndim):
        if f.shape[ax] < 2:
            continue
        lo, ok_lo = _shift(f, ax, -1)
        hi, ok_hi = _shift(f, ax, +1)
        navail += ok_lo.astype(np.int32) + ok_hi.astype(np.int32)
        all_gt &= ~ok_lo | (lo > f)
        all_gt &= ~ok_hi | (hi > f)
        all_lt &= ~ok_lo | (lo < f)
        all_lt &= ~ok_hi | (hi < f)
        up = ok_lo & ok_hi & (lo > f) & (hi > f)
        dn = ok_lo & ok_hi & (lo < f) & (hi < f)
        pair_ok &= up | dn
        any_up |= up
        any_dn |= dn
    sad = pair_ok & any_up & any_dn
    out = np.full(f.shape, R, np.uint8)
    out[sad] = SAD
    out[all_lt] = MAX
    out[all_gt] = MIN
    out[navail == 0] = R
    return out


def q_exact(a: float, e: float) -> int:
    """floor((a + e) / (2e)) with exact rationals (Section II-C)."""
    A, E = Fraction(float(a)), Fraction(float(e))
    return int((A + E) // (2 * E))


def quantize_np(f: np.ndarray, e: float) -> np.ndarray:
    """Vectorised exact quantizer: float64 estimate, then exact edge tests.

    (2q +- 1) e is exact in float64 for |q| < 2^22 and float32 e."""
    a = np.asarray(f, dtype=np.float64)
    ed = float(np.float32(e))
    q = np.floor(a / (2 * ed) + 0.5).astype(np.int64)
    for _ in range(2):
        q += ((2 * q + 1) * ed <= a).astype(np.int64)
        q -= ((2 * q - 1) * ed > a).astype(np.int64)
    return q


def recon_np(q: np.ndarray, e: float) -> np.ndarray:
    return (2 * np.asarray(q)).astype(np.float32) * np.float32(e)


def face_neighbour_same_bin(q: np.ndarray) -> np.ndarray:
    """True where some face neighbour has the same bin index."""
    out = np.zeros(q.shape, bool)
    for ax in range(q.ndim):
        if q.shape[ax] < 2:
            continue
        for step in (-1, 1):
            g, ok = _shift(q, ax, step)
            out |= ok & (g == q)
    return out
