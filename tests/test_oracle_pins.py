"""Pins of the oracle's decompression against what the paper and the
mathematics fix, each chosen so that a plausible slip in the oracle fails it:

- relative order (Section III-C, Section IV-B (2)): restored extrema of one
  class and bin keep the order of their original values, for minima as for
  maxima, and extrema the quantizer kept are not moved;
- the refinement window (Section IV-B (3), Eq. (1)-(2)): an isolated refined
  saddle equals the normalised Gaussian mean over the Euclidean ball of
  radius floor(k/2), computed here in exact rational arithmetic, for k = 5
  and 7 in 2D and 3D;
- the schedule: within a colour phase every candidate reads the phase-start
  values (Jacobi), across phases a later colour reads the earlier commits;
- the evaluation counts (Section III-B) against a recount from an
  independently written classifier;
- the rank reading (a flattened and an unflattened maximum in one bin and
  block): only flattened extrema are ranked, and the unflattened one stays.

Every expected value comes from numpy, Fraction arithmetic or the field
itself, never from the oracle's own helpers.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2602_17552_amd import datagen
from np_ref import MAX, MIN, R, SAD, classify_np, face_neighbour_same_bin, quantize_np, recon_np
import stream_format as sf


def _decoded(ora, f, eb, mode="rel", **params):
    rc, s = ora.compress(f, eb, mode, **params)
    assert rc == ora.OK
    b = bytes(s)
    h = sf.parse_header(b)
    rc, out, st = ora.decompress(s, f.shape)
    assert rc == ora.OK
    e = np.float32(h["e"])
    q = quantize_np(f, e)
    return h, q, recon_np(q, e), out, st


# --- relative order -------------------------------------------------------

ORDER_CASES = [
    ("noise2d_block", lambda: datagen.noise((60, 64), seed=21), 0.6, 0),
    ("noise2d_field", lambda: datagen.noise((40, 50), seed=22), 0.6, 1),
    ("noise3d_block", lambda: datagen.noise((12, 14, 16), seed=23), 0.5, 0),
    ("noise3d_field", lambda: datagen.noise((10, 12, 14), seed=24), 0.5, 1),
]


@pytest.mark.parametrize("name,gen,eb,scope", ORDER_CASES, ids=[c[0] for c in ORDER_CASES])
def test_restored_extrema_keep_their_order(ora, name, gen, eb, scope):
    f = gen()
    h, q, rq, out, st = _decoded(ora, f, eb, "abs", rank_scope=scope)
    assert st["budget_skips"] == 0
    lab = classify_np(f).reshape(-1)
    flat = face_neighbour_same_bin(q).reshape(-1)
    a, d, qq, r0 = f.reshape(-1), out.reshape(-1), q.reshape(-1), rq.reshape(-1)
    ext = (lab == MIN) | (lab == MAX)
    # extrema the quantizer kept are not moved; lost ones are moved
    assert np.array_equal(d[ext & ~flat].view(np.uint32), r0[ext & ~flat].view(np.uint32))
    assert np.all(d[ext & flat] != r0[ext & flat])
    # every pair of lost extrema of one class, bin and scope keeps the order
    # (or the tie) of its original values
    pairs = {MIN: [0, 0], MAX: [0, 0]}
    idx = np.nonzero(ext & flat)[0]
    groups = {}
    for p in idx:
        key = (int(lab[p]), int(qq[p]), int(p // 64) if scope == 0 else 0)
        groups.setdefault(key, []).append(p)
    for (cls, _, _), members in groups.items():
        for i, j in itertools.combinations(members, 2):
            so, sd = np.sign(float(a[i]) - float(a[j])), np.sign(float(d[i]) - float(d[j]))
            assert so == sd, (name, cls, i, j, a[i], a[j], d[i], d[j])
            pairs[cls][0 if so != 0 else 1] += 1
    # the check is not vacuous for either class
    assert pairs[MIN][0] >= 5 and pairs[MAX][0] >= 5, pairs


# --- refinement window ----------------------------------------------------

def ball(ndim, r):
    """Offsets of {q != p : |q - p|_2 <= r}, enumerated directly."""
    rng = range(-r, r + 1)
    axes = [rng] * ndim
    return [o for o in itertools.product(*axes) if 0 < sum(x * x for x in o) <= r * r]


def test_window_sizes():
    assert [len(ball(2, r)) for r in (1, 2, 3)] == [4, 12, 28]
    assert [len(ball(3, r)) for r in (1, 2, 3)] == [6, 32, 122]


def _f32_nearest(x: Fraction) -> np.float32:
    """The float32 nearest to the rational x (ties to even)."""
    c = np.float32(float(x))
    cands = [np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))]
    best = min(cands, key=lambda v: (abs(Fraction(float(v)) - x), int(v.view(np.uint32)) & 1))
    return np.float32(best)


def _candidate(vals, shape, p, r, w, override=None):
    """Normalised Gaussian mean over the in-grid ball around p, exactly:
    sum w[d2] * value / sum w[d2], the weights being the stored float32
    values of exp(-d2 / (2 sigma^2))."""
    num, den = Fraction(0), Fraction(0)
    for o in ball(len(shape), r):
        c = tuple(pi + oi for pi, oi in zip(p, o))
        if any(ci < 0 or ci >= n for ci, n in zip(c, shape)):
            continue
        v = override[c] if override and c in override else vals[c]
        wt = Fraction(float(w[sum(x * x for x in o)]))
        num += wt * Fraction(float(v))
        den += wt
    return num / den


def _ulps(a, b):
    ia, ib = int(np.float32(a).view(np.int32)), int(np.float32(b).view(np.int32))
    ka = ia if ia >= 0 else -(ia & 0x7FFFFFFF)
    kb = ib if ib >= 0 else -(ib & 0x7FFFFFFF)
    return abs(ka - kb)


WINDOW_CASES = [
    ("2d_k5", lambda: datagen.sinusoids_2d(80, 96, 8, seed=12, noise_sd=2e-3), 5e-2, 2, 5),
    ("2d_k7", lambda: datagen.checker_2d(60, 64, seed=1), 0.3, 2, 7),
    ("3d_k5", lambda: datagen.grf_3d(24, 28, 32, seed=13), 0.1, 3, 5),
    ("3d_k7", lambda: datagen.grf_3d(24, 28, 32, seed=13), 0.3, 3, 7),
]


def _refined(h, lab, rq, out):
    return (lab == SAD) & (out != rq)


@pytest.mark.parametrize("name,gen,eb,ndim,k", WINDOW_CASES, ids=[c[0] for c in WINDOW_CASES])
def test_isolated_refined_saddle_is_the_window_mean(ora, name, gen, eb, ndim, k):
    f = gen()
    h, q, rq, out, st = _decoded(ora, f, eb)
    assert (f.ndim, h["k_size"]) == (ndim, k)
    sigma = {3: 0.5, 5: 0.75, 7: 1.0}[k]
    w = [np.float32(math.exp(-d2 / (2 * sigma * sigma))) for d2 in range(10)]
    assert [float(x) for x in w] == h["w"]
    r = k // 2
    lab = classify_np(f)
    ref = _refined(h, lab, rq, out)
    pts = [tuple(int(x) for x in p) for p in np.argwhere(ref)]
    exact = near = 0
    for p in pts:
        if any(ref[tuple(pi + oi for pi, oi in zip(p, o))] for o in ball(ndim, r)
               if all(0 <= pi + oi < n for pi, oi, n in zip(p, o, f.shape))):
            continue  # another refined point in the window: not isolated
        want = _f32_nearest(_candidate(out, f.shape, p, r, w))
        u = _ulps(out[p], want)
        assert u <= 1, (name, p, out[p], want)
        exact += u == 0
        near += 1
    assert near >= 5, (name, near, len(pts))
    assert exact >= 0.9 * near, (name, exact, near)


# --- schedule -------------------------------------------------------------

SCHED_CASES = [
    ("2d_k7", lambda: datagen.checker_2d(60, 64, seed=1), 0.3),
    ("2d_k7_waves", lambda: datagen.sinusoids_2d(120, 128, 8, seed=14, noise_sd=2e-3), 0.3),
    ("3d_k7", lambda: datagen.grf_3d(24, 28, 32, seed=13), 0.3),
    ("3d_k5", lambda: datagen.checker_3d(16, 20, 24, seed=1), 0.1),
]


def _colour(p):
    if len(p) == 2:
        y, x = p
        return (x + 2 * y) % 5
    z, y, x = p
    return (x + 2 * y + 3 * z) % 7


def test_schedule_cases_and_counts():
    # two points of one colour are at L1 distance >= 3 (2D and 3D), so a
    # same-colour pair shares a window only from radius sqrt(3) on
    for ndim, ncol in ((2, 5), (3, 7)):
        for o in itertools.product(range(-4, 5), repeat=ndim):
            if any(o) and sum(abs(x) for x in o) < 3:
                p = (5,) * ndim
                assert _colour(p) != _colour(tuple(a + b for a, b in zip(p, o)))


def test_phase_schedule(ora):
    """One round (max_rounds = 1), pairs of refined saddles inside each
    other's window and with no other refined point in either window: a pair
    of one colour must match Jacobi (both candidates from the phase-start
    values); a pair of two colours must match the lower colour first, the
    higher reading its commit.  The other schedule must differ by more than
    an ulp on some pairs of each kind, so that the pin can fail."""
    seen = {"same": 0, "diff": 0}
    for name, gen, eb in SCHED_CASES:
        f = gen()
        h, q, rq, out, st = _decoded(ora, f, eb, max_rounds=1)
        assert st["rounds"] == 1
        k = h["k_size"]
        r = k // 2
        w = [np.float32(x) for x in h["w"]]
        lab = classify_np(f)
        ref = _refined(h, lab, rq, out)
        shape = f.shape
        pts = [tuple(int(x) for x in p) for p in np.argwhere(ref)]
        offs = ball(f.ndim, r)

        def window(p):
            return [tuple(pi + oi for pi, oi in zip(p, o)) for o in offs
                    if all(0 <= pi + oi < n for pi, oi, n in zip(p, o, shape))]

        for p1 in pts:
            w1 = window(p1)
            others = [c for c in w1 if ref[c]]
            if len(others) != 1:
                continue
            p2 = others[0]
            if p2 < p1:
                continue
            w2 = window(p2)
            if [c for c in w2 if ref[c] and c != p1]:
                continue
            pre1, pre2 = rq[p1], rq[p2]  # a lost saddle's pre-refinement value
            if _colour(p1) == _colour(p2):
                v1 = _f32_nearest(_candidate(out, shape, p1, r, w, {p2: pre2}))
                v2 = _f32_nearest(_candidate(out, shape, p2, r, w, {p1: pre1}))
                alt2 = _f32_nearest(_candidate(out, shape, p2, r, w, {p1: v1}))  # sequential
                kind = "same"
            else:
                a, b = (p1, p2) if _colour(p1) < _colour(p2) else (p2, p1)
                va = _f32_nearest(_candidate(out, shape, a, r, w, {b: rq[b]}))
                vb = _f32_nearest(_candidate(out, shape, b, r, w, {a: va}))
                alt2 = _f32_nearest(_candidate(out, shape, b, r, w, {a: rq[a]}))  # Jacobi across phases
                (v1, v2), p1, p2 = (va, vb), a, b
                kind = "diff"
            assert _ulps(out[p1], v1) <= 1 and _ulps(out[p2], v2) <= 1, (name, kind, p1, p2)
            if _ulps(alt2, v2) > 1:
                seen[kind] += 1
    assert seen["same"] >= 1 and seen["diff"] >= 1, seen


# --- evaluation counts ----------------------------------------------------

def _recount(orig, recon):
    lo, lr = classify_np(orig).reshape(-1), classify_np(recon).reshape(-1)
    fn = (lo != R) & (lr == R)
    c = [int(fn.sum()), int(((lo == R) & (lr != R)).sum()), int(((lo != R) & (lr != R) & (lo != lr)).sum())]
    c += [int((lo == k).sum()) for k in (R, MIN, SAD, MAX)]
    c += [int((fn & (lo == k)).sum()) for k in (R, MIN, SAD, MAX)]
    err = float(np.max(np.abs(orig.astype(np.float64) - recon.astype(np.float64))))
    return c, err


def test_eval_against_recount(ora):
    rng = np.random.default_rng(31)
    cases = []
    f = datagen.sinusoids_2d(50, 70, 8, seed=32)
    rc, s = ora.compress(f, 1e-2, "rel")
    cases.append((f, ora.decompress(s, f.shape)[1]))
    rc, s = ora.compress(f, 1e-2, "rel", topo=False)
    cases.append((f, ora.decompress(s, f.shape)[1]))
    g = datagen.grf_3d(10, 12, 14, seed=33)
    cases.append((g, (g + rng.normal(0, 0.05, g.shape)).astype(np.float32)))  # FP and FT too
    n = datagen.noise((30, 40), seed=34)
    cases.append((n, np.round(n * 2).astype(np.float32) / 2))
    for orig, recon in cases:
        ev = ora.eval_topology(orig, recon)
        c, err = _recount(orig, recon)
        got = [ev["FN"], ev["FP"], ev["FT"], ev["n_r"], ev["n_min"], ev["n_sad"], ev["n_max"],
               0, ev["FN_min"], ev["FN_sad"], ev["FN_max"]]
        assert got == c
        assert ev["max_abs_err"] == err
    # the random perturbation produces every error class
    c, _ = _recount(*cases[2])
    assert c[0] > 0 and c[1] > 0 and c[2] > 0


# --- rank reading ---------------------------------------------------------

def test_flattened_and_kept_maxima_in_one_bin_and_block(ora):
    """Row y = 1 of a 3 x 64 grid is one block.  With e = 0.5 (bin 0 is
    [-0.5, 0.5)) and a background of -0.6 (bin -1): maximum u = 0.25 keeps
    every neighbour in a lower bin; maxima p = 0.3 and p2 = 0.2 each have a
    neighbour in bin 0, so plain SZp flattens them.  p ranks above p2 only:
    delta = 2, 1 and u is unranked and unmoved.  (Counting u as well would
    give p delta 3 and leave every pairwise order as it is: u stays at the
    bin centre below both moved maxima either way.)"""
    f = np.full((3, 64), -0.6, np.float32)
    f[1, 10] = 0.25          # u
    f[1, 20] = 0.3           # p
    f[1, 21] = 0.1           # p's neighbour in bin 0
    f[1, 30] = 0.2           # p2
    f[1, 31] = 0.05          # p2's neighbour in bin 0
    lab = classify_np(f)
    assert lab[1, 10] == lab[1, 20] == lab[1, 30] == MAX
    rc, s = ora.compress(f, 0.5, "abs")
    assert rc == ora.OK
    b = bytes(s)
    h = sf.parse_header(b)
    delta = sf.decode_map(b, h, "R").reshape(f.shape)
    assert (delta[1, 10], delta[1, 20], delta[1, 30]) == (0, 2, 1)
    rc, out, _ = ora.decompress(s, f.shape)
    zero = np.float32(0.0)
    up = lambda v, k: v if k == 0 else up(np.nextafter(v, np.float32(np.inf)), k - 1)
    assert out[1, 10] == zero and out[1, 20] == up(zero, 2) and out[1, 30] == up(zero, 1)
    assert classify_np(out)[1, 10] == classify_np(out)[1, 20] == classify_np(out)[1, 30] == MAX
