"""Oracle streams against the byte table of the stream format (parsed with
tests/stream_format.py, which restates the table and nothing else), and the
decoder's rule for which points it restores, on streams whose rank map is
rewritten to disagree with the decoded field."""
import math
import struct
import zlib

import numpy as np
import pytest

from paper_2602_17552_amd import datagen
from np_ref import MAX, MIN, R, SAD, classify_np, face_neighbour_same_bin, quantize_np, recon_np
import stream_format as sf

CASES = [
    ("bumps_rel", lambda: datagen.gaussian_bumps_2d(45, 70, 8, seed=1), 1e-2, "rel", {}),
    ("waves_abs", lambda: datagen.sinusoids_2d(33, 130, 8, seed=2), 0.004, "abs", {}),
    ("grf3d", lambda: datagen.grf_3d(9, 14, 23, seed=3), 3e-3, "rel", {}),
    ("field_scope", lambda: datagen.noise((31, 37), seed=4), 0.3, "abs", {"rank_scope": 1}),
    ("plain_szp", lambda: datagen.gaussian_bumps_2d(40, 41, 5, seed=5), 1e-3, "rel", {"topo": False}),
    ("tiny", lambda: np.array([[0.5, -1.25, 3.0]], np.float32), 0.1, "abs", {}),
    ("smooth_k7", lambda: datagen.gaussian_bumps_2d(60, 64, 3, seed=6, noise_sd=0.0), 5e-2, "rel", {}),
]


def _eps_float(eps: float) -> float:
    """Largest float32 <= eps (computed here from its definition)."""
    f = np.float32(eps)
    if float(f) > eps:
        f = np.nextafter(f, np.float32(0))
    return float(f)


def _ranks_by_definition(f, q, lab, lost, scope):
    """delta of Section IV-A (2) as read by R8: 1 + the flattened extrema of
    the same class and bin (in the block, or the field) that are less
    extreme; 1 for a flattened saddle; 0 elsewhere."""
    ff, fq, fl, fo = f.reshape(-1), q.reshape(-1), lab.reshape(-1), lost.reshape(-1)
    out = np.zeros(ff.size, np.int64)
    idx = np.nonzero(fo)[0]
    for p in idx:
        if fl[p] == SAD:
            out[p] = 1
            continue
        grp = idx[(fl[idx] == fl[p]) & (fq[idx] == fq[p])]
        if scope == 0:
            grp = grp[grp // 64 == p // 64]
        less = ff[grp] < ff[p] if fl[p] == MAX else ff[grp] > ff[p]
        out[p] = 1 + int(np.count_nonzero(less))
    return out


@pytest.mark.parametrize("name,gen,eb,mode,params", CASES, ids=[c[0] for c in CASES])
def test_header_follows_the_table(ora, name, gen, eb, mode, params):
    f = gen()
    rc, s = ora.compress(f, eb, mode, **params)
    assert rc == ora.OK
    b = bytes(s)
    h = sf.parse_header(b)
    topo = 0 if params.get("topo") is False else 1
    scope = params.get("rank_scope", 0) if topo else 0
    assert h["magic"] == b"TSZ1" and h["version"] == 1
    assert h["ndim"] == f.ndim and h["flags"] == topo | (scope << 1)
    assert h["dims"] == list(f.shape) and [h["dim0"], h["dim1"], h["dim2"]][f.ndim:] == [1] * (3 - f.ndim)
    n = f.size
    assert h["n"] == n and h["nb"] == -(-n // 64) and h["nch"] == -(-h["nb"] // 64) and h["block"] == 64
    assert h["eb_mode"] == (1 if mode == "rel" else 0) and h["eb"] == eb and h["max_rounds"] == 16
    if mode == "rel":
        vmin, vmax = float(f.min()), float(f.max())
        assert (h["vmin"], h["vmax"]) == (vmin, vmax)
        assert h["eps"] == (eb * (vmax - vmin) if vmax > vmin else eb)
    else:
        assert (h["vmin"], h["vmax"], h["eps"]) == (0.0, 0.0, eb)
    assert h["e"] == _eps_float(h["eps"])
    # the adaptive kernel rule on the data plane total (R12)
    W, nb = h["wdata"], h["nb"]
    k, sigma = (7, 1.0) if W <= nb else ((5, 0.75) if W <= 3 * nb else (3, 0.5))
    assert (h["k_size"], h["sigma"]) == (k, sigma)
    assert h["w"] == [float(np.float32(math.exp(-d2 / (2 * sigma * sigma)))) for d2 in range(10)]
    offs, lens, total = sf.layout(n, topo, W, h["wrank"])
    assert h["off"] == offs and h["len"] == lens and h["total"] == total == len(b)
    assert h["adler32"] == zlib.adler32(b[:sf.SUMMED]) and h["zero380"] == 0
    listed = np.zeros(sf.HDR, bool)
    for off, code, _ in sf.FIELDS:
        listed[off: off + struct.calcsize(code)] = True
    assert not any(b[i] for i in range(sf.HDR) if not listed[i])
    # gaps between segments are zero
    for i, name_ in enumerate(sf.SEGS[:-1]):
        end, nxt = offs[name_] + lens[name_], offs[sf.SEGS[i + 1]]
        assert b[end:nxt] == bytes(nxt - end)


@pytest.mark.parametrize("name,gen,eb,mode,params", CASES, ids=[c[0] for c in CASES])
def test_segments_hold_their_definitions(ora, name, gen, eb, mode, params):
    f = gen()
    rc, s = ora.compress(f, eb, mode, **params)
    b = bytes(s)
    h = sf.parse_header(b)
    q = quantize_np(f, h["e"]).reshape(-1)
    assert np.array_equal(sf.decode_map(b, h, "S"), q)
    widths = np.frombuffer(sf.seg(b, h, "S2"), np.uint8)
    const = np.frombuffer(sf.seg(b, h, "S1"), np.uint8)
    assert all(((const[k // 8] >> (k % 8)) & 1) == (widths[k] == 0) for k in range(h["nb"]))
    x1 = np.frombuffer(sf.seg(b, h, "X1"), "<u8")
    csum = np.concatenate([[0], np.cumsum(widths.astype(np.int64))])
    assert np.array_equal(x1, 8 * csum[0: h["nb"]: 64])
    assert 8 * int(csum[-1]) == h["len"]["S5"]
    if not h["topo"]:
        return
    lab = classify_np(f).reshape(-1)
    assert np.array_equal(sf.decode_labels(b, h), lab)
    lost = (lab != R) & face_neighbour_same_bin(q.reshape(f.shape)).reshape(-1)
    delta = sf.decode_map(b, h, "R")
    assert np.array_equal(delta, _ranks_by_definition(f, q, lab, lost, h["field_scope"]))
    # re-encoding the decoded rank map gives the same bytes back
    assert sf.with_ranks(b, delta) == b


def _float_steps(v: np.float32, k: int, up: bool) -> np.float32:
    for _ in range(k):
        v = np.nextafter(v, np.float32(np.inf if up else -np.inf))
        if v == 0:
            v = np.float32(0.0)
    return v


def test_decoder_follows_the_stored_ranks(ora):
    """Which points the decoder restores is read from the stream: an extremum
    or saddle label with delta > 0.  On streams the compressor writes these
    are the labelled points that read as regular in the decoded field; on a
    rewritten rank map the decoder follows delta, not its own classification
    of the decoded values."""
    f = datagen.sinusoids_2d(48, 64, 8, seed=7)
    rc, s = ora.compress(f, 5e-3, "rel")
    b = bytes(s)
    h = sf.parse_header(b)
    e = np.float32(h["e"])
    q = sf.decode_map(b, h, "S")
    rq = recon_np(q, e)
    lab = sf.decode_labels(b, h)
    delta = sf.decode_map(b, h, "R")
    cls_hat = classify_np(rq.reshape(f.shape)).reshape(-1)
    # the compressor's marks are the paper's lost set
    assert np.array_equal(delta > 0, (lab != R) & (cls_hat == R))
    rc, base, st0 = ora.decompress(np.frombuffer(b, np.uint8), f.shape)
    assert rc == ora.OK
    base = base.reshape(-1)

    kept_max = np.nonzero((lab == MAX) & (delta == 0))[0]      # unflattened maxima
    lost_max = np.nonzero((lab == MAX) & (delta > 0))[0]
    regular = np.nonzero((lab == R) & (cls_hat == R))[0]
    kept_sad = np.nonzero((lab == SAD) & (delta == 0) & (cls_hat == SAD))[0]
    assert kept_max.size and lost_max.size and regular.size and kept_sad.size

    # (1) an unflattened maximum given delta 3 moves 3 float steps up from
    # its bin centre, although it is already a maximum of the decoded field
    p = int(kept_max[0])
    d2 = delta.copy()
    d2[p] = 3
    rc, out, st = ora.decompress(np.frombuffer(sf.with_ranks(b, d2), np.uint8), f.shape)
    out = out.reshape(-1)
    assert rc == ora.OK and out[p] == _float_steps(rq[p], 3, True) and base[p] == rq[p]
    assert st["stencil_moves"] == st0["stencil_moves"] + 1

    # (2) a flattened maximum given delta 0 stays at its bin centre
    p = int(lost_max[0])
    d2 = delta.copy()
    d2[p] = 0
    rc, out, st = ora.decompress(np.frombuffer(sf.with_ranks(b, d2), np.uint8), f.shape)
    assert rc == ora.OK and out.reshape(-1)[p] == rq[p] and base[p] != rq[p]
    assert st["stencil_moves"] == st0["stencil_moves"] - 1

    # (3) a regular point given delta 2 is ignored: the output is unchanged
    d2 = delta.copy()
    d2[int(regular[0])] = 2
    rc, out, st = ora.decompress(np.frombuffer(sf.with_ranks(b, d2), np.uint8), f.shape)
    assert rc == ora.OK and np.array_equal(out.reshape(-1).view(np.uint32), base.view(np.uint32))

    # (4) a saddle of the decoded field given delta 1 is queued, and skipped
    # by every round (it is already a saddle): the output is unchanged
    d2 = delta.copy()
    d2[int(kept_sad[0])] = 1
    rc, out, st = ora.decompress(np.frombuffer(sf.with_ranks(b, d2), np.uint8), f.shape)
    assert rc == ora.OK and np.array_equal(out.reshape(-1).view(np.uint32), base.view(np.uint32))
    assert st["worklist0"] == st0["worklist0"] + 1


def test_rank_out_of_range_is_corrupt(ora):
    f = datagen.gaussian_bumps_2d(20, 30, 4, seed=8)
    rc, s = ora.compress(f, 1e-2, "rel")
    b = bytes(s)
    h = sf.parse_header(b)
    delta = sf.decode_map(b, h, "R")
    d2 = delta.copy()
    d2[5] = 65  # block-scope ranks lie in [0, 64]
    rc, _, _ = ora.decompress(np.frombuffer(sf.with_ranks(b, d2), np.uint8), f.shape)
    assert rc == ora.E_CORRUPT
    d2 = delta.copy()
    d2[7] = -1
    rc, _, _ = ora.decompress(np.frombuffer(sf.with_ranks(b, d2), np.uint8), f.shape)
    assert rc == ora.E_CORRUPT


def _corrupt_source(ora):
    f = datagen.sinusoids_2d(75, 120, 8, seed=9)  # 141 blocks: 3 chunks, the last partial
    rc, s = ora.compress(f, 5e-3, "rel")
    assert rc == ora.OK
    return f, bytes(s)


def test_segment_corruption_is_reported(ora):
    f, b = _corrupt_source(ora)
    cases = sf.corruptions(b)
    assert len(cases) >= 18
    for name, t in cases:
        rc, _, _ = ora.decompress(np.frombuffer(t, np.uint8).copy(), f.shape)
        assert rc == ora.E_CORRUPT, name
