"""Both decoders on streams the compressor never writes: rank maps rewritten
(tests/stream_format.py) so that delta marks points the decoded field does
not show as lost, or leaves lost points unmarked.  The decoders take the lost
set from delta alone, so the GPU reconstruction and counters must equal the
oracle's bit for bit on every such stream, as on canonical ones."""
import numpy as np
import pytest

from paper_2602_17552_amd import datagen
from np_ref import R, SAD
import stream_format as sf
from test_gpu_parity import gpu_decompress

pytestmark = pytest.mark.gpu

FIELDS = [
    ("waves2d", lambda: datagen.sinusoids_2d(48, 64, 8, seed=7), 5e-3, {}),
    ("bumps2d", lambda: datagen.gaussian_bumps_2d(40, 72, 10, seed=3, noise_sd=3e-2), 1e-2, {}),
    ("grf3d", lambda: datagen.grf_3d(12, 20, 24, seed=4), 1e-2, {}),
    ("noise_field_scope", lambda: datagen.noise((30, 44), seed=5), 0.3, {"rank_scope": 1}),
    ("coarse_k7", lambda: datagen.gaussian_bumps_2d(50, 64, 4, seed=6, noise_sd=2e-3), 5e-2, {}),
]


def _variants(b, seed):
    h = sf.parse_header(b)
    lab = sf.decode_labels(b, h)
    delta = sf.decode_map(b, h, "R")
    rng = np.random.default_rng(seed)
    dmax = 64 if not h["field_scope"] else 200
    n = delta.size
    out = []
    d = delta.copy()  # random ranks at labelled points
    idx = np.nonzero(lab != R)[0]
    pick = rng.choice(idx, size=min(40, idx.size), replace=False)
    d[pick] = rng.integers(0, 6, pick.size)
    out.append(("labelled_random", d))
    out.append(("all_zero", np.zeros(n, np.int64)))
    d = delta.copy()  # every saddle queued
    d[lab == SAD] = 1
    out.append(("all_saddles", d))
    d = delta.copy()  # the largest ranks at random extrema
    ext = np.nonzero((lab == 1) | (lab == 3))[0]
    pick = rng.choice(ext, size=min(25, ext.size), replace=False)
    d[pick] = dmax
    out.append(("extrema_max_rank", d))
    d = delta.copy()  # ranks on regular points only
    reg = np.nonzero(lab == R)[0]
    pick = rng.choice(reg, size=min(50, reg.size), replace=False)
    d[pick] = rng.integers(1, dmax + 1, pick.size)
    out.append(("regular_marked", d))
    return out


@pytest.mark.parametrize("name,gen,eb,params", FIELDS, ids=[f[0] for f in FIELDS])
def test_rewritten_rank_maps_decode_alike(tsz, ora, name, gen, eb, params):
    f = gen()
    rc, s = ora.compress(f, eb, "rel", **params)
    assert rc == ora.OK
    b = bytes(s)
    for k, (vname, d) in enumerate(_variants(b, 100 + len(name))):
        print("case %s / %s" % (name, vname), flush=True)
        s2 = np.frombuffer(sf.with_ranks(b, d), np.uint8).copy()
        rc_o, rec_o, st_o = ora.decompress(s2, f.shape)
        st_g, rec_g, stats_g = gpu_decompress(tsz, s2, f.shape)
        assert st_g == rc_o == ora.OK, (vname, st_g, rc_o)
        bad = np.nonzero(rec_g.reshape(-1).view(np.uint32) != rec_o.reshape(-1).view(np.uint32))[0]
        assert bad.size == 0, "%s/%s: %d values differ, first at %d" % (name, vname, bad.size, bad[0])
        for key in ("rounds", "commits", "stencil_moves", "budget_skips"):
            assert stats_g[key] == st_o[key], (vname, key, stats_g, st_o)
        assert stats_g["queued"] == st_o["worklist0"], (vname, stats_g, st_o)


def test_rank_out_of_range_is_corrupt_on_both(tsz, ora):
    f = datagen.gaussian_bumps_2d(20, 30, 4, seed=8)
    rc, s = ora.compress(f, 1e-2, "rel")
    b = bytes(s)
    h = sf.parse_header(b)
    delta = sf.decode_map(b, h, "R")
    for pos, val in [(5, 65), (7, -1), (599, 1000)]:
        d = delta.copy()
        d[pos] = val
        s2 = np.frombuffer(sf.with_ranks(b, d), np.uint8).copy()
        rc_o, _, _ = ora.decompress(s2, f.shape)
        st_g, _, _ = gpu_decompress(tsz, s2, f.shape)
        assert rc_o == st_g == ora.E_CORRUPT, (pos, val, rc_o, st_g)


def test_segment_corruption_on_both(tsz, ora):
    """Each segment rule of the format table broken once (chunk offsets,
    constant bitmaps, widths, first values, ranks, truncation): both decoders
    report the stream corrupt.  The GPU decoder checks widths, bitmaps and
    chunk offsets before it reads a chunk's planes, and reads only inside the
    header-checked layout."""
    f = datagen.sinusoids_2d(75, 120, 8, seed=9)
    rc, s = ora.compress(f, 5e-3, "rel")
    for name, t in sf.corruptions(bytes(s)):
        print("corruption:", name, flush=True)
        arr = np.frombuffer(t, np.uint8).copy()
        rc_o, _, _ = ora.decompress(arr, f.shape)
        st_g, _, _ = gpu_decompress(tsz, arr, f.shape)
        assert rc_o == st_g == ora.E_CORRUPT, (name, rc_o, st_g)
