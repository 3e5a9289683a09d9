"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Compressed streams must be byte-identical and reconstructions bit-identical
(every decision is integer or fixed-order IEEE arithmetic); device status
codes and refinement counters must match the oracle's."""
import sys

import numpy as np
import pytest

from paper_2602_17552_amd import datagen

pytestmark = pytest.mark.gpu

SEG_NAMES = ["S1 const", "S2 widths", "S3 signs", "S4 first", "S6 labels", "R1", "R2", "R3", "R4",
             "X1", "X2", "S5 payload", "R5 rank payload"]


def _where(ora, s, k):
    if k < 512:
        return "header byte %d" % k
    rc, info = ora.inspect(s)
    if rc != 0:
        return "byte %d" % k
    for i, (o, L) in enumerate(zip(info["seg_off"], info["seg_len"])):
        if o <= k < o + max(L, 1):
            return "%s +%d" % (SEG_NAMES[i], k - o)
    return "gap byte %d" % k


def gpu_compress(tsz, f, eb, mode, **params):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    st, s = tsz.compress(d, eb, mode, **params)
    return st, s.cpu().numpy()


def gpu_decompress(tsz, s, shape):
    import torch
    ws = tsz.Workspace(shape)
    st, rec = tsz.decompress(torch.from_numpy(np.ascontiguousarray(s)).cuda(), shape, ws=ws)
    return st, rec.cpu().numpy(), tsz.decompress_stats(ws)


def check(tsz, ora, name, f, eb, mode="rel", **params):
    print("case %s shape %s eb %g %s %s" % (name, f.shape, eb, mode, params), flush=True)
    rc_o, s_o = ora.compress(f, eb, mode, **params)
    st, s_g = gpu_compress(tsz, f, eb, mode, **params)
    assert st == rc_o, (name, st, rc_o)
    if rc_o != 0:
        return None
    if s_g.size != s_o.size or not np.array_equal(s_g, s_o):
        n = min(s_g.size, s_o.size)
        diff = np.nonzero(s_g[:n] != s_o[:n])[0]
        k = int(diff[0]) if diff.size else n
        raise AssertionError("%s: stream differs (sizes %d/%d), first at %s, %d bytes differ" %
                             (name, s_g.size, s_o.size, _where(ora, s_o, k), diff.size))
    st, rec_g, stats_g = gpu_decompress(tsz, s_o, f.shape)
    rc, rec_o, stats_o = ora.decompress(s_o, f.shape)
    assert st == rc == 0
    bad = np.nonzero(rec_g.reshape(-1).view(np.uint32) != rec_o.reshape(-1).view(np.uint32))[0]
    assert bad.size == 0, "%s: %d reconstructed values differ, first at %d: gpu %r oracle %r" % (
        name, bad.size, bad[0], rec_g.reshape(-1)[bad[0]], rec_o.reshape(-1)[bad[0]])
    for k in ("rounds", "commits", "stencil_moves", "budget_skips"):
        assert stats_g[k] == stats_o[k], (name, k, stats_g, stats_o)
    assert stats_g["queued"] == stats_o["worklist0"], (name, stats_g, stats_o)
    return s_o, rec_o, stats_o


SMALL = [
    ("bumps", lambda: datagen.gaussian_bumps_2d(96, 160, 10, seed=1), 1e-3, "rel"),
    ("waves", lambda: datagen.sinusoids_2d(90, 180, 16, seed=4, noise_sd=1e-2), 1e-3, "rel"),
    ("noise_abs", lambda: datagen.noise((77, 91), seed=5), 0.3, "abs"),
    ("noise_fine", lambda: datagen.noise((77, 91), seed=6), 1e-4, "abs"),
    ("bumps_1e-2", lambda: datagen.gaussian_bumps_2d(130, 70, 6, seed=2), 1e-2, "rel"),
    ("bumps_1e-4", lambda: datagen.gaussian_bumps_2d(64, 200, 6, seed=3), 1e-4, "rel"),
    ("grf3d", lambda: datagen.grf_3d(20, 24, 28, seed=6), 1e-3, "abs"),
    ("noise3d", lambda: datagen.noise((9, 17, 23), seed=7), 0.2, "abs"),
    ("grf3d_rel", lambda: datagen.grf_3d(16, 16, 16, seed=8), 1e-2, "rel"),
]


@pytest.mark.parametrize("name,gen,eb,mode", SMALL, ids=[c[0] for c in SMALL])
def test_parity_small(tsz, ora, name, gen, eb, mode):
    check(tsz, ora, name, gen(), eb, mode)


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (3, 3), (5, 9), (63, 65), (64, 64), (65, 63), (1, 4097),
          (4097, 1), (130, 200), (2, 3, 4), (5, 6, 7), (1, 9, 9), (9, 1, 9), (17, 1, 13), (3, 3, 1),
          (33, 33, 33), (1, 1, 70)]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s) for s in SHAPES])
def test_parity_shapes(tsz, ora, shape):
    f = datagen.noise(shape, seed=len(shape) * 1000 + int(np.prod(shape)) % 997)
    check(tsz, ora, "noise", f, 0.25, "abs")
    g = (0.05 * f + np.float32(3.0)).astype(np.float32)
    check(tsz, ora, "offset", g, 1e-2, "rel")


def test_parity_kernel_sizes(tsz, ora):
    """Every adaptive window: k_size 3, 5 and 7 in 2D and in 3D (the fields
    and bounds below are chosen to reach each one), the fixed k_size 3
    policy and a one-round cap."""
    smooth = datagen.gaussian_bumps_2d(120, 150, 4, seed=11, noise_sd=2e-4)
    waves = datagen.sinusoids_2d(80, 96, 8, seed=12, noise_sd=2e-3)
    checker = datagen.checker_2d(60, 64, seed=1)
    g3 = datagen.grf_3d(24, 28, 32, seed=13)
    cases = [("waves_k3", waves, 1e-2), ("waves_k5", waves, 5e-2), ("checker_k7", checker, 0.3),
             ("grf3d_k3", g3, 3e-2), ("grf3d_k5", g3, 0.1), ("grf3d_k7", g3, 0.3)]
    ks = set()
    for name, f, eb in cases:
        s_o, _, _ = check(tsz, ora, name, f, eb, "rel")
        ks.add((f.ndim, ora.inspect(s_o)[1]["k"]))
    print("kernel sizes covered:", sorted(ks), flush=True)
    assert ks == {(2, 3), (2, 5), (2, 7), (3, 3), (3, 5), (3, 7)}
    check(tsz, ora, "fixed3", smooth, 1e-3, "rel", rbf_policy=1)
    check(tsz, ora, "rounds1", smooth, 1e-3, "rel", max_rounds=1)
    check(tsz, ora, "checker_k7_rounds1", checker, 0.3, "rel", max_rounds=1)


def _checker_patches(m, counts, gap=4):
    # checker_3d blocks of m^3 cells, `gap` constant cells apart (beyond any
    # read set): one cluster of queued saddles per block at coarse bounds
    p = m + gap
    f = np.zeros(tuple(c * p for c in counts), np.float32)
    for n, (i, j, k) in enumerate(np.ndindex(*counts)):
        f[p * i:p * i + m, p * j:p * j + m, p * k:p * k + m] = datagen.checker_3d(m, m, m, seed=100 + n)
    return f


def test_parity_large_clusters(tsz, ora):
    # queued saddles linked into clusters beyond the refine workgroup's 64
    # members (the 3D checker: one of several hundred), with commits:
    # replayed by the tail from LDS
    res = check(tsz, ora, "checker2d", datagen.checker_2d(40, 48, seed=0), 2.0, "abs")
    assert res[2]["commits"] > 0
    res = check(tsz, ora, "checker3d", datagen.checker_3d(10, 12, 14, seed=11), 1.0, "abs")
    assert res[2]["commits"] > 0
    # the same patterns tiled next to smooth regions: large and small
    # clusters in one field
    f = datagen.gaussian_bumps_2d(120, 150, 12, seed=9)
    f[30:70, 40:88] = datagen.checker_2d(40, 48, seed=1) * 0.05 + f[30:70, 40:88]
    check(tsz, ora, "checker_in_bumps", f, 2e-2, "rel")


def test_parity_tail_clusters(tsz, ora):
    # thirty separate over-size clusters, gathered together by the tail
    res = check(tsz, ora, "patches30", _checker_patches(6, (2, 3, 5)), 1.0, "abs")
    assert 30 * 40 < res[2]["worklist0"] < 4096


def test_parity_whole_field_replay(tsz, ora):
    # over-size clusters beyond what the tail holds in LDS: the whole-field
    # replay.  One cluster of more than 4096 queued saddles ...
    res = check(tsz, ora, "checker3d_big", datagen.checker_3d(24, 26, 28, seed=1), 1.0, "abs")
    assert res[2]["worklist0"] > 4096
    # ... and 150 over-size clusters, more than the 128 candidates the
    # refine kernel records
    res = check(tsz, ora, "patches150", _checker_patches(7, (5, 5, 6)), 1.0, "abs")
    assert res[2]["worklist0"] > 150 * 65
    # with one round allowed: the clusters the refine kernel stopped at the
    # cap must not get more rounds from the whole-field replay
    check(tsz, ora, "checker_cap1", datagen.checker_2d(145, 167, seed=309451577), 1.43446, "abs", max_rounds=1)
    check(tsz, ora, "checker_cap1_field", datagen.checker_2d(785, 286, seed=450909876), 1.51062, "abs",
          rank_scope=1, rbf_policy=1, max_rounds=1)
    check(tsz, ora, "checker3d_big_cap2", datagen.checker_3d(24, 26, 28, seed=1), 1.0, "abs", max_rounds=2)


def _all_lost(shape, seed):
    rng = np.random.default_rng(seed)
    par = np.indices(shape).sum(axis=0) % 2
    return (0.5 + 0.01 * par + rng.uniform(0, 0.001, shape)).astype(np.float32)


FIELD_SCOPE = [
    ("bumps", lambda: datagen.gaussian_bumps_2d(96, 160, 10, seed=1), 1e-3, "rel"),
    ("noise_abs", lambda: datagen.noise((77, 91), seed=5), 0.3, "abs"),
    ("grf3d", lambda: datagen.grf_3d(20, 24, 28, seed=6), 1e-3, "abs"),
    ("near_single_bin", lambda: datagen.noise((150, 170), seed=11), 2.5, "abs"),
    ("ties", lambda: (np.round(datagen.noise((90, 130), seed=12) * 3) / 3).astype(np.float32), 0.2, "abs"),
    ("tiny", lambda: datagen.noise((3, 3), seed=13), 0.5, "abs"),
    ("cfg1_1800x3600_rel1e-3", datagen.cfg1, 1e-3, "rel"),
    # nothing flattened: the sort is skipped
    ("none_lost", lambda: datagen.gaussian_bumps_2d(64, 80, 4, seed=2), 1e-7, "abs"),
    # every point a flattened extremum (a jittered checkerboard inside one bin)
    ("all_lost_2d", lambda: _all_lost((130, 150), seed=14), 0.1, "abs"),
    ("all_lost_3d", lambda: _all_lost((17, 19, 23), seed=15), 0.1, "abs"),
]


@pytest.mark.parametrize("name,gen,eb,mode", FIELD_SCOPE, ids=[c[0] for c in FIELD_SCOPE])
def test_parity_field_scope(tsz, ora, name, gen, eb, mode):
    # ranks among the flattened extrema of the whole field (sorted on the GPU)
    res = check(tsz, ora, name + "_field", gen(), eb, mode, rank_scope=1)
    assert res is not None
    rc, info = ora.inspect(res[0])
    assert rc == 0 and info["scope"] == 1


def test_parity_plain_szp(tsz, ora):
    check(tsz, ora, "plain", datagen.gaussian_bumps_2d(90, 110, 5, seed=9), 1e-3, "rel", topo=False)
    check(tsz, ora, "plain3d", datagen.grf_3d(10, 12, 14, seed=9), 1e-3, "rel", topo=False)
    # rows of at least 64 points: interior blocks, x-boundary ones included,
    # take the fast path (several chunks and a partial last one)
    check(tsz, ora, "plain_waves", datagen.sinusoids_2d(210, 333, 16, seed=10, noise_sd=1e-2), 1e-3, "rel",
          topo=False)
    check(tsz, ora, "plain_noise_abs", datagen.noise((130, 257), seed=11), 1e-2, "abs", topo=False)
    check(tsz, ora, "plain3d_wide", datagen.grf_3d(12, 30, 70, seed=12), 1e-4, "rel", topo=False)


def test_parity_rank_groups(tsz, ora):
    """Block-scope ranks where flattened extrema crowd three bins 32 apart
    (10, 42, 74 at bin width 1): their (class, bin) keys agree in the low six
    bits, so distinct keys meet on one slot of the shared-key test, and each
    block also holds several flattened extrema of one class and bin, whose
    ranks then exceed 1 (Section IV-A (2))."""
    rng = np.random.default_rng(21)
    centres = np.array([10.0, 42.0, 74.0])
    f2 = (rng.choice(centres, (70, 300)) + rng.uniform(-0.45, 0.45, (70, 300))).astype(np.float32)
    check(tsz, ora, "rank_groups_2d", f2, 0.5, "abs")
    f3 = (rng.choice(centres, (10, 12, 90)) + rng.uniform(-0.45, 0.45, (10, 12, 90))).astype(np.float32)
    check(tsz, ora, "rank_groups_3d", f3, 0.5, "abs")


def test_parity_adversarial_values(tsz, ora):
    """Values on and next to bin edges, a power-of-two bound, signed zeros,
    denormals and ties."""
    rng = np.random.default_rng(0)
    e = np.float32(2.0 ** -8)
    k = rng.integers(-300, 300, (70, 90))
    edge = ((2 * k + 1) * np.float64(e)).astype(np.float32)
    jitter = rng.integers(-1, 2, edge.shape)
    f = np.where(jitter == 0, edge, np.nextafter(edge, np.where(jitter > 0, np.inf, -np.inf).astype(np.float32)))
    f = f.astype(np.float32)
    check(tsz, ora, "edges_pow2", f, float(e), "abs")
    check(tsz, ora, "edges_0.01", (f * np.float32(3.1)).astype(np.float32), 0.01 * 3.1 / 2 ** 8 * 2, "abs")
    z = rng.choice(np.array([0.0, -0.0, 1e-45, -1e-45, 1e-40, 3e-39, -2e-38], np.float32), (40, 50))
    check(tsz, ora, "denormals", z, 1e-30, "abs")
    t = rng.integers(0, 4, (60, 70)).astype(np.float32)
    check(tsz, ora, "ties", t, 0.3, "abs")
    check(tsz, ora, "ties_rel", t, 0.2, "rel")
    c = np.full((33, 47), 1.5, np.float32)
    check(tsz, ora, "constant", c, 1e-3, "rel")
    top = np.float32((2 ** 22 - 1) * 2)
    m = np.linspace(-top, top, 64 * 9, dtype=np.float32).reshape(24, 24)
    check(tsz, ora, "q_range_edge", m, 1.0, "abs")


def test_status_codes(tsz, ora):
    f = datagen.noise((40, 50), seed=1)
    g = f.copy()
    g[3, 7] = np.nan
    assert check(tsz, ora, "nan", g, 0.1, "abs") is None
    g[3, 7] = np.inf
    assert check(tsz, ora, "inf_rel", g, 0.1, "rel") is None
    assert check(tsz, ora, "range", f * np.float32(1e30), 1e-3, "abs") is None
    assert check(tsz, ora, "tiny_bound", f, 1e-35, "abs") is None
    # the workspace is reusable after an error
    check(tsz, ora, "after_errors", f, 0.1, "abs")


def test_field_scope_stream_decodes(tsz, ora):
    f = datagen.noise((50, 60), seed=4)
    rc, s = ora.compress(f, 0.4, "abs", rank_scope=1)
    assert rc == 0
    st, rec, _ = gpu_decompress(tsz, s, f.shape)
    rc, rec_o, _ = ora.decompress(s, f.shape)
    assert st == 0 and np.array_equal(rec.view(np.uint32), rec_o.view(np.uint32))


def test_corrupt_headers(tsz, ora):
    """Header corruption is reported, never acted on."""
    f = datagen.noise((30, 40), seed=3)
    rc, s = ora.compress(f, 0.05, "abs")
    rng = np.random.default_rng(1)
    for off in list(range(0, 384, 7)) + [376, 377, 380]:
        t = s.copy()
        t[off] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, _, _ = gpu_decompress(tsz, t, f.shape)
        assert st == -5, off
    st, _, _ = gpu_decompress(tsz, s[:300], f.shape)
    assert st == -5
    st, _, _ = gpu_decompress(tsz, s, (10, 10))
    assert st == -4
    # payload chain / widths
    _, info = ora.inspect(s)
    t = s.copy()
    t[info["seg_off"][1]] = 40
    assert gpu_decompress(tsz, t, f.shape)[0] == -5
    st, rec, _ = gpu_decompress(tsz, s, f.shape)
    assert st == 0


def test_determinism_and_reuse(tsz, ora):
    import torch
    f1 = datagen.sinusoids_2d(120, 240, 8, seed=3)
    f2 = datagen.grf_3d(12, 20, 30, seed=4)
    ws = tsz.Workspace((64, 64, 64))
    outs = []
    for f, eb, mode in [(f1, 1e-3, "rel"), (f2, 1e-2, "abs"), (f1, 1e-3, "rel"), (f2, 1e-2, "abs")]:
        st, s = tsz.compress(torch.from_numpy(f).cuda(), eb, mode, ws=ws)
        assert st == 0
        outs.append(s.cpu().numpy().copy())
    assert np.array_equal(outs[0], outs[2]) and np.array_equal(outs[1], outs[3])
    for f, s in [(f1, outs[0]), (f2, outs[1]), (f1, outs[2])]:
        st, rec = tsz.decompress(torch.from_numpy(s).cuda(), f.shape, ws=ws)
        rc, rec_o, _ = ora.decompress(s, f.shape)
        assert st == 0 and np.array_equal(rec.cpu().numpy().view(np.uint32), rec_o.view(np.uint32))


FULL = [
    ("cfg0_512x512_rel1e-3", datagen.cfg0, 1e-3),
    ("cfg1_1800x3600_rel1e-2", datagen.cfg1, 1e-2),
    ("cfg1_1800x3600_rel1e-3", datagen.cfg1, 1e-3),
    ("cfg1_1800x3600_rel1e-4", datagen.cfg1, 1e-4),
    ("cfg1_1800x3600_rel5e-2_k7", datagen.cfg1, 5e-2),   # the widest window, at scale
    ("cfg2_256cube_rel1e-3", datagen.cfg2, 1e-3),
    ("cfg2_256cube_rel3e-2_k5", datagen.cfg2, 3e-2),     # a 3D k=5 window, at scale
    # the widest 3D window (k=7, 122 cells) on a field of 512 chunks
    ("grf_128cube_rel0.3_k7", lambda: datagen.grf_3d(128, 128, 128, seed=21), 0.3),
    # more than 4096 chunks (16,842,752 points): the separate scan kernel and
    # the unfused finalize
    ("grf_257x256x256_rel1e-3_scan", lambda: datagen.grf_3d(257, 256, 256, seed=2), 1e-3),
    ("waves_4100x4100_rel1e-3_scan", lambda: datagen.sinusoids_2d(4100, 4100, 64, seed=22), 1e-3),
]
_cache = {}


@pytest.mark.parametrize("name,gen,eb", FULL, ids=[c[0] for c in FULL])
def test_parity_full_size(tsz, ora, name, gen, eb):
    key = gen.__name__ if gen.__name__ != "<lambda>" else name
    if key not in _cache:
        _cache.clear()
        _cache[key] = gen()
    f = _cache[key]
    r = check(tsz, ora, name, f, eb, "rel")
    s, rec, stats = r
    ev = ora.eval_topology(f, rec)
    print(name, "bytes", s.size, "ratio %.2f" % (f.nbytes / s.size), ev, stats, flush=True)
    assert ev["FP"] == 0 and ev["FT"] == 0


def test_stats_follow_last_decompression(tsz, ora):
    # the counters are gathered on request from what the last decompression
    # left in the workspace: asking twice gives the same numbers, and a later
    # decompression on the same workspace replaces them
    import torch
    shape = (130, 150)
    ws = tsz.Workspace(shape)
    cases = [(datagen.gaussian_bumps_2d(*shape, 12, seed=9), 2e-2, {}),
             (datagen.noise(shape, seed=4), 0.3, {}),
             (datagen.noise(shape, seed=5), 0.3, {"topo": False})]
    for f, eb, params in cases:
        rc, s_o = ora.compress(f, eb, "abs", **params)
        assert rc == 0
        st, rec = tsz.decompress(torch.from_numpy(s_o).cuda(), shape, ws=ws)
        assert st == tsz.OK
        first = tsz.decompress_stats(ws)
        again = tsz.decompress_stats(ws)
        _, rec_o, stats_o = ora.decompress(s_o, shape)
        assert np.array_equal(rec.cpu().numpy().view(np.uint32), rec_o.view(np.uint32))
        assert first == again
        for k in ("rounds", "commits", "stencil_moves", "budget_skips"):
            assert first[k] == stats_o[k], (k, first, stats_o)
