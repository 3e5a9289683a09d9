"""Pins of the oracle's B + LZ + BE codec and stream layout (Sections II-C,
IV-A).  The byte layout itself is this project's format: the paper lists the
parts (1)-(7) without giving their bytes, so the layout is checked against the
format description, not against the paper."""
import numpy as np
import pytest


def _direct_encode(v):
    """Definition: r_0 = 0, r_i = v_i - v_{i-1}; w = bit length of max |r_i|;
    sign bit i set for r_i < 0; plane j holds bit j of |r_i| at bit i."""
    v = np.asarray(v, dtype=np.int64)
    r = np.zeros(64, np.int64)
    r[1:] = np.diff(v)
    mag = np.abs(r)
    w = int(mag.max()).bit_length()
    sign = sum(1 << i for i in range(64) if r[i] < 0)
    planes = [sum(((int(mag[i]) >> j) & 1) << i for i in range(64)) for j in range(w)]
    return w, int(v[0]), sign, planes


@pytest.mark.parametrize("width", [0, 1, 2, 5, 8, 13, 22, 23])
def test_block_codec_definition_and_round_trip(ora, width):
    rng = np.random.default_rng(width)
    for _ in range(30):
        if width == 0:
            v = np.full(64, rng.integers(-1000, 1000), np.int32)
        else:
            hi = (1 << width) - 1
            steps = rng.integers(-(hi // 2), hi // 2 + 1, 64)
            steps[rng.integers(1, 64)] = hi if rng.uniform() < 0.5 else -hi
            v = np.cumsum(steps).astype(np.int64)
            v = np.clip(v, -(2 ** 22 - 1), 2 ** 22 - 1).astype(np.int32)
        w, first, sign, planes = ora.encode_block(v)
        dw, dfirst, dsign, dplanes = _direct_encode(v)
        assert (w, first, sign) == (dw, dfirst, dsign)
        assert [int(p) for p in planes] == dplanes
        assert np.array_equal(ora.decode_block(w, first, sign, planes), v)


def _spec_layout(n, topo, wdata, wrank):
    nb = -(-n // 64)
    nch = -(-nb // 64)
    lens = [8 * nch, nb, 8 * nb, 4 * nb, 16 * nb if topo else 0, 8 * nch if topo else 0,
            nb if topo else 0, 8 * nb if topo else 0, 4 * nb if topo else 0, 8 * nch,
            8 * nch if topo else 0, 8 * wdata, 8 * wrank if topo else 0]
    offs = [512]
    for L in lens[:-1]:
        offs.append((offs[-1] + L + 7) // 8 * 8)
    return offs, lens, offs[-1] + lens[-1]


@pytest.mark.parametrize("shape,topo", [((37, 41), True), ((64, 64), False), ((3, 5, 7), True),
                                        ((1, 1), True), ((1, 4097), True)])
def test_stream_layout_and_round_trip(ora, shape, topo):
    f = np.random.default_rng(1).standard_normal(shape).astype(np.float32)
    rc, s = ora.compress(f, 0.05, "abs", topo=topo)
    assert rc == ora.OK
    assert bytes(s[:4]) == b"TSZ1"
    rc, info = ora.inspect(s)
    assert rc == ora.OK
    offs, lens, total = _spec_layout(f.size, topo, info["wdata"], info["wrank"])
    assert info["seg_off"] == offs and info["seg_len"] == lens and info["total"] == total == s.size
    rc, rec, _ = ora.decompress(s, f.shape)
    assert rc == ora.OK
    # every point inside the relaxed bound
    assert np.all(np.abs(rec.astype(np.float64) - f) <= 2 * info["e"] * (1 + 2 ** -22))


def test_labels_segment_packing(ora):
    """Part (6): 2 bits per point, point i at byte i//4, bits 2(i%4)."""
    f = np.random.default_rng(2).standard_normal((9, 13)).astype(np.float32)
    rc, s = ora.compress(f, 1e-4, "abs")
    _, info = ora.inspect(s)
    lab = ora.classify(f).reshape(-1)
    seg = s[info["seg_off"][4]: info["seg_off"][4] + info["seg_len"][4]]
    got = np.array([(seg[i >> 2] >> (2 * (i & 3))) & 3 for i in range(f.size)])
    assert np.array_equal(got, lab)
    assert not seg[(f.size + 3) // 4:].any()


def test_chunk_index_matches_widths(ora):
    f = np.random.default_rng(4).standard_normal((130, 200)).astype(np.float32)
    rc, s = ora.compress(f, 1e-3, "rel")
    _, info = ora.inspect(s)
    nb = info["nb"]
    widths = s[info["seg_off"][1]: info["seg_off"][1] + nb].astype(np.int64)
    x1 = s[info["seg_off"][9]: info["seg_off"][9] + info["seg_len"][9]].view(np.uint64)
    pref = np.concatenate([[0], np.cumsum(widths)])
    assert np.array_equal(x1.astype(np.int64), 8 * pref[0:nb:64])
    bitmap = s[info["seg_off"][0]: info["seg_off"][0] + info["seg_len"][0]]
    const = np.array([(bitmap[b >> 3] >> (b & 7)) & 1 for b in range(nb)])
    assert np.array_equal(const, (widths == 0).astype(int))


def test_header_checksum_is_adler32(ora):
    """The header's bytes [0, 376) are covered by an Adler-32 (RFC 1950)
    checksum stored at byte 376; zlib's implementation is the reference."""
    import zlib
    f = np.random.default_rng(6).standard_normal((20, 30)).astype(np.float32)
    rc, s = ora.compress(f, 0.01, "rel")
    assert int(s[376:380].view(np.uint32)[0]) == zlib.adler32(bytes(s[:376]))
    assert not s[380:512].any()
