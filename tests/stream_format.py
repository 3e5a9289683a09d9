"""The stream format, written out from its byte table alone (tests only).

This module restates the layout of a compressed stream (the header table and
segment rules of the design notes, section 5) in plain Python: it parses a
stream, decodes its block-coded maps, and re-encodes a rank map into a stream.
It shares no code with the oracle or the GPU library, so a test that parses
an oracle stream with it checks the oracle's bytes against the table, and a
stream it rewrites can be fed to both decoders.
"""
import struct
import zlib

import numpy as np

HDR = 512
SUMMED = 376
SEGS = ["S1", "S2", "S3", "S4", "S6", "R1", "R2", "R3", "R4", "X1", "X2", "S5", "R5"]

# (offset, struct code, name) of every header field; bytes not listed are 0
FIELDS = [
    (0, "4s", "magic"), (4, "<H", "version"), (6, "<B", "ndim"), (7, "<B", "flags"),
    (8, "<Q", "dim0"), (16, "<Q", "dim1"), (24, "<Q", "dim2"),
    (32, "<Q", "n"), (40, "<Q", "nb"), (48, "<I", "block"),
    (52, "<B", "eb_mode"), (53, "<B", "k_size"), (54, "<H", "max_rounds"),
    (56, "<d", "eb"), (64, "<d", "eps"), (72, "<f", "e"), (76, "<f", "vmin"),
    (80, "<f", "vmax"), (84, "<f", "sigma"),
] + [(88 + 4 * j, "<f", "w%d" % j) for j in range(10)] + [
    (128, "<Q", "total"), (136, "<Q", "wdata"), (144, "<Q", "wrank"), (152, "<Q", "nch"),
] + [(160 + 8 * s, "<Q", "off_" + SEGS[s]) for s in range(13)] + [
    (264 + 8 * s, "<Q", "len_" + SEGS[s]) for s in range(13)] + [
    (376, "<I", "adler32"), (380, "<I", "zero380"),
]


def parse_header(b: bytes) -> dict:
    h = {}
    for off, code, name in FIELDS:
        h[name] = struct.unpack_from(code, b, off)[0]
    h["topo"] = h["flags"] & 1
    h["field_scope"] = (h["flags"] >> 1) & 1
    h["dims"] = [h["dim0"], h["dim1"], h["dim2"]][: h["ndim"]]
    h["w"] = [h["w%d" % j] for j in range(10)]
    h["off"] = {s: h["off_" + s] for s in SEGS}
    h["len"] = {s: h["len_" + s] for s in SEGS}
    return h


def layout(n: int, topo: int, wdata: int, wrank: int):
    """Segment lengths and offsets: fixed-size parts first, each start
    rounded up to 8 bytes after the previous end, the first at byte 512."""
    nb = -(-n // 64)
    nch = -(-nb // 64)
    t = 1 if topo else 0
    lens = {"S1": 8 * nch, "S2": nb, "S3": 8 * nb, "S4": 4 * nb, "S6": t * 16 * nb,
            "R1": t * 8 * nch, "R2": t * nb, "R3": t * 8 * nb, "R4": t * 4 * nb,
            "X1": 8 * nch, "X2": t * 8 * nch, "S5": 8 * wdata, "R5": t * 8 * wrank}
    offs, pos = {}, HDR
    for s in SEGS:
        offs[s] = pos
        pos = (pos + lens[s] + 7) // 8 * 8 if s != SEGS[-1] else pos + lens[s]
    return offs, lens, pos


def seg(b: bytes, h: dict, name: str) -> bytes:
    return bytes(b[h["off"][name]: h["off"][name] + h["len"][name]])


def decode_map(b: bytes, h: dict, which: str) -> np.ndarray:
    """Values of the data map (which='S': bin indices) or the rank map
    (which='R') for the n points: per 64-point block a width byte, a sign
    word, a first value and w bit planes; residual i of a block has bit j of
    its magnitude at bit i of plane j and its sign at bit i of the sign word;
    value 0 of a block is its first value, value i the sum of the first
    value and residuals 1..i."""
    nb, n = h["nb"], h["n"]
    widths = np.frombuffer(seg(b, h, which + "2"), np.uint8)
    signs = np.frombuffer(seg(b, h, which + "3"), "<u8")
    firsts = np.frombuffer(seg(b, h, which + "4"), "<i4")
    planes = np.frombuffer(seg(b, h, which + "5" if which == "R" else "S5"), "<u8")
    out = np.zeros(nb * 64, np.int64)
    pos = 0
    for blk in range(nb):
        w = int(widths[blk])
        mag = np.zeros(64, np.int64)
        for j in range(w):
            pl = int(planes[pos + j])
            mag |= np.array([(pl >> i) & 1 for i in range(64)], np.int64) << j
        pos += w
        sg = int(signs[blk])
        r = np.where(np.array([(sg >> i) & 1 for i in range(64)], bool), -mag, mag)
        r[0] = int(firsts[blk])
        out[blk * 64: blk * 64 + 64] = np.cumsum(r)
    return out[:n]


def decode_labels(b: bytes, h: dict) -> np.ndarray:
    raw = np.frombuffer(seg(b, h, "S6"), np.uint8)
    i = np.arange(h["n"])
    return (raw[i >> 2] >> (2 * (i & 3))) & 3


def encode_map(v: np.ndarray):
    """Block coding of an integer map (the inverse of decode_map): returns
    (constant bitmap, widths, sign words, first values, chunk offsets,
    planes) as bytes, and the plane count."""
    n = v.size
    nb = -(-n // 64)
    nch = -(-nb // 64)
    pad = np.empty(nb * 64, np.int64)
    pad[:n] = v
    pad[n:] = v[-1]  # the last block repeats its last value
    const = bytearray(8 * nch)
    widths = bytearray(nb)
    signs, firsts, xoff, planes = [], [], [], []
    for blk in range(nb):
        if blk % 64 == 0:
            xoff.append(8 * len(planes))
        x = pad[blk * 64: blk * 64 + 64]
        r = np.zeros(64, np.int64)
        r[1:] = np.diff(x)
        mag = np.abs(r)
        w = int(mag.max()).bit_length()
        if w == 0:
            const[blk // 8] |= 1 << (blk % 8)
        widths[blk] = w
        signs.append(sum(1 << i for i in range(64) if r[i] < 0))
        firsts.append(int(x[0]))
        for j in range(w):
            planes.append(sum(((int(mag[i]) >> j) & 1) << i for i in range(64)))
    return (bytes(const), bytes(widths), struct.pack("<%dQ" % nb, *signs),
            struct.pack("<%di" % nb, *firsts), struct.pack("<%dQ" % nch, *xoff),
            struct.pack("<%dQ" % len(planes), *planes), len(planes))


def with_ranks(b: bytes, delta: np.ndarray) -> bytes:
    """The stream b with its rank map replaced by delta (n integers): the
    rank segments, the header's rank-plane count, total size and R5 length
    are rewritten and the header checksum recomputed."""
    h = parse_header(b)
    assert h["topo"] == 1
    r1, r2, r3, r4, x2, r5, wr = encode_map(np.asarray(delta, np.int64).reshape(-1))
    offs, lens, total = layout(h["n"], 1, h["wdata"], wr)
    assert all(offs[s] == h["off"][s] for s in SEGS)
    out = bytearray(total)
    out[: offs["R5"]] = b[: offs["R5"]]
    for name, data in (("R1", r1), ("R2", r2), ("R3", r3), ("R4", r4), ("X2", x2), ("R5", r5)):
        assert len(data) == lens[name]
        out[offs[name]: offs[name] + len(data)] = data
    struct.pack_into("<Q", out, 128, total)
    struct.pack_into("<Q", out, 144, wr)
    struct.pack_into("<Q", out, 264 + 8 * SEGS.index("R5"), lens["R5"])
    struct.pack_into("<I", out, SUMMED, zlib.adler32(bytes(out[:SUMMED])))
    return bytes(out)


def corruptions(b: bytes):
    """(name, stream) pairs, each breaking one segment rule of the table
    while the header stays valid: chunk offsets, constant bitmaps (a wrong
    bit, a bit past the last block), widths, a first value out of the bin
    index range, and a truncated stream.  Needs a topology stream of more
    than one chunk whose last chunk is partial."""
    h = parse_header(b)
    assert h["topo"] == 1 and h["nch"] >= 2 and h["nb"] % 64 != 0
    out = []

    def put(name, segname, off, fmt, value):
        t = bytearray(b)
        struct.pack_into(fmt, t, h["off"][segname] + off, value)
        out.append((name, bytes(t)))

    x1 = np.frombuffer(seg(b, h, "X1"), "<u8")
    x2 = np.frombuffer(seg(b, h, "X2"), "<u8")
    put("X1 chunk 1 off by 8", "X1", 8, "<Q", int(x1[1]) + 8)
    put("X1 chunk 0 not 0", "X1", 0, "<Q", 8)
    put("X1 last past S5", "X1", 8 * (h["nch"] - 1), "<Q", h["len"]["S5"] + 8)
    put("X2 chunk 1 off by 8", "X2", 8, "<Q", int(x2[1]) + 8)
    put("X2 chunk 1 minus 8", "X2", 8, "<Q", max(int(x2[1]) - 8, 0) if int(x2[1]) else 8)
    widths = np.frombuffer(seg(b, h, "S2"), np.uint8)
    rwidths = np.frombuffer(seg(b, h, "R2"), np.uint8)
    k = int(np.nonzero(widths)[0][0])
    t = bytearray(b)
    t[h["off"]["S1"] + k // 8] ^= 1 << (k % 8)
    out.append(("S1 bit set on a coded block", bytes(t)))
    nz = np.nonzero(rwidths == 0)[0]
    k = int(nz[0])
    t = bytearray(b)
    t[h["off"]["R1"] + k // 8] ^= 1 << (k % 8)
    out.append(("R1 bit cleared on a constant block", bytes(t)))
    for segname in ("S1", "R1"):
        t = bytearray(b)
        k = h["nb"]  # first block past the end
        t[h["off"][segname] + k // 8] |= 1 << (k % 8)
        out.append((segname + " bit past the last block", bytes(t)))
    put("S2 width 24", "S2", 0, "<B", 24)
    put("S2 width +1", "S2", int(np.argmax(widths)), "<B", int(widths.max()) + 1)
    put("R2 width 32", "R2", 1, "<B", 32)
    put("R2 width +1", "R2", int(np.argmax(rwidths)), "<B", int(rwidths.max()) + 1)
    put("S4 first value 2^22", "S4", 4, "<i", 1 << 22)
    put("S4 first value -2^22", "S4", 0, "<i", -(1 << 22))
    put("R4 rank 65", "R4", 8, "<i", 65)
    put("R4 rank -1", "R4", 0, "<i", -1)
    out.append(("truncated by one byte", b[:-1]))
    out.append(("truncated to the header", b[:HDR]))
    return out
