"""ctypes binding of the TopoSZp CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
module.  It builds `liboracle.so` from `toposzp_oracle.c` with gcc if no build
is present.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "toposzp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID_ARG, E_NONFINITE, E_RANGE, E_CAPACITY, E_CORRUPT, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -7
R, MIN, SAD, MAX = 0, 1, 2, 3

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile the oracle shared library (plain gcc, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("topo", C.c_int), ("rank_scope", C.c_int),
                ("rbf_policy", C.c_int), ("max_rounds", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("commits", C.c_int64),
                ("worklist0", C.c_int64), ("stencil_moves", C.c_int64),
                ("budget_skips", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L.ora_compress_bound.restype = C.c_size_t
        L.ora_compress_bound.argtypes = [C.c_int, u64p, C.c_int]
        L.ora_compress.restype = C.c_int
        L.ora_compress.argtypes = [f32p, C.c_int, u64p, C.c_int, C.c_double,
                                   C.POINTER(Params), u8p, C.c_size_t, C.POINTER(C.c_size_t)]
        L.ora_decompress.restype = C.c_int
        L.ora_decompress.argtypes = [u8p, C.c_size_t, f32p, C.c_size_t, C.POINTER(Stats)]
        L.ora_eval.restype = None
        L.ora_eval.argtypes = [f32p, f32p, C.c_int, u64p, i64p, C.POINTER(C.c_double)]
        L.ora_eps_float.restype = C.c_float
        L.ora_eps_float.argtypes = [C.c_double]
        L.ora_quantize.restype = C.c_int
        L.ora_quantize.argtypes = [C.c_float, C.c_float, C.POINTER(C.c_int32)]
        L.ora_recon.restype = C.c_float
        L.ora_recon.argtypes = [C.c_int32, C.c_float]
        L.ora_classify.restype = None
        L.ora_classify.argtypes = [f32p, C.c_int, u64p, u8p]
        L.ora_quantize_field.restype = C.c_int
        L.ora_quantize_field.argtypes = [f32p, C.c_size_t, C.c_float, i32p]
        L.ora_labels_ranks.restype = None
        L.ora_labels_ranks.argtypes = [f32p, i32p, C.c_int, u64p, C.c_int, u8p, i32p]
        L.ora_rbf_weights.restype = None
        L.ora_rbf_weights.argtypes = [C.c_double, f32p]
        L.ora_encode_block.restype = C.c_int
        L.ora_encode_block.argtypes = [i32p, C.POINTER(C.c_int32), C.POINTER(C.c_uint64), u64p]
        L.ora_decode_block.restype = None
        L.ora_decode_block.argtypes = [C.c_int, C.c_int32, C.c_uint64, u64p, i32p]
        L.ora_inspect.restype = C.c_int
        L.ora_inspect.argtypes = [u8p, C.c_size_t, i64p, f64p, u64p, u64p]
        _lib = L
    return _lib


def _dims(shape):
    d = np.ones(3, dtype=np.uint64)
    d[: len(shape)] = shape
    return d


def compress(field: np.ndarray, eb: float, mode: str = "rel", topo: bool = True,
             rank_scope: int = 0, rbf_policy: int = 0, max_rounds: int = 16):
    """Returns (status, stream bytes as uint8 array)."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    dims = _dims(f.shape)
    cap = lib().ora_compress_bound(f.ndim, dims, rank_scope)
    if cap == 0:
        cap = 1 << 12
    out = np.zeros(cap, dtype=np.uint8)
    size = C.c_size_t(0)
    p = Params(int(topo), rank_scope, rbf_policy, max_rounds)
    rc = lib().ora_compress(f.reshape(-1), f.ndim, dims, 1 if mode == "rel" else 0,
                            float(eb), C.byref(p), out, cap, C.byref(size))
    return rc, out[: size.value].copy() if rc == OK else out[:0]


def decompress(stream: np.ndarray, shape):
    """Returns (status, reconstruction, stats dict)."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    n = int(np.prod(shape))
    out = np.zeros(max(n, 1), dtype=np.float32)
    st = Stats()
    rc = lib().ora_decompress(s if s.size else np.zeros(1, np.uint8), s.size, out, n, C.byref(st))
    stats = {k: getattr(st, k) for k, _ in Stats._fields_}
    return rc, out[:n].reshape(shape), stats


def eval_topology(orig: np.ndarray, recon: np.ndarray):
    """FN/FP/FT counts (Section III-B) and max |orig - recon|."""
    o = np.ascontiguousarray(orig, dtype=np.float32)
    r = np.ascontiguousarray(recon, dtype=np.float32)
    counts = np.zeros(11, dtype=np.int64)
    mx = C.c_double(0.0)
    lib().ora_eval(o.reshape(-1), r.reshape(-1), o.ndim, _dims(o.shape), counts, C.byref(mx))
    return {"FN": int(counts[0]), "FP": int(counts[1]), "FT": int(counts[2]),
            "n_r": int(counts[3]), "n_min": int(counts[4]), "n_sad": int(counts[5]),
            "n_max": int(counts[6]), "FN_min": int(counts[8]), "FN_sad": int(counts[9]),
            "FN_max": int(counts[10]), "max_abs_err": mx.value}


def classify(field: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(field, dtype=np.float32)
    out = np.zeros(f.size, dtype=np.uint8)
    lib().ora_classify(f.reshape(-1), f.ndim, _dims(f.shape), out)
    return out.reshape(f.shape)


def eps_float(eps_d: float) -> float:
    return float(np.float32(lib().ora_eps_float(float(eps_d))))


def quantize(a: float, e: float):
    q = C.c_int32(0)
    rc = lib().ora_quantize(float(np.float32(a)), float(np.float32(e)), C.byref(q))
    return rc, q.value


def recon(q: int, e: float) -> np.float32:
    return np.float32(lib().ora_recon(int(q), float(np.float32(e))))


def quantize_field(field: np.ndarray, e: float):
    f = np.ascontiguousarray(field, dtype=np.float32).reshape(-1)
    q = np.zeros(f.size, dtype=np.int32)
    rc = lib().ora_quantize_field(f, f.size, float(np.float32(e)), q)
    return rc, q.reshape(np.shape(field))


def labels_ranks(field: np.ndarray, q: np.ndarray, rank_scope: int = 0):
    f = np.ascontiguousarray(field, dtype=np.float32)
    qq = np.ascontiguousarray(q, dtype=np.int32)
    lab = np.zeros(f.size, dtype=np.uint8)
    dl = np.zeros(f.size, dtype=np.int32)
    lib().ora_labels_ranks(f.reshape(-1), qq.reshape(-1), f.ndim, _dims(f.shape), rank_scope, lab, dl)
    return lab.reshape(f.shape), dl.reshape(f.shape)


def rbf_weights(sigma: float) -> np.ndarray:
    w = np.zeros(10, dtype=np.float32)
    lib().ora_rbf_weights(float(sigma), w)
    return w


def encode_block(v):
    v = np.ascontiguousarray(v, dtype=np.int32)
    first = C.c_int32(0)
    sign = C.c_uint64(0)
    planes = np.zeros(32, dtype=np.uint64)
    w = lib().ora_encode_block(v, C.byref(first), C.byref(sign), planes)
    return w, first.value, sign.value, planes[:w].copy()


def decode_block(w, first, sign, planes):
    p = np.zeros(32, dtype=np.uint64)
    p[:w] = planes
    v = np.zeros(64, dtype=np.int32)
    lib().ora_decode_block(int(w), int(first), int(sign), p, v)
    return v


def inspect(stream: np.ndarray):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    iv = np.zeros(16, dtype=np.int64)
    dv = np.zeros(4, dtype=np.float64)
    so = np.zeros(13, dtype=np.uint64)
    sl = np.zeros(13, dtype=np.uint64)
    rc = lib().ora_inspect(s if s.size else np.zeros(1, np.uint8), s.size, iv, dv, so, sl)
    if rc != OK:
        return rc, None
    keys = ["ndim", "topo", "scope", "eb_mode", "k", "max_rounds", "d0", "d1", "d2",
            "n", "nb", "nchunks", "total", "wdata", "wrank"]
    info = {k: int(iv[i]) for i, k in enumerate(keys)}
    info.update(eb=float(dv[0]), eps_d=float(dv[1]), e=float(dv[2]), sigma=float(dv[3]),
                seg_off=[int(x) for x in so], seg_len=[int(x) for x in sl])
    return rc, info
