"""TopoSZp on MI355X: Python binding of libtoposzp.so.

Argument marshalling only: every step of compression and decompression runs in
the library's HIP kernels.  PyTorch provides device memory and the current
stream.  Importing the package does not load the library; the first call does,
and raises if the library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtoposzp.so")

OK, E_INVALID_ARG, E_NONFINITE, E_RANGE, E_CAPACITY, E_CORRUPT, E_DEVICE, E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
EB_ABS, EB_REL = 0, 1
SYMBOLS = [
    "toposzp_version", "toposzp_strerror", "toposzp_compress_bound", "toposzp_workspace_size",
    "toposzp_workspace_init", "toposzp_compress", "toposzp_decompress", "toposzp_compress_sync",
    "toposzp_decompress_sync", "toposzp_inspect", "toposzp_decompress_stats",
    "toposzp_set_timing", "toposzp_kernel_times",
    "toposzp_compress_batch_workspace_size", "toposzp_decompress_batch_workspace_size",
    "toposzp_compress_batch", "toposzp_decompress_batch", "toposzp_decompress_batch_stats",
    "toposzp_set_tuning", "toposzp_get_tuning", "toposzp_autotune_compress_batch",
    "toposzp_autotune_decompress_batch", "toposzp_eval", "toposzp_compress_bound_ex",
    "toposzp_workspace_size_ex", "toposzp_compress_noalloc",
]
NOALLOC_MAX_POINTS = 1 << 24


class Params(C.Structure):
    _fields_ = [("block", C.c_uint32), ("rank_scope", C.c_int32), ("rbf_policy", C.c_int32),
                ("max_rounds", C.c_int32), ("topo", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("topo", C.c_int32), ("rank_scope", C.c_int32),
                ("eb_mode", C.c_int32), ("k_size", C.c_int32), ("max_rounds", C.c_int32),
                ("dims", C.c_uint64 * 3), ("n", C.c_uint64), ("nblocks", C.c_uint64),
                ("total_bytes", C.c_uint64), ("data_planes", C.c_uint64),
                ("rank_planes", C.c_uint64), ("eb", C.c_double), ("eps", C.c_double),
                ("e", C.c_float), ("vmin", C.c_float), ("vmax", C.c_float),
                ("sigma", C.c_float)]


class CompressJob(C.Structure):
    _fields_ = [("d_field", C.c_void_p), ("ndim", C.c_uint32), ("dims", C.c_uint64 * 3),
                ("eb_mode", C.c_int32), ("eb", C.c_double), ("d_out", C.c_void_p),
                ("out_cap", C.c_size_t), ("d_out_size", C.c_void_p), ("d_status", C.c_void_p)]


class DecompressJob(C.Structure):
    _fields_ = [("d_in", C.c_void_p), ("in_size", C.c_size_t), ("d_out", C.c_void_p),
                ("out_cap_elems", C.c_size_t), ("d_status", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("encode_waves", C.c_int32), ("decode_waves", C.c_int32),
                ("compress_wgs_per_cu", C.c_int32), ("decompress_wgs_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded libtoposzp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        u64p = C.POINTER(C.c_uint64)
        vp = C.c_void_p
        L.toposzp_version.restype = C.c_int
        L.toposzp_strerror.restype = C.c_char_p
        L.toposzp_strerror.argtypes = [C.c_int]
        L.toposzp_compress_bound.restype = C.c_size_t
        L.toposzp_compress_bound.argtypes = [C.c_uint32, u64p]
        L.toposzp_workspace_size.restype = C.c_size_t
        L.toposzp_workspace_size.argtypes = [C.c_uint32, u64p]
        L.toposzp_workspace_init.restype = C.c_int
        L.toposzp_workspace_init.argtypes = [vp, C.c_size_t, vp]
        L.toposzp_compress.restype = C.c_int
        L.toposzp_compress.argtypes = [vp, C.c_uint32, u64p, C.c_int, C.c_double,
                                       C.POINTER(Params), vp, C.c_size_t, vp, C.c_size_t,
                                       vp, vp, vp]
        L.toposzp_compress_noalloc.restype = C.c_int
        L.toposzp_compress_noalloc.argtypes = [vp, C.c_uint32, u64p, C.c_int, C.c_double,
                                               C.POINTER(Params), vp, C.c_size_t, vp, vp, vp]
        L.toposzp_decompress.restype = C.c_int
        L.toposzp_decompress.argtypes = [vp, C.c_size_t, vp, C.c_size_t, vp, C.c_size_t, vp, vp]
        L.toposzp_compress_sync.restype = C.c_int
        L.toposzp_compress_sync.argtypes = [vp, C.c_uint32, u64p, C.c_int, C.c_double,
                                            C.POINTER(Params), vp, C.c_size_t, vp, C.c_size_t,
                                            C.POINTER(C.c_uint64), vp]
        L.toposzp_decompress_sync.restype = C.c_int
        L.toposzp_decompress_sync.argtypes = [vp, C.c_size_t, vp, C.c_size_t, vp, C.c_size_t, vp]
        L.toposzp_inspect.restype = C.c_int
        L.toposzp_inspect.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(Info)]
        L.toposzp_decompress_stats.restype = C.c_int
        L.toposzp_decompress_stats.argtypes = [vp, C.POINTER(C.c_int64), vp]
        L.toposzp_set_timing.restype = C.c_int
        L.toposzp_set_timing.argtypes = [C.c_int]
        L.toposzp_kernel_times.restype = C.c_int
        L.toposzp_kernel_times.argtypes = [C.POINTER(C.c_float), C.c_int]
        L.toposzp_compress_bound_ex.restype = C.c_size_t
        L.toposzp_compress_bound_ex.argtypes = [C.c_uint32, u64p, C.c_int32]
        L.toposzp_workspace_size_ex.restype = C.c_size_t
        L.toposzp_workspace_size_ex.argtypes = [C.c_uint32, u64p, C.c_int32]
        L.toposzp_eval.restype = C.c_int
        L.toposzp_eval.argtypes = [vp, vp, C.c_uint32, u64p, vp, vp, vp]
        cjp, djp = C.POINTER(CompressJob), C.POINTER(DecompressJob)
        L.toposzp_compress_batch_workspace_size.restype = C.c_size_t
        L.toposzp_compress_batch_workspace_size.argtypes = [C.c_uint32, cjp]
        L.toposzp_decompress_batch_workspace_size.restype = C.c_size_t
        L.toposzp_decompress_batch_workspace_size.argtypes = [C.c_uint32, djp]
        L.toposzp_compress_batch.restype = C.c_int
        L.toposzp_compress_batch.argtypes = [C.c_uint32, cjp, C.POINTER(Params), vp, C.c_size_t, vp]
        L.toposzp_decompress_batch.restype = C.c_int
        L.toposzp_decompress_batch.argtypes = [C.c_uint32, djp, vp, C.c_size_t, vp]
        L.toposzp_decompress_batch_stats.restype = C.c_int
        L.toposzp_decompress_batch_stats.argtypes = [C.c_uint32, djp, vp, C.c_uint32,
                                                     C.POINTER(C.c_int64), vp]
        L.toposzp_set_tuning.restype = C.c_int
        L.toposzp_set_tuning.argtypes = [C.POINTER(Tuning)]
        L.toposzp_get_tuning.restype = C.c_int
        L.toposzp_get_tuning.argtypes = [C.POINTER(Tuning)]
        L.toposzp_autotune_compress_batch.restype = C.c_int
        L.toposzp_autotune_compress_batch.argtypes = [C.c_uint32, cjp, C.POINTER(Params), vp,
                                                      C.c_size_t, vp, C.POINTER(Tuning)]
        L.toposzp_autotune_decompress_batch.restype = C.c_int
        L.toposzp_autotune_decompress_batch.argtypes = [C.c_uint32, djp, vp, C.c_size_t, vp,
                                                        C.POINTER(Tuning)]
        _lib = L
    return _lib


def _dims(shape):
    if len(shape) not in (2, 3):
        raise ValueError(f"fields are 2D or 3D, got shape {tuple(shape)}")
    arr = (C.c_uint64 * 3)(1, 1, 1)
    for k, d in enumerate(shape):
        if int(d) < 1:
            raise ValueError(f"every extent must be >= 1, got shape {tuple(shape)}")
        arr[k] = int(d)
    return arr


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def strerror(status: int) -> str:
    return lib().toposzp_strerror(int(status)).decode()


def compress_bound(shape, rank_scope: int = 0) -> int:
    return int(lib().toposzp_compress_bound_ex(len(shape), _dims(shape), int(rank_scope)))


def workspace_size(shape, rank_scope: int = 0) -> int:
    return int(lib().toposzp_workspace_size_ex(len(shape), _dims(shape), int(rank_scope)))


class Workspace:
    """Device workspace sized for fields up to `shape` (compress and
    decompress), cleared once on creation."""

    def __init__(self, shape, device="cuda", stream=None, rank_scope: int = 0):
        import torch
        nbytes = workspace_size(shape, rank_scope)
        if nbytes == 0:
            raise ValueError(f"invalid field shape {shape}")
        self.shape = tuple(shape)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes
        rc = lib().toposzp_workspace_init(C.c_void_p(self.buf.data_ptr()), nbytes, _stream(stream))
        if rc != OK:
            raise RuntimeError(strerror(rc))

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


def _params(topo=True, rank_scope=0, rbf_policy=0, max_rounds=16):
    return Params(64, int(rank_scope), int(rbf_policy), int(max_rounds), int(bool(topo)))


def compress_async(field, eb, mode="rel", ws=None, out=None, size=None, status=None,
                   stream=None, **params):
    """Enqueues compression of a float32 CUDA tensor.  Returns
    (out uint8 tensor, size uint64[1] tensor, status int32[1] tensor); the
    first size[0] bytes of out are the stream once the call has completed."""
    import torch
    if field.dtype != torch.float32 or not field.is_cuda or not field.is_contiguous():
        raise TypeError("field must be a contiguous float32 CUDA tensor")
    shape = tuple(field.shape)
    scope = int(params.get("rank_scope", 0)) if params.get("topo", True) else 0
    ws = ws or Workspace(shape, field.device, stream, scope)
    if out is None:
        out = torch.empty(compress_bound(shape, scope), dtype=torch.uint8, device=field.device)
    if size is None:
        size = torch.zeros(1, dtype=torch.int64, device=field.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=field.device)
    p = _params(**params)
    rc = lib().toposzp_compress(C.c_void_p(field.data_ptr()), len(shape), _dims(shape),
                                EB_REL if mode == "rel" else EB_ABS, float(eb), C.byref(p),
                                ws.ptr, ws.nbytes, C.c_void_p(out.data_ptr()), out.numel(),
                                C.c_void_p(size.data_ptr()), C.c_void_p(status.data_ptr()),
                                _stream(stream))
    if rc != OK:
        raise RuntimeError(f"toposzp_compress: {strerror(rc)} ({rc})")
    return out, size, status


def compress_noalloc_async(field, out, size, status, eb, mode="rel", stream=None, **params):
    """Enqueues the allocation-free compression (the library's scratch, no
    workspace) into caller buffers: out uint8, size int64[1], status
    int32[1], all CUDA tensors.  Fields of at most NOALLOC_MAX_POINTS points,
    block-scope ranks only."""
    import torch
    if field.dtype != torch.float32 or not field.is_cuda or not field.is_contiguous():
        raise TypeError("field must be a contiguous float32 CUDA tensor")
    shape = tuple(field.shape)
    p = _params(**params)
    rc = lib().toposzp_compress_noalloc(C.c_void_p(field.data_ptr()), len(shape), _dims(shape),
                                        EB_REL if mode == "rel" else EB_ABS, float(eb), C.byref(p),
                                        C.c_void_p(out.data_ptr()), out.numel(), C.c_void_p(size.data_ptr()),
                                        C.c_void_p(status.data_ptr()), _stream(stream))
    if rc != OK:
        raise RuntimeError(f"toposzp_compress_noalloc: {strerror(rc)} ({rc})")
    return out, size, status


def compress(field, eb, mode="rel", ws=None, stream=None, **params):
    """Synchronous compression: returns (status, stream bytes as a uint8 CUDA
    tensor view of the output buffer)."""
    import torch
    out, size, status = compress_async(field, eb, mode, ws=ws, stream=stream, **params)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    st = int(status.item())
    return st, out[: int(size.item())] if st == OK else out[:0]


def decompress_async(stream_bytes, nbytes, out, ws=None, status=None, stream=None):
    """Enqueues decompression into the float32 CUDA tensor `out` (its numel is
    the capacity).  Returns the status int32[1] tensor."""
    import torch
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous():
        raise TypeError("out must be a contiguous float32 CUDA tensor")
    ws = ws or Workspace(tuple(out.shape), out.device, stream)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=out.device)
    rc = lib().toposzp_decompress(C.c_void_p(stream_bytes.data_ptr()), int(nbytes),
                                  C.c_void_p(out.data_ptr()), out.numel(), ws.ptr, ws.nbytes,
                                  C.c_void_p(status.data_ptr()), _stream(stream))
    if rc != OK:
        raise RuntimeError(f"toposzp_decompress: {strerror(rc)} ({rc})")
    return status


def decompress(stream_bytes, shape, ws=None, nbytes=None, stream=None):
    """Synchronous decompression: returns (status, float32 CUDA tensor)."""
    import torch
    out = torch.empty(tuple(shape), dtype=torch.float32, device=stream_bytes.device)
    nb = stream_bytes.numel() if nbytes is None else nbytes
    status = decompress_async(stream_bytes, nb, out, ws=ws, stream=stream)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return int(status.item()), out


def decompress_stats(ws, stream=None):
    arr = (C.c_int64 * 5)()
    rc = lib().toposzp_decompress_stats(ws.ptr, arr, _stream(stream))
    if rc != OK:
        raise RuntimeError(strerror(rc))
    keys = ["rounds", "commits", "queued", "stencil_moves", "budget_skips"]
    return {k: int(arr[i]) for i, k in enumerate(keys)}


def inspect(header: bytes):
    info = Info()
    rc = lib().toposzp_inspect(header, len(header), C.byref(info))
    if rc != OK:
        return rc, None
    d = {k: getattr(info, k) for k, _ in Info._fields_}
    d["dims"] = [int(x) for x in info.dims]
    return rc, d


def eval_topology(orig, recon, stream=None):
    """False negatives / positives / types of `recon` against `orig` (Section
    III-B) on the GPU: dict with FN, FP, FT, critical points of the original
    by class, FN by class, and the largest absolute error."""
    import torch
    if orig.shape != recon.shape or orig.dtype != torch.float32 or recon.dtype != torch.float32:
        raise TypeError("orig and recon must be float32 tensors of one shape")
    counts = torch.zeros(11, dtype=torch.int64, device=orig.device)
    mx = torch.zeros(1, dtype=torch.float64, device=orig.device)
    shape = tuple(orig.shape)
    rc = lib().toposzp_eval(C.c_void_p(orig.data_ptr()), C.c_void_p(recon.data_ptr()), len(shape), _dims(shape),
                            C.c_void_p(counts.data_ptr()), C.c_void_p(mx.data_ptr()), _stream(stream))
    if rc != OK:
        raise RuntimeError(f"toposzp_eval: {strerror(rc)} ({rc})")
    c = counts.cpu().tolist()
    return {"FN": c[0], "FP": c[1], "FT": c[2], "cp_r": c[3], "cp_min": c[4], "cp_sad": c[5], "cp_max": c[6],
            "FN_r": c[7], "FN_min": c[8], "FN_sad": c[9], "FN_max": c[10], "max_err": float(mx.item())}


def set_timing(enable: bool):
    lib().toposzp_set_timing(int(bool(enable)))


def kernel_times():
    """ms of the last call's kernels: range, encode, finalize, decode, refine
    (-1 where a kernel did not run); valid after the stream is synchronised."""
    arr = (C.c_float * 5)()
    k = lib().toposzp_kernel_times(arr, 5)
    names = ["range", "encode", "finalize", "decode", "refine"]
    return {names[i]: float(arr[i]) for i in range(k)}


# ---------------------------------------------------------------------------
# Batched form.

def get_tuning() -> dict:
    t = Tuning()
    lib().toposzp_get_tuning(C.byref(t))
    return t.as_dict()


def set_tuning(encode_waves=4, decode_waves=4, compress_wgs_per_cu=8, decompress_wgs_per_cu=8):
    t = Tuning(int(encode_waves), int(decode_waves), int(compress_wgs_per_cu), int(decompress_wgs_per_cu))
    rc = lib().toposzp_set_tuning(C.byref(t))
    if rc != OK:
        raise ValueError(f"toposzp_set_tuning: {strerror(rc)}")


class CompressBatch:
    """Compression of several float32 CUDA fields in one batched call.

    fields: list of contiguous float32 CUDA tensors (2D or 3D); ebs: one bound
    per field; modes: "rel"/"abs" per field (or one for all).  Output buffers,
    sizes, statuses and the workspace are allocated once here and reused by
    every run()."""

    def __init__(self, fields, ebs, modes="rel", device=None, **params):
        import torch
        n = len(fields)
        if n < 1:
            raise ValueError("empty batch")
        if isinstance(modes, str):
            modes = [modes] * n
        self.fields = list(fields)
        device = device or self.fields[0].device
        self.outs, self.caps = [], []
        self.sizes = torch.zeros(n, dtype=torch.int64, device=device)
        self.status = torch.zeros(n, dtype=torch.int32, device=device)
        self.jobs = (CompressJob * n)()
        for i, f in enumerate(self.fields):
            if f.dtype != torch.float32 or not f.is_cuda or not f.is_contiguous() or f.dim() not in (2, 3):
                raise TypeError("fields must be contiguous 2D/3D float32 CUDA tensors")
            cap = compress_bound(tuple(f.shape))
            out = torch.empty(cap, dtype=torch.uint8, device=device)
            self.outs.append(out)
            j = self.jobs[i]
            j.d_field = f.data_ptr()
            j.ndim = f.dim()
            j.dims = _dims(tuple(f.shape))
            j.eb_mode = EB_REL if modes[i] == "rel" else EB_ABS
            j.eb = float(ebs[i])
            j.d_out = out.data_ptr()
            j.out_cap = cap
            j.d_out_size = self.sizes.data_ptr() + 8 * i
            j.d_status = self.status.data_ptr() + 4 * i
        self.params = _params(**params)
        nbytes = int(lib().toposzp_compress_batch_workspace_size(n, self.jobs))
        if nbytes == 0:
            raise ValueError("invalid batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        rc = lib().toposzp_workspace_init(C.c_void_p(self.ws.data_ptr()), nbytes, _stream(None))
        if rc != OK:
            raise RuntimeError(strerror(rc))

    def run(self, stream=None):
        rc = lib().toposzp_compress_batch(len(self.fields), self.jobs, C.byref(self.params),
                                          C.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream(stream))
        if rc != OK:
            raise RuntimeError(f"toposzp_compress_batch: {strerror(rc)} ({rc})")

    def autotune(self, stream=None) -> dict:
        t = Tuning()
        rc = lib().toposzp_autotune_compress_batch(len(self.fields), self.jobs, C.byref(self.params),
                                                   C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                   _stream(stream), C.byref(t))
        if rc != OK:
            raise RuntimeError(f"toposzp_autotune_compress_batch: {strerror(rc)} ({rc})")
        return t.as_dict()

    def results(self):
        """(statuses, [stream bytes views]) after the stream has been synchronised."""
        st = self.status.cpu().tolist()
        sz = self.sizes.cpu().tolist()
        return st, [o[: int(z)] for o, z in zip(self.outs, sz)]


class DecompressBatch:
    """Decompression of several streams (uint8 CUDA tensors) into float32
    CUDA tensors of the given shapes, in one batched call."""

    def __init__(self, streams, shapes, device=None):
        import torch
        n = len(streams)
        if n < 1 or len(shapes) != n:
            raise ValueError("streams and shapes must be non-empty and of equal length")
        device = device or streams[0].device
        self.streams = list(streams)
        self.recs = [torch.empty(tuple(sh), dtype=torch.float32, device=device) for sh in shapes]
        self.status = torch.zeros(n, dtype=torch.int32, device=device)
        self.jobs = (DecompressJob * n)()
        for i, (sb, r) in enumerate(zip(self.streams, self.recs)):
            j = self.jobs[i]
            j.d_in = sb.data_ptr()
            j.in_size = sb.numel()
            j.d_out = r.data_ptr()
            j.out_cap_elems = r.numel()
            j.d_status = self.status.data_ptr() + 4 * i
        nbytes = int(lib().toposzp_decompress_batch_workspace_size(n, self.jobs))
        if nbytes == 0:
            raise ValueError("invalid batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        rc = lib().toposzp_workspace_init(C.c_void_p(self.ws.data_ptr()), nbytes, _stream(None))
        if rc != OK:
            raise RuntimeError(strerror(rc))

    def run(self, stream=None):
        rc = lib().toposzp_decompress_batch(len(self.streams), self.jobs, C.c_void_p(self.ws.data_ptr()),
                                            self.ws.numel(), _stream(stream))
        if rc != OK:
            raise RuntimeError(f"toposzp_decompress_batch: {strerror(rc)} ({rc})")

    def autotune(self, stream=None) -> dict:
        t = Tuning()
        rc = lib().toposzp_autotune_decompress_batch(len(self.streams), self.jobs,
                                                     C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                     _stream(stream), C.byref(t))
        if rc != OK:
            raise RuntimeError(f"toposzp_autotune_decompress_batch: {strerror(rc)} ({rc})")
        return t.as_dict()

    def stats(self, index, stream=None):
        arr = (C.c_int64 * 5)()
        rc = lib().toposzp_decompress_batch_stats(len(self.streams), self.jobs, C.c_void_p(self.ws.data_ptr()),
                                                  int(index), arr, _stream(stream))
        if rc != OK:
            raise RuntimeError(strerror(rc))
        keys = ["rounds", "commits", "queued", "stencil_moves", "budget_skips"]
        return {k: int(arr[i]) for i, k in enumerate(keys)}
