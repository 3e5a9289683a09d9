"""The allocation-free compression entry point (the library's per-device
scratch instead of a caller workspace) against toposzp_compress, through the
C ABI: streams, sizes and statuses must be equal byte for byte, on calls in a
row that reuse the scratch, the later ones on smaller fields."""
import ctypes as C

import numpy as np
import pytest

from paper_2602_17552_amd import datagen

pytestmark = pytest.mark.gpu


def _both(tsz, f, eb, mode, **params):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    shape = tuple(f.shape)
    cap = tsz.compress_bound(shape)
    # reference: the workspace entry point
    out_r, size_r, st_r = tsz.compress_async(d, eb, mode, **params)
    # the scratch entry point, into buffers pre-filled with garbage
    out = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
    size = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    tsz.compress_noalloc_async(d, out, size, st, eb, mode, **params)
    torch.cuda.synchronize()
    assert int(st.item()) == int(st_r.item())
    assert int(size.item()) == int(size_r.item())
    n = int(size.item())
    assert np.array_equal(out[:n].cpu().numpy(), out_r[:n].cpu().numpy())
    return int(st.item()), n


def test_noalloc_equals_workspace_call(tsz):
    # two calls in a row on one device: the second, smaller one reuses the
    # scratch the first left behind
    big = datagen.sinusoids_2d(1200, 2500, seed=5)
    small = datagen.gaussian_bumps_2d(97, 131, 12, seed=6)
    for f, eb, mode in [(big, 1e-3, "rel"), (small, 1e-2, "rel")]:
        st, n = _both(tsz, f, eb, mode)
        assert st == tsz.OK and n > 512


def test_noalloc_more_cases(tsz):
    cases = [
        (datagen.grf_3d(70, 64, 66, seed=7), 1e-3, "rel", {}),
        (datagen.sinusoids_2d(300, 700, seed=8), 0.004, "abs", {"topo": False}),
        (datagen.gaussian_bumps_2d(5, 3, 2, seed=9), 1e-3, "rel", {"rbf_policy": 1}),
        (datagen.grf_3d(256, 256, 256, seed=2), 1e-3, "rel", {}),  # the largest size class
        (datagen.gaussian_bumps_2d(33, 65, 4, seed=10), 1e-3, "rel", {}),
    ]
    for f, eb, mode, params in cases:
        st, n = _both(tsz, f, eb, mode, **params)
        assert st == tsz.OK and n > 512
    # a device-side error (non-finite input) is reported like the reference call's
    bad = datagen.gaussian_bumps_2d(40, 50, 4, seed=11)
    bad[3, 4] = np.nan
    st, n = _both(tsz, bad, 1e-3, "rel")
    assert st == tsz.E_NONFINITE and n == 0


def test_noalloc_host_rejections(tsz):
    import torch
    L = tsz.lib()
    fake = C.c_void_p(4096)
    p = tsz.Params(64, 0, 0, 16, 1)
    too_big = (C.c_uint64 * 3)(4097, 4096, 1)
    assert L.toposzp_compress_noalloc(fake, 2, too_big, 1, 1e-3, C.byref(p), fake, 1 << 40, fake, fake,
                                      None) == tsz.E_CAPACITY
    pf = tsz.Params(64, 1, 0, 16, 1)
    ok_dims = (C.c_uint64 * 3)(64, 64, 1)
    assert L.toposzp_compress_noalloc(fake, 2, ok_dims, 1, 1e-3, C.byref(pf), fake, 1 << 40, fake, fake,
                                      None) == tsz.E_UNSUPPORTED
    # an output buffer below the bound is rejected on the host
    f = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    out = torch.empty(100, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        tsz.compress_noalloc_async(f, out, size, st, 1e-3, "rel")
