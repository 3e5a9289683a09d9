"""Batched form on the GPU: many uneven 2D/3D fields per call.

Every field's stream must equal, byte for byte, both the CPU oracle's and the
one-field GPU call's; every reconstruction must equal the oracle's bit for
bit; launch shapes (tuning, autotuner) must change no byte.
"""
import numpy as np
import pytest

from paper_2602_17552_amd import datagen

pytestmark = pytest.mark.gpu


def _cuda(tsz, fields):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in fields]


def _run_batch(tsz, fields, ebs, modes="rel", **params):
    import torch
    b = tsz.CompressBatch(_cuda(tsz, fields), ebs, modes, **params)
    b.run()
    torch.cuda.synchronize()
    st, streams = b.results()
    return b, st, [s.cpu().numpy() for s in streams]


def _small_batch(seed=21, count2d=10, count3d=4):
    return datagen.batch_fields(count2d, count3d, seed=seed, scale=0.12)


def test_batch_matches_oracle_and_single(tsz, ora):
    import torch
    batch = _small_batch()
    fields = [f for f, _ in batch]
    ebs = [eb for _, eb in batch]
    print("batch shapes", [f.shape for f in fields], flush=True)
    b, st, streams = _run_batch(tsz, fields, ebs)
    assert st == [0] * len(fields)
    for i, (f, eb) in enumerate(batch):
        rc, s_o = ora.compress(f, eb, "rel")
        assert rc == 0
        assert np.array_equal(streams[i], s_o), "field %d %s: batch stream differs from the oracle" % (i, f.shape)
        st1, s1 = tsz.compress(torch.from_numpy(f).cuda(), eb, "rel")
        assert st1 == 0 and np.array_equal(s1.cpu().numpy(), s_o)
    # batched decompression of the batch's own streams
    d = tsz.DecompressBatch([torch.from_numpy(s).cuda() for s in streams], [f.shape for f in fields])
    d.run()
    torch.cuda.synchronize()
    assert d.status.cpu().tolist() == [0] * len(fields)
    for i, f in enumerate(fields):
        rc, rec_o, stats_o = ora.decompress(streams[i], f.shape)
        assert rc == 0
        rec_g = d.recs[i].cpu().numpy()
        assert np.array_equal(rec_g.view(np.uint32), rec_o.view(np.uint32)), "field %d reconstruction" % i
        sg = d.stats(i)
        for k in ("rounds", "commits", "stencil_moves", "budget_skips"):
            assert sg[k] == stats_o[k], (i, k, sg, stats_o)


def test_batch_scan_path(tsz, ora):
    """A job of more than 4096 chunks (16,842,752 points) beside small ones:
    the batch's separate scan kernel and the unfused finalize, against the
    oracle byte for byte and bit for bit."""
    import torch
    fields = [datagen.grf_3d(257, 256, 256, seed=2), datagen.gaussian_bumps_2d(70, 90, 6, seed=23),
              datagen.grf_3d(20, 22, 24, seed=24)]
    ebs = [1e-3, 1e-2, 3e-3]
    b, st, streams = _run_batch(tsz, fields, ebs)
    assert st == [0] * len(fields)
    d = tsz.DecompressBatch([torch.from_numpy(s).cuda() for s in streams], [f.shape for f in fields])
    d.run()
    torch.cuda.synchronize()
    assert d.status.cpu().tolist() == [0] * len(fields)
    for i, (f, eb) in enumerate(zip(fields, ebs)):
        print("scan-path batch job %d %s" % (i, f.shape), flush=True)
        rc, s_o = ora.compress(f, eb, "rel")
        assert rc == 0 and np.array_equal(streams[i], s_o), i
        rc, rec_o, stats_o = ora.decompress(s_o, f.shape)
        assert np.array_equal(d.recs[i].cpu().numpy().view(np.uint32), rec_o.view(np.uint32)), i
        sg = d.stats(i)
        for k in ("rounds", "commits", "stencil_moves", "budget_skips"):
            assert sg[k] == stats_o[k], (i, k, sg, stats_o)


def test_batch_mixed_modes_and_params(tsz, ora):
    fields = [datagen.noise((33, 47), seed=3), datagen.grf_3d(9, 10, 11, seed=4),
              datagen.gaussian_bumps_2d(70, 130, 8, seed=5), datagen.noise((1, 1), seed=6),
              datagen.noise((65, 1), seed=7)]
    ebs = [0.2, 1e-2, 1e-3, 0.1, 0.05]
    modes = ["abs", "rel", "rel", "abs", "abs"]
    for params in ({}, {"topo": False}, {"rbf_policy": 1, "max_rounds": 3}):
        _, st, streams = _run_batch(tsz, fields, ebs, modes, **params)
        assert st == [0] * len(fields), params
        for i, f in enumerate(fields):
            rc, s_o = ora.compress(f, ebs[i], modes[i], **params)
            assert rc == 0 and np.array_equal(streams[i], s_o), (params, i)


def test_batch_per_job_errors(tsz, ora):
    good = datagen.noise((40, 50), seed=8)
    bad = good.copy()
    bad[3, 4] = np.nan
    _, st, streams = _run_batch(tsz, [good, bad, good], [1e-3, 1e-3, 1e-3])
    assert st == [0, tsz.E_NONFINITE, 0]
    rc, s_o = ora.compress(good, 1e-3, "rel")
    assert np.array_equal(streams[0], s_o) and np.array_equal(streams[2], s_o)


def test_batch_host_errors(tsz):
    import ctypes as C
    import torch
    f = torch.from_numpy(datagen.noise((20, 30), seed=9)).cuda()
    b = tsz.CompressBatch([f, f], [1e-3, 1e-3])
    jobs = (tsz.CompressJob * 2)(*b.jobs)
    jobs[1].ndim = 4
    L = tsz.lib()
    assert L.toposzp_compress_batch_workspace_size(2, jobs) == 0
    rc = L.toposzp_compress_batch(2, jobs, C.byref(b.params), C.c_void_p(b.ws.data_ptr()), b.ws.numel(),
                                  tsz._stream(None))
    assert rc == tsz.E_INVALID_ARG
    rc = L.toposzp_compress_batch(2, b.jobs, C.byref(b.params), C.c_void_p(b.ws.data_ptr()), 1024,
                                  tsz._stream(None))
    assert rc == tsz.E_CAPACITY
    assert L.toposzp_compress_batch(0, b.jobs, C.byref(b.params), C.c_void_p(b.ws.data_ptr()),
                                    b.ws.numel(), tsz._stream(None)) == tsz.E_INVALID_ARG
    bad = tsz.Tuning(5, 4, 8, 8)
    assert L.toposzp_set_tuning(C.byref(bad)) == tsz.E_INVALID_ARG


def test_tuning_changes_no_byte(tsz, ora):
    import torch
    batch = _small_batch(seed=22, count2d=6, count3d=3)
    fields = [f for f, _ in batch]
    ebs = [eb for _, eb in batch]
    saved = tsz.get_tuning()
    try:
        ref_streams = None
        ref_recs = None
        for t in [(4, 4, 8, 8), (8, 8, 1, 1), (8, 4, 2, 16), (4, 8, 32, 3)]:
            tsz.set_tuning(*t)
            b, st, streams = _run_batch(tsz, fields, ebs)
            assert st == [0] * len(fields)
            d = tsz.DecompressBatch([torch.from_numpy(s).cuda() for s in streams], [f.shape for f in fields])
            d.run()
            torch.cuda.synchronize()
            recs = [r.cpu().numpy() for r in d.recs]
            # the one-field calls use the same shapes
            st1, s1 = tsz.compress(torch.from_numpy(fields[0]).cuda(), ebs[0], "rel")
            st2, r1 = tsz.decompress(s1, fields[0].shape)
            assert st1 == 0 and st2 == 0
            rc, rec_o, _ = ora.decompress(s1.cpu().numpy(), fields[0].shape)
            r1 = r1.cpu().numpy()
            for name, r in (("one-field", r1), ("batched", recs[0])):
                bad = np.nonzero(r.reshape(-1).view(np.uint32) != rec_o.reshape(-1).view(np.uint32))[0]
                assert bad.size == 0, "%s %s: %d values differ from the oracle, first %s: %r vs %r" % (
                    t, name, bad.size, bad[:5].tolist(), r.reshape(-1)[bad[:5]].tolist(),
                    rec_o.reshape(-1)[bad[:5]].tolist())
            if ref_streams is None:
                ref_streams, ref_recs = streams, recs
                for i, f in enumerate(fields):
                    rc, s_o = ora.compress(f, ebs[i], "rel")
                    assert np.array_equal(streams[i], s_o)
            else:
                for i in range(len(fields)):
                    assert np.array_equal(streams[i], ref_streams[i]), (t, i)
                    assert np.array_equal(recs[i].view(np.uint32), ref_recs[i].view(np.uint32)), (t, i)
    finally:
        tsz.set_tuning(**saved)


def test_autotuner(tsz, ora):
    import torch
    batch = _small_batch(seed=23, count2d=8, count3d=2)
    fields = [f for f, _ in batch]
    ebs = [eb for _, eb in batch]
    saved = tsz.get_tuning()
    try:
        b = tsz.CompressBatch(_cuda(tsz, fields), ebs)
        t = b.autotune()
        assert t["encode_waves"] in (4, 8) and 1 <= t["compress_wgs_per_cu"] <= 32
        torch.cuda.synchronize()
        st, streams = b.results()
        assert st == [0] * len(fields)
        streams = [s.cpu().numpy() for s in streams]
        for i, f in enumerate(fields):
            rc, s_o = ora.compress(f, ebs[i], "rel")
            assert np.array_equal(streams[i], s_o), i
        d = tsz.DecompressBatch([torch.from_numpy(s).cuda() for s in streams], [f.shape for f in fields])
        t2 = d.autotune()
        assert t2["decode_waves"] in (4, 8)
        torch.cuda.synchronize()
        assert d.status.cpu().tolist() == [0] * len(fields)
        for i, f in enumerate(fields):
            rc, rec_o, _ = ora.decompress(streams[i], f.shape)
            assert np.array_equal(d.recs[i].cpu().numpy().view(np.uint32), rec_o.view(np.uint32)), i
    finally:
        tsz.set_tuning(**saved)


@pytest.mark.slow
def test_batch_full_size(tsz, ora):
    """The 64-field batch at full size: every field against its one-field GPU
    call; a sample (the largest 2D and 3D fields and a few others) against the
    oracle; no false or type-changed critical point anywhere (sampled)."""
    import torch
    batch = datagen.batch_fields(48, 16, seed=3)
    fields = [f for f, _ in batch]
    ebs = [eb for _, eb in batch]
    print("full batch: %d fields, %.1f MB" % (len(fields), sum(f.nbytes for f in fields) / 1e6), flush=True)
    b, st, streams = _run_batch(tsz, fields, ebs)
    assert st == [0] * len(fields)
    d = tsz.DecompressBatch([torch.from_numpy(s).cuda() for s in streams], [f.shape for f in fields])
    d.run()
    torch.cuda.synchronize()
    assert d.status.cpu().tolist() == [0] * len(fields)
    for i, f in enumerate(fields):
        st1, s1 = tsz.compress(torch.from_numpy(f).cuda(), ebs[i], "rel")
        assert st1 == 0 and np.array_equal(s1.cpu().numpy(), streams[i]), i
    sizes = [f.size for f in fields]
    big2 = max((i for i in range(len(fields)) if fields[i].ndim == 2), key=lambda i: sizes[i])
    big3 = max((i for i in range(len(fields)) if fields[i].ndim == 3), key=lambda i: sizes[i])
    for i in sorted({big2, big3, 0, 1, 2}):
        print("oracle check field %d %s" % (i, fields[i].shape), flush=True)
        rc, s_o = ora.compress(fields[i], ebs[i], "rel")
        assert rc == 0 and np.array_equal(streams[i], s_o), i
        rc, rec_o, _ = ora.decompress(s_o, fields[i].shape)
        rec_g = d.recs[i].cpu().numpy()
        assert np.array_equal(rec_g.view(np.uint32), rec_o.view(np.uint32)), i
        ev = ora.eval_topology(fields[i], rec_g)
        assert ev["FP"] == 0 and ev["FT"] == 0
