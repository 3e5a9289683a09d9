"""Calls on different workspaces from several host threads at once: every
thread's streams and reconstructions equal the oracle's, while another
thread changes the launch shapes (which change no byte)."""
import threading

import numpy as np
import pytest

from paper_2602_17552_amd import datagen

pytestmark = pytest.mark.gpu


def test_threads_on_separate_workspaces(tsz, ora):
    import torch
    fields = [datagen.gaussian_bumps_2d(150 + 10 * k, 170, 6, seed=40 + k) for k in range(3)] + \
             [datagen.grf_3d(20, 22, 24, seed=44)]
    expect = []
    for f in fields:
        rc, s = ora.compress(f, 1e-3, "rel")
        assert rc == 0
        rc, rec, _ = ora.decompress(s, f.shape)
        assert rc == 0
        expect.append((s, rec))
    saved = tsz.get_tuning()
    errors = []

    def work(k):
        try:
            f = fields[k]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):  # this thread's allocations and work on its own stream
                ws = tsz.Workspace(f.shape, torch.device("cuda:0"), stream=st)
                d = torch.from_numpy(f).cuda()
                for _ in range(5):
                    rc, s = tsz.compress(d, 1e-3, "rel", ws=ws, stream=st)
                    assert rc == 0
                    rc, rec = tsz.decompress(s, f.shape, ws=ws, stream=st)
                    assert rc == 0
                    assert np.array_equal(s.cpu().numpy(), expect[k][0]), "thread %d stream" % k
                    assert np.array_equal(rec.cpu().numpy().view(np.uint32), expect[k][1].view(np.uint32)), k
        except Exception as exc:  # reported by the main thread
            errors.append((k, repr(exc)))

    def retune():
        for t in [(8, 8, 4, 4), (4, 4, 8, 8)] * 10:
            tsz.set_tuning(*t)

    try:
        threads = [threading.Thread(target=work, args=(k,)) for k in range(len(fields))]
        threads.append(threading.Thread(target=retune))
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=100)
        assert not any(t.is_alive() for t in threads), "a thread did not finish"
        assert not errors, errors
    finally:
        tsz.set_tuning(**saved)
