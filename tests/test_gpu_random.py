"""GPU parity on seeded random cases: mixed shapes (2D and 3D, from one cell
to a few hundred thousand points), generators, bound modes and magnitudes,
rank scopes, RBF policies and round caps. Every stream byte, every
reconstructed bit and the refinement counters must equal the oracle's."""
import numpy as np
import pytest

from paper_2602_17552_amd import datagen

pytestmark = pytest.mark.gpu


def _case(rng):
    nd = 2 if rng.random() < 0.7 else 3
    if nd == 2 and rng.random() < 0.1:
        shape = (int(rng.integers(200, 700)), int(rng.integers(200, 700)))
    elif nd == 2:
        shape = (int(rng.integers(1, 200)), int(rng.integers(1, 200)))
    else:
        shape = tuple(int(rng.integers(1, 32)) for _ in range(3))
    kind = int(rng.integers(0, 4))
    seed = int(rng.integers(0, 1 << 30))
    if kind == 1 and nd == 2:
        f = datagen.checker_2d(*shape, seed=seed)
    elif kind == 1:
        f = datagen.checker_3d(*shape, seed=seed)
    elif kind == 2 and nd == 2 and min(shape) > 8:
        f = datagen.gaussian_bumps_2d(*shape, int(rng.integers(2, 30)), seed=seed)
    elif kind == 2 and nd == 3 and min(shape) > 4:
        f = datagen.grf_3d(*shape, seed=seed)
    elif kind == 3:
        ramp = np.linspace(0.0, 1.0, int(np.prod(shape))).reshape(shape)
        f = (0.1 * datagen.noise(shape, seed=seed) + ramp).astype(np.float32)
    else:
        f = datagen.noise(shape, seed=seed)
    if rng.random() < 0.5:
        mode, eb = "rel", float(10 ** rng.uniform(-4, -1.0))
    else:
        mode, eb = "abs", float(10 ** rng.uniform(-3, 0.5))
    params = {}
    # field-scope ranks on small fields only: the oracle moves an extremum
    # one float step at a time, and field-scope ranks grow with the field
    if rng.random() < 0.15 and f.size <= 100000:
        params["rank_scope"] = 1
    if rng.random() < 0.1:
        params["rbf_policy"] = 1
    if rng.random() < 0.1:
        params["max_rounds"] = int(rng.integers(1, 6))
    return f, eb, mode, params, "shape %s kind %d seed %d %s %g %s" % (shape, kind, seed, mode, eb, params)


def test_random_cases(tsz, ora):
    import torch
    rng = np.random.default_rng(20260217)
    failures = []
    for it in range(150):
        f, eb, mode, params, tag = _case(rng)
        print("case", it, tag, flush=True)
        rc_o, s_o = ora.compress(f, eb, mode, **params)
        st, s_g = tsz.compress(torch.from_numpy(np.ascontiguousarray(f)).cuda(), eb, mode, **params)
        if st != rc_o:
            failures.append((it, tag, "status %d, oracle %d" % (st, rc_o)))
            continue
        if rc_o != 0:
            continue
        s_g = s_g.cpu().numpy()
        if s_g.size != s_o.size or not np.array_equal(s_g, s_o):
            failures.append((it, tag, "stream differs"))
            continue
        ws = tsz.Workspace(f.shape)
        st, rec = tsz.decompress(torch.from_numpy(s_o).cuda(), f.shape, ws=ws)
        stats = tsz.decompress_stats(ws)
        rc, rec_o, stats_o = ora.decompress(s_o, f.shape)
        if st != 0 or rc != 0:
            failures.append((it, tag, "decompress status %d, oracle %d" % (st, rc)))
            continue
        if not np.array_equal(rec.cpu().numpy().view(np.uint32), rec_o.view(np.uint32)):
            failures.append((it, tag, "reconstruction differs"))
            continue
        for k in ("rounds", "commits", "stencil_moves", "budget_skips"):
            if stats[k] != stats_o[k]:
                failures.append((it, tag, "%s %d, oracle %d" % (k, stats[k], stats_o[k])))
                break
    assert not failures, failures[:5]
