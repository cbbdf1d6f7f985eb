"""Multi-instance runtime: uneven datasets in one persistent launch, graph
capture and replay, and the autotuner with its cache."""
import json
import os

import numpy as np
import pytest

import synth
from tests.gpu_util import have_gpu, tol

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="no GPU")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (n, B, n_k): ragged sizes on both sides of tile boundaries
SHAPES = [(70, 5, 3), (150, 9, 4), (257, 3, 5), (300, 12, 6), (64, 7, 2), (500, 4, 12), (33, 6, 1)]


def _contexts(shapes, seed=100):
    import torch
    import paper_2501_12928_amd as eor
    insts, ctxs = [], []
    for k, (n, B, nk) in enumerate(shapes):
        inst = synth.small(seed=seed + k, m=4 * n, n=n, n_k=nk, n_theta=B)
        ctx = eor.Context(0)
        ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                       torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
        insts.append(inst)
        ctxs.append(ctx)
    return insts, ctxs


def _thetas(insts):
    import torch
    return [torch.from_numpy(i.theta).cuda() for i in insts]


@pytest.fixture(scope="module")
def problem(orc):
    insts, ctxs = _contexts(SHAPES)
    refs = [orc.loglike_instance(i)[0] for i in insts]
    return insts, ctxs, refs


def _check_all(outs, refs):
    for got, ref in zip(outs, refs):
        g = got.cpu().numpy()
        assert np.all(np.abs(g - ref) <= tol(ref)), np.max(np.abs(g - ref))
        assert np.all(np.abs(g - ref) <= 1e-10 * np.abs(ref))


def test_group_eager_matches_oracle(problem):
    import paper_2501_12928_amd as eor
    import torch
    insts, ctxs, refs = problem
    print("gpu: group eager, 7 uneven instances", flush=True)
    g = eor.Group(ctxs)
    g.set_graph(False)
    outs, infos = g.loglike(_thetas(insts))
    torch.cuda.synchronize()
    assert all(bool((i == 0).all()) for i in infos)
    _check_all(outs, refs)
    g.close()


def test_group_equals_single_context(problem):
    """Same kernel, same per-theta arithmetic: the grouped launch gives
    bit-identical results to one context at a time."""
    import paper_2501_12928_amd as eor
    import torch
    insts, ctxs, refs = problem
    g = eor.Group(ctxs)
    outs, _ = g.loglike(_thetas(insts))
    singles = [c.loglike_batch(t)[0] for c, t in zip(ctxs, _thetas(insts))]
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)
    g.close()


def test_group_two_tiles_per_pass(problem):
    """Eight-wave workgroups updating two tiles per pass: same bits as
    four-wave workgroups, eager and from a graph."""
    import paper_2501_12928_amd as eor
    import torch
    insts, ctxs, refs = problem
    g = eor.Group(ctxs)
    g.set_graph(False)
    g.set_tuning(4, 2, 1)
    base, _ = g.loglike(_thetas(insts))
    torch.cuda.synchronize()
    base = [b.clone() for b in base]
    g.set_tuning(4, 1, 2)
    assert g.tuning()[:3] == (4, 1, 2)
    print("gpu: group, two tiles per pass", flush=True)
    outs, infos = g.loglike(_thetas(insts))
    torch.cuda.synchronize()
    assert all(bool((i == 0).all()) for i in infos)
    for a, b in zip(outs, base):
        assert torch.equal(a, b)
    g.set_graph(True)
    outs, infos = g.loglike(_thetas(insts))
    outs, infos = g.loglike(_thetas(insts), outs=outs, infos=infos)
    torch.cuda.synchronize()
    for a, b in zip(outs, base):
        assert torch.equal(a, b)
    _check_all(outs, refs)
    with pytest.raises(eor.EorError):
        g.set_tuning(4, 2, 2)
    g.close()


def test_graph_replays_match_eager(problem):
    """The captured graph is replayed several times with unrelated eager
    work and synchronisations in between; every replay must equal the eager
    launch exactly."""
    import paper_2501_12928_amd as eor
    import torch
    insts, ctxs, refs = problem
    th = _thetas(insts)
    g = eor.Group(ctxs)
    g.set_graph(False)
    eager, _ = g.loglike(th)
    torch.cuda.synchronize()
    eager = [e.clone() for e in eager]
    g.set_graph(True)
    launches0, captures0 = g.tuning()[3:]
    outs, infos = g.loglike(th)          # capture
    for r in range(4):
        print(f"gpu: graph replay {r}", flush=True)
        outs, infos = g.loglike(th, outs=outs, infos=infos)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2.0).sum().item()
        ctxs[r % len(ctxs)].loglike_batch(th[r % len(ctxs)])
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert torch.equal(a, b)
    launches, captures = g.tuning()[3:]
    assert launches - launches0 == 5 and captures - captures0 == 1
    _check_all(eager, refs)
    g.close()


def test_graph_follows_new_buffers(problem):
    """New theta values written into the same buffers replay the captured
    graph (no new capture) and give the oracle's values for the new theta."""
    import paper_2501_12928_amd as eor
    import torch
    from oracle import get as oracle_get
    insts, ctxs, refs = problem
    g = eor.Group(ctxs)
    th = _thetas(insts)
    outs, infos = g.loglike(th)
    rng = np.random.default_rng(5)
    new = [rng.uniform(-1, 3, size=i.theta.shape) for i in insts]
    for t, v in zip(th, new):
        t.copy_(torch.from_numpy(v))
    outs, _ = g.loglike(th, outs=outs, infos=infos)     # same buffers: replay
    torch.cuda.synchronize()
    assert g.tuning()[4] == 1
    orc = oracle_get()
    refs2 = [orc.loglike_instance(i, theta=v)[0] for i, v in zip(insts, new)]
    _check_all(outs, refs2)
    g.close()


def test_autotune_and_cache(problem, tmp_path):
    import paper_2501_12928_amd as eor
    import torch
    insts, ctxs, refs = problem
    cache = tmp_path / "tune.json"
    g = eor.Group(ctxs)
    print("gpu: autotune", flush=True)
    st, wg, tp = g.autotune(_thetas(insts), cache_path=cache)
    assert (st, wg, tp) in [(s, w, p) for s in (2, 4) for (p, w) in ((1, 1), (1, 2), (2, 1))]
    data = json.loads(cache.read_text())
    key = [k for k in data if k.endswith("|n<=512|group")]
    assert len(key) == 1 and key[0].startswith("gfx950")
    assert (data[key[0]]["stages"], data[key[0]]["wg_per_cu"], data[key[0]]["tiles"]) == (st, wg, tp)
    # a second group reads the cached choice (no timing)
    data[key[0]] = {"stages": 2, "wg_per_cu": 1, "tiles": 2, "ms": 1.0}
    cache.write_text(json.dumps(data))
    g2 = eor.Group(ctxs)
    assert g2.autotune(_thetas(insts), cache_path=cache) == (2, 1, 2)
    # the tile side of the one bucket this batch holds (n <= 512) is cached too
    tk = [k for k in data if k.endswith("|n<=512|tile")]
    assert len(tk) == 1 and data[tk[0]]["tile"] in (32, 64)
    assert g.tile_sizes()[0] == data[tk[0]]["tile"]
    assert g2.tile_sizes()[0] == data[tk[0]]["tile"]
    # a cached tile side is taken as it stands
    data[tk[0]] = {"tile": 96 - data[tk[0]]["tile"], "ms64": 1.0, "ms32": 1.0}
    cache.write_text(json.dumps(data))
    g3 = eor.Group(ctxs)
    g3.autotune(_thetas(insts), cache_path=cache)
    assert g3.tile_sizes()[0] == data[tk[0]]["tile"]
    outs, _ = g3.loglike(_thetas(insts))
    torch.cuda.synchronize()
    _check_all(outs, refs)
    outs, _ = g2.loglike(_thetas(insts))
    torch.cuda.synchronize()
    _check_all(outs, refs)
    g.close()
    g2.close()
    g3.close()


def test_group_mixed_tile_sides(orc):
    """Instances in three size buckets, factored with 32-wide tiles in two of
    them and 64-wide in the third, in one launch (eager and from a graph):
    each matches the oracle, and each equals a lone context with the same
    tile side bit for bit."""
    import paper_2501_12928_amd as eor
    import torch
    shapes = [(700, 5, 4), (130, 9, 3), (1100, 4, 6), (200, 6, 2)]   # buckets 1, 0, 2, 0
    insts, ctxs = _contexts(shapes, seed=300)
    refs = [orc.loglike_instance(i)[0] for i in insts]
    sides = [32, 64, 32, 64, 64]
    g = eor.Group(ctxs)
    g.set_tile_sizes(sides)
    assert g.tile_sizes() == sides
    with pytest.raises(eor.EorError):
        g.set_tile_sizes([32, 64, 16, 64, 64])
    for graph in (False, True):
        g.set_graph(graph)
        print(f"gpu: group with mixed tile sides, graph {graph}", flush=True)
        outs, infos = g.loglike(_thetas(insts))
        torch.cuda.synchronize()
        assert all(bool((i == 0).all()) for i in infos)
        _check_all(outs, refs)
    for inst, ctx, out in zip(insts, ctxs, outs):
        ctx.set_tile_size(32 if inst.n <= 512 else (64 if inst.n <= 1024 else 32))
        single, _ = ctx.loglike_batch(torch.from_numpy(inst.theta).cuda())
        torch.cuda.synchronize()
        assert torch.equal(single, out)
        ctx.set_tile_size(64)
    g.close()
    for c in ctxs:
        c.close()


def test_group_argument_errors(problem):
    import ctypes
    import paper_2501_12928_amd as eor
    insts, ctxs, refs = problem
    L = eor.lib()
    out = ctypes.c_void_p()
    assert L.eor_group_create(0, None, ctypes.byref(out)) == eor.EOR_ERR_ARG
    arr = (ctypes.c_void_p * 65)(*([ctxs[0].handle] * 65))
    assert L.eor_group_create(65, arr, ctypes.byref(out)) == eor.EOR_ERR_ARG
    fresh = eor.Context(0)   # never precomputed
    g = eor.Group([ctxs[0], fresh])
    B = (ctypes.c_int64 * 2)(1, 1)
    tp = (ctypes.c_void_p * 2)(1, 1)
    op = (ctypes.c_void_p * 2)(1, 1)
    assert L.eor_group_loglike(g._h, B, tp, op, None, None) == eor.EOR_ERR_STATE
    g.close()
    g = eor.Group(ctxs[:1])
    B = (ctypes.c_int64 * 1)(-1)
    assert L.eor_group_loglike(g._h, B, tp, op, None, None) == eor.EOR_ERR_ARG
    g.close()
    fresh.close()


@pytest.mark.slow
def test_uneven_subband_workload_sampled(orc):
    """The 48-instance uneven workload (n from 266 to 4057, 3097 theta) in
    one launch; three instances checked against stored oracle values."""
    import paper_2501_12928_amd as eor
    import torch
    path = os.path.join(GOLDEN, "c2_oracle_sample.json")
    if not os.path.exists(path):
        pytest.skip("c2 oracle sample not generated")
    gold = json.load(open(path))["instances"]
    ctxs, thetas = [], []
    print("gpu: 48-instance workload, precompute", flush=True)
    for idx, inst in enumerate(synth.gen_group()):
        ctx = eor.Context(0)
        ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                       torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
        torch.cuda.synchronize()
        if str(idx) in gold:
            assert inst.digest() == gold[str(idx)]["digest"]
        ctxs.append(ctx)
        thetas.append(torch.from_numpy(inst.theta).cuda())
    g = eor.Group(ctxs)
    for sides in ([64] * 5, [32] * 5, [32, 32, 64, 64, 64]):
        print(f"gpu: 48-instance workload, group launch, tile sides {sides}", flush=True)
        g.set_tile_sizes(sides)
        outs, infos = g.loglike(thetas)
        torch.cuda.synchronize()
        assert all(bool((i == 0).all()) for i in infos)
        for k, v in gold.items():
            got = outs[int(k)].cpu().numpy()[:len(v["logL"])]
            ref = np.array(v["logL"])
            assert np.all(np.abs(got - ref) <= tol(ref)), (k, np.abs(got - ref).max())
            assert np.all(np.abs(got - ref) <= 1e-10 * np.abs(ref)), (k, np.abs(got - ref).max())
    g.close()
    for c in ctxs:
        c.close()


def test_group_invalid_theta_mixed(problem):
    """Regression: non-finite theta spread through a group launch. Each is
    reported (info -1, logL -inf) and the persistent workgroups move on to
    the remaining tasks; every valid theta still matches the oracle."""
    import paper_2501_12928_amd as eor
    import torch
    from oracle import get as oracle_get
    insts, ctxs, refs = problem
    bad_th = []
    for k, i in enumerate(insts):
        th = i.theta.copy()
        th[k % th.shape[0], 0] = [np.nan, np.inf, -np.inf, 500.0][k % 4]
        bad_th.append(th)
    g = eor.Group(ctxs)
    print("gpu: group with invalid theta", flush=True)
    outs, infos = g.loglike([torch.from_numpy(t).cuda() for t in bad_th])
    torch.cuda.synchronize()
    orc = oracle_get()
    for k, (i, th, o, f) in enumerate(zip(insts, bad_th, outs, infos)):
        ref, rinfo = orc.loglike_instance(i, theta=th)
        f = f.cpu().numpy()
        o = o.cpu().numpy()
        np.testing.assert_array_equal(f, rinfo)
        assert f[k % th.shape[0]] == -1 and o[k % th.shape[0]] == -np.inf
        ok = f == 0
        assert np.all(np.abs(o[ok] - ref[ok]) <= tol(ref[ok]))
    g.close()
