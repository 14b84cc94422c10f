"""GPU: visited-series discovery (Sec. III, the frame algorithm's steps 2-4:
each series of faces the rays visit is tried against every target), through
the C ABI, against the CPU oracle's visited-series frames.

Checked: per-ray hits and lengths; every GPU candidate is an oracle (series,
target) pair or comes from a ray the oracle marks uncertain; every certain
valid oracle path is on the GPU with the same length, delay, directions and
field; received powers; the dense static scene against exhaustive
enumeration; forward and backward; coherent frames against full re-traces;
the full-size urban frame on sampled rays."""
import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes
from tests import parity
from tests.gpu_frames import assert_comparable, compare_frame, log, radius_of, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.build()
    return oracle


@pytest.fixture()
def ctx():
    c = dcem.Context(0)
    yield c
    c.close()


def _valid_set(keys, valid):
    return {tuple(int(x) for x in k) for k, v in zip(keys, valid) if v}


def test_static_toy_visited_finds_every_enumerated_path(ctx, O):
    s = scenes.static_toy()
    st, out, ofr = run_pair(ctx, O, s, n_rays=1024, K=2, visited=True)
    assert_comparable(st)
    keys = O.enumerate_keys(s.n_faces, 1, s.rx.shape[0], 2)
    p = O.refine(O.OracleScene(s), s.tx, s.rx, keys, 2, s.freqs_hz, s.tx_power_w)
    gp = ctx.paths()
    assert _valid_set(gp["keys"], gp["valid"]) == _valid_set(keys, p.valid)
    assert ctx.stats()["captures"] == 0


def test_visited_ragged_and_backward(ctx, O):
    s = scenes.static_toy()
    s2 = scenes.Scene(**{**s.__dict__, "tx": np.array([[0, 0, 5], [-60, 10, 3]], np.float32),
                         "freqs_hz": [28e9, 60e9]})
    for n, K, bw in [(1, 2, False), (63, 0, False), (65, 3, True), (1000, 4, False), (700, 2, True)]:
        dirs = scenes.random_sphere_dirs(n, seed=500 + n)
        st, out, ofr = run_pair(ctx, O, s2, dirs=dirs, K=K, visited=True, backward=bw)
        assert_comparable(st)
    # no direct paths requested: order-0 keys absent
    st, out, ofr = run_pair(ctx, O, s2, dirs=scenes.random_sphere_dirs(500, seed=9), K=2, visited=True,
                            los_always=False)
    assert (ctx.paths()["keys"][:, 2] > 0).all()


def test_visited_urban_frames(ctx, O):
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(4096, seed=43)
    for frame in [0, 30]:
        st, out, ofr = run_pair(ctx, O, s, frame=frame, dirs=dirs, visited=True)
        assert st["rays_fully_certain"] > 0.99 * st["rays"]
        assert_comparable(st)
        assert st["valid_paths"] > 150


def test_visited_backward_urban(ctx, O):
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(64, seed=45)   # 64 rays from each of the 256 receivers
    st, out, ofr = run_pair(ctx, O, s, frame=12, dirs=dirs, visited=True, backward=True)
    assert_comparable(st)


def test_visited_contains_captured_paths(ctx):
    """With the same rays, every valid path capture spheres find is also
    found through the visited series."""
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(1 << 16, seed=47)
    ctx.scene_upload(s)
    dcem.trace_scene_frame(ctx, s, frame=3, ray_dirs=dirs)
    gc = ctx.paths()
    dcem.trace_scene_frame(ctx, s, frame=3, ray_dirs=dirs, discovery=dcem.DISCOVER_VISITED)
    gv = ctx.paths()
    cap, vis = _valid_set(gc["keys"], gc["valid"]), _valid_set(gv["keys"], gv["valid"])
    log("capture valid", len(cap), "visited valid", len(vis))
    assert cap <= vis and len(vis) > 2 * len(cap)


def test_visited_coherent_frames_equal_full_retraces():
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(1 << 15, seed=49)
    coh, full = dcem.Context(0), dcem.Context(0)
    coh.scene_upload(s)
    full.scene_upload(s)
    for frame in range(8):
        dcem.trace_scene_frame(coh, s, frame=frame, ray_dirs=dirs, mode=dcem.MODE_COHERENT,
                               discovery=dcem.DISCOVER_VISITED)
        dcem.trace_scene_frame(full, s, frame=frame, ray_dirs=dirs, rebuild=True, discovery=dcem.DISCOVER_VISITED)
        for x, y in zip(coh.received_power(), full.received_power()):
            assert np.array_equal(x, y)
        ga, gb = coh.paths(), full.paths()
        for k in ("keys", "valid", "length", "tau", "aod", "aoa", "amp", "first_ray"):
            assert np.array_equal(ga[k], gb[k]), k
        st = coh.stats()
        if frame > 0:
            assert st["coherent"] == 1 and st["rays_traced"] < st["rays_total"]
    coh.close()
    full.close()


@pytest.mark.timeout(600)
def test_visited_full_size_urban_sampled(ctx, O):
    """The benchmark's urban frame (2^20 Fibonacci rays, K = 4, 256
    receivers) with visited series: every 64th ray is traced by the oracle, and
    every certain series of those rays, tried against every receiver and
    refined by the oracle, must give the GPU's path (valid ones present, same
    attributes)."""
    s = scenes.dynamic_urban()
    frame = 20
    log("case urban full size, visited series, frame", frame)
    ctx.scene_upload(s)
    dcem.trace_scene_frame(ctx, s, frame=frame, record_trace_log=True, discovery=dcem.DISCOVER_VISITED)
    st = ctx.stats()
    log("  unique candidates", st["unique_candidates"], "valid", st["valid_paths"])
    g_tri, g_t, g_len = ctx.trace_log()
    ids = np.arange(0, s.n_rays, 64, dtype=np.int64)
    osc = O.OracleScene(s, s.transforms(frame))
    dirs = O.fibonacci(s.n_rays)
    otr = O.trace(osc, s.tx, s.rx, s.rx_radius, dirs, s.max_reflections, ray_ids=ids)
    parity.compare_trace(g_tri[:, ids], g_t[:, ids], g_len[:, ids], otr, s.tri_face, radius=radius_of(s))
    keys, certain, _ = O.visited_candidates(otr, 1, s.rx.shape[0], s.max_reflections)
    keys = keys[certain]
    op = O.refine(osc, s.tx, s.rx, keys, s.max_reflections, s.freqs_hz, s.tx_power_w)
    gp = ctx.paths()
    gk = {tuple(int(x) for x in k): i for i, k in enumerate(gp["keys"])}
    checked = 0
    for j, k in enumerate(keys):
        if not op.valid[j] or op.marginal[j]:
            continue
        i = gk.get(tuple(int(x) for x in k))
        assert i is not None, "oracle path %s missing on the GPU" % (k,)
        bad = parity.compare_path_attrs(gp, i, op, j)
        assert not bad, (k, bad)
        checked += 1
    log("  oracle series", len(keys) // s.rx.shape[0], "valid paths checked", checked)
    assert checked > 200
    assert st["valid_paths"] >= checked
