"""GPU: backward tracing from the receivers (Sec. III, "Backward ray
tracing"), through the C ABI, against the CPU oracle tracing the same rays
from the receivers.

Checked element by element as forward frames are: per-ray hits and lengths
(per receiver), captures at the transmitter spheres, candidate keys (the
path's key from the transmitter), refined paths and received powers; the
dense-ray corner scene against exhaustive enumeration; coherent backward
frames against full backward re-traces, with moving vehicles and with moving
transmitters (the capture spheres of a backward frame)."""
import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes
from tests.gpu_frames import assert_comparable, compare_frame, log, run_pair

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


def test_static_toy_backward(ctx, O):
    # one transmitter sphere to capture 16 receivers' rays: a 2 m radius
    s = scenes.Scene(**{**scenes.static_toy().__dict__, "rx_radius": 2.0})
    dirs = scenes.random_sphere_dirs(20_000, seed=31)
    st, out, ofr = run_pair(ctx, O, s, dirs=dirs, backward=True)
    assert ctx.trace_log()[0].shape[0] == s.rx.shape[0]
    assert st["rays_fully_certain"] > 0.98 * st["rays"]
    assert_comparable(st)
    assert ofr.paths.valid.sum() > 25


def test_backward_multi_tx_multi_freq_ragged(ctx, O):
    s = scenes.static_toy()
    s2 = scenes.Scene(**{**s.__dict__, "tx": np.array([[0, 0, 5], [-60, 10, 3], [30, -40, 8]], np.float32),
                         "freqs_hz": [28e9, 60e9]})
    for n, K in [(1, 2), (63, 0), (4097, 3)]:
        dirs = scenes.random_sphere_dirs(n, seed=300 + n)
        run_pair(ctx, O, s2, dirs=dirs, K=K, backward=True)
    st, out, ofr = run_pair(ctx, O, s2, dirs=scenes.random_sphere_dirs(30_000, seed=33), backward=True)
    assert out.p_coh.shape == (2, 3, 16)
    assert_comparable(st)


def test_backward_urban_frames(ctx, O):
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(256, seed=35)   # 256 rays from each of the 256 receivers
    for frame in [0, 45]:
        st, out, ofr = run_pair(ctx, O, s, frame=frame, dirs=dirs, backward=True)
        assert st["rays_fully_certain"] > 0.99 * st["rays"]
        assert_comparable(st)


def test_backward_dense_corner_matches_enumeration(ctx, O):
    """Dense rays from the receivers find exactly the valid paths of the
    exhaustive image-method enumeration, two-bounce face orders included."""
    s = scenes.corner([[3.0, 5.0, 1.0], [12.0, 7.0, 2.0]], [[8.0, 2.0, 1.5], [5.0, 11.0, 1.2], [9.0, 9.0, 2.5]],
                      n_rays=400_000, max_reflections=2)
    s.rx_radius = 0.25
    keys = O.enumerate_keys(s.n_faces, 2, 3, 2)
    p = O.refine(O.OracleScene(s), s.tx, s.rx, keys, 2, s.freqs_hz, s.tx_power_w)
    want = {tuple(k) for k, v in zip(keys.tolist(), p.valid) if v}
    ctx.scene_upload(s)
    dcem.trace_scene_frame(ctx, s, los_always=False, trace_from_rx=True)
    gp = ctx.paths()
    got = {tuple(int(x) for x in k) for k, v in zip(gp["keys"], gp["valid"]) if v}
    assert len(want) == 24 and got == want


def _same_frame(a, b):
    pa, pb = a.received_power(), b.received_power()
    for x, y in zip(pa, pb):
        assert np.array_equal(x, y)
    ga, gb = a.paths(), b.paths()
    for k in ("keys", "valid", "length", "tau", "aod", "aoa", "amp", "first_ray"):
        assert np.array_equal(ga[k], gb[k]), k


def test_backward_coherent_frames_equal_full_retraces(O):
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(1024, seed=37)
    coh, full = dcem.Context(0), dcem.Context(0)
    coh.scene_upload(s)
    full.scene_upload(s)
    for frame in range(10):
        a = dcem.trace_scene_frame(coh, s, frame=frame, ray_dirs=dirs, mode=dcem.MODE_COHERENT,
                                   trace_from_rx=True, record_trace_log=True)
        dcem.trace_scene_frame(full, s, frame=frame, ray_dirs=dirs, rebuild=True, trace_from_rx=True)
        _same_frame(coh, full)
        st = coh.stats()
        log("backward coherent frame", frame, "traced", st["rays_traced"], "of", st["rays_total"])
        if frame > 0:
            assert st["coherent"] == 1 and st["rays_traced"] < st["rays_total"]
        if frame == 9:
            ofr = O.frame(s, frame_index=frame, dirs=dirs, backward=True)
            st = compare_frame(coh, s, ofr, a, len(dirs))
            assert_comparable(st)
    coh.close()
    full.close()


def test_backward_coherent_frames_with_moving_transmitters(O):
    """In a backward frame the transmitters are the capture spheres: moving
    them keeps the cached rays and takes their captures again."""
    s = scenes.static_toy()
    dirs = scenes.random_sphere_dirs(8192, seed=39)
    coh, full = dcem.Context(0), dcem.Context(0)
    coh.scene_upload(s)
    full.scene_upload(s)
    for frame in range(6):
        tx = s.tx + np.array([[1.5 * frame, -0.7 * frame, 0.0]], np.float32)
        kw = dict(rx_radius=s.rx_radius, n_rays=len(dirs), ray_dirs=dirs, max_reflections=s.max_reflections,
                  freqs_hz=s.freqs_hz, tx_power_w=s.tx_power_w, trace_from_rx=True, record_trace_log=True)
        coh.trace_frame(tx, s.rx, mode=dcem.MODE_COHERENT, **kw)
        full.trace_frame(tx, s.rx, mode=dcem.MODE_FULL, **kw)
        _same_frame(coh, full)
        st = coh.stats()
        if frame > 0:
            assert st["coherent"] == 1 and st["rays_traced"] == 0
        if frame == 5:
            s5 = scenes.Scene(**{**s.__dict__, "tx": tx})
            ofr = O.frame(s5, dirs=dirs, backward=True)
            stc = compare_frame(coh, s5, ofr, dcem.FrameOutput(*coh.received_power()), len(dirs))
            assert_comparable(stc)
    coh.close()
    full.close()
