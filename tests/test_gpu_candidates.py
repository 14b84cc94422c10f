"""GPU: the sort-based candidate path sized from the last frame's capture
count (counts read on the device, no host round trip) against the path that
reads the count first, bitwise, and the host's exact redo when a frame's
captures outgrow the sizing."""
import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes

pytestmark = pytest.mark.gpu


def _frame(ctx, s, dirs, rx):
    ctx.trace_frame(s.tx, rx, s.rx_radius, len(dirs), ray_dirs=dirs, max_reflections=s.max_reflections,
                    freqs_hz=s.freqs_hz, tx_power_w=s.tx_power_w, record_trace_log=True)
    pc, pi = ctx.received_power()
    return pc, pi, ctx.paths()


def _same(a, b):
    for x, y in zip(a[:2], b[:2]):
        assert np.array_equal(x, y)
    for k in ("keys", "valid", "length", "amp", "first_ray"):
        assert np.array_equal(a[2][k], b[2][k]), k


def test_sized_path_equals_exact_path():
    s = scenes.Scene(**{**scenes.static_toy().__dict__, "rx_radius": 2.0})
    dirs = scenes.random_sphere_dirs(400_000, seed=81)
    a = dcem.Context(0)
    a.scene_upload(s)
    first = _frame(a, s, dirs, s.rx)        # count read back (no previous frame)
    assert a.stats()["captures"] > 2048
    second = _frame(a, s, dirs, s.rx)       # sized from the first frame's count
    _same(first, second)
    fresh = dcem.Context(0)
    fresh.scene_upload(s)
    _same(second, _frame(fresh, s, dirs, s.rx))
    a.close()
    fresh.close()


def test_outgrown_sizing_is_redone_exactly():
    s = scenes.Scene(**{**scenes.static_toy().__dict__, "rx_radius": 2.0})
    dirs = scenes.random_sphere_dirs(400_000, seed=83)
    a = dcem.Context(0)
    a.scene_upload(s)
    _frame(a, s, dirs, s.rx)
    few = a.stats()["captures"]
    # receivers gathered close to the transmitter: many more captures than
    # the sizing taken from the last frame (2 x count + 4096)
    rx2 = np.array(s.tx[0], np.float32) + np.array([[3.0 + 0.2 * i, 0.5 * (i % 4), -2.0] for i in range(16)],
                                                   np.float32)
    got = _frame(a, s, dirs, rx2)
    many = a.stats()["captures"]
    assert many > 2 * few + 4096
    fresh = dcem.Context(0)
    fresh.scene_upload(s)
    _same(got, _frame(fresh, s, dirs, rx2))
    a.close()
    fresh.close()
