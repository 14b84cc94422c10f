"""GPU: argument validation, call order and capacity errors surface as status
codes (forced from the host; every kernel still exits normally)."""
import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes

pytestmark = pytest.mark.gpu


def expect(status, fn, *a, **k):
    with pytest.raises(dcem.DcemError) as e:
        fn(*a, **k)
    assert e.value.status == status, str(e.value)


def test_call_order():
    c = dcem.Context(0)
    expect(dcem.E_STATE, c.trace_frame, [[0, 0, 1]], [[1, 1, 1]], 0.5, 16)
    expect(dcem.E_STATE, c.received_power)
    s = scenes.dynamic_urban(n_rays=1024)
    c.scene_upload(s)
    c.set_object_transforms(s.transforms(3))
    expect(dcem.E_STATE, c.trace_frame, s.tx, s.rx, 0.5, 1024, max_reflections=4)
    c.refit_bvh()
    c.trace_frame(s.tx, s.rx, 0.5, 1024, max_reflections=4)
    c.received_power()
    c.close()


def test_bad_arguments():
    c = dcem.Context(0)
    s = scenes.static_toy()
    bad = scenes.Scene(**{**s.__dict__, "tris": np.where(s.tris == 5, 10_000, s.tris).astype(np.int32)})
    expect(dcem.E_INVALID_ARG, c.scene_upload, bad)
    nanv = s.vertices.copy()
    nanv[3, 1] = np.nan
    expect(dcem.E_INVALID_ARG, c.scene_upload, scenes.Scene(**{**s.__dict__, "vertices": nanv}))
    badf = scenes.Scene(**{**s.__dict__, "tri_face": np.full_like(s.tri_face, 99)})
    expect(dcem.E_INVALID_ARG, c.scene_upload, badf)
    c.scene_upload(s)
    expect(dcem.E_INVALID_ARG, c.trace_frame, s.tx, s.rx, 0.5, 64, max_reflections=11)
    expect(dcem.E_INVALID_ARG, c.trace_frame, s.tx, s.rx, -1.0, 64)
    expect(dcem.E_INVALID_ARG, c.trace_frame, s.tx, s.rx, 0.5, 64, freqs_hz=[0.0])
    expect(dcem.E_INVALID_ARG, c.set_object_transforms, np.zeros((3, 3, 4), np.float32))
    c.close()


def test_capture_capacity_overflow_is_reported():
    c = dcem.Context(0)
    s = scenes.static_toy()
    c.scene_upload(s)
    c.set_capture_capacity(4)
    c.trace_frame(s.tx, s.rx, s.rx_radius, 100_000, max_reflections=2, los_always=True)
    expect(dcem.E_CAPACITY, c.received_power)
    c.set_capture_capacity(1 << 20)
    c.trace_frame(s.tx, s.rx, s.rx_radius, 100_000, max_reflections=2, los_always=True)
    c.received_power()
    c.close()
