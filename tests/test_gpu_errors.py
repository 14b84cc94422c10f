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


def test_stack_overflow_is_reported():
    """A traversal stack capped at one entry overflows on the urban tree: the
    frame reports DCEM_E_CAPACITY (forced from the host; the traversals drop
    what does not fit and exit normally); the full depth traces again."""
    s = scenes.dynamic_urban(n_rays=4096)
    c = dcem.Context(0)
    c.scene_upload(s)
    c.set_stack_limit(1)
    c.trace_frame(s.tx, s.rx, s.rx_radius, 4096, max_reflections=4)
    expect(dcem.E_CAPACITY, c.received_power)
    # the group re-trace of a coherent frame too
    c.set_object_transforms(s.transforms(1))
    c.refit_bvh()
    c.set_stack_limit(0)
    c.trace_frame(s.tx, s.rx, s.rx_radius, 4096, max_reflections=4, keep_cache=True)
    c.received_power()
    c.set_object_transforms(s.transforms(2))
    c.refit_bvh()
    c.set_stack_limit(1)
    c.trace_frame(s.tx, s.rx, s.rx_radius, 4096, max_reflections=4, mode=dcem.MODE_COHERENT)
    expect(dcem.E_CAPACITY, c.received_power)
    st = c.stats()   # the error is reported once
    assert st["trace_kernel"] == 1 and st["coherent"] == 1
    c.set_stack_limit(0)
    c.trace_frame(s.tx, s.rx, s.rx_radius, 4096, max_reflections=4)
    pc, _ = c.received_power()
    fresh = dcem.Context(0)
    fresh.scene_upload(s)
    out = dcem.trace_scene_frame(fresh, s, frame=2, n_rays=4096)
    assert np.array_equal(pc, out.p_coh)
    expect(dcem.E_INVALID_ARG, c.set_stack_limit, -1)
    fresh.close()
    c.close()


def test_nonfinite_transform_is_reported():
    """Finite transform entries whose products overflow FP32, and (device
    memory, not checked on the host) NaN entries: the transform kernel flags
    the non-finite vertices and the next synchronising call reports
    DCEM_E_INVALID_ARG; valid transforms then restore the scene."""
    import torch
    s = scenes.dynamic_urban(n_rays=4096)
    c = dcem.Context(0)
    c.scene_upload(s)
    big = s.transforms(0).copy()
    big[0, :, :3] *= np.float32(1e37)
    c.set_object_transforms(big)
    expect(dcem.E_INVALID_ARG, c.vertices)
    bad = torch.tensor(s.transforms(0), device="cuda")
    bad[1, 2, 3] = float("nan")
    c.set_object_transforms(bad)
    torch.cuda.synchronize()
    expect(dcem.E_INVALID_ARG, c.vertices)
    c.set_object_transforms(s.transforms(4))
    c.refit_bvh()
    c.trace_frame(s.tx, s.rx, s.rx_radius, 4096, max_reflections=4)
    pc, _ = c.received_power()
    fresh = dcem.Context(0)
    fresh.scene_upload(s)
    out = dcem.trace_scene_frame(fresh, s, frame=4, n_rays=4096)
    assert np.array_equal(pc, out.p_coh)
    fresh.close()
    c.close()
