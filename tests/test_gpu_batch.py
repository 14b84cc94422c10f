"""GPU: batched frames (dcem_batch_*): several ragged scenes traced with one
persistent launch equal the same frames traced one context at a time,
bitwise; each scene's batched frame against the oracle on sampled rays; the
captured-graph mode and the autotuner."""
import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes
from tests.gpu_frames import check_full_size_sampled, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.build()
    return oracle


def small_batch(n=6, seed=11, budget_range=(1 << 14, 1 << 17), rx_range=(32, 256)):
    return scenes.batched_workload(n, seed=seed, tri_range=(8_000, 60_000), budget_range=budget_range,
                                   rx_range=rx_range, tx_range=(1, 3), k_range=(2, 4))


def outputs(ctx):
    pc, pi = ctx.received_power()
    return pc, pi, ctx.paths(), ctx.trace_log()


def assert_same(a, b):
    for x, y in zip(a[:2], b[:2]):
        assert np.array_equal(x, y)
    for k in ("keys", "valid", "length", "tau", "aod", "aoa", "amp", "first_ray"):
        assert np.array_equal(a[2][k], b[2][k]), k
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y, equal_nan=True)


def place(ctx, s, frame):
    ctx.set_object_transforms(s.transforms(frame))
    ctx.refit_bvh(threshold=float("inf"))


def run_batched_and_single(ws, frames, graph=False, modes=None, stream=None):
    modes = modes or [dcem.MODE_FULL] * len(ws)
    bctx = [dcem.Context(0, stream=stream) for _ in ws]
    sctx = [dcem.Context(0, stream=stream) for _ in ws]
    for c, d, s in zip(bctx, sctx, ws):
        c.scene_upload(s)
        d.scene_upload(s)
    batch = dcem.Batch(bctx)
    batch.set_graph(graph)
    for f in frames:
        for c, s in zip(bctx, ws):
            place(c, s, f)
        batch.trace([dcem.scene_frame_args(s, mode=m, record_trace_log=True) for s, m in zip(ws, modes)])
        for j, (c, d, s, m) in enumerate(zip(bctx, sctx, ws, modes)):
            place(d, s, f)
            d.trace_frame(**dcem.scene_frame_args(s, mode=m, record_trace_log=True))
            assert_same(outputs(c), outputs(d))
        log("frame", f, "batched == single for", len(ws), "scenes;", batch.info())
    return batch, bctx, sctx


def test_batch_equals_single_scene_frames():
    ws = small_batch()
    log("scenes", [(s.n_tris, s.tx.shape[0], s.n_rays, s.max_reflections, s.rx.shape[0], s.freqs_hz[0]) for s in ws])
    batch, b, s = run_batched_and_single(ws, [0, 1, 2])
    batch.close()


def test_batch_with_coherent_contexts():
    ws = small_batch(4, seed=12)
    modes = [dcem.MODE_COHERENT, dcem.MODE_FULL, dcem.MODE_COHERENT, dcem.MODE_FULL]
    batch, b, s = run_batched_and_single(ws, [0, 1, 2, 3], modes=modes)
    assert b[0].stats()["coherent"] == 1 and b[2].stats()["coherent"] == 1
    batch.close()


def test_batch_as_one_captured_graph():
    import torch
    stream = torch.cuda.Stream()
    # few enough captures per frame for the one-workgroup candidate path, so
    # that frames after the first need no host round trip
    ws = small_batch(5, seed=13, budget_range=(1 << 12, 1 << 14), rx_range=(32, 96))
    with torch.cuda.stream(stream):
        batch, b, s = run_batched_and_single(ws, [0, 1, 2, 3, 4], graph=True, stream=stream.cuda_stream)
        info = batch.info()
        assert info["graph_frames"] >= 3, info   # frames after the first run on the device-only path
        batch.close()
    torch.cuda.synchronize()


def test_batch_autotune_keeps_results():
    ws = small_batch(6, seed=14)
    bctx = [dcem.Context(0) for _ in ws]
    for c, s in zip(bctx, ws):
        c.scene_upload(s)
        place(c, s, 0)
    batch = dcem.Batch(bctx)
    frames = [dcem.scene_frame_args(s, record_trace_log=True) for s in ws]
    info = batch.tune(frames, repeats=1)
    log("tuned", info)
    assert info["tuned"] == 1 and info["ms_trace_tuned"] > 0
    for c, s in zip(bctx, ws):
        d = dcem.Context(0)
        d.scene_upload(s)
        place(d, s, 0)
        d.trace_frame(**dcem.scene_frame_args(s, record_trace_log=True))
        assert_same(outputs(c), outputs(d))
        d.close()
    batch.close()


def test_batch_scenes_against_oracle_sampled(O):
    ws = small_batch(4, seed=15)
    bctx = [dcem.Context(0) for _ in ws]
    for c, s in zip(bctx, ws):
        c.scene_upload(s)
        place(c, s, 2)
    batch = dcem.Batch(bctx)
    batch.trace([dcem.scene_frame_args(s, record_trace_log=True) for s in ws])
    for c, s in zip(bctx, ws):
        log("scene", s.n_tris, "tris", s.tx.shape[0], "tx", s.n_rays, "rays K", s.max_reflections)
        check_full_size_sampled(c, O, s, 2, stride=max(1, s.n_rays // 16384), min_keys=3)
    batch.close()


def test_batch_of_large_capture_lists_as_one_graph():
    """Scenes with more captures than the one-workgroup path holds: after the
    first frame their candidates take the sort-based path sized from the last
    frame's count, with every count read on the device, so the whole batch is
    captured as one graph too."""
    import torch
    stream = torch.cuda.Stream()
    ws = small_batch(4, seed=16, budget_range=(1 << 20, 1 << 21), rx_range=(768, 1024))
    with torch.cuda.stream(stream):
        batch, b, s = run_batched_and_single(ws, [0, 1, 2, 3], graph=True, stream=stream.cuda_stream)
        info = batch.info()
        caps = [c.stats()["captures"] for c in b]
        log("captures per scene", caps, info)
        assert max(caps) > 2048
        assert info["graph_frames"] >= 2, info
        batch.close()
    torch.cuda.synchronize()
