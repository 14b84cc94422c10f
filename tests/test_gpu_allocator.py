"""GPU: every device buffer of a context comes from the caller's allocator
(dcem_allocator; here torch's caching allocator through the binding), and the
results do not depend on where the memory comes from."""
import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes

pytestmark = pytest.mark.gpu


def run_frames(ctx, s, n):
    ctx.scene_upload(s)
    outs = []
    for frame in range(4):
        out = dcem.trace_scene_frame(ctx, s, frame=frame, n_rays=n, mode=dcem.MODE_COHERENT)
        outs.append((out.p_coh.copy(), out.p_inc.copy()))
    g = ctx.power_gradients()
    return outs, g


def test_torch_allocator_owns_the_buffers():
    import torch
    s = scenes.dynamic_urban()
    n = 1 << 18
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = dcem.Context(0)
    assert ctx.allocator is not None
    outs, g = run_frames(ctx, s, n)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - base
    held = sum(ctx.allocator.live.values())
    # at least the segment cache of the coherent frames: 2 x (K + 1) x n x 16 B
    assert held >= 2 * 5 * n * 16
    assert grown >= held
    print("library buffers through torch: %.1f MB in %d blocks" % (held / 1e6, len(ctx.allocator.live)))
    ctx.close()
    torch.cuda.synchronize()
    assert not ctx.allocator.live
    assert torch.cuda.memory_allocated() == base
    # the same frames with hipMalloc'd buffers: bitwise equal
    plain = dcem.Context(0, allocator=None)
    assert plain.allocator is None
    outs2, g2 = run_frames(plain, s, n)
    plain.close()
    for (a, b), (c, d) in zip(outs, outs2):
        assert np.array_equal(a, c) and np.array_equal(b, d)
    for a, b in zip(g, g2):
        assert np.array_equal(a, b)
