"""GPU: code paths the urban workload does not reach.

- A refit of a 300k-triangle scene built by a forced rebuild, whose nodes
  spanning refit blocks are too many for the last-block pass (the block pass
  then uses device-wide arrival counters for them): exact boxes, and the same
  hits as a rebuild.
- More moving objects than the coherence pass bins on its grid (they are then
  tested one by one): coherent frames equal the full re-trace bitwise.
- The build at upload keeps each moving object, and each face, in a subtree of
  its own.
"""
import sys

import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes

pytestmark = pytest.mark.gpu

REFIT_BLOCK = 1024      # leaves per refit block
LAST_BLOCK_NODES = 1024  # nodes spanning blocks that the last block finishes in LDS
GRID_OBJECTS = 256      # moving objects the coherence grid holds


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def leaf_ranges(child):
    """(lo, hi) sorted-leaf range of every internal node (child [n][2], leaves ~index)."""
    n = child.shape[0]
    lo = np.zeros(n, np.int64)
    hi = np.zeros(n, np.int64)
    order, stack = [], [0]
    while stack:
        x = stack.pop()
        order.append(x)
        for c in child[x]:
            if c >= 0:
                stack.append(int(c))
    for x in reversed(order):
        l, r = int(child[x, 0]), int(child[x, 1])
        lo[x] = ~l if l < 0 else lo[l]
        hi[x] = ~r if r < 0 else hi[r]
    return lo, hi


def exact_boxes(child, box, leaf_tri, V, T, pad):
    """Vectorised: every internal child box is the union of its children, every
    leaf box the triangle box grown by pad (FP32)."""
    lo_s, hi_s = box[:, :, 0:3], box[:, :, 3:6]
    inner = child >= 0
    c = np.where(inner, child, 0)
    ulo = np.minimum(lo_s[c, 0], lo_s[c, 1])
    uhi = np.maximum(hi_s[c, 0], hi_s[c, 1])
    ok_inner = np.all((ulo == lo_s) & (uhi == hi_s), axis=-1) | ~inner
    li = np.where(inner, 0, ~child)
    tv = V[T[leaf_tri[li]]]                        # [n, 2, 3 vertices, 3]
    tlo = tv.min(axis=2) - np.float32(pad)
    thi = tv.max(axis=2) + np.float32(pad)
    ok_leaf = np.all((tlo == lo_s) & (thi == hi_s), axis=-1) | inner
    return bool(np.all(ok_inner) and np.all(ok_leaf))


def outputs(ctx):
    pc, pi = ctx.received_power()
    tri, t, length = ctx.trace_log()
    return pc, pi, ctx.paths(), tri, t, length


def assert_same(a, b):
    pc0, pi0, p0, tri0, t0, l0 = a
    pc1, pi1, p1, tri1, t1, l1 = b
    assert np.array_equal(tri0, tri1)
    assert np.array_equal(t0, t1, equal_nan=True) and np.array_equal(l0, l1, equal_nan=True)
    for k in ["keys", "valid", "length", "amp"]:
        assert np.array_equal(p0[k], p1[k]), k
    assert np.array_equal(pc0, pc1) and np.array_equal(pi0, pi1)


def test_large_scene_refit_equals_rebuild():
    s = scenes.box_field(25000, 20)
    log("box field", s.n_tris, "triangles")
    a, b = dcem.Context(0), dcem.Context(0)
    a.scene_upload(s)
    b.scene_upload(s)
    # a forced rebuild orders all triangles along one Morton curve, whose nodes
    # straddle the refit blocks' boundaries at every level
    a.refit_bvh(force_rebuild=True)
    child, box, leaf = a.bvh()
    lo, hi = leaf_ranges(child)
    n_cross = int(np.sum(lo // REFIT_BLOCK != hi // REFIT_BLOCK))
    log("nodes spanning refit blocks", n_cross)
    assert n_cross > LAST_BLOCK_NODES
    pad = 4e-6 * (2.0 * float(np.abs(s.vertices).max()) + 1.0)
    dirs = scenes.random_sphere_dirs(1 << 16, seed=11)
    for frame in [1, 3]:
        xf = s.transforms(frame)
        a.set_object_transforms(xf)
        rebuilt, _ = a.refit_bvh(threshold=float("inf"))
        assert not rebuilt
        b.set_object_transforms(xf)
        b.refit_bvh(force_rebuild=True)
        child, box, leaf = a.bvh()
        assert exact_boxes(child, box, leaf, a.vertices(), s.tris, pad)
        for c in (a, b):
            c.trace_frame(s.tx, s.rx, s.rx_radius, dirs.shape[0], ray_dirs=dirs, max_reflections=s.max_reflections,
                          record_trace_log=True)
        assert_same(outputs(a), outputs(b))
        log("frame", frame, "refit == rebuild")
    a.close()
    b.close()


def test_very_large_scene_refit_cross_pass():
    """More than 512k triangles: the refit's cross nodes are finished by a
    launch of their own, beyond the LDS capacity through device memory.  The
    refitted boxes are exact unions, the coherent launch's refit equals the
    plain one, and hits equal those of a rebuilt tree."""
    s = scenes.box_field(52000, 400)
    log("box field", s.n_tris, "triangles")
    assert s.n_tris > 524288
    a, b = dcem.Context(0), dcem.Context(0)
    a.scene_upload(s)
    b.scene_upload(s)
    a.refit_bvh(force_rebuild=True)
    child, box, leaf = a.bvh()
    lo, hi = leaf_ranges(child)
    n_cross = int(np.sum(lo // REFIT_BLOCK != hi // REFIT_BLOCK))
    log("nodes spanning refit blocks", n_cross)
    assert n_cross > LAST_BLOCK_NODES
    pad = 4e-6 * (2.0 * float(np.abs(s.vertices).max()) + 1.0)
    dirs = scenes.random_sphere_dirs(1 << 16, seed=12)
    for frame in [1, 2, 3]:
        xf = s.transforms(frame)
        a.set_object_transforms(xf)
        rebuilt, ratio = a.refit_bvh(threshold=float("inf"))
        assert not rebuilt
        b.set_object_transforms(xf)
        b.refit_bvh(force_rebuild=True)
        # coherent frames run the refit inside the revalidation launch
        a.trace_frame(s.tx, s.rx, s.rx_radius, dirs.shape[0], ray_dirs=dirs, max_reflections=s.max_reflections,
                      record_trace_log=True, mode=dcem.MODE_COHERENT)
        b.trace_frame(s.tx, s.rx, s.rx_radius, dirs.shape[0], ray_dirs=dirs, max_reflections=s.max_reflections,
                      record_trace_log=True)
        assert_same(outputs(a), outputs(b))
        child, box, leaf = a.bvh()
        assert exact_boxes(child, box, leaf, a.vertices(), s.tris, pad)
        log("frame", frame, "refit == rebuild, SAH ratio", a.stats()["sah_ratio"])
    a.close()
    b.close()


def test_upload_build_keeps_objects_in_own_subtrees():
    """The build at upload gives every moving object (and the static geometry)
    a subtree of its own, and every face one inside it: a node whose leaf
    range is exactly its triangles."""
    s = scenes.dynamic_urban(n_rays=1 << 10)
    ctx = dcem.Context(0)
    ctx.scene_upload(s)
    child, box, leaf = ctx.bvh()
    lo, hi = leaf_ranges(child)
    spans = set(zip(lo.tolist(), hi.tolist()))
    tri_obj = s.face_object[s.tri_face][leaf]      # object of each sorted leaf (-1 static)
    for o in range(-1, s.n_objects):
        pos = np.flatnonzero(tri_obj == o)
        assert pos.size and pos[-1] - pos[0] + 1 == pos.size, o
        assert (int(pos[0]), int(pos[-1])) in spans, o
    # and every face inside its group
    tri_face = s.tri_face[leaf]
    for f in range(s.face_object.shape[0]):
        pos = np.flatnonzero(tri_face == f)
        if pos.size > 1:
            assert pos[-1] - pos[0] + 1 == pos.size, f
            assert (int(pos[0]), int(pos[-1])) in spans, f
    log("objects and faces in own subtrees:", s.n_objects, s.face_object.shape[0])
    ctx.close()


def test_many_moving_objects_coherent_equals_full():
    s = scenes.box_field(200, 300)
    assert s.n_objects > GRID_OBJECTS
    full, coh = dcem.Context(0), dcem.Context(0)
    full.scene_upload(s)
    coh.scene_upload(s)
    n = 1 << 15
    for frame in range(s.n_frames):
        xf = s.transforms(frame)
        for c, mode in ((full, dcem.MODE_FULL), (coh, dcem.MODE_COHERENT)):
            c.set_object_transforms(xf)
            c.refit_bvh(force_rebuild=mode == dcem.MODE_FULL)
            c.trace_frame(s.tx, s.rx, s.rx_radius, n, max_reflections=s.max_reflections, mode=mode,
                          record_trace_log=True)
        assert_same(outputs(full), outputs(coh))
        st = coh.stats()
        log("frame", frame, "traced", st["rays_traced"], "of", n)
        if frame > 0:
            assert st["coherent"] == 1 and st["rays_traced"] < n
    full.close()
    coh.close()
