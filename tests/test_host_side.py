"""CPU-only checks: the C ABI library loads and exports what include/dcem.h
declares, the struct layouts seen by the binding match the header, the scene
generator is deterministic, and the BVH invariant checker catches planted
mistakes."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes
from tests.bvh_check import check_bvh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcem.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dcem_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = dcem.load_library()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(n for n, _, _ in dcem.SIGNATURES) == names


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "dcem.h"
#define P(T, f) printf("%s.%s %zu\\n", #T, #f, offsetof(T, f));
int main(void) {
  printf("dcem_scene_desc %zu\\n", sizeof(dcem_scene_desc));
  printf("dcem_trace_params %zu\\n", sizeof(dcem_trace_params));
  printf("dcem_frame_stats %zu\\n", sizeof(dcem_frame_stats));
  printf("dcem_allocator %zu\\n", sizeof(dcem_allocator));
  P(dcem_scene_desc, mem_kind) P(dcem_scene_desc, n_objects) P(dcem_scene_desc, materials)
  P(dcem_trace_params, rx_radius) P(dcem_trace_params, n_rays) P(dcem_trace_params, tx_power_w)
  P(dcem_trace_params, mem_kind) P(dcem_frame_stats, sah_ratio) P(dcem_frame_stats, ms_reduce)
  P(dcem_allocator, free) P(dcem_allocator, user)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(got["dcem_scene_desc"]) == ctypes.sizeof(dcem.SceneDesc)
    assert int(got["dcem_trace_params"]) == ctypes.sizeof(dcem.TraceParams)
    assert int(got["dcem_frame_stats"]) == ctypes.sizeof(dcem.FrameStats)
    assert int(got["dcem_allocator"]) == ctypes.sizeof(dcem.AllocatorDesc)
    for key, cls in [("dcem_scene_desc", dcem.SceneDesc), ("dcem_trace_params", dcem.TraceParams),
                     ("dcem_frame_stats", dcem.FrameStats), ("dcem_allocator", dcem.AllocatorDesc)]:
        for k, v in got.items():
            if k.startswith(key + "."):
                assert getattr(cls, k.split(".")[1]).offset == int(v), k


def test_scenes_deterministic_and_sized():
    a, b = scenes.dynamic_urban(), scenes.dynamic_urban()
    assert np.array_equal(a.vertices, b.vertices) and np.array_equal(a.rx, b.rx)
    assert a.n_tris == 32002 and a.n_faces == 625 and a.n_objects == 40
    assert np.array_equal(a.transforms(17), b.transforms(17))
    s = scenes.static_toy()
    assert s.n_tris == 50 and s.n_faces == 25 and s.rx.shape == (16, 3)
    # faces are planar groups: every triangle of a face lies in one axis plane here
    for f in range(a.n_faces):
        v = a.vertices[a.tris[a.tri_face == f]].reshape(-1, 3)
        assert np.any(np.ptp(v, axis=0) == 0.0)


def test_vehicles_move_and_wrap():
    s = scenes.dynamic_urban(n_frames=60)
    x0, x59 = s.transforms(0), s.transforms(59)
    assert np.all(x0[:, :, 3] == 0)
    moved = np.abs(x59[:, :2, 3]).max(axis=1)
    assert np.all(moved > 0)
    assert np.all(np.abs(x59[:, 2, 3]) == 0)


def _toy_tree():
    # 3 triangles, hand-built tree: root(0) -> [node 1, leaf 2]; node 1 -> [leaf 0, leaf 1]
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [2, 0, 0], [3, 0, 0], [2, 1, 0],
                  [5, 5, 5], [6, 5, 5], [5, 6, 5]], np.float32)
    T = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)
    child = np.array([[1, ~2], [~0, ~1]], np.int32)
    leaf_tri = np.array([0, 1, 2], np.int32)

    def tb(t):
        v = V[T[t]]
        return np.concatenate([v.min(0), v.max(0)])
    box = np.zeros((2, 2, 6), np.float32)
    box[1, 0], box[1, 1] = tb(0), tb(1)
    box[0, 0] = np.concatenate([np.minimum(tb(0)[:3], tb(1)[:3]), np.maximum(tb(0)[3:], tb(1)[3:])])
    box[0, 1] = tb(2)
    return child, box, leaf_tri, V, T


def test_bvh_checker_accepts_sound_tree():
    child, box, leaf_tri, V, T = _toy_tree()
    assert check_bvh(child, box, leaf_tri, V, T, exact=True) == []


@pytest.mark.parametrize("mistake", ["shrunk_leaf", "shrunk_parent", "dup_leaf", "bad_perm", "loose_union"])
def test_bvh_checker_catches_mistakes(mistake):
    child, box, leaf_tri, V, T = _toy_tree()
    if mistake == "shrunk_leaf":
        box[1, 1, 3] -= 0.5
    elif mistake == "shrunk_parent":
        box[0, 0, 3] -= 0.5
    elif mistake == "dup_leaf":
        child[1, 1] = ~0
    elif mistake == "bad_perm":
        leaf_tri[2] = 0
    elif mistake == "loose_union":
        box[0, 0, 0] -= 1.0
    exact = mistake == "loose_union"
    assert check_bvh(child, box, leaf_tri, V, T, exact=exact) != []
