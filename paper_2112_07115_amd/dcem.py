"""Python binding of libdcem (ctypes): argument marshalling only.

Every step of a frame runs in the HIP kernels behind include/dcem.h; this
module converts NumPy arrays or torch tensors to pointers, passes the caller's
HIP stream, and turns status codes into exceptions.  It raises at import of a
context if the shared library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcem.so")

OK = 0
E_INVALID_ARG, E_OUT_OF_MEMORY, E_DEVICE, E_STATE, E_CAPACITY, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
MODE_FULL, MODE_COHERENT = 0, 1
FORCE_REBUILD = 1
DISCOVER_CAPTURE, DISCOVER_VISITED = 0, 1
REBUILD_SUBTREES = 2
REFITTED, REBUILT_FULL, REBUILT_SUBTREES = 0, 1, 2
MAX_REFLECTIONS = 10
PATTERN_TAPS = 16

_P = ctypes.c_void_p
_I32, _I64, _F32, _F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double


class SceneDesc(ctypes.Structure):
    _fields_ = [("vertices", _P), ("n_vertices", _I64), ("tris", _P), ("tri_face", _P), ("n_tris", _I64),
                ("face_material", _P), ("face_object", _P), ("n_faces", _I32), ("materials", _P),
                ("n_materials", _I32), ("object_vertex_range", _P), ("n_objects", _I32), ("mem_kind", _I32)]


class TraceParams(ctypes.Structure):
    _fields_ = [("tx_pos", _P), ("n_tx", _I32), ("rx_pos", _P), ("n_rx", _I32), ("rx_radius", _F32),
                ("n_rays", _I64), ("ray_dirs", _P), ("max_reflections", _I32), ("freqs_hz", _P),
                ("n_freqs", _I32), ("tx_power_w", _F64), ("atten_db_per_km", _F64), ("mode", _I32),
                ("los_always", _I32), ("keep_cache", _I32), ("record_trace_log", _I32), ("mem_kind", _I32),
                ("trace_from_rx", _I32), ("discovery", _I32), ("max_transmissions", _I32)]


class FrameStats(ctypes.Structure):
    _fields_ = [("rays_total", _I64), ("rays_traced", _I64), ("rays_reused", _I64), ("segments", _I64),
                ("captures", _I64), ("unique_candidates", _I64), ("valid_paths", _I64),
                ("nodes_visited", _I64), ("tri_tests", _I64), ("rebuilt", _I32),
                ("coherent", _I32), ("sah_ratio", _F64), ("ms_refit", _F32), ("ms_coherence", _F32),
                ("ms_trace", _F32), ("ms_candidates", _F32), ("ms_refine", _F32), ("ms_reduce", _F32),
                ("trace_kernel", _I32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_ALLOC_FN = ctypes.CFUNCTYPE(_P, ctypes.c_size_t, _P, _P)
_FREE_FN = ctypes.CFUNCTYPE(None, _P, ctypes.c_size_t, _P, _P)


class AllocatorDesc(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", _P)]


class TorchAllocator:
    """dcem_allocator backed by torch's CUDA caching allocator: the library's
    device buffers are then torch's memory (counted by
    torch.cuda.memory_allocated, reused through its pools)."""

    def __init__(self, device: int):
        import torch
        self.device = device
        self.live = {}

        def alloc(nbytes, stream, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=int(stream or 0))
            except Exception:   # reported by the library as out of memory
                return None
            self.live[p] = int(nbytes)
            return p

        def free(p, nbytes, stream, user):
            if self.live.pop(p, None) is not None and not sys.is_finalizing():
                try:
                    torch.cuda.caching_allocator_delete(p)
                except Exception:   # interpreter shutdown: torch already torn down
                    pass

        self._alloc, self._free = _ALLOC_FN(alloc), _FREE_FN(free)   # kept alive with the context
        self.desc = AllocatorDesc(self._alloc, self._free, None)


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_ctx", _I32), ("lds_stack", _I32), ("blocks_per_cu", _I32), ("chunk", _I32), ("tuned", _I32),
                ("graph_frames", _I32), ("ms_trace_tuned", _F32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) of every exported entry point of include/dcem.h
SIGNATURES = [
    ("dcem_create", _I32, [ctypes.POINTER(_P), _I32, _P, ctypes.POINTER(AllocatorDesc)]),
    ("dcem_destroy", None, [_P]),
    ("dcem_last_error", ctypes.c_char_p, [_P]),
    ("dcem_set_capture_capacity", _I32, [_P, _I64]),
    ("dcem_set_timing", _I32, [_P, _I32]),
    ("dcem_set_stack_limit", _I32, [_P, _I32]),
    ("dcem_scene_upload", _I32, [_P, ctypes.POINTER(SceneDesc)]),
    ("dcem_set_object_transforms", _I32, [_P, _P, _I32, _I32]),
    ("dcem_refit_bvh", _I32, [_P, _I32, _F64, ctypes.POINTER(_I32), ctypes.POINTER(_F64)]),
    ("dcem_trace_frame", _I32, [_P, ctypes.POINTER(TraceParams)]),
    ("dcem_received_power", _I32, [_P, _P, _P, _I32]),
    ("dcem_set_tx_pattern", _I32, [_P, _P, _I32]),
    ("dcem_set_materials", _I32, [_P, _P, _I32]),
    ("dcem_set_penetration_loss", _I32, [_P, _P, _I32]),
    ("dcem_power_gradients", _I32, [_P, _P, _P, _P, _P]),
    ("dcem_power_gradients_noalloc", _I32, [_P, _P, _P, _P, _P]),
    ("dcem_get_paths", _I32, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_I64)]),
    ("dcem_get_trace_log", _I32, [_P, _P, _P, _P]),
    ("dcem_get_captures", _I32, [_P, _I64, _P, ctypes.POINTER(_I64)]),
    ("dcem_get_bvh", _I32, [_P, _I64, ctypes.POINTER(_I32), _P, _P, _P]),
    ("dcem_get_vertices", _I32, [_P, _P]),
    ("dcem_get_ray_dirs", _I32, [_P, _P]),
    ("dcem_get_stats", _I32, [_P, ctypes.POINTER(FrameStats)]),
    ("dcem_batch_create", _I32, [ctypes.POINTER(_P), ctypes.POINTER(_P), _I32]),
    ("dcem_batch_destroy", None, [_P]),
    ("dcem_batch_set_graph", _I32, [_P, _I32]),
    ("dcem_batch_set_shape", _I32, [_P, _I32, _I32, _I32]),
    ("dcem_batch_trace", _I32, [_P, ctypes.POINTER(TraceParams)]),
    ("dcem_batch_tune", _I32, [_P, ctypes.POINTER(TraceParams), _I32]),
    ("dcem_batch_get_info", _I32, [_P, ctypes.POINTER(BatchInfo)]),
]

_lib = None

# Contexts and batches still open: closed at interpreter exit while torch (whose
# allocator may own their buffers) is still alive; batches before contexts.
_live_batches = weakref.WeakSet()
_live_contexts = weakref.WeakSet()


@atexit.register
def _close_all():
    for b in list(_live_batches):
        b.close()
    for c in list(_live_contexts):
        c.close()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdcem.so; raises if it is missing (build it with paper_2112_07115_amd.build)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libdcem.so not built (%s); run `python -m paper_2112_07115_amd.build`" % path)
    # torch carries its own HIP runtime with the same soname: loaded first, it is
    # the one runtime of the process and libdcem binds to it, so torch's streams
    # and tensors are valid here.  Loaded after libdcem, torch would bind to the
    # system runtime and find no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


class DcemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("dcem status %d: %s" % (status, message))
        self.status = status


def _addr(a) -> Optional[int]:
    """Address of a contiguous NumPy array or torch tensor (None passes NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def _kind(a) -> int:
    if a is None or isinstance(a, np.ndarray):
        return MEM_HOST
    return MEM_DEVICE if a.is_cuda else MEM_HOST


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Context:
    """One dcem context: a device, a HIP stream and the scene, BVH and ray cache on it.

    allocator: "torch" (default when torch is loaded) takes every device
    buffer from torch's caching allocator, None uses hipMalloc; any other
    object supplies its own dcem_allocator as `.desc` (an AllocatorDesc whose
    callbacks it keeps alive)."""

    def __init__(self, device: int = 0, stream=None, allocator="torch"):
        self.lib = load_library()
        torch = sys.modules.get("torch")
        if stream is None:
            # follow torch's current stream when torch is in use; else the null stream
            stream = torch.cuda.current_stream(device).cuda_stream if torch is not None else 0
        if isinstance(allocator, str):
            if allocator != "torch":
                raise ValueError("allocator: 'torch', None or an object with .desc")
            self.allocator = TorchAllocator(device) if torch is not None else None
        else:
            self.allocator = allocator
        self.handle = _P()
        st = self.lib.dcem_create(ctypes.byref(self.handle), device, _P(stream or None),
                                  ctypes.byref(self.allocator.desc) if self.allocator else None)
        if st != OK:
            raise DcemError(st, "dcem_create failed (device %d)" % device)
        _live_contexts.add(self)
        self._keep = []
        self._batches = []
        self.K = 0
        self.n_freqs = 1
        self.n_tx = self.n_rx = self.n_src = 0
        self.n_branch = 1
        self.n_rays = 0

    def close(self):
        for b in list(getattr(self, "_batches", [])):
            b.close()   # a batch holds the context's handle
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.dcem_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            raise DcemError(st, self.lib.dcem_last_error(self.handle).decode())

    def set_capture_capacity(self, n: int):
        self._check(self.lib.dcem_set_capture_capacity(self.handle, int(n)))

    def set_stack_limit(self, entries: int = 0):
        """Cap the traversal stacks (0: full depth); an overflow is reported as E_CAPACITY."""
        self._check(self.lib.dcem_set_stack_limit(self.handle, int(entries)))

    def set_timing(self, on: bool = True):
        self._check(self.lib.dcem_set_timing(self.handle, 1 if on else 0))

    def scene_upload(self, scene):
        """Upload a scene (object with the arrays of paper_2112_07115_amd.scenes.Scene)."""
        arrs = [_host(scene.vertices, np.float32), _host(scene.tris, np.int32),
                _host(scene.tri_face, np.int32), _host(scene.face_material, np.int32),
                _host(scene.face_object, np.int32), _host(scene.materials, np.float64),
                _host(scene.object_vertex_range, np.int64)]
        V, T, TF, FM, FO, M, OR = arrs
        d = SceneDesc(_addr(V), V.shape[0], _addr(T), _addr(TF), T.shape[0], _addr(FM), _addr(FO),
                      FM.shape[0], _addr(M), M.shape[0], _addr(OR), OR.shape[0], MEM_HOST)
        self._check(self.lib.dcem_scene_upload(self.handle, ctypes.byref(d)))
        pen = getattr(scene, "penetration_db", None)   # per material, +inf opaque (Table II losses)
        if pen is not None:
            self.set_penetration_loss(pen)
        self.n_vertices = V.shape[0]
        self.n_tris = T.shape[0]
        self.n_objects = OR.shape[0]
        self.n_materials = M.shape[0]

    def set_object_transforms(self, xf):
        a = xf if not isinstance(xf, np.ndarray) else _host(xf, np.float32)
        n = int(a.shape[0])
        self._check(self.lib.dcem_set_object_transforms(self.handle, _addr(a), n, _kind(a)))

    def refit_bvh(self, force_rebuild: bool = False, threshold: float = 1.5, subtrees: bool = False):
        """Refit (or rebuild) the tree for the current vertices; returns
        (decision, SAH ratio): REFITTED, REBUILT_FULL or REBUILT_SUBTREES."""
        rb = _I32(0)
        ratio = _F64(0.0)
        flags = (FORCE_REBUILD if force_rebuild else 0) | (REBUILD_SUBTREES if subtrees else 0)
        self._check(self.lib.dcem_refit_bvh(self.handle, flags, float(threshold), ctypes.byref(rb),
                                            ctypes.byref(ratio)))
        return int(rb.value), float(ratio.value)

    def _params(self, tx, rx, rx_radius: float, n_rays: int, ray_dirs=None, max_reflections: int = 2,
                freqs_hz: Sequence[float] = (28e9,), tx_power_w: float = 5.0, atten_db_per_km: float = 0.0,
                mode: int = MODE_FULL, los_always: bool = True, keep_cache: bool = False,
                record_trace_log: bool = False, trace_from_rx: bool = False, discovery: int = 0,
                max_transmissions: int = 0):
        """dcem_trace_params of one frame (arrays kept alive on the context).
        A frame called with the same array objects and values as the last one
        reuses its parameter block (the library reads the arrays at each call)."""
        key = (rx_radius, n_rays, max_reflections, tx_power_w, atten_db_per_km, mode, los_always, keep_cache,
               record_trace_log, trace_from_rx, discovery, max_transmissions)
        fkey = tuple(float(f) for f in np.asarray(freqs_hz, dtype=np.float64).reshape(-1))
        last = getattr(self, "_pcache", None)
        if (last is not None and last[0] is tx and last[1] is rx and last[2] is ray_dirs and last[3] == fkey
                and last[4] == key):
            return last[5], last[6]
        dev = ray_dirs is not None and not isinstance(ray_dirs, np.ndarray) and ray_dirs.is_cuda
        if dev:
            txa, rxa, dirs = tx, rx, ray_dirs
        else:
            txa, rxa = _host(tx, np.float32).reshape(-1, 3), _host(rx, np.float32).reshape(-1, 3)
            dirs = None if ray_dirs is None else _host(ray_dirs, np.float32).reshape(-1, 3)
        fr = _host(freqs_hz, np.float64).reshape(-1)
        self._keep = [txa, rxa, dirs, fr]
        p = TraceParams(_addr(txa), int(txa.shape[0]), _addr(rxa), int(rxa.shape[0]), float(rx_radius),
                        int(n_rays), _addr(dirs), int(max_reflections), _addr(fr), int(fr.shape[0]),
                        float(tx_power_w), float(atten_db_per_km), int(mode), int(bool(los_always)),
                        int(bool(keep_cache)), int(bool(record_trace_log)), MEM_DEVICE if dev else MEM_HOST,
                        int(bool(trace_from_rx)), int(discovery), int(max_transmissions))
        n_tx, n_rx = int(txa.shape[0]), int(rxa.shape[0])
        shape = (int(max_reflections) + int(max_transmissions), int(fr.shape[0]), n_tx, n_rx, int(n_rays),
                 n_rx if trace_from_rx else n_tx, n_branches(int(max_reflections), int(max_transmissions)))
        # reusable only while the block points at the caller's own arrays (a
        # converted copy would not follow later changes to them)
        def same_buffer(a, b):
            return b is None or (isinstance(a, np.ndarray) and a.ctypes.data == b.ctypes.data)
        cacheable = not dev and same_buffer(tx, txa) and same_buffer(rx, rxa) and \
            (ray_dirs is None or same_buffer(ray_dirs, dirs))
        self._pcache = (tx, rx, ray_dirs, fkey, key, p, shape) if cacheable else None
        return p, shape

    def _traced(self, shape):
        # K: interactions per path at most; n_src: the rays' origins (the
        # receivers when tracing backward); n_branch: traces per ray
        self.K, self.n_freqs, self.n_tx, self.n_rx, self.n_rays, self.n_src, self.n_branch = shape

    def trace_frame(self, tx, rx, rx_radius: float, n_rays: int, ray_dirs=None,
                    max_reflections: int = 2, freqs_hz: Sequence[float] = (28e9,),
                    tx_power_w: float = 5.0, atten_db_per_km: float = 0.0, mode: int = MODE_FULL,
                    los_always: bool = True, keep_cache: bool = False, record_trace_log: bool = False,
                    trace_from_rx: bool = False, discovery: int = 0, max_transmissions: int = 0):
        p, shape = self._params(tx, rx, rx_radius, n_rays, ray_dirs, max_reflections, freqs_hz, tx_power_w,
                                atten_db_per_km, mode, los_always, keep_cache, record_trace_log, trace_from_rx,
                                discovery, max_transmissions)
        self._check(self.lib.dcem_trace_frame(self.handle, ctypes.byref(p)))
        self._traced(shape)

    def received_power(self, out=None):
        """(p_coh, p_inc) [n_freqs, n_tx, n_rx] FP64; host arrays unless `out` tensors are given."""
        shape = (self.n_freqs, self.n_tx, self.n_rx)
        if out is None:
            pc = np.empty(shape, np.float64)
            pi = np.empty(shape, np.float64)
        else:
            pc, pi = out
        self._check(self.lib.dcem_received_power(self.handle, _addr(pc), _addr(pi), _kind(pc)))
        return pc, pi

    def set_tx_pattern(self, weights=None):
        """Transmit pattern weights (16 azimuth hats) for the next frames;
        None restores the isotropic antenna."""
        if weights is None:
            self._check(self.lib.dcem_set_tx_pattern(self.handle, None, 0))
            return
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        self._check(self.lib.dcem_set_tx_pattern(self.handle, _addr(w), int(w.shape[0])))

    def set_penetration_loss(self, loss_db):
        """Penetration loss in dB per material (+inf: opaque) for the next frames."""
        v = _host(loss_db, np.float64).reshape(-1)
        self._check(self.lib.dcem_set_penetration_loss(self.handle, _addr(v), int(v.shape[0])))

    def set_materials(self, materials):
        """New material table [n_materials, 3] (eps_r, sigma, const_gamma) for
        the next frames; geometry and caches stay."""
        m = np.ascontiguousarray(materials, dtype=np.float64).reshape(-1, 3)
        self._check(self.lib.dcem_set_materials(self.handle, _addr(m), int(m.shape[0])))

    def power_gradients(self):
        """Derivatives of the last frame's coherent power along its paths:
        (d_eps_r, d_sigma) [n_freqs, n_tx, n_rx, n_materials], d_tx_power
        [n_freqs, n_tx, n_rx] and d_pattern [n_freqs, n_tx, n_rx, 16], FP64
        host arrays."""
        shape = (self.n_freqs, self.n_tx, self.n_rx)
        de = np.empty(shape + (self.n_materials,), np.float64)
        ds = np.empty(shape + (self.n_materials,), np.float64)
        dp = np.empty(shape, np.float64)
        dw = np.empty(shape + (PATTERN_TAPS,), np.float64)
        self._check(self.lib.dcem_power_gradients(self.handle, _addr(de), _addr(ds), _addr(dp), _addr(dw)))
        return de, ds, dp, dw

    def power_gradients_noalloc(self, out=None):
        """power_gradients() through the entry point that allocates nothing
        (fixed per-GPU workspace); `out`: four preallocated host arrays of the
        shapes power_gradients returns (allocated here when None)."""
        shape = (self.n_freqs, self.n_tx, self.n_rx)
        if out is None:
            out = (np.empty(shape + (self.n_materials,), np.float64), np.empty(shape + (self.n_materials,), np.float64),
                   np.empty(shape, np.float64), np.empty(shape + (PATTERN_TAPS,), np.float64))
        de, ds, dp, dw = out
        self._check(self.lib.dcem_power_gradients_noalloc(self.handle, _addr(de), _addr(ds), _addr(dp), _addr(dw)))
        return de, ds, dp, dw

    def stats(self) -> dict:
        s = FrameStats()
        self._check(self.lib.dcem_get_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def paths(self) -> dict:
        n = _I64(0)
        self._check(self.lib.dcem_get_paths(self.handle, 0, None, None, None, None, None, None, None, None,
                                            ctypes.byref(n)))
        m = int(n.value)
        K, nf = self.K, self.n_freqs
        out = {"keys": np.zeros((m, 3 + K), np.int32), "valid": np.zeros(m, np.uint8),
               "length": np.zeros(m), "tau": np.zeros(m), "aod": np.zeros((m, 3)), "aoa": np.zeros((m, 3)),
               "amp": np.zeros((m, nf, 3, 2)), "first_ray": np.zeros(m, np.int32)}
        if m:
            self._check(self.lib.dcem_get_paths(self.handle, m, _addr(out["keys"]), _addr(out["valid"]),
                                                _addr(out["length"]), _addr(out["tau"]), _addr(out["aod"]),
                                                _addr(out["aoa"]), _addr(out["amp"]), _addr(out["first_ray"]),
                                                ctypes.byref(n)))
        out["valid"] = out["valid"].astype(bool)
        out["amp"] = out["amp"][..., 0] + 1j * out["amp"][..., 1]
        return out

    def trace_log(self):
        shp = (self.n_src, self.n_branch * self.n_rays, self.K + 1)
        tri = np.empty(shp, np.int32)
        t = np.empty(shp, np.float32)
        length = np.empty(shp, np.float32)
        self._check(self.lib.dcem_get_trace_log(self.handle, _addr(tri), _addr(t), _addr(length)))
        return tri, t, length

    def captures(self) -> np.ndarray:
        n = _I64(0)
        self._check(self.lib.dcem_get_captures(self.handle, 0, None, ctypes.byref(n)))
        rows = np.zeros((int(n.value), 4 + self.K), np.int32)
        if n.value:
            self._check(self.lib.dcem_get_captures(self.handle, rows.shape[0], _addr(rows), ctypes.byref(n)))
        return rows

    def bvh(self):
        ni = _I32(0)
        self._check(self.lib.dcem_get_bvh(self.handle, 0, ctypes.byref(ni), None, None, None))
        n = int(ni.value)
        child = np.zeros((n, 2), np.int32)
        box = np.zeros((n, 2, 6), np.float32)
        leaf_tri = np.zeros(self.n_tris, np.int32)
        self._check(self.lib.dcem_get_bvh(self.handle, n, ctypes.byref(ni), _addr(child), _addr(box),
                                          _addr(leaf_tri)))
        return child, box, leaf_tri

    def vertices(self) -> np.ndarray:
        out = np.empty((self.n_vertices, 3), np.float32)
        self._check(self.lib.dcem_get_vertices(self.handle, _addr(out)))
        return out

    def ray_dirs(self) -> np.ndarray:
        out = np.empty((self.n_rays, 3), np.float32)
        self._check(self.lib.dcem_get_ray_dirs(self.handle, _addr(out)))
        return out


class Batch:
    """One frame of several contexts (each with its own scene) traced together:
    one persistent launch carries every full trace (dcem_batch_*)."""

    def __init__(self, contexts):
        self.ctxs = list(contexts)
        self.lib = self.ctxs[0].lib
        arr = (_P * len(self.ctxs))(*[c.handle.value for c in self.ctxs])
        self.handle = _P()
        st = self.lib.dcem_batch_create(ctypes.byref(self.handle), arr, len(self.ctxs))
        if st != OK:
            raise DcemError(st, self.ctxs[0].lib.dcem_last_error(self.ctxs[0].handle).decode())
        _live_batches.add(self)
        for c in self.ctxs:
            c._batches.append(self)

    def _check(self, st):
        if st != OK:
            msgs = {c.lib.dcem_last_error(c.handle).decode() for c in self.ctxs} - {""}
            raise DcemError(st, "; ".join(sorted(msgs)))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.dcem_batch_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _params(self, frames):
        """frames: one dict of Context.trace_frame keyword arguments per context."""
        arr = (TraceParams * len(self.ctxs))()
        shapes = []
        for j, (c, kw) in enumerate(zip(self.ctxs, frames)):
            p, shape = c._params(**kw)
            arr[j] = p
            shapes.append(shape)
        return arr, shapes

    def trace(self, frames):
        arr, shapes = self._params(frames)
        self._check(self.lib.dcem_batch_trace(self.handle, arr))
        for c, sh in zip(self.ctxs, shapes):
            c._traced(sh)

    def tune(self, frames, repeats: int = 1):
        arr, shapes = self._params(frames)
        self._check(self.lib.dcem_batch_tune(self.handle, arr, int(repeats)))
        for c, sh in zip(self.ctxs, shapes):
            c._traced(sh)
        return self.info()

    def set_graph(self, on: bool = True):
        self._check(self.lib.dcem_batch_set_graph(self.handle, 1 if on else 0))

    def set_shape(self, lds_stack: int, blocks_per_cu: int, chunk: int):
        self._check(self.lib.dcem_batch_set_shape(self.handle, int(lds_stack), int(blocks_per_cu), int(chunk)))

    def info(self) -> dict:
        out = BatchInfo()
        self._check(self.lib.dcem_batch_get_info(self.handle, ctypes.byref(out)))
        return out.as_dict()


def n_branches(max_reflections: int, max_transmissions: int) -> int:
    """Traces per ray: sets of at most max_transmissions of the first
    max_reflections + max_transmissions interactions (dcem_trace_params)."""
    from math import comb
    slots = max_reflections + max_transmissions
    return sum(comb(slots, t) for t in range(max_transmissions + 1))


def scene_frame_args(scene, frame: int = 0, mode: int = MODE_FULL, **kw) -> dict:
    """Context.trace_frame keyword arguments of one frame of a scene."""
    args = dict(tx=scene.tx, rx=scene.rx_at(frame) if hasattr(scene, "rx_at") else scene.rx,
                rx_radius=scene.rx_radius, n_rays=scene.n_rays,
                max_reflections=scene.max_reflections, freqs_hz=scene.freqs_hz, tx_power_w=scene.tx_power_w,
                mode=mode, max_transmissions=getattr(scene, "max_transmissions", 0))
    args.update(kw)
    return args


@dataclass
class FrameOutput:
    p_coh: np.ndarray
    p_inc: np.ndarray


def trace_scene_frame(ctx: Context, scene, frame: int = 0, mode: int = MODE_FULL, ray_dirs=None,
                      n_rays: Optional[int] = None, K: Optional[int] = None, rebuild: bool = False,
                      keep_cache: bool = False, record_trace_log: bool = False, los_always: bool = True,
                      threshold: float = 1.5, atten_db_per_km: float = 0.0,
                      trace_from_rx: bool = False, discovery: int = 0,
                      max_transmissions: Optional[int] = None) -> FrameOutput:
    """Convenience: place the scene's objects for `frame`, update the BVH, trace, read power."""
    if scene.object_vertex_range.shape[0]:
        ctx.set_object_transforms(scene.transforms(frame))
        ctx.refit_bvh(force_rebuild=rebuild, threshold=threshold)
    n = scene.n_rays if n_rays is None else n_rays
    if ray_dirs is not None:
        n = ray_dirs.shape[0]
    rx = scene.rx_at(frame) if hasattr(scene, "rx_at") else scene.rx
    ctx.trace_frame(scene.tx, rx, scene.rx_radius, n, ray_dirs=ray_dirs,
                    max_reflections=scene.max_reflections if K is None else K, freqs_hz=scene.freqs_hz,
                    tx_power_w=scene.tx_power_w, atten_db_per_km=atten_db_per_km, mode=mode,
                    los_always=los_always, keep_cache=keep_cache, record_trace_log=record_trace_log,
                    trace_from_rx=trace_from_rx, discovery=discovery,
                    max_transmissions=getattr(scene, "max_transmissions", 0) if max_transmissions is None
                    else max_transmissions)
    pc, pi = ctx.received_power()
    return FrameOutput(pc, pi)
