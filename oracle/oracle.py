"""Python front end of the CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain FP64 brute-force implementation of what one frame of the
dynamic EM ray tracer computes (paper Sec. III: ray sphere, specular bounces,
per-depth visited-path tables, image-method refinement, path validation, and
per-path distance / attenuation / phase).  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import this module.  It never imports
the GPU library and shares no code with it.

Scene objects are taken by duck typing (attributes ``vertices``, ``tris``,
``tri_face``, ``face_material``, ``face_object``, ``materials``,
``object_vertex_range``, ``tx``, ``rx``, ``rx_radius``, ...), so this module
does not import the package either.

Functions and the passages they follow:
  fibonacci          ray sphere (step 1 of the frame algorithm)
  trace              bounces + capture spheres (steps 1-2); rays start at the
                     sources and are captured at spheres around the targets
  visited_candidates every distinct series of faces the rays visit, tried
                     against every target (steps 2-4 without capture spheres)
  candidates         de-duplicated (tx, rx, order, faces) keys (step 2's tables);
                     records traced backward from the receivers (Sec. III,
                     "Backward ray tracing": sources = receivers, targets =
                     transmitters) are turned into the path's key from the
                     transmitter: pair swapped, faces in reverse order
  refine             image method, validity, field per path (steps 3, 4, 6;
                     Eq. (3) with n = 2 for the free-space magnitude)
  received_power     phase-coherent sum per receiver ("phase calculation")
  frame              all of the above for one frame
  refine_grad,       derivatives of each receiver's coherent power along the
  power_gradients    frame's paths with respect to every material's eps_r and
                     sigma (the Fresnel coefficients of the field model,
                     differentiated in closed form) and the transmit power
  pattern_gain,      the transmit field pattern (an extension of the paper's
  pattern_gradients  isotropic antenna: 16 periodic azimuth hats, weights 1 =
                     isotropic) and dP/dw of its weights along the paths
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dcem_oracle.cpp")
_LIB = os.environ.get("DCEM_ORACLE_LIB") or os.path.join(_HERE, "libdcem_oracle.so")

SEG_TIE, SEG_EDGE, SEG_TRI = 1, 2, 4
CAP_HIT, CAP_MARGINAL, CAP_UNCERTAIN = 1, 2, 4

T_MIN = 1e-4          # metres; hits closer than this to a segment start are ignored
EPS_TRACE = 4e-6      # relative position tolerance of an FP32 tracer (see flags)
EPS_REFINE = 1e-9     # relative tolerance of an FP64 validation
EPS0 = 8.8541878128e-12   # vacuum permittivity [F/m]
PATTERN_TAPS = 16         # azimuth hats of the transmit pattern


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math)."""
    if os.environ.get("DCEM_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.oracle_scene_new.restype = P
        lib.oracle_scene_new.argtypes = [P, I64, P, P, I64, P, P, I32, P, I32, P, I32, P]
        lib.oracle_scene_free.argtypes = [P]
        lib.oracle_scene_radius.argtypes = [P, P]
        lib.oracle_fibonacci.argtypes = [I64, P]
        lib.oracle_trace.restype = I64
        lib.oracle_trace.argtypes = [P, P, I32, P, I32, F64, P, I64, P, I64, I32, I32, P, I32, F64, F64, I32,
                                     P, P, P, P, P, P, P, I64]
        lib.oracle_scene_set_penetration.argtypes = [P, P, I32]
        lib.oracle_refine.argtypes = [P, P, P, P, I64, I32, P, I32, F64, F64, F64, F64, I32,
                                      P, P, P, P, P, P, P, P]
        lib.oracle_fresnel.argtypes = [F64, F64, F64, F64, F64, P]
        lib.oracle_refine_grad.argtypes = [P, P, P, P, I64, I32, P, I32, F64, F64, F64, F64, I32, P, P]
        lib.oracle_pattern_gain.restype = F64
        lib.oracle_pattern_gain.argtypes = [P, F64, F64, F64]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class OracleScene:
    """FP64 copy of a scene at one frame (object transforms applied)."""

    def __init__(self, scene, xf: Optional[np.ndarray] = None):
        lib = _load()
        self._keep = [
            np.ascontiguousarray(scene.vertices, dtype=np.float32),
            np.ascontiguousarray(scene.tris, dtype=np.int32),
            np.ascontiguousarray(scene.tri_face, dtype=np.int32),
            np.ascontiguousarray(scene.face_material, dtype=np.int32),
            np.ascontiguousarray(scene.face_object, dtype=np.int32),
            np.ascontiguousarray(scene.materials, dtype=np.float64),
            np.ascontiguousarray(scene.object_vertex_range, dtype=np.int64),
        ]
        V, T, TF, FM, FO, M, OR = self._keep
        xfa = None if xf is None else np.ascontiguousarray(xf, dtype=np.float32)
        self.n_faces = FM.shape[0]
        self.handle = lib.oracle_scene_new(
            _ptr(V), V.shape[0], _ptr(T), _ptr(TF), T.shape[0], _ptr(FM), _ptr(FO), FM.shape[0],
            _ptr(M), M.shape[0], _ptr(OR), OR.shape[0], _ptr(xfa))
        # penetration loss per material in dB (+inf opaque; Table II)
        pen = getattr(scene, "penetration_db", None)
        if pen is not None:
            pa = np.ascontiguousarray(pen, dtype=np.float64).reshape(-1)
            self._keep.append(pa)
            lib.oracle_scene_set_penetration(self.handle, _ptr(pa), pa.shape[0])

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.oracle_scene_free(self.handle)
            self.handle = None


def fibonacci(n: int) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float32)
    _load().oracle_fibonacci(n, _ptr(out))
    return out


def fresnel(eps_r: float, sigma: float, freq: float, cos_theta: float,
            const_gamma: float = float("nan")):
    out = np.empty(4, dtype=np.float64)
    _load().oracle_fresnel(eps_r, sigma, const_gamma, freq, cos_theta, _ptr(out))
    return complex(out[0], out[1]), complex(out[2], out[3])


@dataclass
class TraceResult:
    # per (source, branch * nsel + ray, segment); K = interactions at most
    tri: np.ndarray        # i32 [ntx, nb * nsel, K+1]  (-1 miss, -2 not traced)
    face: np.ndarray       # i32 [ntx, nb * nsel, K+1]
    t: np.ndarray          # f64 [ntx, nb * nsel, K+1]
    length: np.ndarray     # f64 [ntx, nb * nsel, K+1]
    flags: np.ndarray      # i32 [ntx, nb * nsel, K+1]  SEG_*
    caps: np.ndarray       # i32 [ncap, 4 + K]     (ray, tx, rx, order, faces...)
    cap_flags: np.ndarray  # i32 [ncap]            CAP_*
    sets: tuple = (0,)     # transmitting interactions of each branch (bit j: interaction j)


def branch_sets(slots: int, max_t: int) -> list:
    """The branches of a ray that may transmit at up to max_t of its first
    `slots` interactions: every such set of interaction indices as a bit mask,
    by size and then lexicographically (branch 0: the ray that only reflects;
    Sec. III, "Reflected and transmitted rays")."""
    out = [0]
    for t in range(1, max_t + 1):
        for combo in itertools.combinations(range(slots), t):
            out.append(sum(1 << j for j in combo))
    return out


def trace(osc: OracleScene, tx, rx, radius: float, dirs: np.ndarray, K: int,
          ray_ids: Optional[np.ndarray] = None, t_min: float = T_MIN,
          eps_rel: float = EPS_TRACE, nthreads: Optional[int] = None,
          max_transmissions: int = 0) -> TraceResult:
    """Rays from every source (tx), captured at spheres around the targets
    (rx).  K: reflections at most; with max_transmissions > 0 every ray is
    traced once per branch (branch_sets) and paths hold up to K +
    max_transmissions interactions, a transmission through face f recorded as
    -2 - f; capture rows name ray b * len(dirs) + id for branch b."""
    lib = _load()
    max_refl = K
    K = max_refl + max_transmissions
    sets = np.array(branch_sets(K, max_transmissions), dtype=np.uint32)
    nb = sets.shape[0]
    tx = np.ascontiguousarray(tx, dtype=np.float32).reshape(-1, 3)
    rx = np.ascontiguousarray(rx, dtype=np.float32).reshape(-1, 3)
    dirs = np.ascontiguousarray(dirs, dtype=np.float32).reshape(-1, 3)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, dtype=np.int64)
    nsel = dirs.shape[0] if ids is None else ids.shape[0]
    ntx = tx.shape[0]
    shp = (ntx, nb * nsel, K + 1)
    tri = np.empty(shp, np.int32)
    face = np.empty(shp, np.int32)
    t = np.empty(shp, np.float64)
    length = np.empty(shp, np.float64)
    flags = np.empty(shp, np.int32)
    cap = max(1024, 4 * ntx * nb * nsel)
    nthreads = nthreads or default_threads()
    while True:
        rows = np.empty((cap, 4 + K), np.int32)
        cflags = np.empty(cap, np.int32)
        n = lib.oracle_trace(osc.handle, _ptr(tx), ntx, _ptr(rx), rx.shape[0], float(radius),
                             _ptr(dirs), dirs.shape[0], _ptr(ids), nsel, K, max_refl, _ptr(sets), nb,
                             t_min, eps_rel, nthreads,
                             _ptr(tri), _ptr(face), _ptr(t), _ptr(length), _ptr(flags),
                             _ptr(rows), _ptr(cflags), cap)
        if n <= cap:
            return TraceResult(tri, face, t, length, flags, rows[:n].copy(), cflags[:n].copy(),
                               tuple(int(x) for x in sets))
        cap = int(n)


def los_keys(ntx: int, nrx: int, K: int) -> np.ndarray:
    """Direct-path keys (tx, rx, 0, -1...) for every pair: direct rays are their own mechanism."""
    keys = np.full((ntx * nrx, 3 + K), -1, dtype=np.int32)
    keys[:, 0] = np.repeat(np.arange(ntx), nrx)
    keys[:, 1] = np.tile(np.arange(nrx), ntx)
    keys[:, 2] = 0
    return keys


def path_rows(rows: np.ndarray, K: int, backward: bool) -> np.ndarray:
    """Capture rows (src, tgt, order, faces in traced order) as path keys
    (tx, rx, order, faces from the transmitter).  Forward rows are keys
    already; a row traced from a receiver names (rx, tx) and lists the faces
    from the receiver's end, so the pair is swapped and the first `order`
    faces are reversed."""
    rows = np.asarray(rows, dtype=np.int32).reshape(-1, 3 + K)
    if not backward:
        return rows
    out = rows.copy()
    out[:, 0], out[:, 1] = rows[:, 1], rows[:, 0]
    for o in range(2, K + 1):
        sel = rows[:, 2] == o
        out[sel, 3:3 + o] = rows[sel, 3:3 + o][:, ::-1]
    return out


def candidates(tr: TraceResult, ntx: int, nrx: int, K: int, los_always: bool = True,
               backward: bool = False):
    """Unique keys from exact captures, sorted by (tx, rx, order, f1..fK).
    ntx, nrx: the paths' transmitters and receivers; backward: tr was traced
    from the receivers (its rows name (rx, tx) and faces from the receiver).

    Returns (keys, certain, possible):
      keys      the oracle's own candidate set (captures with distance <= r)
      certain   bool per key: produced by at least one capture that no FP32
                tracer can decide differently
      possible  every key seen by any capture within r + eps (marginal and
                uncertain ones included); an FP32 tracer can only find keys
                outside this set on rays whose path the oracle marks uncertain
    """
    rows = path_rows(tr.caps[:, 1:], K, backward)
    hit = (tr.cap_flags & CAP_HIT) != 0
    sure = tr.cap_flags == CAP_HIT
    parts = [rows[hit]]
    if los_always:
        parts.append(los_keys(ntx, nrx, K))
    allk = np.concatenate(parts) if parts else np.zeros((0, 3 + K), np.int32)
    keys = np.unique(allk, axis=0) if len(allk) else allk
    sure_rows = rows[sure]
    if los_always:
        sure_rows = np.concatenate([sure_rows, los_keys(ntx, nrx, K)])
    certain = _member(keys, sure_rows)
    poss = [rows] + parts[1:]
    possible = np.unique(np.concatenate(poss), axis=0) if sum(len(x) for x in poss) \
        else np.zeros((0, 3 + K), np.int32)
    return keys, certain, possible


def visited_candidates(tr: TraceResult, ntx: int, nrx: int, K: int, los_always: bool = True,
                       backward: bool = False):
    """Visited-series discovery (Sec. III, the frame algorithm's steps 2-4):
    every series of faces a ray reflects on, up to the reflection limit, is
    entered in the visited table of its depth, and each distinct series is
    tried against every target (its images checked for a valid path); no
    capture sphere is involved.  The series of depth d of a ray are the faces
    of its first d hits (all of them hits).  Traced from the receivers
    (backward), a series lists the faces from the receiver's end and its key
    from the transmitter reverses them.  With los_always the empty series of
    every source gives the direct paths.

    Returns (keys, certain, possible) as candidates() does: keys = every
    distinct (source, series) times every target, sorted; certain = the series
    was visited by a ray whose first d hits no FP32 tracer can decide
    differently; possible = keys."""
    nsrc = tr.face.shape[0]
    ntgt = nrx if not backward else ntx
    unc = (tr.flags & (SEG_TIE | SEG_EDGE)) != 0
    K1 = tr.flags.shape[-1]
    fu = np.where(unc.any(axis=-1), unc.argmax(axis=-1), K1)
    # interactions each traced branch performed: its segments but the last
    n_int = (tr.tri != -2).sum(axis=-1) - 1
    nb = len(tr.sets)
    nsel = tr.face.shape[1] // nb
    # per row: its branch's transmitting interactions, and the first depth
    # that branch adds (shorter series are those of the branch without its
    # last transmission)
    tset = np.repeat(np.array(tr.sets, dtype=np.int64), nsel)[None, :]
    d0 = np.array([1 + max([j for j in range(32) if (s >> j) & 1] or [-1]) for s in tr.sets])
    d0 = np.repeat(d0, nsel)[None, :]
    series = {}
    for d in range(1, K + 1):
        ok = (n_int >= d) & (d0 <= d)
        src_i, row_i = np.nonzero(ok)
        faces = tr.face[src_i, row_i, :d].astype(np.int64)
        tbits = (tset[0, row_i][:, None] >> np.arange(d)[None, :]) & 1
        faces = np.where(tbits == 1, -2 - faces, faces)
        if backward:
            faces = faces[:, ::-1]
        sure = fu[src_i, row_i] >= d
        for sc, fs, su in zip(src_i.tolist(), faces.tolist(), sure.tolist()):
            k = (sc, d) + tuple(fs)
            series[k] = series.get(k, False) or su
    if los_always:
        for sc in range(nsrc):
            series[(sc, 0)] = True
    rows, cert = [], []
    for k, su in series.items():
        src, d, fs = k[0], k[1], list(k[2:])
        for tg in range(ntgt):
            tx, rx = (tg, src) if backward else (src, tg)
            rows.append([tx, rx, d] + fs + [-1] * (K - d))
            cert.append(su)
    if not rows:
        z = np.zeros((0, 3 + K), np.int32)
        return z, np.zeros(0, bool), z
    keys = np.array(rows, dtype=np.int32)
    order = np.lexsort(keys.T[::-1])
    keys, certain = keys[order], np.array(cert, bool)[order]
    return keys, certain, keys


def _member(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    if len(a) == 0:
        return np.zeros(0, bool)
    if len(b) == 0:
        return np.zeros(len(a), bool)
    sb = {tuple(r) for r in b.tolist()}
    return np.array([tuple(r) in sb for r in a.tolist()], dtype=bool)


@dataclass
class Paths:
    keys: np.ndarray      # i32 [n, 3 + K]
    valid: np.ndarray     # bool [n]
    marginal: np.ndarray  # bool [n]
    length: np.ndarray    # f64 [n]
    tau: np.ndarray       # f64 [n]
    aod: np.ndarray       # f64 [n, 3]
    aoa: np.ndarray       # f64 [n, 3]
    amp: np.ndarray       # c128 [n, nfreq, 3]


def _pattern(pattern) -> Optional[np.ndarray]:
    if pattern is None:
        return None
    w = np.ascontiguousarray(pattern, dtype=np.float64).reshape(-1)
    assert w.shape[0] == PATTERN_TAPS
    return w


def pattern_gain(pattern, u) -> float:
    """Transmit field gain of departure direction u (1 without a pattern)."""
    w = _pattern(pattern)
    return _load().oracle_pattern_gain(_ptr(w), float(u[0]), float(u[1]), float(u[2]))


def pattern_basis(aod: np.ndarray) -> np.ndarray:
    """B_j(phi) of each departure direction, [n, 16]: periodic hats of
    half-width 2 pi / 16 centred on azimuth 2 pi j / 16."""
    phi = np.arctan2(aod[:, 1], aod[:, 0])
    step = 2.0 * np.pi / PATTERN_TAPS
    centres = step * np.arange(PATTERN_TAPS)
    d = np.abs(np.remainder(phi[:, None] - centres[None, :] + np.pi, 2.0 * np.pi) - np.pi)
    return np.maximum(0.0, 1.0 - d / step)


def refine(osc: OracleScene, tx, rx, keys: np.ndarray, K: int, freqs, tx_power_w: float,
           atten_db_per_km: float = 0.0, t_min: float = T_MIN, eps_rel: float = EPS_REFINE,
           nthreads: Optional[int] = None, pattern=None) -> Paths:
    """Image-method refinement and field of each candidate; pattern: the 16
    transmit pattern weights (None: the paper's isotropic antenna)."""
    lib = _load()
    pattern = _pattern(pattern)
    tx = np.ascontiguousarray(tx, dtype=np.float32).reshape(-1, 3)
    rx = np.ascontiguousarray(rx, dtype=np.float32).reshape(-1, 3)
    keys = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, 3 + K)
    freqs = np.ascontiguousarray(freqs, dtype=np.float64).reshape(-1)
    n = keys.shape[0]
    nf = freqs.shape[0]
    valid = np.zeros(n, np.uint8)
    marginal = np.zeros(n, np.uint8)
    length = np.zeros(n)
    tau = np.zeros(n)
    aod = np.zeros((n, 3))
    aoa = np.zeros((n, 3))
    amp = np.zeros((n, nf, 3, 2))
    if n:
        lib.oracle_refine(osc.handle, _ptr(tx), _ptr(rx), _ptr(keys), n, K, _ptr(freqs), nf,
                          float(tx_power_w), float(atten_db_per_km), t_min, eps_rel,
                          nthreads or default_threads(), _ptr(valid), _ptr(marginal),
                          _ptr(length), _ptr(tau), _ptr(aod), _ptr(aoa), _ptr(amp), _ptr(pattern))
    return Paths(keys, valid.astype(bool), marginal.astype(bool), length, tau, aod, aoa,
                 amp[..., 0] + 1j * amp[..., 1])


def refine_grad(osc: OracleScene, tx, rx, keys: np.ndarray, K: int, freqs, tx_power_w: float, n_mat: int,
                atten_db_per_km: float = 0.0, t_min: float = T_MIN, eps_rel: float = EPS_REFINE,
                nthreads: Optional[int] = None, pattern=None) -> np.ndarray:
    """d amp / d eps_c of each material, c128 [n, nfreq, n_mat, 3] (zero for an
    invalid candidate): the same candidates and validity as refine()."""
    lib = _load()
    pattern = _pattern(pattern)
    tx = np.ascontiguousarray(tx, dtype=np.float32).reshape(-1, 3)
    rx = np.ascontiguousarray(rx, dtype=np.float32).reshape(-1, 3)
    keys = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, 3 + K)
    freqs = np.ascontiguousarray(freqs, dtype=np.float64).reshape(-1)
    n, nf = keys.shape[0], freqs.shape[0]
    damp = np.zeros((n, nf, n_mat, 3, 2))
    if n:
        lib.oracle_refine_grad(osc.handle, _ptr(tx), _ptr(rx), _ptr(keys), n, K, _ptr(freqs), nf,
                               float(tx_power_w), float(atten_db_per_km), t_min, eps_rel,
                               nthreads or default_threads(), _ptr(damp), _ptr(pattern))
    return damp[..., 0] + 1j * damp[..., 1]


def power_gradients(paths: Paths, damp: np.ndarray, ntx: int, nrx: int, freqs, tx_power_w: float):
    """Derivatives of the coherent power P = sum_c |A_c|^2, A = sum_p a_p, per
    (freq, tx, rx): dP/d theta = 2 Re sum_c conj(A_c) dA_c/d theta.  With
    eps_c = eps_r - j sigma / (2 pi f eps0): d/d eps_r = d/d eps_c and
    d/d sigma = -j / (2 pi f eps0) d/d eps_c.  P is proportional to the transmit
    power: dP/dP_t = P / P_t.  Returns (d_eps_r, d_sigma) [nfreq, ntx, nrx, n_mat]
    and d_pt [nfreq, ntx, nrx]."""
    freqs = np.asarray(freqs, dtype=np.float64).reshape(-1)
    nf, n_mat = len(freqs), damp.shape[2]
    acc = np.zeros((nf, ntx, nrx, 3), dtype=np.complex128)
    dacc = np.zeros((nf, ntx, nrx, n_mat, 3), dtype=np.complex128)
    for i in range(len(paths.keys)):
        if paths.valid[i]:
            t, r = int(paths.keys[i, 0]), int(paths.keys[i, 1])
            acc[:, t, r] += paths.amp[i]
            dacc[:, t, r] += damp[i]
    g = 2.0 * np.real(np.sum(np.conj(acc)[:, :, :, None, :] * dacc, axis=-1))
    dsig_fac = -1j / (2.0 * np.pi * freqs * EPS0)
    g_sig = 2.0 * np.real(np.sum(np.conj(acc)[:, :, :, None, :] * dacc * dsig_fac[:, None, None, None, None], axis=-1))
    p_coh = np.sum(np.abs(acc) ** 2, axis=-1)
    return g, g_sig, p_coh / tx_power_w


def pattern_gradients(paths: Paths, paths_iso: Paths, ntx: int, nrx: int) -> np.ndarray:
    """dP/dw_j of the coherent power, [nfreq, ntx, nrx, 16].  A path's field is
    a_p = g(phi_p) a_p^iso with g = sum_j w_j B_j, so
    dP/dw_j = 2 Re sum_c conj(A_c) sum_p B_j(phi_p) a_pc^iso.  paths: the
    frame's paths under the pattern; paths_iso: the same candidates refined
    without one."""
    nf = paths.amp.shape[1]
    acc = np.zeros((nf, ntx, nrx, 3), dtype=np.complex128)
    dacc = np.zeros((nf, ntx, nrx, PATTERN_TAPS, 3), dtype=np.complex128)
    basis = pattern_basis(paths.aod)
    for i in range(len(paths.keys)):
        if paths.valid[i]:
            t, r = int(paths.keys[i, 0]), int(paths.keys[i, 1])
            acc[:, t, r] += paths.amp[i]
            dacc[:, t, r] += basis[i][None, :, None] * paths_iso.amp[i][:, None, :]
    return 2.0 * np.real(np.sum(np.conj(acc)[:, :, :, None, :] * dacc, axis=-1))


def received_power(paths: Paths, ntx: int, nrx: int, nfreq: int):
    """Per (freq, tx, rx): coherent P = sum_c |sum_p a_pc|^2 and incoherent sum_p |a_p|^2.

    Paths are summed in key order (keys are sorted)."""
    p_coh = np.zeros((nfreq, ntx, nrx))
    p_inc = np.zeros((nfreq, ntx, nrx))
    for i in range(len(paths.keys)):
        if not paths.valid[i]:
            continue
        t, r = int(paths.keys[i, 0]), int(paths.keys[i, 1])
        p_inc[:, t, r] += np.sum(np.abs(paths.amp[i]) ** 2, axis=-1)
    acc = np.zeros((nfreq, ntx, nrx, 3), dtype=np.complex128)
    for i in range(len(paths.keys)):
        if paths.valid[i]:
            acc[:, int(paths.keys[i, 0]), int(paths.keys[i, 1])] += paths.amp[i]
    p_coh[:] = np.sum(np.abs(acc) ** 2, axis=-1)
    return p_coh, p_inc


@dataclass
class FrameResult:
    trace: TraceResult
    keys: np.ndarray
    certain: np.ndarray
    possible: np.ndarray
    paths: Paths
    p_coh: np.ndarray
    p_inc: np.ndarray


def frame(scene, frame_index: int = 0, dirs: Optional[np.ndarray] = None, K: Optional[int] = None,
          freqs=None, tx_power_w: Optional[float] = None, atten_db_per_km: float = 0.0,
          los_always: bool = True, nthreads: Optional[int] = None, pattern=None,
          backward: bool = False, visited: bool = False,
          max_transmissions: Optional[int] = None) -> FrameResult:
    """One frame, from scratch: the oracle keeps nothing between frames.
    backward: rays cast from the receivers and captured at spheres around the
    transmitters (Sec. III, "Backward ray tracing"); the trace result is then
    per receiver.  visited: candidates by visited-series discovery
    (visited_candidates) instead of capture spheres."""
    K = scene.max_reflections if K is None else K
    T = getattr(scene, "max_transmissions", 0) if max_transmissions is None else max_transmissions
    freqs = scene.freqs_hz if freqs is None else freqs
    tx_power_w = scene.tx_power_w if tx_power_w is None else tx_power_w
    if dirs is None:
        dirs = fibonacci(scene.n_rays)
    xf = scene.transforms(frame_index) if scene.object_vertex_range.shape[0] else None
    osc = OracleScene(scene, xf)
    # receivers of this frame (vehicle-mounted receivers move with their vehicles)
    rx = scene.rx_at(frame_index) if hasattr(scene, "rx_at") else scene.rx
    src, tgt = (rx, scene.tx) if backward else (scene.tx, rx)
    tr = trace(osc, src, tgt, scene.rx_radius, dirs, K, nthreads=nthreads, max_transmissions=T)
    ntx, nrx = scene.tx.shape[0], rx.shape[0]
    slots = K + T   # interactions per path at most: the key's face entries
    if visited:
        keys, certain, possible = visited_candidates(tr, ntx, nrx, slots, los_always, backward)
    else:
        keys, certain, possible = candidates(tr, ntx, nrx, slots, los_always, backward)
    paths = refine(osc, scene.tx, rx, keys, slots, freqs, tx_power_w, atten_db_per_km,
                   nthreads=nthreads, pattern=pattern)
    p_coh, p_inc = received_power(paths, ntx, nrx, len(freqs))
    return FrameResult(tr, keys, certain, possible, paths, p_coh, p_inc)


def enumerate_keys(n_faces: int, ntx: int, nrx: int, K: int, T: int = 0) -> np.ndarray:
    """Every interaction sequence with at most K reflections and T
    transmissions (a transmission through face f written -2 - f) and no face
    met twice in a row, for every (tx, rx); keys [n][3 + K + T]."""
    width = K + T
    seqs = [([], 0, 0)]   # (entries, reflections, transmissions)
    out = []
    for order in range(width + 1):
        for s, _, _ in seqs:
            for t in range(ntx):
                for r in range(nrx):
                    out.append([t, r, order] + s + [-1] * (width - order))
        nxt = []
        for s, nr, nt in seqs:
            last = None if not s else (s[-1] if s[-1] >= 0 else -2 - s[-1])
            for f in range(n_faces):
                if f == last:
                    continue
                if nr < K:
                    nxt.append((s + [f], nr + 1, nt))
                if nt < T:
                    nxt.append((s + [-2 - f], nr, nt + 1))
        seqs = nxt
    return np.array(out, dtype=np.int32).reshape(-1, 3 + width)
