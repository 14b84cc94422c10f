"""Helpers of the GPU parity tests: trace a frame through the C ABI and compare
everything the oracle computes for it (per-ray hits and lengths, captures,
candidate keys, refined paths, coherent and incoherent received power)."""
from __future__ import annotations

import sys

import numpy as np

from paper_2112_07115_amd import dcem
from tests import parity

# share of receivers whose path sets must be certain on both sides (the rest
# sit within the FP32 uncertainty of a capture or a hit): at most 5% of them,
# or one receiver, may be excluded
MAX_EXCLUDED = 0.05


def assert_comparable(st):
    excluded = st["pairs"] - st["comparable_pairs"]
    assert excluded <= max(1, int(MAX_EXCLUDED * st["pairs"])), \
        "%d of %d receivers not comparable" % (excluded, st["pairs"])


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def radius_of(scene):
    pts = np.concatenate([scene.vertices, scene.tx, scene.rx]).astype(np.float64)
    return float(np.linalg.norm(pts, axis=1).max())


def compare_frame(ctx, scene, ofr, out, n_rays, check_log=True, check_captures=True, check_paths=True,
                  visited=False):
    """Compare the context's last frame with the oracle's FrameResult `ofr`
    (traced over the same n_rays directions).  visited: the frame's candidates
    came from visited-series discovery (no capture records; keys compared by
    parity.compare_visited).  Returns a dict of statistics."""
    st = {}
    # rays are traced once per transmission branch: the logs' rows and the
    # ray ids run over branch * n_rays + ray
    n_rays = n_rays * getattr(ctx, "n_branch", 1)
    if check_log:
        g_tri, g_t, g_len = ctx.trace_log()
        st = parity.compare_trace(g_tri, g_t, g_len, ofr.trace, scene.tri_face, radius=radius_of(scene))
        log("  trace", st)
    if check_captures and not visited:
        g_caps = ctx.captures()
        g_caps = g_caps[g_caps[:, 0] >= 0]
        cs = parity.compare_captures(g_caps, ofr.trace, np.arange(n_rays), n_rays)
        log("  captures", cs)
    if check_paths:
        gp = ctx.paths()
        if visited:
            comparable, n_common = parity.compare_visited(gp, ofr, n_rays)
        else:
            comparable, n_common = parity.compare_paths(gp, ofr, n_rays)
        worst = parity.compare_power(out.p_coh, ofr.p_coh, comparable)
        worst_inc = parity.compare_power(out.p_inc, ofr.p_inc, comparable)
        log("  paths: gpu %d oracle %d common %d valid %d; comparable rx %d/%d; worst %.2e dB (P_inc %.2e dB)" %
            (len(gp["keys"]), len(ofr.keys), n_common, int(ofr.paths.valid.sum()), comparable.sum(),
             comparable.size, worst, worst_inc))
        st["comparable"] = float(comparable.mean())
        st["comparable_pairs"] = int(comparable.sum())
        st["pairs"] = int(comparable.size)
        st["valid_paths"] = int(ofr.paths.valid.sum())
    return st


def run_pair(ctx, O, scene, frame=0, dirs=None, K=None, n_rays=None, check_captures=True, check_paths=True,
             los_always=True, atten_db_per_km=0.0, upload=True, backward=False, visited=False):
    """Trace one FULL frame on both sides and compare everything; returns
    (stats, GPU output, oracle FrameResult).  backward: rays cast from the
    receivers on both sides (trace logs and captures are then per receiver)."""
    K = scene.max_reflections if K is None else K
    log("case", scene.name, "frame", frame, "K", K, "rays", n_rays if dirs is None else len(dirs),
        "atten", atten_db_per_km, "backward" if backward else "forward", "visited" if visited else "capture")
    if upload:
        ctx.scene_upload(scene)
    out = dcem.trace_scene_frame(ctx, scene, frame=frame, ray_dirs=dirs, n_rays=n_rays, K=K,
                                 record_trace_log=True, los_always=los_always, atten_db_per_km=atten_db_per_km,
                                 trace_from_rx=backward, discovery=dcem.DISCOVER_VISITED if visited else 0)
    if dirs is None:
        g_dirs = ctx.ray_dirs()
        o_dirs = O.fibonacci(n_rays or scene.n_rays)
        assert np.array_equal(g_dirs, o_dirs), "Fibonacci directions differ"
    else:
        o_dirs = dirs
    ofr = O.frame(scene, frame_index=frame, dirs=o_dirs, K=K, los_always=los_always,
                  atten_db_per_km=atten_db_per_km, backward=backward, visited=visited)
    st = compare_frame(ctx, scene, ofr, out, o_dirs.shape[0], check_captures=check_captures,
                       check_paths=check_paths, visited=visited)
    return st, out, ofr


def check_full_size_sampled(ctx, O, s, frame, stride=16, min_keys=10):
    """The context's last frame of scene `s` (its Fibonacci rays) against the
    oracle on every `stride`-th ray of every transmitter: per-ray hits, lengths and captures, then
    every key the sampled rays' certain captures give, refined by the oracle
    and compared with the GPU's path (validity, length, delay, directions,
    field).  The GPU's powers are the coherent and incoherent sums of its own
    valid paths in key order."""
    g_tri, g_t, g_len = ctx.trace_log()
    g_dirs = ctx.ray_dirs()
    o_dirs = O.fibonacci(s.n_rays)
    assert np.array_equal(g_dirs, o_dirs)
    ids = np.arange(0, s.n_rays, stride, dtype=np.int64)
    osc = O.OracleScene(s, s.transforms(frame))
    otr = O.trace(osc, s.tx, s.rx, s.rx_radius, o_dirs, s.max_reflections, ray_ids=ids)
    st = parity.compare_trace(g_tri[:, ids], g_t[:, ids], g_len[:, ids], otr, s.tri_face, radius=radius_of(s))
    log("  sampled trace", st)
    g_caps = ctx.captures()
    sel = (g_caps[:, 0] >= 0) & np.isin(g_caps[:, 0] % s.n_rays, ids)
    pos = {int(r): i for i, r in enumerate(ids)}
    parity.compare_captures(g_caps[sel], otr, pos, s.n_rays)
    # oracle-derived keys: certain captures of the sampled rays, refined by the oracle
    hit = otr.caps[otr.cap_flags == parity.CAP_HIT][:, 1:]
    keys = np.unique(np.concatenate([hit, O.los_keys(s.tx.shape[0], s.rx.shape[0], s.max_reflections)]), axis=0)
    gp = ctx.paths()
    gk = {tuple(int(x) for x in k): i for i, k in enumerate(gp["keys"])}
    op = O.refine(osc, s.tx, s.rx, keys, s.max_reflections, s.freqs_hz, s.tx_power_w)
    checked = 0
    for j, k in enumerate(keys):
        i = gk.get(tuple(int(x) for x in k))
        assert i is not None, "oracle key %s not found on the GPU" % (k,)
        if op.marginal[j]:
            continue
        bad = parity.compare_path_attrs(gp, i, op, j)
        assert not bad, (k, bad)
        checked += int(op.valid[j])
    log("  oracle-derived valid paths checked", checked, "of", len(keys), "keys")
    assert len(keys) >= min_keys and checked >= min_keys
    # powers: sums of the GPU's own valid paths in key order
    pc, pi = ctx.received_power()
    nf, ntx = len(s.freqs_hz), s.tx.shape[0]
    acc = np.zeros((nf, ntx, s.rx.shape[0], 3), complex)
    inc = np.zeros((nf, ntx, s.rx.shape[0]))
    for i, k in enumerate(gp["keys"]):
        if gp["valid"][i]:
            acc[:, k[0], k[1]] += gp["amp"][i]
            inc[:, k[0], k[1]] += np.sum(np.abs(gp["amp"][i]) ** 2, axis=-1)
    np.testing.assert_allclose(pc, np.sum(np.abs(acc) ** 2, axis=-1), rtol=1e-9, atol=0)
    np.testing.assert_allclose(pi, inc, rtol=1e-9, atol=0)
