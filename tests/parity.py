"""Comparison of the GPU library's outputs with the CPU oracle.

The oracle marks, per ray segment, the decisions an FP32 tracer may take
differently (hits within eps of a face silhouette, near misses before the hit,
ties within 1e-6 relative, hits near t_min, capture distances within eps of the
radius).  Everything else must agree exactly:
  - hit triangle ids and reflection orders bit-exact on every segment before
    the first uncertain one (only the face is compared where the oracle marks
    the triangle id alone as uncertain);
  - hit distances and cumulative lengths within the FP32 tolerance;
  - per-ray captures: every certain oracle capture is found, nothing outside
    the oracle's possible set before an uncertain segment;
  - candidate keys: every certain key found; every extra key traced back to a
    ray whose path is uncertain;
  - refined paths (FP64 on both sides): validity, length within 1e-9
    relative, field amplitude within 1e-6 relative;
  - received power within 0.01 dB for every receiver none of whose keys is
    marginal, or uncertain and valid on a side that has it (its power is the
    same sum of the same valid paths on both sides).
"""
from __future__ import annotations

import numpy as np

SEG_TIE, SEG_EDGE, SEG_TRI = 1, 2, 4
CAP_HIT, CAP_MARGINAL, CAP_UNCERTAIN = 1, 2, 4


def first_uncertain(flags: np.ndarray) -> np.ndarray:
    """Index of the first segment with SEG_TIE/SEG_EDGE (K+1 if none); flags [..., K+1]."""
    unc = (flags & (SEG_TIE | SEG_EDGE)) != 0
    K1 = flags.shape[-1]
    idx = np.where(unc.any(axis=-1), unc.argmax(axis=-1), K1)
    return idx


def compare_trace(g_tri, g_t, g_len, o, tri_face, eps_rel=4e-6, radius=1.0):
    """g_*: GPU log rows for the same rays as the oracle TraceResult `o` ([ntx, n, K+1]).

    Returns a dict of counts; raises AssertionError listing the first mismatches."""
    K1 = o.tri.shape[-1]
    fu = first_uncertain(o.flags)
    ks = np.arange(K1)
    check = ks[None, None, :] < fu[..., None]
    o_tri, g_tri = o.tri, g_tri
    same_tri = o_tri == g_tri
    tri_only = (o.flags & SEG_TRI) != 0
    tf = np.concatenate([np.asarray(tri_face, np.int64), [-3]])   # index -> face, sentinel for empty scenes
    o_face = np.where(o_tri >= 0, tf[np.clip(o_tri, 0, len(tf) - 1)], o_tri)
    g_face = np.where(g_tri >= 0, tf[np.clip(g_tri, 0, len(tf) - 1)], g_tri)
    ok = np.where(tri_only, o_face == g_face, same_tri)
    bad = check & ~ok
    msgs = []
    if bad.any():
        for (t, r, k) in np.argwhere(bad)[:10]:
            msgs.append("tx %d ray %d bounce %d: oracle tri %d (flags %d) gpu tri %d" %
                        (t, r, k, o_tri[t, r, k], o.flags[t, r, k], g_tri[t, r, k]))
    hit = check & (o_tri >= 0) & ok
    # FP32 distances against FP64: positions agree to eps_rel * (k+1) * (R + L)
    # (misses carry infinities on both sides: compared only where the oracle hit,
    # and a NaN on the GPU side fails the check)
    o_t = np.where(hit, o.t, 0.0)
    o_l = np.where(hit, o.length, 0.0)
    tol = eps_rel * (ks[None, None, :] + 1) * (radius + o_l)
    dt = np.abs(np.where(hit, g_t.astype(np.float64), 0.0) - o_t)
    dl = np.abs(np.where(hit, g_len.astype(np.float64), 0.0) - o_l)
    bad_t = hit & ~((dt <= tol) & (dl <= tol))
    if bad_t.any():
        for (t, r, k) in np.argwhere(bad_t)[:10]:
            msgs.append("tx %d ray %d bounce %d: t %.9g vs %.9g, len %.9g vs %.9g" %
                        (t, r, k, g_t[t, r, k], o.t[t, r, k], g_len[t, r, k], o.length[t, r, k]))
    rel_len = np.where(hit, dl / np.maximum(o_l, 1e-30), 0.0)
    stats = {
        "rays": int(np.prod(fu.shape)),
        "rays_fully_certain": int((fu == K1).sum()),
        "segments_checked": int(check.sum()),
        "segments_hit_checked": int(hit.sum()),
        "tri_only": int((check & tri_only).sum()),
        "max_rel_len_err": float(rel_len.max()) if hit.any() else 0.0,
        "max_abs_t_err": float(np.where(hit, dt, 0).max()) if hit.any() else 0.0,
    }
    assert not msgs, "\n".join(msgs)
    return stats


def _cap_tuples(rows, ray_col, n_rays_total=None):
    return {tuple(int(x) for x in r) for r in rows}


def compare_captures(g_rows, o, ray_index, n_rays):
    """g_rows: GPU captures (ray=work, tx, rx, order, faces...) restricted to the
    compared rays; o: oracle TraceResult over those rays (caps' ray column holds the
    ray index); ray_index: mapping oracle ray id -> row position in o's arrays."""
    fu = first_uncertain(o.flags)
    K = o.tri.shape[-1] - 1
    # normalise GPU rows to (tx, ray, rx, order, faces...)
    g = set()
    for r in g_rows:
        work, tx = int(r[0]), int(r[1])
        ray = work - tx * n_rays
        g.add((tx, ray, int(r[2]), int(r[3])) + tuple(int(x) for x in r[4:4 + K]))
    certain, possible, late = set(), set(), set()
    for row, fl in zip(o.caps, o.cap_flags):
        ray, tx, rx, order = int(row[0]), int(row[1]), int(row[2]), int(row[3])
        key = (tx, ray, rx, order) + tuple(int(x) for x in row[4:4 + K])
        possible.add(key)
        if fl == CAP_HIT:
            certain.add(key)
    missing = certain - g
    extra = set()
    for key in g - possible:
        tx, ray, order = key[0], key[1], key[3]
        if order < fu[tx, ray_index[ray]]:
            extra.add(key)
    assert not missing, "certain oracle captures not found on the GPU: %s" % sorted(missing)[:10]
    assert not extra, "GPU captures outside the oracle's possible set: %s" % sorted(extra)[:10]
    return {"gpu_captures": len(g), "oracle_certain": len(certain), "oracle_possible": len(possible)}


C0 = 299792458.0


def compare_path_attrs(gp: dict, i: int, op, j: int, eps_len=1e-9, eps_amp=1e-6, eps_dir=1e-9):
    """Attributes of GPU path i against oracle path j (both FP64): validity,
    length and delay within eps_len relative, departure and arrival unit
    vectors within eps_dir, field within eps_amp relative.  Returns a list of
    mismatch descriptions (NaN never passes)."""
    bad = []
    if bool(gp["valid"][i]) != bool(op.valid[j]):
        return [("valid", bool(gp["valid"][i]), bool(op.valid[j]))]
    if not op.valid[j]:
        return bad
    lo = op.length[j]
    if not abs(gp["length"][i] - lo) <= eps_len * lo:
        bad.append(("length", gp["length"][i], lo))
    if not abs(gp["tau"][i] - op.tau[j]) <= eps_len * op.tau[j]:
        bad.append(("tau", gp["tau"][i], op.tau[j]))
    if not abs(op.tau[j] - lo / C0) <= 1e-12 * op.tau[j]:
        bad.append(("oracle tau", op.tau[j], lo / C0))
    for name in ("aod", "aoa"):
        g, o = np.asarray(gp[name][i]), np.asarray(getattr(op, name)[j])
        if not np.linalg.norm(g - o) <= eps_dir:
            bad.append((name, g.tolist(), o.tolist()))
    ao = op.amp[j]
    if not np.linalg.norm(gp["amp"][i] - ao) <= eps_amp * np.linalg.norm(ao) + 1e-300:
        bad.append(("amp", gp["amp"][i].tolist(), ao.tolist()))
    return bad


def compare_paths(gp: dict, ofr, n_rays: int, eps_len=1e-9, eps_amp=1e-6, tol_db=0.01,
                  min_comparable=0.9):
    """Candidate keys, refined paths and per-receiver power of one frame."""
    K = ofr.keys.shape[1] - 3
    gk = {tuple(int(x) for x in k): i for i, k in enumerate(gp["keys"])}
    ok_ = {tuple(int(x) for x in k): i for i, k in enumerate(ofr.keys)}
    cert = {k for k, i in ok_.items() if ofr.certain[i]}
    poss = {tuple(int(x) for x in k) for k in ofr.possible}
    missing = cert - set(gk)
    assert not missing, "certain keys missing on the GPU: %s" % sorted(missing)[:10]
    fu = first_uncertain(ofr.trace.flags)
    unexplained = []
    for k, i in gk.items():
        if k in poss:
            continue
        fr = int(gp["first_ray"][i])
        if fr < 0:
            unexplained.append(k)
            continue
        tx, ray = fr // n_rays, fr % n_rays
        if k[2] < fu[tx, ray]:
            unexplained.append(k)
    assert not unexplained, "GPU keys the oracle cannot explain: %s" % unexplained[:10]
    # path attributes for common keys
    n_common = 0
    bad = []
    for k, i in gk.items():
        j = ok_.get(k)
        if j is None:
            continue
        n_common += 1
        if ofr.paths.marginal[j]:
            continue
        for b in compare_path_attrs(gp, i, ofr.paths, j, eps_len=eps_len, eps_amp=eps_amp):
            bad.append((k,) + b)
    assert not bad, "path mismatches: %s" % bad[:5]
    # per-receiver power: a receiver's power is the sum over its valid paths,
    # so it is comparable unless one of its keys is marginal, or uncertain
    # (either side may or may not have it) and valid on a side that has it
    ntx, nrx = ofr.p_coh.shape[1], ofr.p_coh.shape[2]
    comparable = np.ones((ntx, nrx), bool)
    for k, i in ok_.items():
        if ofr.paths.marginal[i] or (not ofr.certain[i] and ofr.paths.valid[i]):
            comparable[k[0], k[1]] = False
    for k, i in gk.items():
        if k not in cert and gp["valid"][i]:
            comparable[k[0], k[1]] = False
    return comparable, n_common


def compare_power(g_pc, o_pc, comparable, tol_db=0.01):
    """Largest |10 log10(g / o)| over the comparable receivers (every
    frequency); fails above tol_db, and on a NaN."""
    both0 = (g_pc == 0) & (o_pc == 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        db = np.abs(10 * np.log10(g_pc / o_pc))
    db = np.where(both0, 0.0, db)
    sel = np.broadcast_to(comparable, db.shape)
    worst = float(np.max(db[sel])) if sel.any() else 0.0
    assert worst <= tol_db, "power differs by %.4g dB on a comparable receiver" % worst
    assert not np.isnan(g_pc).any(), "NaN power on the GPU"
    return worst


def compare_visited(gp: dict, ofr, n_rays: int, eps_len=1e-9, eps_amp=1e-6):
    """Candidates of visited-series discovery against the oracle's.

    The oracle refines every (series, target) pair; the GPU keeps those whose
    image-method points lie inside their segments and faces, then validates
    them.  Checked: every GPU key is one of the oracle's or comes from a ray
    whose first `order` hits the oracle marks uncertain; every certain, valid,
    non-marginal oracle path is on the GPU; keys on both sides agree on
    validity and attributes (marginal ones excepted).  Returns the (tx, rx)
    pairs whose power is comparable: a pair is excluded when one of its keys is
    marginal, or uncertain and valid on either side."""
    gk = {tuple(int(x) for x in k): i for i, k in enumerate(gp["keys"])}
    ok_ = {tuple(int(x) for x in k): i for i, k in enumerate(ofr.keys)}
    fu = first_uncertain(ofr.trace.flags)
    unexplained = []
    for k, i in gk.items():
        if k in ok_:
            continue
        fr = int(gp["first_ray"][i])
        if fr < 0 or k[2] < fu[fr // n_rays, fr % n_rays]:
            unexplained.append(k)
    assert not unexplained, "GPU keys the oracle cannot explain: %s" % unexplained[:10]
    missing = [k for k, j in ok_.items()
               if ofr.certain[j] and ofr.paths.valid[j] and not ofr.paths.marginal[j] and k not in gk]
    assert not missing, "certain valid oracle paths missing on the GPU: %s" % sorted(missing)[:10]
    bad = []
    n_common = 0
    for k, i in gk.items():
        j = ok_.get(k)
        if j is None or ofr.paths.marginal[j]:
            continue
        n_common += 1
        for b in compare_path_attrs(gp, i, ofr.paths, j, eps_len=eps_len, eps_amp=eps_amp):
            bad.append((k,) + b)
    assert not bad, "path mismatches: %s" % bad[:5]
    ntx, nrx = ofr.p_coh.shape[1], ofr.p_coh.shape[2]
    comparable = np.ones((ntx, nrx), bool)
    for k, j in ok_.items():
        if ofr.paths.marginal[j]:
            comparable[k[0], k[1]] = False
        elif not ofr.certain[j]:
            i = gk.get(k)
            if ofr.paths.valid[j] or (i is not None and gp["valid"][i]):
                comparable[k[0], k[1]] = False
    for k, i in gk.items():
        if k not in ok_ and gp["valid"][i]:
            comparable[k[0], k[1]] = False
    return comparable, n_common
