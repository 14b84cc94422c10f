"""Structural invariants of a BVH downloaded from the library (plain NumPy).

Checks, for a binary tree with child-box-in-parent layout:
  - n_tris - 1 internal nodes (one for a single triangle), root 0;
  - every internal node except the root and every leaf is referenced exactly
    once; leaf_tri is a permutation of the triangles;
  - each leaf box contains its triangle; each internal child box contains both
    of its own child boxes; with exact=True a child box must equal the union of
    its children (refit boxes are exact min/max) and a leaf box must equal the
    triangle box grown by `pad`.
Returns a list of human-readable violations (empty when the tree is sound).
"""
import numpy as np


def check_bvh(child, box, leaf_tri, vertices, tris, pad=0.0, exact=False):
    bad = []
    nt = tris.shape[0]
    ni = child.shape[0]
    if nt == 0:
        return bad if ni == 0 else ["internal nodes without triangles"]
    want = nt - 1 if nt > 1 else 1
    if ni != want:
        return ["%d internal nodes, expected %d" % (ni, want)]
    if sorted(leaf_tri.tolist()) != list(range(nt)):
        bad.append("leaf_tri is not a permutation of the triangles")
    ref_int = np.zeros(ni, int)
    ref_leaf = np.zeros(nt, int)
    for p in range(ni):
        for s in range(2):
            c = int(child[p, s])
            if c >= 0:
                if c >= ni:
                    bad.append("node %d slot %d: child %d out of range" % (p, s, c))
                    continue
                ref_int[c] += 1
            else:
                li = ~c
                if li >= nt:
                    bad.append("node %d slot %d: leaf %d out of range" % (p, s, li))
                    continue
                ref_leaf[li] += 1
    if nt > 1:
        if ref_int[0] != 0:
            bad.append("root is referenced as a child")
        if np.any(ref_int[1:] != 1):
            bad.append("internal nodes referenced %s times" % sorted(set(ref_int[1:].tolist())))
        if np.any(ref_leaf != 1):
            bad.append("leaves referenced %s times" % sorted(set(ref_leaf.tolist())))
    V = vertices.astype(np.float64)
    lo_slot = box[:, :, 0:3].astype(np.float64)
    hi_slot = box[:, :, 3:6].astype(np.float64)
    if np.any(lo_slot > hi_slot):
        bad.append("inverted child box")
    for p in range(ni):
        for s in range(2):
            c = int(child[p, s])
            lo, hi = lo_slot[p, s], hi_slot[p, s]
            if c >= 0:
                if c >= ni:
                    continue
                clo = np.minimum(lo_slot[c, 0], lo_slot[c, 1])
                chi = np.maximum(hi_slot[c, 0], hi_slot[c, 1])
                if np.any(clo < lo) or np.any(chi > hi):
                    bad.append("node %d slot %d does not contain node %d" % (p, s, c))
                elif exact and (np.any(clo != lo) or np.any(chi != hi)):
                    bad.append("node %d slot %d is not the union of node %d" % (p, s, c))
            else:
                li = ~c
                if li >= nt:
                    continue
                t = int(leaf_tri[li])
                tv = V[tris[t]]
                tlo, thi = tv.min(axis=0), tv.max(axis=0)
                if np.any(tlo < lo) or np.any(thi > hi):
                    bad.append("leaf %d (triangle %d) outside its box" % (li, t))
                elif exact:
                    plo = (tlo.astype(np.float32) - np.float32(pad)).astype(np.float64)
                    phi = (thi.astype(np.float32) + np.float32(pad)).astype(np.float64)
                    if np.any(plo != lo) or np.any(phi != hi):
                        bad.append("leaf %d box is not its triangle box grown by the padding" % li)
        if len(bad) > 20:
            break
    return bad
