"""Pins of the oracle's paper variants (Sec. III): backward tracing from the
receivers and visited-series discovery.

Expected values come from brute force: every face sequence up to the
reflection limit is refined by the image method (the exhaustive enumeration of
the visited-path tables), and with rays dense enough that every path has
several capturing rays, a traced frame must find exactly the valid ones.
"""
import numpy as np
import pytest

from paper_2112_07115_amd import scenes

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _valid_set(keys, valid):
    return {tuple(k) for k, v in zip(np.asarray(keys).tolist(), valid) if v}


def _enumerated(O, sc, K):
    keys = O.enumerate_keys(sc.n_faces, sc.tx.shape[0], sc.rx.shape[0], K)
    osc = O.OracleScene(sc)
    p = O.refine(osc, sc.tx, sc.rx, keys, K, sc.freqs_hz, sc.tx_power_w)
    return _valid_set(keys, p.valid)


def _corner(tx, rx):
    sc = scenes.corner(tx, rx, n_rays=400000, max_reflections=2)
    sc.rx_radius = 0.25
    return sc


@pytest.mark.parametrize("tx,rx", [
    ([[3.0, 5.0, 1.0], [12.0, 7.0, 2.0]], [[8.0, 2.0, 1.5], [5.0, 11.0, 1.2], [9.0, 9.0, 2.5]]),
    ([[6.0, 1.0, 2.0], [2.0, 14.0, 1.0]], [[1.0, 9.0, 1.0], [10.0, 4.0, 3.0], [7.0, 7.0, 1.5]]),
])
def test_backward_frame_finds_every_corner_path(oracle_mod, tx, rx):
    """Rays cast from the receivers and captured at the transmitters find the
    same valid paths (keys from the transmitter, the two-bounce face order
    included) as exhaustive enumeration; so does the forward frame."""
    sc = _corner(tx, rx)
    want = _enumerated(oracle_mod, sc, 2)
    assert len(want) == 24    # per pair: direct, one bounce on each wall, one double bounce
    bwd = oracle_mod.frame(sc, los_always=False, backward=True)
    fwd = oracle_mod.frame(sc, los_always=False)
    assert _valid_set(bwd.keys, bwd.paths.valid) == want
    assert _valid_set(fwd.keys, fwd.paths.valid) == want
    # the backward trace is per receiver: its log has one row block per receiver
    assert bwd.trace.tri.shape[0] == len(rx)


def test_backward_records_name_receiver_then_transmitter(oracle_mod):
    """A ray cast from a receiver straight at a transmitter's sphere is a direct
    path of that (tx, rx) pair: the record names (rx, tx), the key (tx, rx)."""
    sc = scenes.free_space([[0.0, 0.0, 0.0], [0.0, 40.0, 0.0]], [[30.0, 0.0, 0.0]])
    osc = oracle_mod.OracleScene(sc)
    d = np.array([[-1.0, 0.0, 0.0], [-30.0, 40.0, 0.0]], np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tr = oracle_mod.trace(osc, sc.rx, sc.tx, 0.5, d, 1)
    hit = tr.caps[(tr.cap_flags & oracle_mod.CAP_HIT) != 0]
    assert sorted(map(tuple, hit[:, :4].tolist())) == [(0, 0, 0, 0), (1, 0, 1, 0)]
    keys, _, _ = oracle_mod.candidates(tr, 2, 1, 1, los_always=False, backward=True)
    assert keys.tolist() == [[0, 0, 0, -1], [1, 0, 0, -1]]


def test_visited_series_find_every_static_toy_path(oracle_mod):
    """Visited-series discovery with only 1024 rays finds every valid path of
    the exhaustive enumeration (37 up to two reflections), where capture
    spheres of 0.5 m find a third of them."""
    s = scenes.static_toy()
    want = _enumerated(oracle_mod, s, 2)
    assert len(want) == 37
    dirs = oracle_mod.fibonacci(1024)
    vis = oracle_mod.frame(s, dirs=dirs, K=2, visited=True)
    cap = oracle_mod.frame(s, dirs=dirs, K=2)
    got_v = _valid_set(vis.keys, vis.paths.valid)
    got_c = _valid_set(cap.keys, cap.paths.valid)
    assert got_v == want
    assert got_c < got_v and len(got_c) < 20


def test_visited_series_contain_capture_candidates(oracle_mod):
    """A capturing ray visited its candidate's series: with the same rays,
    every capture-discovered key is also a visited-series key."""
    s = scenes.dynamic_urban()
    dirs = scenes.random_sphere_dirs(2048, seed=41)
    vis = oracle_mod.frame(s, dirs=dirs, visited=True)
    cap = oracle_mod.frame(s, dirs=dirs)
    kv = {tuple(k) for k in vis.keys.tolist()}
    kc = {tuple(k) for k in cap.keys.tolist()}
    assert kc <= kv
    assert _valid_set(cap.keys, cap.paths.valid) <= _valid_set(vis.keys, vis.paths.valid)
    # each key is a series of the source's rays tried against every receiver
    assert len(vis.keys) % s.rx.shape[0] == 0


def test_backward_visited_series_find_every_corner_path(oracle_mod):
    """From the receivers, 2000 rays (the paper's shooting-ray count) and
    visited series find every valid corner path, two-bounce orders included."""
    sc = _corner([[3.0, 5.0, 1.0], [12.0, 7.0, 2.0]], [[8.0, 2.0, 1.5], [5.0, 11.0, 1.2], [9.0, 9.0, 2.5]])
    want = _enumerated(oracle_mod, sc, 2)
    dirs = oracle_mod.fibonacci(2000)
    bwd = oracle_mod.frame(sc, dirs=dirs, backward=True, visited=True)
    assert _valid_set(bwd.keys, bwd.paths.valid) == want


def test_backward_visited_series_find_every_static_toy_path(oracle_mod):
    """1024 rays from each receiver: the receivers' visited series, reversed
    into keys from the transmitter, give every enumerated valid path."""
    s = scenes.static_toy()
    want = _enumerated(oracle_mod, s, 2)
    fr = oracle_mod.frame(s, dirs=oracle_mod.fibonacci(1024), K=2, backward=True, visited=True)
    assert _valid_set(fr.keys, fr.paths.valid) == want


# ---------------------------------------------------------- transmission ----
# Table II: indoor wall 10 mm, reflection 0.7, penetration 20 dB; indoor glass
# 5 mm, 0.74, 5 dB (tests/golden/table2_materials.txt).

def _table2():
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "table2_materials.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, th, refl, pen = line.split()
                rows[name] = (float(th), float(refl), float(pen))
    return rows


def _friis_w(pt, f, d):
    """Received power of Eq. (3) in free space (n = 2), in watts, from the dB form."""
    import math
    fspl_db = 20.0 * math.log10(4.0 * math.pi * f / 299792458.0) + 20.0 * math.log10(d)
    return pt * 10.0 ** (-fspl_db / 10.0)


def _power(paths, i):
    return float(np.sum(np.abs(paths.amp[i]) ** 2))


@pytest.mark.parametrize("name", ["wall_indoor", "glass_indoor"])
def test_transmission_through_one_slab(oracle_mod, name):
    """The direct path through one wall of Table II: free-space power of
    Eq. (3) lowered by the material's penetration loss, straight-line length
    and directions; the direct key without the transmission is blocked."""
    import math
    _, refl, pen = _table2()[name]
    tx, rx = [0.0, 0.0, 1.5], [20.0, 3.0, 1.5]
    sc = scenes.slabs([tx], [rx], [(10.0, 0)], [(5.31, 0.48, refl)], [pen], freqs_hz=[30e9],
                      tx_power_w=0.5, max_reflections=1, max_transmissions=1)
    keys = np.array([[0, 0, 1, -2, -1], [0, 0, 0, -1, -1]], np.int32)
    p = oracle_mod.refine(oracle_mod.OracleScene(sc), sc.tx, sc.rx, keys, 2, sc.freqs_hz, sc.tx_power_w)
    d = math.dist(tx, rx)
    assert list(p.valid) == [True, False]
    assert abs(p.length[0] - d) < 1e-12 * d
    want = _friis_w(0.5, 30e9, d) * 10.0 ** (-pen / 10.0)
    assert abs(_power(p, 0) - want) < 1e-9 * want
    u = np.subtract(rx, tx) / d
    assert np.allclose(p.aod[0], u, atol=1e-12) and np.allclose(p.aoa[0], -u, atol=1e-12)


def test_losses_of_two_slabs_add_and_reflections_keep_table2_gamma(oracle_mod):
    """Glass then wall: 5 + 20 dB.  The reflection off the penetrable wall has
    Table II's coefficient 0.7 (power factor 0.49), at the image-source
    distance."""
    import math
    t2 = _table2()
    tx, rx, rx2 = [0.0, 0.0, 1.5], [20.0, 3.0, 1.5], [4.0, 6.0, 1.0]
    mats = [(6.27, 0.0, t2["glass_indoor"][1]), (5.31, 0.48, t2["wall_indoor"][1])]
    sc = scenes.slabs([tx], [rx, rx2], [(8.0, 0), (14.0, 1)], mats,
                      [t2["glass_indoor"][2], t2["wall_indoor"][2]], freqs_hz=[30e9], tx_power_w=0.5,
                      max_reflections=1, max_transmissions=2)
    keys = np.array([[0, 0, 2, -2, -3, -1], [0, 1, 1, 0, -1, -1]], np.int32)
    p = oracle_mod.refine(oracle_mod.OracleScene(sc), sc.tx, sc.rx, keys, 3, sc.freqs_hz, sc.tx_power_w)
    assert p.valid.all()
    d = math.dist(tx, rx)
    want = _friis_w(0.5, 30e9, d) * 10.0 ** (-25.0 / 10.0)
    assert abs(_power(p, 0) - want) < 1e-9 * want
    img = [16.0, 0.0, 1.5]   # the transmitter mirrored in x = 8
    d2 = math.dist(img, rx2)
    want2 = _friis_w(0.5, 30e9, d2) * t2["glass_indoor"][1] ** 2
    assert abs(p.length[1] - d2) < 1e-12 * d2
    assert abs(_power(p, 1) - want2) < 1e-9 * want2


def _slab_room():
    t2 = _table2()
    mats = [(5.31, 0.48, t2["wall_indoor"][1]), (6.27, 0.0, t2["glass_indoor"][1]), (5.31, 0.48, 0.8)]
    inf = float("inf")
    # two penetrable slabs between the transmitter and receivers on both
    # sides, and an opaque back wall
    return scenes.slabs([[0.0, 0.0, 1.5]], [[12.0, 2.0, 1.2], [-3.0, 4.0, 2.0], [5.0, -3.0, 1.0]],
                        [(4.0, 0), (8.0, 1), (-6.0, 2)], mats,
                        [t2["wall_indoor"][2], t2["glass_indoor"][2], inf], half=40.0,
                        freqs_hz=[30e9], tx_power_w=0.5, max_reflections=2, max_transmissions=2)


@pytest.mark.parametrize("T", [1, 2])
def test_transmission_paths_match_enumeration(oracle_mod, T):
    """Every interaction sequence of up to two reflections and T
    transmissions, refined by the image method, against frames traced with
    ray branches: visited series (forward and backward) find exactly the valid
    ones, and dense capture spheres only valid ones."""
    sc = _slab_room()
    sc.max_transmissions = T
    keys = oracle_mod.enumerate_keys(sc.n_faces, 1, 3, 2, T)
    p = oracle_mod.refine(oracle_mod.OracleScene(sc), sc.tx, sc.rx, keys, 2 + T, sc.freqs_hz, sc.tx_power_w)
    want = _valid_set(keys, p.valid)
    n_trans = sum(1 for k in want if any(x <= -2 for x in k[3:]))
    assert n_trans >= 6
    dirs = oracle_mod.fibonacci(4096)
    for bw in (False, True):
        fr = oracle_mod.frame(sc, dirs=dirs, visited=True, backward=bw)
        assert _valid_set(fr.keys, fr.paths.valid) == want
    sc.rx_radius = 0.3
    fc = oracle_mod.frame(sc, dirs=oracle_mod.fibonacci(200_000))
    got = _valid_set(fc.keys, fc.paths.valid)
    assert got <= want and len(got) >= len(want) - 2


def test_branch_log_layout(oracle_mod):
    """Each ray is traced once per branch (sets of at most T of the first K + T
    interactions); a branch transmits exactly at its set's interactions."""
    sc = _slab_room()
    tr = oracle_mod.trace(oracle_mod.OracleScene(sc), sc.tx, sc.rx, 0.3, np.array([[1.0, 0.0, 0.0]], np.float32),
                          2, max_transmissions=2)
    sets = oracle_mod.branch_sets(4, 2)
    assert len(sets) == 1 + 4 + 6 and tr.tri.shape == (1, 11, 5)
    # straight along +x: wall x = 4, glass x = 8 ahead, the back wall behind
    faces = tr.face[0, :, :]
    b_tt = sets.index(0b11)            # transmit at interactions 0 and 1: through both slabs, then nothing
    assert list(faces[b_tt, :3]) == [0, 1, -1]
    b_rt = sets.index(0b10)            # reflect at the wall, then through nothing: the back wall ends it
    assert list(faces[b_rt, :2]) == [0, 2] and tr.tri[0, b_rt, 2] == -2


def test_no_transmission_through_opaque_faces(oracle_mod):
    """A key that transmits through an opaque face is never valid."""
    sc = _slab_room()
    keys = np.array([[0, 1, 1, -4, -1, -1, -1], [0, 1, 0, -1, -1, -1, -1]], np.int32)   # through the back wall
    sc2 = scenes.Scene(**{**sc.__dict__, "rx": np.array([[-9.0, 0.0, 1.5], [-9.0, 0.0, 1.5]], np.float32)})
    p = oracle_mod.refine(oracle_mod.OracleScene(sc2), sc2.tx, sc2.rx, keys, 4, sc2.freqs_hz, sc2.tx_power_w)
    assert not p.valid.any()
