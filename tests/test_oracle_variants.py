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
