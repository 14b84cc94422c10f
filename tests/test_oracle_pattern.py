"""Oracle pins of the transmit pattern (the field gain g = sum_j w_j B_j of the
departure azimuth, 16 periodic hats) and of dP/dw along the frame's paths:
the hats' shape against linear interpolation between the taps, the
isotropic weights against no pattern, a constant pattern against the closed
form c^2 P, and the derivatives against central differences of the forward
power (the forward code does not share the derivative code)."""
import numpy as np
import pytest

from oracle import oracle
from paper_2112_07115_amd import scenes

TAPS = oracle.PATTERN_TAPS


@pytest.fixture(scope="module")
def toy():
    oracle.build()
    s = scenes.static_toy()
    s = scenes.Scene(**{**s.__dict__, "freqs_hz": [28e9, 3.5e9]})
    dirs = scenes.random_sphere_dirs(20000, seed=3)
    fr = oracle.frame(s, dirs=dirs)
    return s, fr


def refine(s, keys, pattern=None, mats=None):
    s2 = s if mats is None else scenes.Scene(**{**s.__dict__, "materials": mats})
    return oracle.refine(oracle.OracleScene(s2), s.tx, s.rx, keys, s.max_reflections, s.freqs_hz,
                         s.tx_power_w, pattern=pattern)


def power(s, keys, pattern=None, mats=None):
    p = refine(s, keys, pattern, mats)
    return oracle.received_power(p, s.tx.shape[0], s.rx.shape[0], len(s.freqs_hz))[0]


def test_gain_is_periodic_linear_interpolation_of_the_weights():
    rng = np.random.default_rng(5)
    w = rng.uniform(-1.0, 2.0, TAPS)
    knots = 2.0 * np.pi * np.arange(TAPS + 1) / TAPS
    for phi in np.concatenate([rng.uniform(-np.pi, np.pi, 200), knots[:-1] - np.pi, [np.pi, -np.pi]]):
        u = (np.cos(phi) * 0.6, np.sin(phi) * 0.6, 0.8)
        ref = np.interp(np.mod(phi, 2.0 * np.pi), knots, np.append(w, w[0]))
        assert oracle.pattern_gain(w, u) == pytest.approx(ref, rel=1e-12, abs=1e-12)
        b = oracle.pattern_basis(np.array([u]))[0]
        assert b.sum() == pytest.approx(1.0, rel=1e-12)
        assert np.dot(b, w) == pytest.approx(ref, rel=1e-12, abs=1e-12)
    # tap 0 points along +x, tap 4 along +y
    e4 = np.eye(TAPS)[4]
    assert oracle.pattern_gain(e4, (0.0, 1.0, 0.0)) == pytest.approx(1.0)
    assert oracle.pattern_gain(e4, (1.0, 0.0, 0.0)) == 0.0
    assert oracle.pattern_gain(None, (0.3, 0.4, 0.5)) == 1.0


def test_isotropic_weights_equal_no_pattern(toy):
    s, fr = toy
    p = power(s, fr.keys, pattern=np.ones(TAPS))
    np.testing.assert_allclose(p, fr.p_coh, rtol=1e-12, atol=0)


def test_constant_pattern_scales_power_by_its_square(toy):
    s, fr = toy
    p = power(s, fr.keys, pattern=np.full(TAPS, 0.3))
    np.testing.assert_allclose(p, 0.09 * fr.p_coh, rtol=1e-12, atol=0)


def test_single_tap_keeps_only_its_sector(toy):
    s, fr = toy
    j = 3
    paths = refine(s, fr.keys, pattern=np.eye(TAPS)[j])
    phi = np.arctan2(fr.paths.aod[:, 1], fr.paths.aod[:, 0])
    d = np.abs(np.angle(np.exp(1j * (phi - 2.0 * np.pi * j / TAPS))))
    hat = np.maximum(0.0, 1.0 - d / (2.0 * np.pi / TAPS))
    v = fr.paths.valid
    assert v.sum() > 10
    np.testing.assert_allclose(paths.amp[v], hat[v, None, None] * fr.paths.amp[v], rtol=1e-12, atol=1e-300)


def test_pattern_gradients_match_central_differences(toy):
    s, fr = toy
    rng = np.random.default_rng(9)
    w = rng.uniform(0.5, 1.5, TAPS)
    paths = refine(s, fr.keys, pattern=w)
    g = oracle.pattern_gradients(paths, fr.paths, s.tx.shape[0], s.rx.shape[0])
    scale = np.abs(fr.p_coh).max()
    moved = 0
    for j in range(TAPS):
        h = 1e-5
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd = (power(s, fr.keys, wp) - power(s, fr.keys, wm)) / (2 * h)
        np.testing.assert_allclose(g[..., j], fd, rtol=1e-5, atol=1e-7 * scale)
        moved += np.abs(fd).max() > 1e-6 * scale
    assert moved >= 4
    # the gain is linear in w: P is a quadratic form, so sum_j w_j dP/dw_j = 2 P
    p = oracle.received_power(paths, s.tx.shape[0], s.rx.shape[0], len(s.freqs_hz))[0]
    np.testing.assert_allclose(np.tensordot(g, w, axes=([3], [0])), 2.0 * p, rtol=1e-9, atol=1e-12 * scale)


def test_material_gradients_under_a_pattern(toy):
    s, fr = toy
    w = np.linspace(0.4, 1.6, TAPS)
    paths = refine(s, fr.keys, pattern=w)
    damp = oracle.refine_grad(oracle.OracleScene(s), s.tx, s.rx, fr.keys, s.max_reflections, s.freqs_hz,
                              s.tx_power_w, s.materials.shape[0], pattern=w)
    g_eps, _, _ = oracle.power_gradients(paths, damp, s.tx.shape[0], s.rx.shape[0], s.freqs_hz, s.tx_power_w)
    m, h = 0, 1e-5 * s.materials[0, 0]
    mp, mm = s.materials.copy(), s.materials.copy()
    mp[m, 0] += h
    mm[m, 0] -= h
    fd = (power(s, fr.keys, w, mp) - power(s, fr.keys, w, mm)) / (2 * h)
    assert np.abs(fd).max() > 0
    np.testing.assert_allclose(g_eps[..., m], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
