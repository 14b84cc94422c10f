"""Oracle pins of the power gradients: the closed-form derivatives along the
frame's fixed paths against central differences of the oracle's own forward
power (the forward code does not share the derivative code), and dP/dP_t
against P / P_t."""
import numpy as np
import pytest

from oracle import oracle
from paper_2112_07115_amd import scenes


@pytest.fixture(scope="module")
def toy():
    oracle.build()
    s = scenes.static_toy()
    # the toy's two materials, plus a constant-gamma one on no face (its
    # derivatives are zero) and a lossy ground far from the defaults
    mats = np.vstack([s.materials, [[3.0, 0.01, 0.8]]])
    s = scenes.Scene(**{**s.__dict__, "materials": mats, "freqs_hz": [28e9, 3.5e9]})
    dirs = scenes.random_sphere_dirs(20000, seed=3)
    fr = oracle.frame(s, dirs=dirs)
    return s, fr


def power_with(s, keys, mats=None, pt=None):
    s2 = scenes.Scene(**{**s.__dict__, "materials": s.materials if mats is None else mats})
    osc = oracle.OracleScene(s2)
    K = s.max_reflections
    p = oracle.refine(osc, s.tx, s.rx, keys, K, s.freqs_hz, s.tx_power_w if pt is None else pt)
    return oracle.received_power(p, s.tx.shape[0], s.rx.shape[0], len(s.freqs_hz))[0]


def gradients(s, fr):
    osc = oracle.OracleScene(s)
    damp = oracle.refine_grad(osc, s.tx, s.rx, fr.keys, s.max_reflections, s.freqs_hz, s.tx_power_w,
                              s.materials.shape[0])
    return oracle.power_gradients(fr.paths, damp, s.tx.shape[0], s.rx.shape[0], s.freqs_hz, s.tx_power_w)


def test_gradients_match_central_differences(toy):
    s, fr = toy
    g_eps, g_sig, _ = gradients(s, fr)
    assert fr.paths.valid.sum() > 10
    scale = np.abs(fr.p_coh).max()
    checked = 0
    for m in range(s.materials.shape[0]):
        for col, g in ((0, g_eps), (1, g_sig)):
            v = s.materials[m, col]
            h = 1e-5 * max(abs(v), 1e-2)
            mp, mm = s.materials.copy(), s.materials.copy()
            mp[m, col] += h
            mm[m, col] -= h
            fd = (power_with(s, fr.keys, mats=mp) - power_with(s, fr.keys, mats=mm)) / (2 * h)
            ref = np.abs(fd).max() + 1e-30
            np.testing.assert_allclose(g[..., m], fd, rtol=1e-5, atol=1e-6 * ref + 1e-12 * scale / max(abs(v), 1e-2))
            if np.abs(fd).max() > 0:
                checked += 1
    assert checked >= 3   # both parameters of the faces' materials move the power


def test_constant_gamma_material_has_no_gradient(toy):
    s, fr = toy
    g_eps, g_sig, _ = gradients(s, fr)
    assert np.all(g_eps[..., 2] == 0) and np.all(g_sig[..., 2] == 0)


def test_transmit_power_derivative(toy):
    s, fr = toy
    _, _, g_pt = gradients(s, fr)
    h = 1e-3
    fd = (power_with(s, fr.keys, pt=s.tx_power_w + h) - power_with(s, fr.keys, pt=s.tx_power_w - h)) / (2 * h)
    np.testing.assert_allclose(g_pt, fd, rtol=1e-7, atol=1e-30)
    np.testing.assert_allclose(g_pt, fr.p_coh / s.tx_power_w, rtol=1e-12)
