"""Host logic of the material calibration (the dB loss, its derivatives and
the Adam loop), driven by the oracle's forward power and gradients on the
toy scene: the loop must recover hidden materials from noise-free powers, and
the loss derivative must match central differences of the loss."""
import numpy as np
import pytest

from oracle import oracle
from paper_2112_07115_amd import calibrate, scenes


@pytest.fixture(scope="module")
def setup():
    oracle.build()
    s = scenes.static_toy()
    s = scenes.Scene(**{**s.__dict__, "freqs_hz": [28e9, 3.5e9]})
    hidden = s.materials.copy()
    hidden[0, :2] = (7.0, 1.0)
    hidden[1, :2] = (10.0, 0.5)
    dirs = scenes.random_sphere_dirs(20000, seed=3)
    fr = oracle.frame(scenes.Scene(**{**s.__dict__, "materials": hidden}), dirs=dirs)
    meas = 10.0 * np.log10(np.where(fr.p_coh > 0, fr.p_coh, np.nan))
    ntx, nrx = s.tx.shape[0], s.rx.shape[0]

    def evaluate(m):
        osc = oracle.OracleScene(scenes.Scene(**{**s.__dict__, "materials": m}))
        p = oracle.refine(osc, s.tx, s.rx, fr.keys, s.max_reflections, s.freqs_hz, s.tx_power_w)
        pc = oracle.received_power(p, ntx, nrx, len(s.freqs_hz))[0]
        damp = oracle.refine_grad(osc, s.tx, s.rx, fr.keys, s.max_reflections, s.freqs_hz, s.tx_power_w,
                                  m.shape[0])
        ge, gs, _ = oracle.power_gradients(p, damp, ntx, nrx, s.freqs_hz, s.tx_power_w)
        return pc, ge, gs

    return s, hidden, meas, evaluate


def test_loss_gradient_matches_central_differences(setup):
    s, _, meas, evaluate = setup
    mask = np.ones(meas.shape, bool)
    p, ge, gs = evaluate(s.materials)
    _, g_eps, g_sig = calibrate.db_loss_and_grad(p, ge, gs, meas, mask)
    for m in range(2):
        for col, g in ((0, g_eps), (1, g_sig)):
            h = 1e-5 * s.materials[m, col]
            mp, mm = s.materials.copy(), s.materials.copy()
            mp[m, col] += h
            mm[m, col] -= h
            lp = calibrate.db_loss_and_grad(*evaluate(mp), meas, mask)[0]
            lm = calibrate.db_loss_and_grad(*evaluate(mm), meas, mask)[0]
            assert g[m] == pytest.approx((lp - lm) / (2 * h), rel=1e-5)


def test_adam_recovers_hidden_materials(setup):
    s, hidden, meas, evaluate = setup
    r = calibrate.adam_fit(evaluate, s.materials, meas, steps=400, lr=0.1)
    assert r.loss_db2[0] > 1e-3 and r.loss_db2[-1] < 1e-12
    np.testing.assert_allclose(r.materials[:, :2], hidden[:, :2], rtol=1e-5)


def test_constant_gamma_materials_stay(setup):
    s, _, meas, evaluate = setup
    m0 = s.materials.copy()
    m0[1, 2] = 0.7   # ground as a constant gamma: nothing to fit there
    r = calibrate.adam_fit(evaluate, m0, meas, steps=5, lr=0.1)
    assert np.array_equal(r.materials[1], m0[1])
    assert not np.array_equal(r.materials[0], m0[0])
