"""GPU: derivatives of the coherent received power along a frame's paths
(dcem_power_gradients) against the FP64 oracle's, through the C ABI, and the
transmit pattern (dcem_set_tx_pattern) in the forward power.

Workloads: the static toy scene (2 frequencies, an added constant-gamma
material) with 20,000 random rays and K = 2, and the dynamic urban grid
(K = 4, moving metal vehicles) with 65,536 random rays, the latter under a
random transmit pattern.  Receivers whose path sets are certain on both sides
are compared; the rest are skipped as in the power parity tests.
"""
import sys

import numpy as np
import pytest

from paper_2112_07115_amd import dcem, scenes
from tests import parity

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.build()
    return oracle


@pytest.fixture()
def ctx():
    c = dcem.Context(0)
    yield c
    c.close()


def oracle_gradients(O, s, frame, dirs, pattern=None):
    ofr = O.frame(s, frame_index=frame, dirs=dirs, pattern=pattern)
    xf = s.transforms(frame) if s.object_vertex_range.shape[0] else None
    osc = O.OracleScene(s, xf)
    ntx, nrx = s.tx.shape[0], s.rx.shape[0]
    damp = O.refine_grad(osc, s.tx, s.rx, ofr.keys, s.max_reflections, s.freqs_hz, s.tx_power_w,
                         s.materials.shape[0], pattern=pattern)
    iso = ofr.paths if pattern is None else O.refine(osc, s.tx, s.rx, ofr.keys, s.max_reflections,
                                                     s.freqs_hz, s.tx_power_w)
    g = O.power_gradients(ofr.paths, damp, ntx, nrx, s.freqs_hz, s.tx_power_w)
    return ofr, g + (O.pattern_gradients(ofr.paths, iso, ntx, nrx),)


def compare(ctx, O, s, frame, dirs, pattern=None):
    log("case", s.name, "frame", frame, "rays", len(dirs), "pattern", pattern is not None)
    ctx.scene_upload(s)
    ctx.set_tx_pattern(pattern)
    dcem.trace_scene_frame(ctx, s, frame=frame, ray_dirs=dirs)
    p_coh, _ = ctx.received_power()
    g_eps, g_sig, g_pt, g_pat = ctx.power_gradients()
    ofr, (o_eps, o_sig, o_pt, o_pat) = oracle_gradients(O, s, frame, dirs, pattern)
    comparable, _ = parity.compare_paths(ctx.paths(), ofr, len(dirs))
    assert (~comparable).sum() <= max(1, int(0.05 * comparable.size))
    n_cmp = 0
    for t in range(s.tx.shape[0]):
        for r in range(s.rx.shape[0]):
            if not comparable[t, r]:
                continue
            np.testing.assert_allclose(p_coh[:, t, r], ofr.p_coh[:, t, r], rtol=1e-6, atol=0)
            for g, o in ((g_eps, o_eps), (g_sig, o_sig), (g_pat, o_pat)):
                ref = np.abs(o[:, t, r]).max()
                np.testing.assert_allclose(g[:, t, r], o[:, t, r], rtol=1e-6, atol=1e-6 * ref + 1e-300)
            np.testing.assert_allclose(g_pt[:, t, r], o_pt[:, t, r], rtol=1e-6, atol=0)
            n_cmp += 1
    nz = int((np.abs(o_eps) > 0).sum())
    log("  compared receivers", n_cmp, "nonzero oracle d/deps_r entries", nz,
        "nonzero d/dw entries", int((np.abs(o_pat) > 0).sum()))
    assert n_cmp > 0 and nz > 0 and np.abs(o_pat).max() > 0
    return g_eps, g_sig, g_pt


def test_toy_gradients(ctx, O):
    s = scenes.static_toy()
    mats = np.vstack([s.materials, [[3.0, 0.01, 0.8]]])
    s = scenes.Scene(**{**s.__dict__, "materials": mats, "freqs_hz": [28e9, 3.5e9]})
    g_eps, g_sig, _ = compare(ctx, O, s, 0, scenes.random_sphere_dirs(20_000, seed=3))
    assert np.all(g_eps[..., 2] == 0) and np.all(g_sig[..., 2] == 0)   # constant gamma, on no face


def test_urban_gradients_under_a_pattern(ctx, O):
    s = scenes.dynamic_urban()
    w = np.random.default_rng(4).uniform(0.5, 1.5, dcem.PATTERN_TAPS)
    compare(ctx, O, s, 7, scenes.random_sphere_dirs(65_536, seed=11), pattern=w)


def test_pattern_applies_from_the_next_frame(ctx):
    """The weights take effect at the next traced frame; all-ones is the
    isotropic antenna bitwise, and a constant 0.5 quarters every power
    exactly (a scale by a power of two)."""
    s = scenes.static_toy()
    ctx.scene_upload(s)
    kw = dict(ray_dirs=scenes.random_sphere_dirs(20_000, seed=3))
    dcem.trace_scene_frame(ctx, s, **kw)
    p_iso, _ = ctx.received_power()
    g_iso = ctx.power_gradients()
    ctx.set_tx_pattern(np.full(dcem.PATTERN_TAPS, 0.5))
    p_same, _ = ctx.received_power()
    assert np.array_equal(p_same, p_iso)            # no frame traced since the call
    for a, b in zip(g_iso, ctx.power_gradients()):
        assert np.array_equal(a, b)
    dcem.trace_scene_frame(ctx, s, **kw)
    p_half, _ = ctx.received_power()
    assert np.array_equal(p_half, 0.25 * p_iso)
    ctx.set_tx_pattern(np.ones(dcem.PATTERN_TAPS))
    dcem.trace_scene_frame(ctx, s, **kw)
    assert np.array_equal(ctx.received_power()[0], p_iso)
    ctx.set_tx_pattern(None)
    dcem.trace_scene_frame(ctx, s, **kw)
    assert np.array_equal(ctx.received_power()[0], p_iso)
    assert p_iso.max() > 0


def test_pattern_argument_errors(ctx):
    for bad in (np.ones(15), np.ones(17), np.array([1.0] * 15 + [np.nan])):
        with pytest.raises(dcem.DcemError):
            ctx.set_tx_pattern(bad)


def test_gradients_after_the_next_frame_started():
    """Gradients read after the next frame's refit and revalidation were
    started (objects moved before the read) equal those read before."""
    s = scenes.dynamic_urban()
    n = 1 << 16
    c = dcem.Context(0)
    c.scene_upload(s)
    kw = dict(max_reflections=s.max_reflections, freqs_hz=s.freqs_hz, tx_power_w=s.tx_power_w)
    for f in range(3):
        c.set_object_transforms(s.transforms(f))
        c.refit_bvh()
        c.trace_frame(s.tx, s.rx, s.rx_radius, n, mode=dcem.MODE_COHERENT, **kw)
        before = c.power_gradients()
        c.received_power()
        c.set_object_transforms(s.transforms(f + 1))
        c.refit_bvh()   # starts the next frame early
        after = c.power_gradients()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)
    c.close()


def toy_two_bands():
    s = scenes.static_toy()
    return scenes.Scene(**{**s.__dict__, "freqs_hz": [28e9, 3.5e9]})


HIDDEN = ((7.0, 1.0), (10.0, 0.5))   # concrete and ground, far from the scene's own


def test_set_materials_applies_from_the_next_frame(ctx, O):
    s = toy_two_bands()
    dirs = scenes.random_sphere_dirs(20_000, seed=3)
    hidden = s.materials.copy()
    hidden[:, :2] = HIDDEN
    sh = scenes.Scene(**{**s.__dict__, "materials": hidden})
    ctx.scene_upload(s)
    dcem.trace_scene_frame(ctx, s, ray_dirs=dirs)
    p0, _ = ctx.received_power()
    g0 = ctx.power_gradients()
    ctx.set_materials(hidden)
    assert np.array_equal(ctx.received_power()[0], p0)   # the last frame keeps its table
    for a, b in zip(g0, ctx.power_gradients()):
        assert np.array_equal(a, b)
    dcem.trace_scene_frame(ctx, s, ray_dirs=dirs)
    p1, _ = ctx.received_power()
    g1 = ctx.power_gradients()
    # the same as a fresh upload of the hidden table, and as the oracle's
    c2 = dcem.Context(0)
    try:
        c2.scene_upload(sh)
        dcem.trace_scene_frame(c2, sh, ray_dirs=dirs)
        assert np.array_equal(c2.received_power()[0], p1)
        for a, b in zip(c2.power_gradients(), g1):
            assert np.array_equal(a, b)
    finally:
        c2.close()
    ofr = O.frame(sh, dirs=dirs)
    comparable, _ = parity.compare_paths(ctx.paths(), ofr, len(dirs))
    assert (~comparable).sum() <= max(1, int(0.05 * comparable.size)) and not np.array_equal(p1, p0)
    np.testing.assert_allclose(p1[:, comparable], ofr.p_coh[:, comparable], rtol=1e-6, atol=0)
    with pytest.raises(dcem.DcemError):
        ctx.set_materials(hidden[:1])
    bad = hidden.copy()
    bad[0, 0] = 0.5   # eps_r below 1
    with pytest.raises(dcem.DcemError):
        ctx.set_materials(bad)


def test_materials_fit_by_adam(ctx, O):
    """Calibration: the materials of the toy scene are fitted by Adam through
    the library's frames and gradients to the oracle's powers at hidden
    materials (noise-free), on the receivers whose path sets are certain."""
    from paper_2112_07115_amd import calibrate
    s = toy_two_bands()
    dirs = scenes.random_sphere_dirs(20_000, seed=3)
    hidden = s.materials.copy()
    hidden[:, :2] = HIDDEN
    ofr = O.frame(scenes.Scene(**{**s.__dict__, "materials": hidden}), dirs=dirs)
    meas = 10.0 * np.log10(np.where(ofr.p_coh > 0, ofr.p_coh, np.nan))
    ctx.scene_upload(s)
    dcem.trace_scene_frame(ctx, s, ray_dirs=dirs)
    # path sets (geometry only) compared at the starting table, amplitudes included
    comparable, _ = parity.compare_paths(ctx.paths(), O.frame(s, dirs=dirs), len(dirs))
    mask = np.broadcast_to(comparable, meas.shape)
    r = calibrate.fit_materials(ctx, s, meas, s.materials, mask=mask, ray_dirs=dirs, steps=400, lr=0.1)
    log("  fit: loss %.3g -> %.3g dB^2 in %d steps" % (r.loss_db2[0], r.loss_db2[-1], r.steps), r.materials[:, :2])
    assert r.loss_db2[0] > 1e-3 and r.loss_db2[-1] < 1e-10
    np.testing.assert_allclose(r.materials[:, :2], hidden[:, :2], rtol=1e-4)


def test_autograd_function_against_the_oracle(ctx, O):
    """torch autograd through the frame's power: the backward pass's
    contraction of a random weighting of the receivers' powers equals the
    same contraction of the oracle's gradients (comparable receivers only)."""
    import torch
    from paper_2112_07115_amd import autograd
    s = toy_two_bands()
    dirs = scenes.random_sphere_dirs(20_000, seed=3)
    w = np.random.default_rng(8).uniform(0.6, 1.4, dcem.PATTERN_TAPS)
    eps = torch.tensor(s.materials[:, 0], dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(s.materials[:, 1], dtype=torch.float64, requires_grad=True)
    pt = torch.tensor(float(s.tx_power_w), dtype=torch.float64, requires_grad=True)
    pat = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    ctx.scene_upload(s)
    p = autograd.received_power(ctx, s, eps, sig, pt, pat, ray_dirs=dirs)
    ofr, (o_eps, o_sig, o_pt, o_pat) = oracle_gradients(O, s, 0, dirs, pattern=w)
    comparable, _ = parity.compare_paths(ctx.paths(), ofr, len(dirs))
    assert (~comparable).sum() <= max(1, int(0.05 * comparable.size))
    wt = np.random.default_rng(2).uniform(0.5, 1.5, p.shape) * comparable[None]
    (p * torch.from_numpy(wt)).sum().backward()
    np.testing.assert_allclose(p.detach().numpy()[:, comparable], ofr.p_coh[:, comparable], rtol=1e-6)
    for got, o in ((eps.grad, o_eps), (sig.grad, o_sig), (pat.grad, o_pat)):
        ref = np.tensordot(wt, o, axes=([0, 1, 2], [0, 1, 2]))
        np.testing.assert_allclose(got.numpy(), ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())
    assert float(pt.grad) == pytest.approx(float((wt * o_pt).sum()), rel=1e-6)


def test_autograd_with_device_parameters(ctx):
    """Parameters on the GPU (a torch training loop's natural place): the
    power comes back on their device and every gradient on its parameter's
    device and dtype, equal to the CPU-parameter run."""
    import torch
    from paper_2112_07115_amd import autograd
    s = toy_two_bands()
    dirs = scenes.random_sphere_dirs(20_000, seed=3)
    ctx.scene_upload(s)
    res = []
    for dev, dt in (("cpu", torch.float64), ("cuda", torch.float64), ("cuda", torch.float32)):
        eps = torch.tensor(s.materials[:, 0], dtype=dt, device=dev, requires_grad=True)
        sig = torch.tensor(s.materials[:, 1], dtype=dt, device=dev, requires_grad=True)
        pt = torch.tensor(float(s.tx_power_w), dtype=dt, device=dev, requires_grad=True)
        pat = torch.ones(dcem.PATTERN_TAPS, dtype=dt, device=dev, requires_grad=True)
        p = autograd.received_power(ctx, s, eps, sig, pt, pat, ray_dirs=dirs, mode=dcem.MODE_FULL)
        assert p.device.type == dev and p.dtype == torch.float64
        (p * torch.arange(p.numel(), device=dev, dtype=torch.float64).reshape(p.shape)).sum().backward()
        for t in (eps, sig, pt, pat):
            assert t.grad.device.type == dev and t.grad.dtype == dt
        res.append([p.detach().cpu().double()] + [t.grad.detach().cpu().double() for t in (eps, sig, pt, pat)])
    assert torch.equal(res[0][0], res[1][0])   # the same frame
    for a, b in zip(res[0][1:], res[1][1:]):   # contractions summed on another device
        np.testing.assert_allclose(b.numpy(), a.numpy(), rtol=1e-12, atol=1e-12 * float(a.abs().max()))
    for a, b in zip(res[0][1:], res[2][1:]):
        np.testing.assert_allclose(b.numpy(), a.numpy(), rtol=1e-6, atol=1e-6 * float(a.abs().max()))


def test_materials_fit_over_moving_frames(ctx, O):
    """Calibration over three frames of the urban scene (moving vehicles,
    65,536 random rays, K = 4): concrete and ground are fitted to the oracle's
    powers at hidden values on every frame's comparable receivers; the metal
    (eps_r = 1) has no eps_r freedom left and keeps its table values."""
    from paper_2112_07115_amd import calibrate
    s = scenes.dynamic_urban()
    s = scenes.Scene(**{**s.__dict__, "freqs_hz": [28e9, 3.5e9]})
    dirs = scenes.random_sphere_dirs(65_536, seed=11)
    hidden = s.materials.copy()
    hidden[0, :2] = HIDDEN[0]
    hidden[1, :2] = HIDDEN[1]
    sh = scenes.Scene(**{**s.__dict__, "materials": hidden})
    frames = [0, 3, 6]
    ctx.scene_upload(s)
    meas, masks = [], []
    for f in frames:
        ofr = O.frame(sh, frame_index=f, dirs=dirs)
        meas.append(10.0 * np.log10(np.where(ofr.p_coh > 0, ofr.p_coh, np.nan)))
        dcem.trace_scene_frame(ctx, s, frame=f, ray_dirs=dirs)
        comparable, _ = parity.compare_paths(ctx.paths(), O.frame(s, frame_index=f, dirs=dirs), len(dirs))
        masks.append(np.broadcast_to(comparable, meas[-1].shape))
    r = calibrate.fit_materials(ctx, s, np.stack(meas), s.materials, mask=np.stack(masks), ray_dirs=dirs,
                                frames=frames, steps=300, lr=0.1)
    log("  fit over frames %s: loss %.3g -> %.3g dB^2 in %d steps" % (frames, r.loss_db2[0], r.loss_db2[-1],
                                                                     r.steps), r.materials[:, :2])
    assert r.loss_db2[-1] < 1e-3 * r.loss_db2[0]
    np.testing.assert_allclose(r.materials[:2, :2], hidden[:2, :2], rtol=1e-2)
    assert r.materials[2, 0] == pytest.approx(s.materials[2, 0], abs=1e-6)
