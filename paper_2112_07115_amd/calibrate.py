"""Material calibration by gradient descent on measured received power.

The traced paths of a frame do not depend on the materials (reflection
points and visibility are geometry only, Sec. III), so a fit of the
materials' eps_r and sigma to measured powers can hold the frame's paths and
follow dcem_power_gradients: each step sets the material table
(dcem_set_materials), re-traces the frame in coherent mode (no ray is
re-shot when nothing moved, only the paths' fields are recomputed), and reads
the powers and their derivatives.

The loss is the mean squared error in dB over the receivers, frequencies and
transmitters selected by `mask` (and with a positive measured and predicted
power); the parameters are a = log(eps_r - 1) and b = log(sigma), so eps_r
stays above 1 and sigma positive, updated with Adam.  Materials with a
constant gamma (third column not NaN) have no eps_r or sigma to fit and stay.
The optimiser runs on the host over a handful of parameters; every frame and
derivative runs in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import dcem

_DB = 10.0 / np.log(10.0)


@dataclass
class FitResult:
    materials: np.ndarray            # [n_materials, 3], the fitted table
    loss_db2: list = field(default_factory=list)   # loss before each step, dB^2
    steps: int = 0


def db_loss_and_grad(p: np.ndarray, d_eps: np.ndarray, d_sig: np.ndarray, measured_db: np.ndarray,
                     mask: np.ndarray):
    """Loss (mean squared dB error over the selected entries) and its
    derivatives with respect to every material's eps_r and sigma."""
    sel = mask & (p > 0) & np.isfinite(measured_db)
    n = max(int(sel.sum()), 1)
    err = np.where(sel, _DB * np.log(np.where(sel, p, 1.0)) - np.where(sel, measured_db, 0.0), 0.0)
    loss = float(np.sum(err ** 2) / n)
    dl_dp = np.where(sel, 2.0 * err * _DB / np.where(sel, p, 1.0) / n, 0.0)
    g_eps = np.tensordot(dl_dp, d_eps, axes=(list(range(dl_dp.ndim)), list(range(dl_dp.ndim))))
    g_sig = np.tensordot(dl_dp, d_sig, axes=(list(range(dl_dp.ndim)), list(range(dl_dp.ndim))))
    return loss, g_eps, g_sig


def adam_fit(evaluate: Callable[[np.ndarray], tuple], materials0: np.ndarray, measured_db: np.ndarray,
             mask: Optional[np.ndarray] = None, steps: int = 300, lr: float = 0.05, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8, tol_db2: float = 0.0) -> FitResult:
    """Adam over (log(eps_r - 1), log(sigma)) of the materials without a
    constant gamma.  evaluate(materials) -> (p_coh, d_eps_r, d_sigma) with the
    layouts of dcem_received_power and dcem_power_gradients."""
    mats = np.array(materials0, dtype=np.float64, copy=True).reshape(-1, 3)
    free = np.isnan(mats[:, 2])
    if mask is None:
        mask = np.ones(measured_db.shape, dtype=bool)
    theta = np.stack([np.log(np.maximum(mats[:, 0] - 1.0, 1e-12)), np.log(np.maximum(mats[:, 1], 1e-12))], axis=1)
    m1 = np.zeros_like(theta)
    m2 = np.zeros_like(theta)
    out = FitResult(mats)
    for k in range(1, steps + 1):
        p, d_eps, d_sig = evaluate(mats)
        loss, g_eps, g_sig = db_loss_and_grad(p, d_eps, d_sig, measured_db, mask)
        out.loss_db2.append(loss)
        if loss <= tol_db2:
            break
        # chain rule to the log parameters: d eps_r / da = eps_r - 1, d sigma / db = sigma
        g = np.stack([g_eps * (mats[:, 0] - 1.0), g_sig * mats[:, 1]], axis=1)
        g[~free] = 0.0
        m1 = beta1 * m1 + (1.0 - beta1) * g
        m2 = beta2 * m2 + (1.0 - beta2) * g * g
        step = lr * (m1 / (1.0 - beta1 ** k)) / (np.sqrt(m2 / (1.0 - beta2 ** k)) + eps)
        theta = theta - step
        mats = mats.copy()
        mats[free, 0] = 1.0 + np.exp(theta[free, 0])
        mats[free, 1] = np.exp(theta[free, 1])
        out.steps = k
    out.materials = mats
    return out


def fit_materials(ctx: "dcem.Context", scene, measured_db: np.ndarray, materials0: np.ndarray,
                  mask: Optional[np.ndarray] = None, frame: int = 0, ray_dirs=None, frames=None,
                  **adam) -> FitResult:
    """Fit the scene's materials to measured powers in dBW: [n_freqs, n_tx,
    n_rx] at one frame of the scene, or, with `frames` (a list of frame
    indices), [len(frames), n_freqs, n_tx, n_rx] over those frames (the loss
    is the mean over all of them).  The context must hold the scene
    (uploaded); the first step traces each frame in full, later steps trace
    coherently (every frame's objects are placed again, so only the rays their
    motion invalidates are re-traced)."""
    state = {"traced": False}
    seq = [frame] if frames is None else list(frames)

    def evaluate(mats):
        ctx.set_materials(mats)
        ps, des, dss = [], [], []
        for f in seq:
            dcem.trace_scene_frame(ctx, scene, frame=f, ray_dirs=ray_dirs,
                                   mode=dcem.MODE_COHERENT if state["traced"] else dcem.MODE_FULL,
                                   keep_cache=True)
            p, _ = ctx.received_power()
            d_eps, d_sig, _, _ = ctx.power_gradients()
            ps.append(p)
            des.append(d_eps)
            dss.append(d_sig)
        state["traced"] = True
        if frames is None:
            return ps[0], des[0], dss[0]
        return np.stack(ps), np.stack(des), np.stack(dss)

    return adam_fit(evaluate, materials0, measured_db, mask, **adam)
