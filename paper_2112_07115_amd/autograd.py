"""The received power of a frame as a differentiable torch function.

`received_power(ctx, scene, eps_r, sigma, tx_power, pattern, ...)` traces the
scene's frame with the given material parameters, transmit power and transmit
pattern weights (dcem_set_materials, dcem_set_tx_pattern, dcem_trace_frame)
and returns the coherent power [n_freqs, n_tx, n_rx] as an FP64 tensor.  Its
backward pass holds the frame's paths and uses dcem_power_gradients (Sec. III,
the field of Eq. (3) with closed-form Fresnel derivatives): the incoming
gradient is contracted with dP/d eps_r, dP/d sigma, dP/dP_t and dP/dw over the
receivers.  Forward and derivatives run in the library's kernels; the
contraction of a few hundred numbers per parameter is host glue.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dcem, scenes


class _ReceivedPower(torch.autograd.Function):
    @staticmethod
    def forward(fctx, eps_r, sigma, tx_power, pattern, dctx, scene, frame, ray_dirs, mode):
        mats = np.array(scene.materials, dtype=np.float64, copy=True)
        mats[:, 0] = eps_r.detach().cpu().double().numpy()
        mats[:, 1] = sigma.detach().cpu().double().numpy()
        s = scenes.Scene(**{**scene.__dict__, "tx_power_w": float(tx_power.detach().cpu())})
        dctx.set_materials(mats)
        dctx.set_tx_pattern(pattern.detach().cpu().double().numpy())
        dcem.trace_scene_frame(dctx, s, frame=frame, ray_dirs=ray_dirs, mode=mode, keep_cache=True)
        p, _ = dctx.received_power()
        de, ds, dp, dw = dctx.power_gradients()
        # gradients are returned on each parameter's device and in its dtype;
        # the power lives where eps_r does
        fctx.like = [(t.device, t.dtype) for t in (eps_r, sigma, tx_power, pattern)]
        dev = eps_r.device
        fctx.save_for_backward(*(torch.from_numpy(a).to(dev) for a in (de, ds, dp, dw)))
        return torch.from_numpy(p).to(dev)

    @staticmethod
    def backward(fctx, grad_p):
        de, ds, dp, dw = fctx.saved_tensors
        g = grad_p.double().to(de.device)
        grads = ((g[..., None] * de).sum((0, 1, 2)), (g[..., None] * ds).sum((0, 1, 2)), (g * dp).sum(),
                 (g[..., None] * dw).sum((0, 1, 2)))
        grads = tuple(x.to(device=d, dtype=t) for x, (d, t) in zip(grads, fctx.like))
        return grads + (None, None, None, None, None)


def received_power(dctx: "dcem.Context", scene, eps_r: torch.Tensor, sigma: torch.Tensor, tx_power: torch.Tensor,
                   pattern: torch.Tensor, frame: int = 0, ray_dirs=None, mode: int = dcem.MODE_COHERENT):
    """Coherent power [n_freqs, n_tx, n_rx] (FP64, on eps_r's device) of
    `scene`'s frame with eps_r, sigma [n_materials], tx_power [] and pattern
    [16] (each on any device; its gradient comes back on that device and in
    its dtype); the context must hold the scene.  Differentiable in all four.
    Materials with a constant gamma ignore their eps_r and sigma (zero
    gradients)."""
    return _ReceivedPower.apply(eps_r, sigma, tx_power, pattern, dctx, scene, frame, ray_dirs, mode)
