"""torch.autograd binding of the filter's log marginal likelihood.

``log_marginal(theta, frames, cfg, truth)`` runs the filter over ``frames``
from ``truth`` with theta = (psf_sigma, I0, q) (I0 is the intensity of the
starting state) and returns J [F], the filter's estimate of
log p(z_1..z_K) per filter.  Its backward runs the library's reverse sweep
(pf_grad_end) over the recorded iterations: the derivative of J with every
discrete choice of the run held fixed.  The forward pass keeps the recording
alive until backward (or until the returned tensor is freed).

Argument marshalling only: every step runs in the HIP library.
"""
from __future__ import annotations

import numpy as np

from .tracker import Tracker


def _function():
    import torch

    class LogMarginal(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, frames, cfg, truth):
            th = theta.detach().to("cpu", torch.float64).numpy()
            c = dict(cfg, psf_sigma=float(th[0]), q=float(th[2]))
            t = np.array(truth, dtype=np.float32, copy=True).reshape(-1, 5)
            t[:, 4] = th[1]
            tr = Tracker(c, t)
            K = frames.shape[0]
            tr.grad_begin(K)
            tr.run(frames)
            ctx.tracker, ctx.frames = tr, frames
            J = torch.from_numpy(tr.grad_value()).to(theta.device)
            return J

        @staticmethod
        def backward(ctx, gJ):
            tr = ctx.tracker
            res = tr.grad_end(ctx.frames)
            tr.close()
            ctx.tracker = ctx.frames = None
            G = torch.from_numpy(res["grad"]).to(gJ.device, gJ.dtype)   # [F][3]
            return (gJ[:, None] * G).sum(0), None, None, None

    return LogMarginal


_FN = None


def log_marginal(theta, frames, cfg: dict, truth):
    """J [F] = log p-hat(z_1..z_K) per filter, differentiable in theta
    (float64 tensor [3]: psf_sigma, I0, q).  frames: CUDA float32 [K][H][W].

    Tracking start only: the information-sharing start draws the intensities
    of PEs other than the first as 2 I0 u (a scaling of I0, not the shift
    the reverse sweep differentiates), so it is refused."""
    from ._native import PF_INIT_INFOSHARE
    if cfg.get("init_mode", 0) == PF_INIT_INFOSHARE:
        raise ValueError("log_marginal differentiates the tracking start only "
                         "(init_mode=PF_INIT_TRACKING)")
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(theta, frames, cfg, truth)
