"""Online calibration as gradient descent (paper, Sec. "Approach for online
calibration" and Sec. "Overview of HLT online calibration": calibration
objects computed from default-transformed clusters, fed back to the
transformation used by tracking).

``Chi2Refit`` is a torch.autograd.Function whose forward calls
tpcca_refit_grad (total Kalman-refit chi2 of a frozen track set under the
correction theta) and whose backward returns the gradient the library
computed in the same call.  ``calibrate`` runs Adam on theta.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np
import torch

from .tracker import FitTracks, Tracker


class Chi2Refit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, tracker: Tracker, fit: FitTracks):
        chi2, ndf, grad = tracker.refit_grad(fit, theta)
        ctx.save_for_backward(grad)
        ctx.ndf = ndf
        return torch.tensor(chi2, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (g * grad).to(torch.float64), None, None


def to_theta(u: torch.Tensor, n_sectors: int, drift_length: float, drift_unit: float = 1e-3) -> torch.Tensor:
    """Optimiser variables -> theta.  u = (drift scale in units of 1e-3,
    drift offset at the central electrode o = tau - L*delta [cm], map [cm]).
    The vertex constrains o directly and the external tan(lambda) constrains
    delta, so these coordinates are nearly decoupled, unlike (delta, tau)."""
    S = n_sectors
    d = u[:S] * drift_unit
    tau = u[S:2 * S] + drift_length * d
    return torch.cat([d, tau, u[2 * S:]])


def from_theta(theta: torch.Tensor, n_sectors: int, drift_length: float,
               drift_unit: float = 1e-3) -> torch.Tensor:
    S = n_sectors
    d = theta[:S]
    return torch.cat([d / drift_unit, theta[S:2 * S] - drift_length * d, theta[2 * S:]])


def calibrate(tracker: Tracker, fit: FitTracks, steps: int = 50, lr=(0.5, 0.02, 0.02),
              theta0: Optional[torch.Tensor] = None, betas=(0.9, 0.999), drift_length: float = 250.0,
              callback: Optional[Callable] = None, state: Optional[dict] = None):
    """Adam on theta from theta0 (default 0) in the variables of to_theta.
    lr = learning rates of the (drift scale [1e-3], drift offset [cm],
    map [cm]) groups.  Returns (theta, history, state); `state` (step,
    moments, variables) allows a resume from a checkpoint."""
    S = tracker.n_sectors
    dev = fit.hit_off.device
    if state is None:
        th0 = torch.zeros(S * 66, dtype=torch.float64, device=dev) if theta0 is None else (
            theta0.to(torch.float64).to(dev))
        u0 = from_theta(th0, S, drift_length)
        state = dict(step=0, u=u0, m=torch.zeros_like(u0), v=torch.zeros_like(u0))
    lr_vec = torch.empty(S * 66, dtype=torch.float64, device=dev)
    lr_vec[:S] = lr[0]; lr_vec[S:2 * S] = lr[1]; lr_vec[2 * S:] = lr[2]
    b1, b2 = betas
    hist = []
    for _ in range(steps):
        u = state["u"].clone().requires_grad_(True)
        chi2 = Chi2Refit.apply(to_theta(u, S, drift_length), tracker, fit)
        chi2.backward()
        gu = u.grad.detach()
        state["step"] += 1
        t = state["step"]
        state["m"] = b1 * state["m"] + (1 - b1) * gu
        state["v"] = b2 * state["v"] + (1 - b2) * gu * gu
        mh = state["m"] / (1 - b1 ** t)
        vh = state["v"] / (1 - b2 ** t)
        state["u"] = state["u"] - lr_vec * mh / (torch.sqrt(vh) + 1e-12)
        hist.append(float(chi2))
        if callback:
            callback(t, float(chi2), state)
    return to_theta(state["u"], S, drift_length).detach(), hist, state


def save_state(path: str, state: dict) -> None:
    np.savez(path, step=state["step"], u=state["u"].cpu().numpy(), m=state["m"].cpu().numpy(),
             v=state["v"].cpu().numpy())


def load_state(path: str, device) -> dict:
    z = np.load(path)
    t = lambda a: torch.from_numpy(a).to(torch.float64).to(device)
    return dict(step=int(z["step"]), u=t(z["u"]), m=t(z["m"]), v=t(z["v"]))
