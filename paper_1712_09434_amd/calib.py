"""Online calibration as gradient descent (paper, Sec. "Approach for online
calibration" and Sec. "Overview of HLT online calibration": calibration
objects computed from default-transformed clusters, fed back to the
transformation used by tracking).

``Chi2Refit`` is a torch.autograd.Function whose forward calls
tpcca_refit_grad (total Kalman-refit chi2 of a frozen track set under the
correction theta) and whose backward returns the gradient the library
computed in the same call.  ``calibrate`` runs Adam on theta;
``calibrate_newton`` takes damped Newton steps on the per-sector Hessian
blocks (the MAP estimate under a Gaussian prior on the miscalibration).
"""
from __future__ import annotations

import math

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


def sector_hessian(tracker: Tracker, fit: FitTracks, theta0: torch.Tensor,
                   steps=(1e-3, 0.05, 0.1)) -> torch.Tensor:
    """Per-sector 66x66 Hessian blocks of chi2 at theta0 by central
    differences of the library gradient.  Parameters of different sectors
    never share a track, so perturbing parameter p of every sector at once
    gives column p of all blocks: 2 x 66 gradient evaluations.
    steps: perturbation of (drift scale, time offset [cm], map [cm]); the
    chi2 is close to quadratic in theta (cluster positions move linearly
    with it), so steps of about half the expected miscalibration keep the
    truncation error small while the FP32 rounding of the gradient is
    divided by a large step."""
    S = tracker.n_sectors
    dev = theta0.device
    th0 = theta0.to(torch.float64)
    H = torch.zeros(S, 66, 66, dtype=torch.float64, device=dev)

    def sp(v):   # [S*66] layout -> [S, 66]
        return torch.cat([v[:S, None], v[S:2 * S, None], v[2 * S:].reshape(S, 64)], dim=1)

    def flat(a):
        return torch.cat([a[:, 0], a[:, 1], a[:, 2:].reshape(-1)])

    for q in range(66):
        h = steps[0] if q == 0 else steps[1] if q == 1 else steps[2]
        e = torch.zeros(S, 66, dtype=torch.float64, device=dev)
        e[:, q] = h
        _, _, gp = tracker.refit_grad(fit, (th0 + flat(e)).to(torch.float32))
        _, _, gm = tracker.refit_grad(fit, (th0 - flat(e)).to(torch.float32))
        H[:, :, q] = (sp(gp) - sp(gm)) / (2.0 * h)
    return 0.5 * (H + H.transpose(1, 2))


def whitening(H: torch.Tensor, floor: float = 1e-9):
    """Symmetric square roots W = H^(1/2) and W^-1 per block (eigenvalues
    floored at floor * the block's largest)."""
    w, V = torch.linalg.eigh(H)
    w = torch.clamp(w, min=floor * w.max(dim=1, keepdim=True).values)
    r = torch.sqrt(w)
    W = V @ torch.diag_embed(r) @ V.transpose(1, 2)
    Wi = V @ torch.diag_embed(1.0 / r) @ V.transpose(1, 2)
    return W, Wi


def default_prior_sigma(n_sectors: int = 36, device=None) -> torch.Tensor:
    """Expected spread of the miscalibration: drift scale 2e-3, time offset
    0.1 cm, map coefficients 0.3/sqrt(3) cm (the sd of U(-0.3, 0.3))."""
    s = torch.empty(n_sectors * 66, dtype=torch.float64, device=device)
    s[:n_sectors] = 2e-3
    s[n_sectors:2 * n_sectors] = 0.1
    s[2 * n_sectors:] = 0.3 / math.sqrt(3.0)
    return s


def calibrate(tracker: Tracker, fit: FitTracks, steps: int = 50, lr=(0.5, 0.02, 0.02),
              theta0: Optional[torch.Tensor] = None, betas=(0.9, 0.999), drift_length: float = 250.0,
              callback: Optional[Callable] = None, state: Optional[dict] = None,
              precondition: bool = False, lr_white: float = 30.0, lr_final: float = 0.1,
              prior_sigma: Optional[torch.Tensor] = None):
    """Adam on theta from theta0 (default 0).

    Loss: the refit chi2 and, if prior_sigma is given, a Gaussian prior
    sum((theta / prior_sigma)^2) on the size of the miscalibration (a MAP
    estimate: directions the tracks cannot see stay near zero instead of
    drifting).

    Without preconditioning the variables are those of to_theta and
    lr = learning rates of the (drift scale [1e-3], drift offset [cm], map
    [cm]) groups.  With a preconditioner the per-sector Hessian blocks of the
    loss at theta0 are estimated once (sector_hessian plus the prior's
    curvature) and Adam runs on linear coordinates u of theta - theta0 with a
    step size decaying from lr_white to lr_final (half cosine over `steps`):
      precondition=True or "white": u = H^(1/2) (theta - theta0), where the
        loss is locally isotropic;
      precondition="eigen": u = V^T D^-1 (theta - theta0) with D the prior
        spread (prior_sigma, required) and V the eigenvectors of D H D: the
        prior-scaled parameters rotated so that each coordinate is an
        independent quadratic to second order.  Adam's per-coordinate
        normalisation then moves every coordinate at the same rate in units
        of the expected miscalibration, so one step-size schedule suits
        strongly and weakly measured directions alike.
    Returns (theta, history, state); `state` (step, moments, variables,
    coordinate map) allows a resume from a checkpoint."""
    S = tracker.n_sectors
    dev = fit.hit_off.device

    def sp(v):
        return torch.cat([v[:S, None], v[S:2 * S, None], v[2 * S:].reshape(S, 64)], dim=1)

    def flat(a):
        return torch.cat([a[:, 0], a[:, 1], a[:, 2:].reshape(-1)])

    if state is None:
        th0 = torch.zeros(S * 66, dtype=torch.float64, device=dev) if theta0 is None else (
            theta0.to(torch.float64).to(dev))
        if precondition:
            H = sector_hessian(tracker, fit, th0)
            if prior_sigma is not None:
                H = H + torch.diag_embed(sp(2.0 / prior_sigma.to(dev) ** 2))
            if precondition == "eigen":
                if prior_sigma is None:
                    raise ValueError('precondition="eigen" needs prior_sigma')
                d = sp(prior_sigma.to(dev).to(torch.float64))             # [S, 66]
                A = d.unsqueeze(2) * H * d.unsqueeze(1)
                _, V = torch.linalg.eigh(0.5 * (A + A.transpose(1, 2)))
                R = d.unsqueeze(2) * V                                    # theta - theta0 = R u
            else:
                _, R = whitening(H)
            u0 = torch.zeros(S * 66, dtype=torch.float64, device=dev)
            state = dict(step=0, u=u0, m=torch.zeros_like(u0), v=torch.zeros_like(u0), R=R, th0=th0,
                         total=torch.tensor(float(steps)))
        else:
            u0 = from_theta(th0, S, drift_length)
            state = dict(step=0, u=u0, m=torch.zeros_like(u0), v=torch.zeros_like(u0))
    white = "R" in state

    def theta_of(u):
        if white:
            du = (state["R"] @ u.reshape(S, 66, 1)).reshape(S, 66)
            return state["th0"] + flat(du)
        return to_theta(u, S, drift_length)

    if not white:
        lr_vec = torch.empty(S * 66, dtype=torch.float64, device=dev)
        lr_vec[:S] = lr[0]; lr_vec[S:2 * S] = lr[1]; lr_vec[2 * S:] = lr[2]
    b1, b2 = betas
    hist = []
    for _ in range(steps):
        u = state["u"].clone().requires_grad_(True)
        theta = theta_of(u)
        loss = Chi2Refit.apply(theta, tracker, fit)
        if prior_sigma is not None:
            loss = loss + ((theta / prior_sigma.to(dev)) ** 2).sum()
        loss.backward()
        gu = u.grad.detach()
        state["step"] += 1
        t = state["step"]
        state["m"] = b1 * state["m"] + (1 - b1) * gu
        state["v"] = b2 * state["v"] + (1 - b2) * gu * gu
        mh = state["m"] / (1 - b1 ** t)
        vh = state["v"] / (1 - b2 ** t)
        if white:
            frac = min(1.0, (t - 1) / max(float(state["total"]) - 1.0, 1.0))
            rate = lr_final + 0.5 * (lr_white - lr_final) * (1.0 + math.cos(math.pi * frac))
            state["u"] = state["u"] - rate * mh / (torch.sqrt(vh) + 1e-12)
        else:
            state["u"] = state["u"] - lr_vec * mh / (torch.sqrt(vh) + 1e-12)
        hist.append(float(loss.detach()))
        if callback:
            callback(t, float(loss), state)
    return theta_of(state["u"]).detach(), hist, state


def _blocks(v: torch.Tensor, S: int) -> torch.Tensor:
    return torch.cat([v[:S, None], v[S:2 * S, None], v[2 * S:].reshape(S, 64)], dim=1)


def _flat(a: torch.Tensor) -> torch.Tensor:
    return torch.cat([a[:, 0], a[:, 1], a[:, 2:].reshape(-1)])


def map_objective(tracker: Tracker, fit: FitTracks, theta: torch.Tensor, prior_sigma: torch.Tensor):
    """(chi2 + sum((theta / sigma)^2), its gradient) at theta (FP64)."""
    chi2, _, g = tracker.refit_grad(fit, theta.to(torch.float32))
    th = theta.to(torch.float64)
    return chi2 + float(((th / prior_sigma) ** 2).sum()), g + 2.0 * th / prior_sigma ** 2


def calibrate_newton(tracker: Tracker, fit: FitTracks, iters: int = 4, prior_sigma: Optional[torch.Tensor] = None,
                     theta0: Optional[torch.Tensor] = None, rehess: bool = True, max_halvings: int = 8,
                     callback: Optional[Callable] = None):
    """MAP calibration by damped Newton steps.

    Loss f = chi2(theta) + sum((theta / prior_sigma)^2).  Every iteration
    takes the per-sector Hessian blocks (sector_hessian, recomputed at the
    current theta when rehess, else kept from theta0), clamps the chi2 part
    to be positive semi-definite per block (eigenvalues < 0 -> 0, so the
    prior alone sets the curvature of directions the tracks do not see),
    solves for the Newton step and halves it until f decreases.  Returns
    (theta, history of f)."""
    S = tracker.n_sectors
    dev = fit.hit_off.device
    sig = (default_prior_sigma(S, dev) if prior_sigma is None else prior_sigma.to(dev)).to(torch.float64)
    th = torch.zeros(S * 66, dtype=torch.float64, device=dev) if theta0 is None else theta0.to(torch.float64).to(dev)
    f, g = map_objective(tracker, fit, th, sig)
    hist = [f]
    curv = torch.diag_embed(_blocks(2.0 / sig ** 2, S))
    H = None
    for it in range(iters):
        if H is None or rehess:
            Hc = sector_hessian(tracker, fit, th)
            w, V = torch.linalg.eigh(Hc)
            Hc = V @ torch.diag_embed(torch.clamp(w, min=0.0)) @ V.transpose(1, 2)
            H = Hc + curv
        step = -torch.linalg.solve(H, _blocks(g, S).unsqueeze(2)).squeeze(2)
        step = _flat(step)
        a = 1.0
        for _ in range(max_halvings + 1):
            tn = th + a * step
            fn, gn = map_objective(tracker, fit, tn, sig)
            if math.isfinite(fn) and fn < f:
                break
            a *= 0.5
        else:
            break                      # no decrease along the step: converged to rounding
        th, f, g = tn, fn, gn
        hist.append(f)
        if callback:
            callback(it + 1, f, th, a)
    return th, hist


def save_state(path: str, state: dict) -> None:
    arrays = {k: v.cpu().numpy() for k, v in state.items() if isinstance(v, torch.Tensor)}
    np.savez(path, step=state["step"], **arrays)


def load_state(path: str, device) -> dict:
    z = np.load(path)
    st = {k: torch.from_numpy(z[k]).to(torch.float64).to(device) for k in z.files if k != "step"}
    st["step"] = int(z["step"])
    return st
