"""Calibration as gradient-based optimisation on the GPU (the paper's
feedback loop, Sec. "Approach for online calibration"), through the
torch.autograd.Function around tpcca_refit_grad.

What the frozen track set determines (per sector, 66 parameters): the drift
offset at the central electrode (tau - L delta) through the vertex, and a
subspace of (drift scale, time offset, map) through the track curvature and
the external tan(lambda); the rest is fixed only by the Gaussian prior.  The
track set holds the segments that reach the inner pad rows (the ones a
TPC-ITS matching would see; the vertex and external tan(lambda) terms stand
in for it) from 20 miscalibrated full events.  The tests check (a) that 50
Adam steps from theta = 0 reach an objective no worse than the injected
truth's and recover the drift offset and the identifiable subspace, (b) the
same for the MAP estimate of damped Newton on the first 10 events, (c) that
Adam in Hessian-whitened coordinates lowers the objective most of the way,
(d) checkpoint/resume of the Adam state.
"""
import os

import numpy as np
import pytest
import torch

import synth
from calibset import calib_subset

pytestmark = pytest.mark.gpu
S = 36
NEV = int(os.environ.get("TPCCA_CALIB_EVENTS", "20"))
NEV_NEWTON = min(NEV, 10)
LR = (0.5, 0.02, 0.02)   # Adam learning rates: drift scale [1e-3], drift offset [cm], map [cm]


def fit_of(parts, dev):
    """One FitTracks over several events: clusters concatenated, hit ids shifted."""
    from paper_1712_09434_amd import FitTracks
    cols = [[] for _ in range(5)]
    offs, ids, k0s, exts = [0], [], [], []
    base = 0
    for ev, cs in parts:
        for L, a in zip(cols, (ev.x, ev.y, ev.z, ev.row, ev.sector)):
            L.append(a)
        for k in range(len(cs["k0"])):
            h = cs["hit_ids"][cs["hit_off"][k]:cs["hit_off"][k + 1]] + base
            ids.append(h)
            offs.append(offs[-1] + len(h))
        k0s.append(cs["k0"]); exts.append(cs["ext_tgl"])
        base += ev.n
    cat = lambda a, dt: torch.from_numpy(np.ascontiguousarray(np.concatenate(a)).astype(dt)).to(dev)
    cl = (cat(cols[0], np.float32), cat(cols[1], np.float32), cat(cols[2], np.float32),
          cat(cols[3], np.int16), cat(cols[4], np.uint8))
    return FitTracks(clusters=cl, hit_off=torch.tensor(offs, dtype=torch.int32, device=dev),
                     hit_id=cat(ids, np.int32), k_prior=cat(k0s, np.float32), ext_tgl=cat(exts, np.float32),
                     use_vertex=torch.ones(len(offs) - 1, dtype=torch.uint8, device=dev))


@pytest.fixture(scope="module")
def events():
    from paper_1712_09434_amd import Tracker
    dev = torch.device("cuda:0")
    print(f"[gpu] generating {NEV} miscalibrated full events", flush=True)
    evs = synth.make_configs("C5", range(NEV))
    trk = Tracker.from_geometry(synth.default_geometry())
    parts = []
    for ev in evs:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        out = trk.track(t(ev.x), t(ev.y), t(ev.z), t(ev.row), t(ev.sector))
        off = out.hit_off.cpu().numpy().astype(np.int64)
        hid = out.hit_id.cpu().numpy().astype(np.int64)
        cs = calib_subset(ev, off, hid, out.sector.cpu().numpy(), out.chi2.cpu().numpy(),
                          out.ndf.cpu().numpy(), out.k_prior.cpu().numpy(), max_inner_row=10)
        parts.append((ev, cs))
    yield trk, parts
    trk.close()


def _dataset(events, n):
    trk, parts = events
    fit = fit_of(parts[:n], torch.device("cuda:0"))
    print(f"[gpu] calibration set: {n} events, {fit.n_tracks} tracks, {int(fit.hit_off[-1])} hits", flush=True)
    return trk, fit, synth.draw_theta().flat()


@pytest.fixture(scope="module")
def dataset(events):
    return _dataset(events, NEV)


@pytest.fixture(scope="module")
def dataset_newton(events):
    return _dataset(events, NEV_NEWTON)


SPREAD = np.array([2e-3, 0.1] + [0.3 / np.sqrt(3.0)] * 64)   # injected spread per parameter kind
DRIFT_L = 250.0


def blocks(v):
    return np.concatenate([v[:S, None], v[S:2 * S, None], v[2 * S:].reshape(S, 64)], 1)


def identifiable_subspace(trk, fit):
    """Per sector: eigenvectors (in units of the injected spread) of the
    chi2 Hessian at theta = 0 whose statistical error is <= 0.1 spread."""
    from paper_1712_09434_amd.calib import sector_hessian
    H = sector_hessian(trk, fit, torch.zeros(S * 66, dtype=torch.float64, device="cuda:0")).cpu().numpy()
    D = np.diag(SPREAD)
    out = []
    for s in range(S):
        w, V = np.linalg.eigh(0.5 * (D @ H[s] @ D + (D @ H[s] @ D).T))
        out.append(V[:, np.sqrt(2.0 / np.maximum(w, 1e-300)) <= 0.1])
    return out


@pytest.fixture(scope="module")
def identifiable(dataset):
    return identifiable_subspace(*dataset[:2])


@pytest.fixture(scope="module")
def identifiable_newton(dataset_newton):
    return identifiable_subspace(*dataset_newton[:2])


def subspace_error(theta, theta_star, P):
    u, us = blocks(theta) / SPREAD, blocks(theta_star) / SPREAD
    num = sum(np.sum((P[s].T @ (u[s] - us[s])) ** 2) for s in range(S))
    den = sum(np.sum((P[s].T @ us[s]) ** 2) for s in range(S))
    return float(np.sqrt(num / den))


def offset_error(theta, theta_star):
    o = lambda a: a[:, 1] - DRIFT_L * a[:, 0]
    return float(np.abs(o(blocks(theta)) - o(blocks(theta_star))).max())


def test_adam_50_steps_recover_injected_miscalibration(dataset, identifiable):
    """50 Adam steps from theta = 0 in prior-scaled Hessian eigen-coordinates
    (the Hessian from 132 gradient calls at theta = 0)."""
    from paper_1712_09434_amd import calibrate
    from paper_1712_09434_amd.calib import default_prior_sigma, map_objective
    trk, fit, theta_star = dataset
    sig = default_prior_sigma(S, "cuda:0")
    f_star = map_objective(trk, fit, torch.from_numpy(theta_star).to("cuda:0"), sig)[0]
    theta, hist, _ = calibrate(trk, fit, steps=50, precondition="eigen", lr_white=0.6, lr_final=1e-3,
                               betas=(0.8, 0.999), prior_sigma=sig)
    th = theta.cpu().numpy()
    zero = np.zeros_like(th)
    sub, sub0 = subspace_error(th, theta_star, identifiable), subspace_error(zero, theta_star, identifiable)
    off, off0 = offset_error(th, theta_star), offset_error(zero, theta_star)
    print(f"[gpu] adam 50: f {hist[0]:.0f} -> {hist[-1]:.0f} (truth {f_star:.0f}); identifiable-subspace "
          f"error {sub0:.3f} -> {sub:.3f}; max drift-offset error {off0:.3f} -> {off:.4f} cm", flush=True)
    assert len(hist) == 50
    assert hist[-1] <= f_star * (1.0 + 1e-3)     # at least as good a fit as the truth
    assert off <= 0.05                           # drift offset: 10 % of its spread (~0.5 cm)
    assert sub <= 0.3 * sub0                     # identifiable subspace: 70 % of the error removed


def test_newton_map_recovers_injected_miscalibration(dataset_newton, identifiable_newton):
    from paper_1712_09434_amd import calibrate_newton
    from paper_1712_09434_amd.calib import default_prior_sigma, map_objective
    trk, fit, theta_star = dataset_newton
    identifiable = identifiable_newton
    sig = default_prior_sigma(S, "cuda:0")
    f_star = map_objective(trk, fit, torch.from_numpy(theta_star).to("cuda:0"), sig)[0]
    theta, hist = calibrate_newton(trk, fit, iters=5, prior_sigma=sig)
    th = theta.cpu().numpy()
    zero = np.zeros_like(th)
    sub, sub0 = subspace_error(th, theta_star, identifiable), subspace_error(zero, theta_star, identifiable)
    off, off0 = offset_error(th, theta_star), offset_error(zero, theta_star)
    print(f"[gpu] newton: f {hist[0]:.0f} -> {hist[-1]:.0f} (truth {f_star:.0f}); identifiable-subspace "
          f"error {sub0:.3f} -> {sub:.3f}; max drift-offset error {off0:.3f} -> {off:.4f} cm", flush=True)
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert hist[-1] <= f_star * (1.0 + 1e-3)     # at least as good a fit as the truth
    assert off <= 0.05                           # drift offset: 10 % of its spread (~0.5 cm)
    assert sub <= 0.3 * sub0                     # identifiable subspace: 70 % of the error removed


def test_adam_lowers_the_objective(dataset):
    from paper_1712_09434_amd import calibrate
    from paper_1712_09434_amd.calib import default_prior_sigma, map_objective
    trk, fit, theta_star = dataset
    sig = default_prior_sigma(S, "cuda:0")
    f_star = map_objective(trk, fit, torch.from_numpy(theta_star).to("cuda:0"), sig)[0]
    theta, hist, _ = calibrate(trk, fit, steps=100, precondition=True, lr_white=100.0, lr_final=0.1,
                               prior_sigma=sig)
    gap = (hist[0] - hist[-1]) / (hist[0] - f_star)
    off, off0 = offset_error(theta.cpu().numpy(), theta_star), offset_error(np.zeros(S * 66), theta_star)
    print(f"[gpu] whitened adam: f {hist[0]:.0f} -> {hist[-1]:.0f} (truth {f_star:.0f}), {100 * gap:.0f} % of "
          f"the gap; max drift-offset error {off0:.3f} -> {off:.3f} cm", flush=True)
    assert gap >= 0.8
    assert off < off0


def test_resume_from_checkpoint(dataset, tmp_path):
    from paper_1712_09434_amd.calib import calibrate, load_state, save_state
    trk, fit, theta_star = dataset
    _, h_all, st_all = calibrate(trk, fit, steps=6, lr=LR)
    _, h1, st1 = calibrate(trk, fit, steps=3, lr=LR)
    save_state(str(tmp_path / "adam.npz"), st1)
    st2 = load_state(str(tmp_path / "adam.npz"), fit.hit_off.device)
    _, h2, st2 = calibrate(trk, fit, steps=3, lr=LR, state=st2)
    assert h1 + h2 == h_all
    assert torch.equal(st2["u"], st_all["u"])
