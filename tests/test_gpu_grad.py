"""GPU parity of tpcca_refit_grad against the oracle's FP64 gradient.

The oracle's gradient is exact reverse-mode differentiation of the FP64
objective and is itself pinned by central finite differences
(test_oracle_calib.py).  The GPU computes the same objective in FP32 with a
hand-written adjoint and reduces in FP64.  Bar: chi2 within 1e-4 relative;
per parameter group ||g - g_ref|| <= 1e-3 ||g_ref||; every component within
1e-3 of the group's largest component.
"""
import numpy as np
import pytest
import torch

import synth
from calibset import calib_subset

pytestmark = pytest.mark.gpu
S = 36


def to_dev(ev, dev="cuda:0"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t(ev.x), t(ev.y), t(ev.z), t(ev.row), t(ev.sector)


@pytest.fixture(scope="module")
def setup():
    from paper_1712_09434_amd import FitTracks, Tracker
    theta_star = synth.draw_theta(77)
    ev = synth.make_event(seed=31, n_primaries=600, noise=0.01, theta=theta_star)
    trk = Tracker.from_geometry(ev.geom)
    cl = to_dev(ev)
    out = trk.track(*cl)
    off = out.hit_off.cpu().numpy().astype(np.int64)
    ids = out.hit_id.cpu().numpy().astype(np.int64)
    cs = calib_subset(ev, off, ids, out.sector.cpu().numpy(), out.chi2.cpu().numpy(),
                      out.ndf.cpu().numpy(), out.k_prior.cpu().numpy())
    cs['k0'] = cs['k0'].astype(np.float32).astype(np.float64)
    cs['ext_tgl'] = cs['ext_tgl'].astype(np.float32).astype(np.float64)
    d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).cuda()
    fit = FitTracks(clusters=cl, hit_off=d(cs['hit_off'], np.int32), hit_id=d(cs['hit_ids'], np.int32),
                    k_prior=d(cs['k0'], np.float32), ext_tgl=d(cs['ext_tgl'], np.float32),
                    use_vertex=d(cs['use_vertex'], np.uint8))
    print(f"[gpu] gradient set: {fit.n_tracks} tracks, {len(cs['hit_ids'])} hits", flush=True)
    yield ev, trk, fit, cs, theta_star
    trk.close()


def oracle_grad(orc, ev, cs, theta):
    th = np.asarray(theta, np.float32).astype(np.float64)
    return orc.calib_chi2(ev.geom, ev.x.astype(np.float64), ev.y.astype(np.float64),
                          ev.z.astype(np.float64), ev.sector, cs['hit_off'], cs['hit_ids'], cs['k0'], th,
                          ext_tgl=cs['ext_tgl'], use_vertex=cs['use_vertex'], grad=True)


def check_groups(g, ref):
    for name, sl in (("drift", slice(0, S)), ("offset", slice(S, 2 * S)), ("map", slice(2 * S, 66 * S))):
        a, b = g[sl], ref[sl]
        nb = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 1e-3 * nb + 1e-9, (name, np.linalg.norm(a - b) / nb)
        assert np.all(np.abs(a - b) <= 1e-3 * np.abs(b).max() + 1e-9), name


@pytest.mark.parametrize("where", ["zero", "half", "truth"])
def test_gradient_matches_oracle(setup, orc, where):
    ev, trk, fit, cs, theta_star = setup
    th = {"zero": np.zeros(S * 66), "half": 0.5 * theta_star.flat(), "truth": theta_star.flat()}[where]
    c2, ndf, g = trk.refit_grad(fit, torch.from_numpy(th.astype(np.float32)).cuda())
    rc2, rndf, _, rg = oracle_grad(orc, ev, cs, th)
    assert ndf == rndf
    assert abs(c2 - rc2) <= 1e-4 * rc2, (c2, rc2)
    if where != "truth":
        check_groups(g.cpu().numpy(), rg)
    else:   # near the optimum the gradient is mostly noise: compare on the scale of theta = 0
        _, _, _, g0 = oracle_grad(orc, ev, cs, np.zeros(S * 66))
        assert np.linalg.norm(g.cpu().numpy() - rg) <= 1e-3 * np.linalg.norm(g0)


def test_checkpoint_stride_does_not_change_results(setup):
    ev, trk, fit, cs, theta_star = setup
    th = torch.from_numpy((0.3 * theta_star.flat()).astype(np.float32)).cuda()
    ref = None
    for K in (1, 5, 12, 40, 160):
        trk.set_tuning(ckpt_every=K)
        c2, ndf, g = trk.refit_grad(fit, th)
        if ref is None:
            ref = (c2, g)
        else:
            assert c2 == ref[0] and torch.equal(g, ref[1]), K
    trk.set_tuning(ckpt_every=160)


def test_deterministic_and_host_mode(setup):
    ev, trk, fit, cs, theta_star = setup
    from paper_1712_09434_amd import FitTracks
    th = torch.from_numpy((0.3 * theta_star.flat()).astype(np.float32)).cuda()
    a = trk.refit_grad(fit, th)
    b = trk.refit_grad(fit, th)
    assert a[0] == b[0] and torch.equal(a[2], b[2])
    hfit = FitTracks(clusters=tuple(t.cpu() for t in fit.clusters), hit_off=fit.hit_off.cpu(),
                     hit_id=fit.hit_id.cpu(), k_prior=fit.k_prior.cpu(), ext_tgl=fit.ext_tgl.cpu(),
                     use_vertex=fit.use_vertex.cpu())
    h = trk.refit_grad(hfit, th.cpu())
    assert h[0] == a[0] and torch.equal(h[2], a[2].cpu())


def test_autograd_function(setup):
    from paper_1712_09434_amd import Chi2Refit
    ev, trk, fit, cs, theta_star = setup
    th = torch.zeros(S * 66, dtype=torch.float64, device="cuda:0", requires_grad=True)
    chi2 = Chi2Refit.apply(th, trk, fit)
    chi2.backward()
    _, _, g = trk.refit_grad(fit, th.detach())
    assert torch.equal(th.grad, g)


def test_empty_track_set(setup):
    from paper_1712_09434_amd import FitTracks
    ev, trk, fit, cs, theta_star = setup
    empty = FitTracks(clusters=fit.clusters, hit_off=torch.zeros(1, dtype=torch.int32, device="cuda:0"),
                      hit_id=torch.zeros(1, dtype=torch.int32, device="cuda:0"),
                      k_prior=torch.zeros(1, device="cuda:0"), ext_tgl=None, use_vertex=None)
    c2, ndf, g = trk.refit_grad(empty, torch.zeros(S * 66, device="cuda:0"))
    assert c2 == 0.0 and ndf == 0 and torch.count_nonzero(g) == 0


def test_bad_hit_ids_rejected(setup):
    from paper_1712_09434_amd import FitTracks, TpccaError
    ev, trk, fit, cs, theta_star = setup
    bad_ids = fit.hit_id.clone()
    bad_ids[3] = ev.n + 5
    bad = FitTracks(clusters=fit.clusters, hit_off=fit.hit_off, hit_id=bad_ids, k_prior=fit.k_prior,
                    ext_tgl=fit.ext_tgl, use_vertex=fit.use_vertex)
    with pytest.raises(TpccaError):
        trk.refit_grad(bad, torch.zeros(S * 66, device="cuda:0"))
