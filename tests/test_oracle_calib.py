"""Pins of the oracle's calibration correction and chi2(theta) gradient.

* theta = 0 is the identity; the B-spline basis is a partition of unity.
* The generator's inverse calibration (its own Cox-de Boor B-splines and a
  fixed-point inverse) followed by the oracle's correction is the identity.
* The reverse-mode gradient of the FP64 objective equals central finite
  differences of the same objective.
* At the injected truth on noiseless data, chi2 and the gradient are tiny
  compared with their values at theta = 0.
"""
import numpy as np
import pytest

import synth
from calibset import calib_subset


def test_identity_and_partition_of_unity(orc):
    ev = synth.make_config('C1')
    th = np.zeros(orc.NPAR)
    xo, zo = orc.calib_apply(ev, ev.sector, ev.x64, ev.y64, ev.z64, th)
    np.testing.assert_array_equal(xo, ev.x64)
    np.testing.assert_allclose(zo, ev.z64, atol=1e-12)
    th[72:72 + 64] = 1.0                    # sector 0 map all ones
    xo, _ = orc.calib_apply(ev, ev.sector, ev.x64, ev.y64, ev.z64, th)
    np.testing.assert_allclose(xo, ev.x64 + 1.0, atol=1e-12)


def test_inverse_round_trip(orc):
    theta = synth.draw_theta(1234)
    ev = synth.make_event(seed=9, n_primaries=300, theta=theta)
    clean = synth.make_event(seed=9, n_primaries=300)
    xo, zo = orc.calib_apply(ev, ev.sector, ev.x64, ev.y64, ev.z64, theta.flat())
    np.testing.assert_allclose(xo, clean.x64, atol=1e-9)
    np.testing.assert_allclose(zo, clean.z64, atol=1e-9)
    assert np.abs(ev.x64 - clean.x64).max() > 0.05       # the map really moved clusters


@pytest.fixture(scope="module")
def small_calib(orc):
    theta = synth.draw_theta(77, sd_delta=2e-3, sd_tau=0.1, amp=0.3)
    ev = synth.make_event(seed=31, n_primaries=400, noise=0.0, theta=theta)
    r = orc.track(ev, precision=32)
    k_prior = r['seed_state'][r['trk_seed'], 4]
    cs = calib_subset(ev, r['hit_off'], r['hit_ids'], r['sector'], r['chi2'], r['ndf'],
                      np.concatenate([k_prior, [0]])[np.arange(len(r['trk_seed']))], max_tracks=60)
    return ev, theta, cs


def _chi2(orc, ev, cs, th, grad=False):
    return orc.calib_chi2(ev.geom, ev.x64, ev.y64, ev.z64, ev.sector, cs['hit_off'], cs['hit_ids'],
                          cs['k0'], th, ext_tgl=cs['ext_tgl'], use_vertex=cs['use_vertex'], grad=grad)


def test_gradient_matches_finite_differences(orc, small_calib):
    ev, theta, cs = small_calib
    assert len(cs['k0']) >= 30
    rng = np.random.default_rng(4)
    th = theta.flat() * 0.5 + rng.normal(0, 1e-4, orc.NPAR)
    c2, ndf, _, g = _chi2(orc, ev, cs, th, grad=True)
    secs = np.unique(ev.sector[cs['hit_ids']])
    s = int(secs[0])
    idx = [s, 36 + s] + [72 + s * 64 + k for k in (0, 9, 18, 27, 36, 45, 54, 63)]
    for i in idx:
        h = 1e-6 if i < 36 else 1e-5
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd = (_chi2(orc, ev, cs, tp)[0] - _chi2(orc, ev, cs, tm)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i])) + 1e-4 * np.abs(g).max() * 1e-2, (i, fd, g[i])
    # parameters of sectors without tracks have zero gradient
    empty = [k for k in range(36) if k not in set(secs.tolist())]
    if empty:
        assert g[empty[0]] == 0.0


def test_truth_is_near_stationary_on_noiseless_data(orc):
    theta = synth.draw_theta(55)
    ev = synth.make_event(seed=41, n_primaries=300, noise=0.0, smear=False, theta=theta)
    r = orc.track(ev, precision=32)
    k_prior = r['seed_state'][r['trk_seed'], 4]
    cs = calib_subset(ev, r['hit_off'], r['hit_ids'], r['sector'], r['chi2'], np.maximum(r['ndf'], 1),
                      k_prior, max_q=1e9, max_tracks=80)
    cs['ext_tgl'] = ev.tracks['tgl'][cs['truth']]           # noiseless external reference
    assert len(cs['k0']) >= 40
    c0, _, _, g0 = _chi2(orc, ev, cs, np.zeros(orc.NPAR), grad=True)
    c1, _, _, g1 = _chi2(orc, ev, cs, theta.flat(), grad=True)
    assert c1 < 1e-3 * c0, (c0, c1)
    assert np.linalg.norm(g1) < 1e-2 * np.linalg.norm(g0)
