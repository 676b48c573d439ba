"""Pins of the oracle's FP32 input correction (calib_apply32), the one the
tracker applies to its clusters when a calibration is installed.

* theta = 0 leaves every cluster bit for bit unchanged (the corrections are
  added to the coordinates).
* Against the FP64 correction (calib_apply, pinned by test_oracle_calib.py)
  on miscalibrated events: within a few FP32 ulps of the coordinate.
* Against the generator's own inverse (independent B-splines, FP64 fixed
  point): the correction of a miscalibrated event returns the clean
  clusters to within FP32 rounding.
* The FP32 basis (de Boor's recursion, reached through a map that is 1 in
  one coefficient) equals the generator's FP64 Cox-de Boor basis to FP32
  accuracy, and a map of all ones moves every cluster by 1 (partition of
  unity).
* Planted mistakes (the drift side flipped, tau dropped, the radial basis
  evaluated at the corrected x) break the FP64 agreement.
* Tracking the miscalibrated event with the injected calibration installed
  brings the median chi2/ndf of its tracks back to the clean event's.
"""
import numpy as np
import pytest

import synth

S = 36


def _f32(ev):
    return ev.x.astype(np.float32), ev.y.astype(np.float32), ev.z.astype(np.float32)


@pytest.fixture(scope="module")
def miscal():
    theta = synth.draw_theta(1234)
    ev = synth.make_event(seed=9, n_primaries=400, noise=0.02, theta=theta)
    clean = synth.make_event(seed=9, n_primaries=400, noise=0.02)
    return ev, clean, theta


def test_zero_theta_is_bitwise_identity(orc):
    ev = synth.make_config('C1')
    x, y, z = _f32(ev)
    xo, zo = orc.calib_apply32(ev, ev.sector, x, y, z, np.zeros(S * 66, np.float32))
    assert np.array_equal(xo.view(np.uint32), x.view(np.uint32))
    assert np.array_equal(zo.view(np.uint32), z.view(np.uint32))


def test_matches_fp64_correction(orc, miscal):
    ev, clean, theta = miscal
    x, y, z = _f32(ev)
    th = theta.flat().astype(np.float32)
    xo, zo = orc.calib_apply32(ev, ev.sector, x, y, z, th)
    xr, zr = orc.calib_apply(ev, ev.sector, x.astype(float), y.astype(float), z.astype(float),
                             th.astype(float))
    ulp_x = np.spacing(np.abs(xr).astype(np.float32)).astype(float)
    ulp_z = np.spacing(np.maximum(np.abs(zr), 1.0).astype(np.float32)).astype(float)
    assert np.all(np.abs(xo - xr) <= 2 * ulp_x), np.abs(xo - xr).max()
    assert np.all(np.abs(zo - zr) <= 2 * ulp_z), np.abs(zo - zr).max()
    assert np.abs(xo - x).max() > 0.05 and np.abs(zo - z).max() > 0.05   # it really corrected


def test_undoes_the_generators_miscalibration(orc, miscal):
    ev, clean, theta = miscal
    x, y, z = _f32(ev)
    xo, zo = orc.calib_apply32(ev, ev.sector, x, y, z, theta.flat())
    # FP32 inputs (rounded after the FP64 inverse) and FP32 arithmetic: a few ulps of 250 cm
    np.testing.assert_allclose(xo, clean.x64, atol=1e-4)
    np.testing.assert_allclose(zo, clean.z64, atol=1e-4)


def test_basis_and_partition_of_unity(orc):
    rng = np.random.default_rng(3)
    n = 20000
    geom = synth.default_geometry()
    sec = np.zeros(n, np.uint8)
    X = geom.row_x.astype(np.float64)
    x = rng.uniform(X[0], X[-1], n).astype(np.float32)
    tan_a = float(geom.tan_half_angle)
    y = (x * rng.uniform(-tan_a, tan_a, n)).astype(np.float32)
    z = rng.uniform(0, 240, n).astype(np.float32)
    xh = (x.astype(float) - X[0]) / (X[-1] - X[0])
    uh = (y.astype(float) / x + tan_a) / (2 * tan_a)
    Ba, Bb = synth.bspline_basis(xh), synth.bspline_basis(uh)
    for a, b in ((0, 0), (3, 5), (7, 7), (2, 6)):
        th = np.zeros(S * 66, np.float32)
        th[2 * S + a * 8 + b] = 1.0
        xo, _ = orc.calib_apply32(geom, sec, x, y, z, th)
        np.testing.assert_allclose(xo.astype(float) - x, Ba[:, a] * Bb[:, b], atol=3e-5)
    th = np.zeros(S * 66, np.float32)
    th[2 * S:2 * S + 64] = 1.0
    xo, _ = orc.calib_apply32(geom, sec, x, y, z, th)
    np.testing.assert_allclose(xo.astype(float) - x, 1.0, atol=3e-5)


def test_planted_mistakes_break_the_fp64_agreement(orc, miscal):
    """The FP64 reference computed with a plausible mistake differs from the
    FP32 correction by far more than the tolerance of the check above."""
    ev, clean, theta = miscal
    x, y, z = _f32(ev)
    th = theta.flat().astype(np.float32)
    xo, zo = orc.calib_apply32(ev, ev.sector, x, y, z, th)
    xd, yd, zd = x.astype(float), y.astype(float), z.astype(float)
    side = np.where(ev.sector < S // 2, 1.0, -1.0)
    dl, tau = th[:S][ev.sector].astype(float), th[S:2 * S][ev.sector].astype(float)
    L = float(ev.geom.z_max)
    good = z + side * (tau - dl * ((L - side * zd) - tau))
    flipped = z - side * (tau - dl * ((L + side * zd) - tau))
    no_tau = z + side * (-dl * (L - side * zd))
    assert np.abs(zo - good).max() < 1e-4
    assert np.abs(zo - flipped).max() > 0.05 and np.abs(zo - no_tau).max() > 0.05
    # radial basis at the corrected instead of the uncorrected x
    xr, _ = orc.calib_apply(ev, ev.sector, xd, yd, zd, th.astype(float))
    xr2, _ = orc.calib_apply(ev, ev.sector, xr, yd, zd, th.astype(float))
    shifted = xd + (xr2 - xr)
    assert np.abs(xo - shifted).max() > 1e-3


def test_tracking_the_corrected_event(orc, miscal):
    """Tracking with the injected calibration installed: the median fit
    quality of the found tracks returns to that of the clean event (the
    smooth miscalibration raises it by a few per cent only: most of it is
    absorbed by the track parameters)."""
    ev, clean, theta = miscal
    q = lambda r: float(np.median(r['chi2'] / np.maximum(r['ndf'], 1)))
    r_raw = orc.track(ev, precision=32)
    r_cor = orc.track(ev, precision=32, theta=theta.flat())
    r_cln = orc.track(clean, precision=32)
    excess = q(r_raw) - q(r_cln)
    assert excess > 0.02
    assert abs(q(r_cor) - q(r_cln)) < 0.1 * excess
    assert abs(len(r_cor['chi2']) - len(r_cln['chi2'])) <= 0.02 * len(r_cln['chi2'])
