"""Checks of the synthetic event generator (input side only)."""
import numpy as np

import synth


def test_noiseless_clusters_inside_acceptance_and_on_rows():
    ev = synth.make_event(seed=3, n_primaries=500, smear=False)
    X = ev.geom.row_x
    assert np.all(ev.x == X[ev.row])
    assert np.all(np.abs(ev.y64) <= X[ev.row].astype(np.float64) * np.tan(np.deg2rad(10)) + 1e-9)
    assert np.all(np.abs(ev.z64) <= 250.0)
    a_side = ev.sector < 18
    assert np.all(ev.z64[a_side] >= 0) and np.all(ev.z64[~a_side] < 0)


def test_clusters_lie_on_the_generating_circle():
    ev = synth.make_event(seed=4, n_primaries=50, smear=False, shuffle=False)
    tr = ev.tracks
    for i in range(50):
        m = np.nonzero(ev.truth_track == i)[0]
        if len(m) == 0:
            continue
        w = ev.sector[m] % 18
        a = (w + 0.5) * np.deg2rad(20.0)
        gx = ev.x64[m] * np.cos(a) - ev.y64[m] * np.sin(a)
        gy = ev.x64[m] * np.sin(a) + ev.y64[m] * np.cos(a)
        R = tr['pt'][i] / (synth.events.C_LIGHT * 0.5)
        # centre of the circle through the origin, tangent direction phi0
        kap = -tr['q'][i] / R
        cx, cy = -np.sin(tr['phi0'][i]) / kap, np.cos(tr['phi0'][i]) / kap
        np.testing.assert_allclose(np.hypot(gx - cx, gy - cy), R, rtol=1e-10)


def test_sizes_and_determinism():
    a = synth.make_config('C1'); b = synth.make_config('C1')
    np.testing.assert_array_equal(a.x, b.x)
    assert 10000 < a.n < 30000
    assert np.all(a.sector == 0)


def test_bspline_partition_of_unity():
    u = np.linspace(-0.1, 1.1, 1001)
    B = synth.bspline_basis(u)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(B >= 0)
