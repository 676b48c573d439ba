"""Pins of the oracle's Kalman filter.

* One update equals Gaussian conditioning written in information form.
* The chi2 increment equals r^T (H C H^T + V)^-1 r.
* A noiseless helix, with the filter started at its true state, stays on the
  generator's exact helix (independent helix code) to 1e-9.
* Over many smeared tracks the pulls are ~N(0,1) and <chi2/ndf> ~ 1.
"""
import numpy as np

import synth


def test_update_equals_information_form(orc):
    rng = np.random.default_rng(11)
    iu = np.triu_indices(5)
    H = np.zeros((2, 5)); H[0, 0] = H[1, 1] = 1
    for _ in range(30):
        A = rng.normal(size=(5, 5)); Cm = A @ A.T + 0.1 * np.eye(5)
        p = rng.normal(size=5)
        m = rng.normal(size=2)
        V = np.diag([0.01, 0.0225])
        op, oc, c2 = orc.kf_update(p, Cm[iu], m[0], m[1], V[0, 0], V[1, 1])
        Ci = np.linalg.inv(Cm)
        Pinv = Ci + H.T @ np.linalg.inv(V) @ H
        Pn = np.linalg.inv(Pinv)
        mean = Pn @ (Ci @ p + H.T @ np.linalg.inv(V) @ m)
        np.testing.assert_allclose(op, mean, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(oc, Pn[iu], rtol=1e-8, atol=1e-10)
        r = m - H @ p
        S = H @ Cm @ H.T + V
        np.testing.assert_allclose(c2, r @ np.linalg.solve(S, r), rtol=1e-10)


def truth_state(tr, i, alpha, x):
    """Local state (y, z, sin phi, tan lambda, q/pT) of truth track i at the
    plane x of the sector frame rotated by alpha (outgoing leg)."""
    kap = -synth.events.C_LIGHT * 0.5 * tr['q'][i] / tr['pt'][i]
    xv = tr['xv'][i] * np.cos(alpha) + tr['yv'][i] * np.sin(alpha)
    yv = -tr['xv'][i] * np.sin(alpha) + tr['yv'][i] * np.cos(alpha)
    psi0 = tr['phi0'][i] - alpha
    v = np.sin(psi0) + kap * (x - xv)
    th = np.arcsin(v)
    dpsi = (th - psi0) if kap > 0 else (psi0 - th)
    dpsi = np.mod(dpsi, 2 * np.pi)
    ell = dpsi / abs(kap)
    y = yv - (np.cos(th) - np.cos(psi0)) / kap
    z = tr['zv'][i] + np.sinh(tr['eta'][i]) * ell
    return np.array([y, z, v, np.sinh(tr['eta'][i]), tr['q'][i] / tr['pt'][i]])


def test_noiseless_helix_filter_stays_on_truth(orc):
    ev = synth.make_event(seed=5, n_primaries=40, single_sector=True, smear=False, shuffle=False,
                          pt_range=(0.3, 10.0))
    alpha = np.deg2rad(10.0)
    iu = np.triu_indices(5)
    checked = 0
    for i in range(40):
        m = np.nonzero(ev.truth_track == i)[0]
        if len(m) < 30:
            continue
        order = m[np.argsort(-ev.row[m])]            # outermost first
        x = ev.x64[order]
        st = truth_state(ev.tracks, i, alpha, x[0])
        assert abs(st[0] - ev.y64[order[0]]) < 1e-9
        p = st.copy()
        cv = np.diag([0.01, 0.0225, 0.25, 0.25, 100.0])[iu]
        for h in range(1, len(order)):
            ok, p, cv, _ = orc.transport(p, cv, x[h - 1], x[h])
            assert ok
            p, cv, c2 = orc.kf_update(p, cv, ev.y64[order[h]], ev.z64[order[h]], 0.01, 0.0225)
            assert c2 < 1e-12
        ref = truth_state(ev.tracks, i, alpha, x[-1])
        np.testing.assert_allclose(p, ref, rtol=1e-9, atol=1e-9)
        checked += 1
    assert checked >= 10


def test_fit_pulls_and_chi2(orc):
    ev = synth.make_event(seed=77, n_primaries=600, single_sector=True, shuffle=False,
                          pt_range=(0.5, 10.0))
    alpha = np.deg2rad(10.0)
    pulls, q = [], []
    for i in range(600):
        m = np.nonzero(ev.truth_track == i)[0]
        if len(m) < 60:
            continue
        order = m[np.argsort(-ev.row[m])]
        k0 = ev.tracks['q'][i] / ev.tracks['pt'][i]
        ok, p, cv, c2 = orc.fit_hits(ev.geom, ev.x64[order], ev.y64[order], ev.z64[order], k0)
        assert ok
        ref = truth_state(ev.tracks, i, alpha, ev.x64[order[-1]])
        Cm = np.zeros((5, 5)); Cm[np.triu_indices(5)] = cv; Cm = Cm + np.triu(Cm, 1).T
        pulls.append((p - ref) / np.sqrt(np.diag(Cm)))
        q.append(c2 / (2 * len(order) - 5))
    pulls = np.array(pulls)
    assert len(pulls) > 200
    assert abs(np.mean(q) - 1.0) < 0.05
    np.testing.assert_array_less(np.abs(pulls.mean(axis=0)), 0.2)
    sd = pulls.std(axis=0)
    assert np.all(sd > 0.85) and np.all(sd < 1.15), sd
