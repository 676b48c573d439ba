"""Pins of the oracle's sector track merger (segments of one track in
adjacent sectors joined and refitted as one track).

* Rotation of a state into another sector's frame: the same point and
  direction computed from first principles in both frames; the Jacobian
  against central finite differences (of the rotation followed by the
  transport back to the fixed new plane); rotating back is the identity.
* A noiseless helix crossing a sector boundary: tracked as two segments,
  merged into one track with all hits, whose refit has chi2 ~ 0 and the
  true q/pT and tan(lambda).
* On a full event (5,000 primaries): every kept link joins two segments of
  one injected particle, and nearly every particle found as two segments in
  adjacent sectors is joined; the merged tracks' median chi2/ndf is 1.
* A planted mistake (the turn of the frame taken with the wrong sign)
  breaks the first-principles rotation check.
"""
import numpy as np
import pytest

import synth
import truth

D20 = np.deg2rad(20.0)


def frame(X, Y, psi, alpha):
    """Point (X, Y) and direction angle psi (global) in the frame of a sector centred at alpha."""
    ca, sa = np.cos(alpha), np.sin(alpha)
    return X * ca + Y * sa, -X * sa + Y * ca, np.sin(psi - alpha)


@pytest.mark.parametrize("turn", [D20, -D20, 3 * D20])
def test_rotation_from_first_principles(orc, turn):
    rng = np.random.default_rng(5)
    for _ in range(50):
        r, phi = rng.uniform(90, 240), rng.uniform(-0.15, 0.15)
        X, Y = r * np.cos(phi), r * np.sin(phi)
        psi = phi + rng.uniform(-0.4, 0.4)
        x1, y1, s1 = frame(X, Y, psi, 0.0)
        x2, y2, s2 = frame(X, Y, psi, turn)
        if abs(s2) >= 0.95:
            continue
        p = np.array([y1, rng.uniform(-100, 100), s1, rng.uniform(-1, 1), rng.uniform(-5, 5)])
        ok, xo, po, _, _ = orc.rotate(x1, p, np.eye(5)[np.triu_indices(5)], turn)
        assert ok
        np.testing.assert_allclose([xo, po[0], po[2]], [x2, y2, s2], atol=1e-10)
        np.testing.assert_array_equal(po[[1, 3, 4]], p[[1, 3, 4]])
        # the planted mistake: the turn with the wrong sign
        _, xw, pw, _, _ = orc.rotate(x1, p, np.eye(5)[np.triu_indices(5)], -turn)
        assert abs(pw[0] - y2) > 1.0 or abs(xw - x2) > 1.0


def test_rotation_jacobian_and_inverse(orc):
    rng = np.random.default_rng(6)
    iu = np.triu_indices(5)
    for _ in range(20):
        x = rng.uniform(90, 240)
        p = np.array([rng.uniform(-0.15, 0.15) * x, rng.uniform(-100, 100), rng.uniform(-0.5, 0.5),
                      rng.uniform(-1, 1), rng.uniform(-5, 5)])
        A = rng.normal(size=(5, 5)) * np.array([0.1, 0.1, 0.01, 0.01, 0.1])
        cov = (A @ A.T + 1e-6 * np.eye(5))[iu]
        turn = rng.choice([D20, -D20])
        ok, x2, p2, c2, J = orc.rotate(x, p, cov, turn)
        assert ok

        def at_plane(q):
            ok, xq, pq, cq, _ = orc.rotate(x, q, cov, turn)
            ok2, pt, _, _ = orc.transport(pq, cq, xq, x2)
            assert ok and ok2
            return pt

        for j in range(5):
            h = 1e-6 * max(1.0, abs(p[j]))
            e = np.zeros(5); e[j] = h
            fd = (at_plane(p + e) - at_plane(p - e)) / (2 * h)
            np.testing.assert_allclose(J[:, j], fd, rtol=1e-6, atol=1e-7, err_msg=f"column {j}")
        C2 = np.zeros((5, 5)); C2[iu] = c2; C2 = C2 + np.triu(C2, 1).T
        C1 = np.zeros((5, 5)); C1[iu] = cov; C1 = C1 + np.triu(C1, 1).T
        np.testing.assert_allclose(C2, J @ C1 @ J.T, rtol=1e-12, atol=1e-15)
        ok, x3, p3, c3, _ = orc.rotate(x2, p2, c2, -turn)
        assert ok
        np.testing.assert_allclose(x3, x, atol=1e-10)
        np.testing.assert_allclose(p3, p, atol=1e-10)
        np.testing.assert_allclose(c3, cov, rtol=1e-9, atol=1e-14)


def crossing_event():
    """A noiseless single helix whose outgoing leg crosses from wedge 0 into
    wedge 1 with at least 20 clusters on each side."""
    for seed in range(200):
        ev = synth.make_event(seed=seed, n_primaries=1, smear=False, pt_range=(0.4, 2.0),
                              eta_range=(-0.5, 0.5), phi_range=(np.deg2rad(12), np.deg2rad(19)), shuffle=False)
        secs, cnt = np.unique(ev.sector, return_counts=True)
        if len(secs) == 2 and cnt.min() >= 20 and abs(int(secs[1]) - int(secs[0])) == 1:
            return ev
    raise AssertionError("no crossing helix found")


def test_noiseless_boundary_crossing_is_one_track(orc):
    ev = crossing_event()
    r = orc.track(ev, precision=32)
    assert len(r['x_ref']) == 2 and len(set(r['sector'].tolist())) == 2
    m = orc.merge(ev, r)
    assert len(m['x_ref']) == 1
    ids = np.sort(m['hit_ids'])
    np.testing.assert_array_equal(ids, np.sort(r['hit_ids']))
    rows = ev.row[m['hit_ids']]
    inner = m['sector'][0]
    # innermost segment's hits first, every pad row at most once, rows rising
    assert ev.sector[m['hit_ids'][0]] == inner and np.all(np.diff(rows) > 0)
    assert m['ndf'][0] == 2 * len(ids) - 5
    assert m['chi2'][0] < 1e-3, m['chi2'][0]
    k_true = ev.tracks['q'][0] / ev.tracks['pt'][0]
    assert abs(m['p'][0, 4] - k_true) <= 2e-4 * abs(k_true), (m['p'][0, 4], k_true)
    assert abs(m['p'][0, 3] - ev.tracks['tgl'][0]) <= 1e-5


@pytest.fixture(scope="module")
def full_event(orc):
    ev = synth.make_config("C2")
    r = orc.track(ev, precision=32)
    return ev, r, orc.merge(ev, r)


def test_links_join_one_particle(full_event):
    ev, r, m = full_event
    lab = truth.match_tracks(ev, r['hit_off'], r['hit_ids'], r['sector']) // 64
    links = [(a, b) for a, b in enumerate(m['link']) if b >= 0]
    assert len(links) > 1000
    bad = [(a, b) for a, b in links if lab[a] < 0 or lab[a] != lab[b]]
    assert len(bad) <= 1e-3 * len(links), bad[:5]
    # particles found as two segments in adjacent sectors of one side, rows in order
    first = ev.row[r['hit_ids'][r['hit_off'][:-1]]]
    last = ev.row[r['hit_ids'][r['hit_off'][1:] - 1]]
    sec = r['sector']
    joined = set(links)
    elig = found = 0
    order = np.argsort(lab, kind='stable')
    for i, j in zip(order[:-1], order[1:]):
        if lab[i] < 0 or lab[i] != lab[j]:
            continue
        a, b = (i, j) if last[i] < first[j] else (j, i)
        same_side = (sec[a] < 18) == (sec[b] < 18)
        adjacent = (sec[a] % 18 - sec[b] % 18) % 18 in (1, 17)
        if same_side and adjacent and last[a] < first[b]:
            elig += 1
            found += (a, b) in joined
    assert elig > 1000 and found >= 0.97 * elig, (found, elig)


def test_merged_tracks_fit_well(full_event):
    ev, r, m = full_event
    multi = np.array([len(set(ev.sector[m['hit_ids'][m['hit_off'][i]:m['hit_off'][i + 1]]].tolist())) > 1
                      for i in range(len(m['x_ref']))])
    assert multi.sum() > 1000
    q = m['chi2'][multi] / m['ndf'][multi]
    assert 0.9 < np.median(q) < 1.1
    # every merged track has at most one hit per pad row
    for i in np.nonzero(multi)[0][:500]:
        rows = ev.row[m['hit_ids'][m['hit_off'][i]:m['hit_off'][i + 1]]]
        assert np.all(np.diff(rows) > 0)
    assert len(m['x_ref']) == len(r['x_ref']) - int((m['link'] >= 0).sum())
