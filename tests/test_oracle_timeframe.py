"""Pins of the oracle's time-frame tracking (continuous readout, the frame
sliced along the time axis, slices tracked as events, their segments merged;
Sec. "Track reconstruction in the TPC").

* The slice's pseudo-coordinate follows from the generator's physics, not
  from the formula: z' = z - side (c - s D) for a cluster at z of a
  collision at c (FP64 truth), within FP32 rounding.
* Slice bounds: s D <= tau < (s + 1) D up to the FP32 quotient's rounding.
* One slice holding a whole collision at c = 0 reduces to tracking the
  event itself: the same tracks, hit for hit.
* On the small frame every merge link joins segments of one particle, the
  particles split by a slice boundary are rejoined, and the merged fits
  have chi2/ndf near 1; a planted sign error in the frame shift of the
  states breaks the joins.
"""
import numpy as np
import pytest

import oracle
import synth

L = 250.0


def _labels(tf, seg):
    ns = len(seg["x_ref"])
    lab = np.full(ns, -1)
    for i in range(ns):
        h = seg["hit_ids"][seg["hit_off"][i]:seg["hit_off"][i + 1]]
        t = tf.truth_track[h]
        t = t[t >= 0]
        if t.size:
            v, c = np.unique(t, return_counts=True)
            if c.max() >= 0.9 * len(h):
                lab[i] = v[np.argmax(c)]
    return lab


def test_pseudo_z_follows_the_collision_time():
    c = 300.0
    tf = synth.make_timeframe(seed=5, n_collisions=1, length=3 * L, times=[c], multiplicity=200, noise=0.0,
                              smear=False)
    s, zp = oracle.timeframe_slices(tf.geom, tf.tau, tf.sector, L)
    side = np.where(tf.sector < 18, 1.0, -1.0)
    want = tf.z64 - side * (c - s * L)
    assert set(np.unique(s)) <= {1, 2}
    np.testing.assert_allclose(zp.astype(np.float64), want, rtol=0, atol=1e-4)


def test_slice_bounds():
    tf = synth.make_tf_config("TF-small")
    D = np.float32(synth.TF_SLICE)
    s, _ = oracle.timeframe_slices(tf.geom, tf.tau, tf.sector, D)
    tau = tf.tau.astype(np.float64)
    ulp = np.spacing(np.float32(tf.length)).astype(np.float64)
    assert s.min() >= 0 and s.max() == 2
    assert np.all(s * float(D) - tau <= ulp)
    assert np.all(tau - (s + 1) * float(D) < ulp)


def test_single_slice_equals_event_tracking():
    tf = synth.make_timeframe(seed=77, n_collisions=1, length=2 * L, times=[0.0], multiplicity=400, noise=0.01)
    r = oracle.timeframe(tf, 2 * L, 1)
    ev = oracle._Clusters(tf.geom, tf.x, tf.y, tf.z64.astype(np.float32), tf.row, tf.sector)
    ref = oracle.track(ev, precision=32)
    a = r["seg"]
    assert len(a["x_ref"]) == len(ref["x_ref"]) > 300
    lists = lambda d: sorted(tuple(d["hit_ids"][d["hit_off"][i]:d["hit_off"][i + 1]]) for i in range(len(d["x_ref"])))
    assert lists(a) == lists(ref)
    assert np.all(r["slice"] == 0)


@pytest.fixture(scope="module")
def small_frame():
    tf = synth.make_tf_config("TF-small")
    return tf, oracle.timeframe(tf, synth.TF_SLICE, 3)


def _slice_pairs(tf, r):
    seg, sl = r["seg"], r["slice"]
    lab = _labels(tf, seg)
    byp = {}
    for i in range(len(lab)):
        if lab[i] >= 0:
            byp.setdefault((lab[i], seg["sector"][i]), []).append(i)
    return [tuple(v) for v in byp.values() if len(v) == 2 and abs(sl[v[0]] - sl[v[1]]) == 1], lab


def test_slice_split_particles_are_rejoined(small_frame):
    tf, r = small_frame
    seg, m = r["seg"], r["merged"]
    pairs, lab = _slice_pairs(tf, r)
    lk = m["link"]
    linked = [a for a in range(len(lk)) if lk[a] >= 0]
    assert all(lab[a] >= 0 and lab[a] == lab[lk[a]] for a in linked)          # every link joins one particle
    joined = sum(1 for a, b in pairs if lk[a] == b or lk[b] == a)
    assert len(pairs) >= 80 and joined >= 0.95 * len(pairs), (joined, len(pairs))
    slice_links = sum(1 for a in linked if seg["sector"][a] == seg["sector"][lk[a]])
    assert slice_links == joined
    q = m["chi2"] / np.maximum(m["ndf"], 1)
    assert 0.8 <= np.median(q) <= 1.25


def test_planted_sign_error_breaks_the_joins(small_frame):
    tf, r = small_frame
    seg = dict(r["seg"])
    side = np.where(seg["sector"] < 18, 1.0, -1.0)
    p = seg["p"].copy()
    p[:, 1] += 2.0 * side * r["slice"] * synth.TF_SLICE          # shift by +side s D instead of -side s D
    seg["p"] = p
    frame = oracle._Clusters(tf.geom, tf.x.astype(np.float64), tf.y.astype(np.float64), r["z_tf"], tf.row,
                             tf.sector)
    bad = oracle.merge(frame, seg, slices=r["slice"])
    lk = bad["link"]
    slice_links = sum(1 for a in range(len(lk)) if lk[a] >= 0 and seg["sector"][a] == seg["sector"][lk[a]])
    assert slice_links < 0.1 * len(_slice_pairs(tf, r)[0])
