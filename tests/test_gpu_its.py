"""GPU parity of the ITS standalone tracker (tpcca_its_track) against the
oracle (oracle.its), on the pp-like, minimum-bias-like and two
central-Pb-Pb-like events.

Both sides evaluate the same FP32 expressions, so the integer results are
compared exactly (vertexer histogram, pair count, peak, tracklets, accepted
tracks, their clusters, layers and staves) and so are the FP32 values (the
vertex z, chi2, the outward and inward states and covariances).  The
vertex fit sums in FP64 in a different order (strided partial sums and a
tree on the GPU, one sequential sum in the oracle): within 1e-9 cm, the same
number of tracks with non-zero weight.  A batch of events in one call
(tpcca_its_track_batch) returns for each event what a call on it alone
returns, bit for bit.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def its_tracker():
    from paper_1712_09434_amd.its import ItsTracker
    trk = ItsTracker(synth.default_its_geometry())
    yield trk
    trk.close()


def dev(ev):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t(ev.x), t(ev.y), t(ev.z), t(ev.layer), t(ev.stave)


EVENTS = [("ITS-pp", 0), ("ITS-mb", 0), ("ITS-central", 0), ("ITS-central", 1)]
_ORACLE = {}


def oracle_its(orc, name, index):
    if (name, index) not in _ORACLE:
        ev = synth.make_its_config(name, index)
        _ORACLE[(name, index)] = (ev, orc.its(ev))
    return _ORACLE[(name, index)]


def check_vs_oracle(out, ref):
    np.testing.assert_array_equal(out.hist.cpu().numpy().astype(np.int64), ref["hist"])
    assert out.n_pairs == ref["n_pairs"] and out.peak == ref["peak"]
    assert out.vz_ok == ref["vz_ok"] and np.float32(out.vz) == np.float32(ref["vz"])
    T = len(ref["tl0"])
    assert out.tl0.shape[0] == T > 0
    g = lambda k: getattr(out, k).cpu().numpy()
    np.testing.assert_array_equal(g("tl0"), ref["tl0"])
    np.testing.assert_array_equal(g("tl1"), ref["tl1"])
    np.testing.assert_array_equal(g("ok"), ref["ok"])
    ok = ref["ok"].astype(bool)
    np.testing.assert_array_equal(g("cls")[ok], ref["cls"][ok])
    np.testing.assert_array_equal(g("ncls")[ok], ref["ncls"][ok])
    np.testing.assert_array_equal(g("out_layer")[ok], ref["olayer"][ok])
    np.testing.assert_array_equal(g("out_stave")[ok], ref["ostave"][ok])
    np.testing.assert_array_equal(g("out_x")[ok], ref["ox"][ok])
    np.testing.assert_array_equal(g("chi2")[ok], ref["chi2"][ok])
    np.testing.assert_array_equal(g("out_p")[ok], ref["op"][ok])
    np.testing.assert_array_equal(g("out_cov")[ok], ref["oc"][ok])
    np.testing.assert_array_equal(g("in_ok")[ok], ref["iok"][ok])
    iok = ok & ref["iok"].astype(bool)
    np.testing.assert_array_equal(g("in_stave")[iok], ref["istave"][iok])
    np.testing.assert_array_equal(g("in_p")[iok], ref["ip"][iok])
    np.testing.assert_array_equal(g("in_cov")[iok], ref["ic"][iok])
    assert out.vfit_ok == ref["vfit_ok"] and out.vfit_n == ref["vfit_n"]
    np.testing.assert_allclose(np.array(out.vertex), ref["vertex"], rtol=0, atol=1e-9)
    assert abs(out.vfit_sumw - ref["vfit_sumw"]) <= 1e-9 * max(1.0, ref["vfit_sumw"])
    return T, int(ok.sum())


@pytest.mark.parametrize("name,index", EVENTS)
def test_its_matches_oracle(its_tracker, orc, name, index):
    ev, ref = oracle_its(orc, name, index)
    print(f"[gpu] ITS {name}/{index}: {ev.n} clusters", flush=True)
    out = its_tracker.track(*dev(ev), hist=True)
    T, nok = check_vs_oracle(out, ref)
    print(f"[gpu] ITS {name}/{index}: {T} tracklets, {nok} tracks, vertex "
          f"{np.array(out.vertex)} (true {ev.vertex})", flush=True)


def assert_same_event(a, b):
    """Every result of two calls on one event, bit for bit (arrays the
    tracker leaves unset for rejected tracks compared under the masks)."""
    assert torch.equal(a.hist, b.hist)
    for k in ("n_pairs", "peak", "vz_ok", "vz", "vfit_ok", "vfit_n", "vertex", "vfit_sumw"):
        assert getattr(a, k) == getattr(b, k), k
    for k in ("tl0", "tl1", "ok", "in_ok"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    m = a.ok.bool()
    for k in ("cls", "ncls", "chi2", "out_layer", "out_stave", "out_x", "out_p", "out_cov"):
        assert torch.equal(getattr(a, k)[m], getattr(b, k)[m]), k
    mi = m & a.in_ok.bool()
    for k in ("in_stave", "in_p", "in_cov"):
        assert torch.equal(getattr(a, k)[mi], getattr(b, k)[mi]), k


def test_its_batch_equals_single_events(its_tracker, orc):
    """One call on several events (an empty one among them, a repeated one)
    returns for each what a call on that event alone returns, and the
    oracle's results."""
    evs = [oracle_its(orc, *k) for k in EVENTS]
    d = [dev(ev) for ev, _ in evs]
    empty = tuple(t[:0] for t in d[0])
    batch_in = [d[0], d[2], empty, d[1], d[3], d[2]]
    print(f"[gpu] ITS batch of {len(batch_in)} events", flush=True)
    got = its_tracker.track_batch(batch_in, hist=True)
    single = [its_tracker.track(*e, hist=True) for e in batch_in]
    for a, b in zip(got, single):
        assert_same_event(a, b)
    assert got[2].tl0.shape[0] == 0 and not got[2].vz_ok and not got[2].vfit_ok
    for slot, i in zip([0, 1, 3, 4, 5], [0, 2, 1, 3, 2]):
        check_vs_oracle(got[slot], evs[i][1])


def test_its_batch_capacity(its_tracker):
    """An event whose output is too small fails the call with every event's
    required count."""
    from paper_1712_09434_amd import _abi as A
    ev = synth.make_its_config("ITS-pp")
    e1 = its_tracker._event(*dev(ev), False)
    e2 = its_tracker._event(*dev(ev), False)
    e2[1].cap = 1
    cls = (A.tpcca_its_clusters * 2)(e1[0], e2[0])
    sts = (A.tpcca_its_tracks * 2)(e1[1], e2[1])
    rc = its_tracker.L.tpcca_its_track_batch(its_tracker.ctx, 2, cls, sts)
    assert rc == A.TPCCA_E_CAPACITY
    assert sts[0].n_tracklets == sts[1].n_tracklets > 1
    assert its_tracker.L.tpcca_its_track_batch(its_tracker.ctx, 0, cls, sts) == A.TPCCA_E_INVALID
    # the tracker still works after the errors
    out = its_tracker.track_batch([dev(ev)])[0]
    assert out.tl0.shape[0] == sts[0].n_tracklets


def test_its_edges(its_tracker):
    from paper_1712_09434_amd import TpccaError
    ev = synth.make_its_config("ITS-pp")
    x, y, z, lay, stv = dev(ev)
    out = its_tracker.track(x[:0], y[:0], z[:0], lay[:0], stv[:0])
    assert out.tl0.shape[0] == 0 and not out.vz_ok and not out.vfit_ok
    bad = stv.clone()
    bad[3] = 99
    with pytest.raises(TpccaError):
        its_tracker.track(x, y, z, lay, bad)
    badz = z.clone()
    badz[0] = float("nan")
    with pytest.raises(TpccaError):
        its_tracker.track(x, y, badz, lay, stv)
    # the tracker still works after the errors, and repeats bit for bit
    a = its_tracker.track(x, y, z, lay, stv)
    b = its_tracker.track(x, y, z, lay, stv)
    m = (a.ok * a.in_ok).bool()
    assert torch.equal(a.ok, b.ok) and torch.equal(a.in_p[m], b.in_p[m]) and a.vertex == b.vertex
