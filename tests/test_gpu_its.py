"""GPU parity of the ITS standalone tracker (tpcca_its_track) against the
oracle (oracle.its), on the pp-like, minimum-bias-like and two
central-Pb-Pb-like events.

Both sides evaluate the same FP32 expressions, so the integer results are
compared exactly (vertexer histogram, pair count, peak, tracklets, accepted
tracks, their clusters, layers and staves) and so are the FP32 values (the
vertex z, chi2, the outward and inward states and covariances).  The
vertex fit sums in FP64 in a different order (strided partial sums and a
tree on the GPU, one sequential sum in the oracle): within 1e-9 cm, the same
number of tracks with non-zero weight.
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


@pytest.mark.parametrize("name,index", [("ITS-pp", 0), ("ITS-mb", 0), ("ITS-central", 0), ("ITS-central", 1)])
def test_its_matches_oracle(its_tracker, orc, name, index):
    ev = synth.make_its_config(name, index)
    print(f"[gpu] ITS {name}/{index}: {ev.n} clusters", flush=True)
    ref = orc.its(ev)
    out = its_tracker.track(*dev(ev), hist=True)
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
    print(f"[gpu] ITS {name}/{index}: {T} tracklets, {int(ok.sum())} tracks, vertex "
          f"{np.array(out.vertex)} (true {ev.vertex})", flush=True)


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
