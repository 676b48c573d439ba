"""GPU parity of the sector track merger (tpcca_merge) against the oracle.

The oracle merges its own segments (its FP32 tracking output, which equals
the library's bit for bit) in FP64; the library merges in FP32.  Bar:
  * links: equal, except where the oracle's decision is ambiguous at FP32
    resolution (its best match chi2 within 1e-3 relative of the cut or of
    the second-best candidate, on either end of the link); at most 1 in
    1,000 links may differ that way;
  * merged output: tracks in the same order with the same hit lists,
    sectors, ndf and x_ref; unmerged segments bit for bit; refitted chains
    against the FP64 refit: |dp| <= 2e-3 max(|p|, floor) (floor 1 cm for
    y, z, 1e-2 for sin phi, tan lambda, q/pT), covariance entries within
    5e-2 sqrt(C_ii C_jj), chi2 within 1e-2 relative (floor 1).  These
    bounds are the spread of an FP32 Kalman fit (first three updates
    compensated) against FP64 over a full event's tracks (largest errors
    3.6e-4, 3.1e-2, 3.8e-3), with margin.
On the one-sector-per-thread oracle of the central-Pb-Pb-shaped event and on
a full event; plus empty input, one segment, capacity and host-memory errors.
"""
import numpy as np
import pytest
import torch

import synth
from test_gpu_track import oracle_by_sector, to_dev

pytestmark = pytest.mark.gpu
FLOOR_P = np.array([1.0, 1.0, 1e-2, 1e-2, 1e-2])


@pytest.fixture(scope="module")
def tracker():
    from paper_1712_09434_amd import Tracker
    trk = Tracker.from_geometry(synth.default_geometry())
    yield trk
    trk.close()


def ambiguous(ref, a, cut):
    def amb(c1, c2):
        return np.isfinite(c1) and (abs(c1 - cut) <= 1e-3 * cut or (np.isfinite(c2) and c2 - c1 <= 1e-3 * c1))
    return amb(ref["chi_out"][a], ref["chi_out2"][a]) or (
        ref["best_out"][a] >= 0 and amb(ref["chi_in"][ref["best_out"][a]], ref["chi_in2"][ref["best_out"][a]]))


def compare_merge(ev, seg, merged, links, ref, cut=50.0, single_rtol=0.0):
    """single_rtol: relative bound (floors as for the refit) on the copied
    parameters of unmerged segments (0: bit for bit)."""
    lk = links.cpu().numpy()
    diff = np.nonzero(lk != ref["link"])[0]
    nl = int((ref["link"] >= 0).sum())
    print(f"[gpu] merge: {len(lk)} segments, {nl} oracle links, {len(diff)} different", flush=True)
    for a in diff:
        assert ambiguous(ref, a, cut) or (lk[a] >= 0 and ambiguous(ref, lk[a], cut)), (a, lk[a], ref["link"][a])
    assert len(diff) <= max(1, nl // 1000)
    if len(diff):
        return    # the chains differ; the rest is compared on agreeing inputs only
    off = merged.hit_off.cpu().numpy().astype(np.int64)
    ids = merged.hit_id.cpu().numpy().astype(np.int64)
    assert merged.n_tracks == len(ref["x_ref"])
    np.testing.assert_array_equal(off, ref["hit_off"])
    np.testing.assert_array_equal(ids, ref["hit_ids"])
    np.testing.assert_array_equal(merged.sector.cpu().numpy(), ref["sector"])
    np.testing.assert_array_equal(merged.ndf.cpu().numpy(), ref["ndf"])
    xr = merged.x_ref.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(xr, ref["x_ref"])
    p = merged.p.cpu().numpy().astype(np.float64)
    cov = merged.cov.cpu().numpy().astype(np.float64)
    chi2 = merged.chi2.cpu().numpy().astype(np.float64)
    chained = np.diff(off) != np.array([seg_len(seg, h) for h in ref["head"]])
    single = ~chained
    if single_rtol:
        assert np.all(np.abs(p[single] - ref["p"][single]) <= single_rtol * np.maximum(np.abs(ref["p"][single]),
                                                                                      FLOOR_P))
    else:
        np.testing.assert_array_equal(p[single], ref["p"][single])
    np.testing.assert_array_equal(cov[single], ref["cov"][single])
    np.testing.assert_array_equal(chi2[single], ref["chi2"][single])
    assert chained.sum() > 0
    rp, rc, rx = ref["p"][chained], ref["cov"][chained], ref["chi2"][chained]
    perr = np.abs(p[chained] - rp) / np.maximum(np.abs(rp), FLOOR_P)
    xerr = np.abs(chi2[chained] - rx) / np.maximum(rx, 1.0)
    w = np.unravel_index(np.argmax(perr), perr.shape)
    print(f"[gpu] merge: parameter error / max(|p|, floor): max {perr.max():.2e} (track {w[0]}, parameter "
          f"{w[1]}: {p[chained][w]} vs {rp[w]}, {int(np.diff(off)[chained][w[0]])} hits); chi2 max {xerr.max():.2e}",
          flush=True)
    assert np.all(perr <= 2e-3), "merged parameters"
    iu = np.triu_indices(5)
    diag = rc[:, [0, 5, 9, 12, 14]]
    scale = np.sqrt(diag[:, iu[0]] * diag[:, iu[1]])        # sqrt(C_ii C_jj) per packed entry
    cerr = np.abs(cov[chained] - rc) / scale
    print(f"[gpu] merge: covariance error / sqrt(C_ii C_jj): median {np.median(cerr):.2e}, max {cerr.max():.2e}",
          flush=True)
    assert np.all(cerr <= 5e-2), "merged covariance"
    assert np.all(np.abs(chi2[chained] - rx) <= 1e-2 * np.maximum(rx, 1.0)), "merged chi2"
    print(f"[gpu] merge: {int(chained.sum())} refitted chains; median |dp|/|p| "
          f"{np.median(np.abs(p[chained] - rp) / np.maximum(np.abs(rp), FLOOR_P)):.2e}", flush=True)


def seg_len(seg, i):
    return int(seg["hit_off"][i + 1] - seg["hit_off"][i])


def test_merge_full_event(tracker, orc):
    ev = synth.make_config("C2")
    cl = to_dev(ev)
    seg = tracker.track(*cl)
    merged, links = tracker.merge(seg, cl, links=True)
    r = orc.track(ev, precision=32)
    ref = orc.merge(ev, r)
    compare_merge(ev, r, merged, links, ref)


def test_merge_headline_event(tracker, orc):
    ev = synth.make_config("C3")
    print(f"[gpu] merge on the central-Pb-Pb-shaped event n={ev.n}: oracle per sector", flush=True)
    refs = oracle_by_sector(orc, ev, range(ev.geom.n_sectors))
    r = {k: [] for k in ("sector", "x_ref", "p", "cov", "chi2", "hit_ids")}
    off = [0]
    for s in range(ev.geom.n_sectors):
        q = refs[s]
        for k in r:
            r[k].append(q[k])
        off += list(off[-1] + q["hit_off"][1:])
    seg = {k: np.concatenate(v) for k, v in r.items()}
    seg["hit_off"] = np.array(off, np.int64)
    ref = orc.merge(ev, seg)
    cl = to_dev(ev)
    out = tracker.track(*cl)
    merged, links = tracker.merge(out, cl, links=True)
    compare_merge(ev, seg, merged, links, ref)


def test_merge_edges(tracker):
    from paper_1712_09434_amd import TpccaError
    ev = synth.make_event(seed=6, n_primaries=300, noise=0.05)
    cl = to_dev(ev)
    seg = tracker.track(*cl)
    # empty input
    import dataclasses
    empty = dataclasses.replace(seg, sector=seg.sector[:0], x_ref=seg.x_ref[:0], p=seg.p[:0], cov=seg.cov[:0],
                                chi2=seg.chi2[:0], ndf=seg.ndf[:0], k_prior=seg.k_prior[:0],
                                hit_off=seg.hit_off[:1], hit_id=seg.hit_id[:0])
    m = tracker.merge(empty, cl)
    assert m.n_tracks == 0 and int(m.hit_off[0]) == 0
    # one segment: copied unchanged
    one = dataclasses.replace(seg, sector=seg.sector[:1], x_ref=seg.x_ref[:1], p=seg.p[:1], cov=seg.cov[:1],
                              chi2=seg.chi2[:1], ndf=seg.ndf[:1], k_prior=seg.k_prior[:1],
                              hit_off=seg.hit_off[:2], hit_id=seg.hit_id[:int(seg.hit_off[1])])
    m = tracker.merge(one, cl)
    assert m.n_tracks == 1 and torch.equal(m.p, one.p) and torch.equal(m.hit_id, one.hit_id)
    # the whole event twice in a row gives the same result
    a = tracker.merge(seg, cl)
    b = tracker.merge(seg, cl)
    for k in ("hit_off", "hit_id", "p", "cov", "chi2", "sector"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert a.n_tracks < seg.n_tracks
    # host memory is rejected
    hseg = dataclasses.replace(seg, **{k: getattr(seg, k).cpu() for k in
                                      ("sector", "x_ref", "p", "cov", "chi2", "ndf", "k_prior", "hit_off", "hit_id")})
    with pytest.raises(TpccaError):
        tracker.merge(hseg, tuple(t.cpu() for t in cl))
