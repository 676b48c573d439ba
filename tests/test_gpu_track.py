"""GPU parity of the tracking path against the oracle (through the C ABI).

Bar (FP32 both sides, same expressions, no contraction):
  * raw and cleaned neighbour links, start hits, tracklet hit lists and
    final hit lists: bit-exact;
  * track parameters, covariance, chi2: |a - b| <= 1e-4 * max(|b|, floor).
C1 and C2 are compared whole; C3 (the headline event) is compared whole,
sector by sector (the oracle takes one sector per host thread), with the
taps on and in the launch configuration the benchmark times.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

FLOOR_P = np.array([1.0, 1.0, 1e-2, 1e-2, 1e-2])


def to_dev(ev, dev="cuda:0"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t(ev.x), t(ev.y), t(ev.z), t(ev.row), t(ev.sector)


@pytest.fixture(scope="module")
def tracker():
    from paper_1712_09434_amd import Tracker
    trk = Tracker.from_geometry(synth.default_geometry())
    yield trk
    trk.close()


def compare(ev, out, tl, ref, sectors=None, check_taps=True):
    n = ev.n
    if sectors is None:
        m = np.ones(n, bool)
    else:
        m = np.isin(ev.sector, sectors)
    if check_taps:
        t = {k: v.cpu().numpy().astype(np.int64) for k, v in out.taps.items()}
        for k in ("up", "dn", "cup", "cdn"):
            np.testing.assert_array_equal(t[k][m], ref[k][m], err_msg=f"link tap {k}")
        starts = t["start"]
        starts = starts[np.isin(ev.sector[starts], sectors)] if sectors is not None else starts
        np.testing.assert_array_equal(starts, ref["starts"], err_msg="start hits")
    if tl is not None:
        ss = tl["seed_start"].astype(np.int64)
        keep = np.isin(ev.sector[ss], sectors) if sectors is not None else np.ones(len(ss), bool)
        np.testing.assert_array_equal(ss[keep], ref["seed_start"], err_msg="seed list")
        np.testing.assert_array_equal(tl["seed_nhits"][keep], ref["seed_nhits"], err_msg="tracklet n_hits")
        gh = tl["seed_hits"][keep].astype(np.int64)
        valid = ref["seed_nhits"] > 0
        np.testing.assert_array_equal(gh[valid], ref["seed_hits"][valid], err_msg="tracklet hit lists")
    sec = out.sector.cpu().numpy().astype(np.int64)
    keep = np.isin(sec, sectors) if sectors is not None else np.ones(len(sec), bool)
    off = out.hit_off.cpu().numpy().astype(np.int64)
    ids = out.hit_id.cpu().numpy().astype(np.int64)
    lists = [ids[off[i]:off[i + 1]] for i in np.nonzero(keep)[0]]
    ref_lists = [ref["hit_ids"][ref["hit_off"][i]:ref["hit_off"][i + 1]] for i in range(len(ref["x_ref"]))]
    assert len(lists) == len(ref_lists), (len(lists), len(ref_lists))
    for a, b in zip(lists, ref_lists):
        np.testing.assert_array_equal(a, b, err_msg="final hit list")
    np.testing.assert_array_equal(sec[keep], ref["sector"])
    np.testing.assert_array_equal(out.ndf.cpu().numpy()[keep], ref["ndf"])
    p = out.p.cpu().numpy().astype(np.float64)[keep]
    assert np.all(np.abs(p - ref["p"]) <= 1e-4 * np.maximum(np.abs(ref["p"]), FLOOR_P)), "track parameters"
    cov = out.cov.cpu().numpy().astype(np.float64)[keep]
    assert np.all(np.abs(cov - ref["cov"]) <= 1e-4 * np.maximum(np.abs(ref["cov"]), 1e-8)), "covariance"
    chi2 = out.chi2.cpu().numpy().astype(np.float64)[keep]
    assert np.all(np.abs(chi2 - ref["chi2"]) <= 1e-4 * np.maximum(ref["chi2"], 1.0)), "chi2"
    xr = out.x_ref.cpu().numpy().astype(np.float64)[keep]
    np.testing.assert_array_equal(xr, ref["x_ref"])
    return float(np.mean(p == ref["p"])) if len(p) else 1.0


@pytest.mark.parametrize("cfg", ["C1", "C2"])
def test_parity_full_event(tracker, orc, cfg):
    ev = synth.make_config(cfg)
    print(f"[gpu] parity {cfg} n={ev.n}", flush=True)
    out = tracker.track(*to_dev(ev), taps=True)
    tl = tracker.debug_tracklets()
    ref = orc.track(ev, precision=32)
    exact = compare(ev, out, tl, ref)
    assert out.n_tracks > 0
    print(f"[gpu] {cfg}: {out.n_tracks} tracks, exact-parameter fraction {exact:.4f}", flush=True)


def host(out):
    """The tracks with every tensor copied to host memory once."""
    import dataclasses
    taps = {k: v.cpu() for k, v in out.taps.items()} if out.taps else out.taps
    return dataclasses.replace(out, **{f.name: getattr(out, f.name).cpu() for f in dataclasses.fields(out)
                                       if f.name != "taps"}, taps=taps)


def oracle_by_sector(orc, ev, sectors, threads=16):
    """The oracle on each sector alone (sectors are independent), one sector
    per host thread; returns {sector: result}."""
    import concurrent.futures

    def one(s):
        mask = np.zeros(ev.geom.n_sectors, np.uint8)
        mask[s] = 1
        return s, orc.track(ev, precision=32, sector_mask=mask)

    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as pool:
        return dict(pool.map(one, sectors))


@pytest.fixture(scope="module")
def c3_reference(orc):
    ev = synth.make_config("C3")
    print(f"[gpu] oracle on the 36 sectors of C3 n={ev.n}", flush=True)
    return ev, oracle_by_sector(orc, ev, range(ev.geom.n_sectors))


def test_parity_c3_whole_event(tracker, c3_reference):
    """The headline event, every sector: links, starts, tracklets and tracks."""
    ev, refs = c3_reference
    print(f"[gpu] parity C3 whole event (taps on) n={ev.n}", flush=True)
    out = host(tracker.track(*to_dev(ev), taps=True))
    tl = tracker.debug_tracklets()
    for s, ref in refs.items():
        compare(ev, out, tl, ref, sectors=[s])
    assert out.n_tracks == sum(len(r["x_ref"]) for r in refs.values())


def test_parity_c3_timed_configuration(tracker, c3_reference):
    """The call the benchmark times (no taps, default tuning, phase timing
    on): final tracks of every sector equal the oracle's."""
    ev, refs = c3_reference
    print(f"[gpu] parity C3 whole event (taps off) n={ev.n}", flush=True)
    tracker.set_phase_timing(True)
    try:
        out = host(tracker.track(*to_dev(ev)))
    finally:
        tracker.set_phase_timing(False)
    for s, ref in refs.items():
        compare(ev, out, None, ref, sectors=[s], check_taps=False)
    assert out.n_tracks == sum(len(r["x_ref"]) for r in refs.values())


def test_deterministic_repeat(tracker):
    ev = synth.make_config("C2")
    a = tracker.track(*to_dev(ev))
    b = tracker.track(*to_dev(ev))
    for k in ("hit_off", "hit_id", "p", "cov", "chi2"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k


def test_batch_equals_single_events(tracker):
    evs = [synth.make_config("C1"), synth.make_event(seed=5, n_primaries=0),
           synth.make_event(seed=6, n_primaries=300, noise=0.05),
           synth.make_event(seed=7, n_primaries=3, single_sector=True)]
    evs[1].meta["empty"] = True
    batch = tracker.track_batch([to_dev(e) for e in evs], taps=True)
    for e, ev in enumerate(evs):
        single = tracker.track(*to_dev(ev), taps=True)
        for k in ("sector", "x_ref", "p", "cov", "chi2", "ndf", "k_prior", "hit_off", "hit_id"):
            assert torch.equal(getattr(batch[e], k), getattr(single, k)), (e, k)
        for k in ("up", "dn", "cup", "cdn", "start"):
            assert torch.equal(batch[e].taps[k], single.taps[k]), (e, k)


def test_host_memory_mode_matches_device(tracker):
    ev = synth.make_config("C1")
    d = tracker.track(*to_dev(ev), taps=True)
    h = tracker.track(*to_dev(ev, "cpu"), taps=True)
    for k in ("sector", "x_ref", "p", "cov", "chi2", "ndf", "hit_off", "hit_id"):
        assert torch.equal(getattr(h, k), getattr(d, k).cpu()), k


def test_empty_and_single_cluster(tracker):
    for n in (0, 1):
        ev = synth.make_event(seed=11, n_primaries=0)
        x = torch.full((n,), 100.0, device="cuda:0")
        row = torch.full((n,), 10, dtype=torch.int16, device="cuda:0")
        sec = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
        out = tracker.track(x, x.clone(), x.clone(), row, sec, taps=True)
        assert out.n_tracks == 0 and out.hit_off.cpu().tolist() == [0]
        assert out.taps["start"].numel() == 0


def _raw_track(tracker, x, y, z, row, sec, cap_t, cap_h):
    from paper_1712_09434_amd import _abi as A
    cl = tracker.clusters_struct(x, y, z, row, sec)
    st, o = tracker._alloc_out(int(x.shape[0]), x.device, False)
    st.cap_tracks, st.cap_hits = cap_t, cap_h
    rc = tracker.L.tpcca_track(tracker.ctx, C.byref(cl), C.byref(st))
    return rc, st


def test_invalid_inputs_rejected(tracker):
    from paper_1712_09434_amd import _abi as A
    ev = synth.make_config("C1")
    base = to_dev(ev)
    bad = [t.clone() for t in base]
    bad[1][17] = float("nan")
    rc, _ = _raw_track(tracker, *bad, 1000, 100000)
    assert rc == A.TPCCA_E_INVALID
    bad = [t.clone() for t in base]
    bad[3][5] = 159
    rc, _ = _raw_track(tracker, *bad, 1000, 100000)
    assert rc == A.TPCCA_E_INVALID
    bad = [t.clone() for t in base]
    bad[4][9] = 36
    rc, _ = _raw_track(tracker, *bad, 1000, 100000)
    assert rc == A.TPCCA_E_INVALID
    # the context still works afterwards
    out = tracker.track(*base)
    assert out.n_tracks > 0


def test_capacity_overflow_reports_required_sizes(tracker):
    from paper_1712_09434_amd import _abi as A
    ev = synth.make_config("C1")
    full = tracker.track(*to_dev(ev))
    rc, st = _raw_track(tracker, *to_dev(ev), 1, 10)
    assert rc == A.TPCCA_E_CAPACITY
    assert st.n_tracks == full.n_tracks and st.n_hits == full.hit_id.numel()


def test_row_limit(tracker):
    from paper_1712_09434_amd import _abi as A
    n = A.TPCCA_MAX_ROW_CLUSTERS + 1
    g = torch.Generator().manual_seed(0)
    y = (torch.rand(n, generator=g) * 20 - 10).to("cuda:0")
    z = (torch.rand(n, generator=g) * 200).to("cuda:0")
    x = torch.full((n,), 100.0, device="cuda:0")
    row = torch.full((n,), 14, dtype=torch.int16, device="cuda:0")
    sec = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    rc, _ = _raw_track(tracker, x, y, z, row, sec, 100, n)
    assert rc == A.TPCCA_E_LIMIT


def test_graph_replay_matches_eager(tracker):
    """Captured tracking graph: every replay equals the eager call, with eager
    GPU work and synchronisations between replays."""
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        evs = [synth.make_config("C1"), synth.make_event(seed=21, n_primaries=400, noise=0.03)]
        tens = [to_dev(e) for e in evs]
        tracker.set_tuning(use_graph=0)
        eager = [tracker.track(*t) for t in tens]
        tracker.set_tuning(use_graph=1)
        try:
            for rep in range(3):
                for e, t in enumerate(tens):
                    out = tracker.track(*t)
                    junk = t[0] * 2.0 + 1.0          # eager work between replays
                    torch.cuda.synchronize()
                    for k in ("hit_off", "hit_id", "p", "cov", "chi2", "sector"):
                        assert torch.equal(getattr(out, k), getattr(eager[e], k)), (rep, e, k)
                    del junk
            batch = tracker.track_batch(tens)
            batch2 = tracker.track_batch(tens)
            for e in range(len(tens)):
                assert torch.equal(batch[e].hit_id, eager[e].hit_id)
                assert torch.equal(batch2[e].p, eager[e].p)
        finally:
            tracker.set_tuning(use_graph=0)


def test_tracklet_grid_does_not_change_results(tracker):
    ev = synth.make_config("C2")
    t = to_dev(ev)
    ref = tracker.track(*t)
    for g in (1, 7, 256, 4096):
        tracker.set_tuning(tracklet_grid=g)
        out = tracker.track(*t)
        for k in ("hit_off", "hit_id", "p"):
            assert torch.equal(getattr(out, k), getattr(ref, k)), (g, k)
    tracker.set_tuning(tracklet_grid=0)


def _with_patches(ev, patches, seed):
    """Copy of `ev` with uniform clusters added in (row, n, y range, z range)
    patches of sector 0, on the row planes."""
    import dataclasses
    rng = np.random.default_rng(seed)
    xs, ys, zs, rows = [ev.x], [ev.y], [ev.z], [ev.row]
    for r, n, (y0, y1), (z0, z1) in patches:
        xs.append(np.full(n, ev.geom.row_x[r], np.float32))
        ys.append(rng.uniform(y0, y1, n).astype(np.float32))
        zs.append(rng.uniform(z0, z1, n).astype(np.float32))
        rows.append(np.full(n, r, np.int16))
    extra = sum(p[1] for p in patches)
    cat = np.concatenate
    return dataclasses.replace(
        ev, x=cat(xs), y=cat(ys), z=cat(zs), row=cat(rows), sector=cat([ev.sector, np.zeros(extra, np.uint8)]),
        x64=cat(xs).astype(np.float64), y64=cat(ys).astype(np.float64), z64=cat(zs).astype(np.float64),
        truth_track=cat([ev.truth_track, np.full(extra, -1, np.int32)]),
        truth_double=cat([ev.truth_double, np.zeros(extra, bool)]))


def test_dense_rows_take_the_fallback_paths(tracker, orc):
    """Rows above the register-sort size (1024), above the neighbour slab
    (896), a 4-row band above the LDS ownership capacity (6144), and windows
    with more than the 15 kept candidates per side in an LDS-staged row:
    every fallback path still matches the oracle."""
    ev = synth.make_event(seed=31, n_primaries=150, noise=0.01, single_sector=True)
    patches = [(r, 1600, (-10.0, 10.0), (40.0, 120.0)) for r in (40, 41, 42, 43)]
    patches += [(r, 650, (-6.0, 6.0), (150.0, 180.0)) for r in (80, 81, 82)]
    ev = _with_patches(ev, patches, seed=32)
    print(f"[gpu] dense rows n={ev.n}", flush=True)
    out = tracker.track(*to_dev(ev), taps=True)
    tl = tracker.debug_tracklets()
    ref = orc.track(ev, precision=32)
    compare(ev, out, tl, ref)
    assert out.n_tracks > 0


def test_lattice_ties_in_slab_rows(tracker, orc):
    """Rows of 300 to 800 clusters (the 896-cluster slab variant of the link
    kernel, which scores a wave's candidate pairs with all of its lanes) on
    a 0.5 cm lattice, a fifth of each row duplicating other clusters of the
    row: equal scores from different pairs are common, and the tie rule
    (smaller up position, then smaller down position) decides.  Links and
    everything after them equal the oracle."""
    import dataclasses
    ev = synth.make_event(seed=33, n_primaries=60, noise=0.0, single_sector=True)
    rng = np.random.default_rng(34)
    xs, ys, zs, rows = [ev.x], [ev.y], [ev.z], [ev.row]
    for r, n in ((60, 500), (61, 700), (62, 600), (63, 800), (64, 300)):
        y = (rng.integers(-20, 21, n) * 0.5).astype(np.float32)
        z = (rng.integers(40, 241, n) * 0.5).astype(np.float32)
        src = rng.integers(n // 5, n, n // 5)
        y[: n // 5] = y[src]
        z[: n // 5] = z[src]
        xs.append(np.full(n, ev.geom.row_x[r], np.float32))
        ys.append(y)
        zs.append(z)
        rows.append(np.full(n, r, np.int16))
    extra = sum(len(a) for a in rows[1:])
    cat = np.concatenate
    ev = dataclasses.replace(
        ev, x=cat(xs), y=cat(ys), z=cat(zs), row=cat(rows), sector=cat([ev.sector, np.zeros(extra, np.uint8)]),
        x64=cat(xs).astype(np.float64), y64=cat(ys).astype(np.float64), z64=cat(zs).astype(np.float64),
        truth_track=cat([ev.truth_track, np.full(extra, -1, np.int32)]),
        truth_double=cat([ev.truth_double, np.zeros(extra, bool)]))
    print(f"[gpu] lattice rows n={ev.n}", flush=True)
    out = tracker.track(*to_dev(ev), taps=True)
    tl = tracker.debug_tracklets()
    ref = orc.track(ev, precision=32)
    compare(ev, out, tl, ref)
    # the patch rows' links are many, so the pair scoring ran on them
    up = out.taps["up"].cpu().numpy()
    patch = (ev.sector == 0) & (ev.row >= 61) & (ev.row <= 63)
    assert (up[patch] >= 0).sum() > 500


def test_batch_with_dense_rows_equals_single_events(tracker):
    """A batch large enough for the row-unit class lists (more than 16,384 row
    units), holding units of every row and link class (a dense event with
    1600- and 650-cluster rows, a one-sector event of ~100 clusters per row,
    a small event): each event's output equals its single-event call."""
    dense = synth.make_event(seed=31, n_primaries=150, noise=0.01, single_sector=True)
    patches = [(r, 1600, (-10.0, 10.0), (40.0, 120.0)) for r in (40, 41, 42, 43)]
    patches += [(r, 650, (-6.0, 6.0), (150.0, 180.0)) for r in (80, 81, 82)]
    evs = [_with_patches(dense, patches, seed=32), synth.make_config("C1"),
           synth.make_event(seed=8, n_primaries=200, noise=0.02)]
    assert len(evs) * evs[0].geom.n_sectors * evs[0].geom.n_rows > 16384
    batch = tracker.track_batch([to_dev(e) for e in evs], taps=True)
    for e, ev in enumerate(evs):
        single = tracker.track(*to_dev(ev), taps=True)
        for k in ("sector", "x_ref", "p", "cov", "chi2", "ndf", "k_prior", "hit_off", "hit_id"):
            assert torch.equal(getattr(batch[e], k), getattr(single, k)), (e, k)
        for k in ("up", "dn", "cup", "cdn", "start"):
            assert torch.equal(batch[e].taps[k], single.taps[k]), (e, k)


def test_batch_of_uneven_events_matches_oracle(tracker, orc):
    """Several events of the batching workload (lognormal multiplicity) in one
    call, each compared with the oracle in full."""
    evs = [synth.make_config("C4", e) for e in range(6)]
    evs = sorted(evs, key=lambda e: e.n)[:4]          # the four smallest, for the oracle's sake
    print("[gpu] batch sizes", [e.n for e in evs], flush=True)
    batch = tracker.track_batch([to_dev(e) for e in evs], taps=True)
    for ev, out in zip(evs, batch):
        ref = orc.track(ev, precision=32)
        compare(ev, out, None, ref)


def test_event_above_2_22_clusters(tracker, orc):
    """An event of more than 2^22 clusters (ids past 22 bits, noise added to
    sectors 1-12 of the headline event): the sampled sectors still match the
    oracle."""
    import dataclasses
    ev = synth.make_config("C3")
    extra = (1 << 22) - ev.n + 20000
    rng = np.random.default_rng(77)
    g = ev.geom
    sec = rng.integers(1, 13, extra).astype(np.uint8)          # noise in sectors 1..12 only
    row = rng.integers(0, g.n_rows, extra).astype(np.int16)
    x = np.asarray(g.row_x, np.float32)[row]
    y = (rng.uniform(-1.0, 1.0, extra) * x * np.float32(g.tan_half_angle)).astype(np.float32)
    z = rng.uniform(-0.98, 0.98, extra).astype(np.float32) * np.float32(g.z_max)
    cat = np.concatenate
    big = dataclasses.replace(
        ev, x=cat([ev.x, x]), y=cat([ev.y, y]), z=cat([ev.z, z]), row=cat([ev.row, row]),
        sector=cat([ev.sector, sec]), x64=cat([ev.x64, x.astype(np.float64)]),
        y64=cat([ev.y64, y.astype(np.float64)]), z64=cat([ev.z64, z.astype(np.float64)]),
        truth_track=cat([ev.truth_track, np.full(extra, -1, np.int32)]),
        truth_double=cat([ev.truth_double, np.zeros(extra, bool)]))
    assert big.n >= 1 << 22
    print(f"[gpu] event above 2^22 clusters n={big.n}", flush=True)
    out = tracker.track(*to_dev(big), taps=True)
    tl = tracker.debug_tracklets()
    sectors = [0, 5, 13]
    mask = np.zeros(36, np.uint8); mask[sectors] = 1
    ref = orc.track(big, precision=32, sector_mask=mask)
    compare(big, out, tl, ref, sectors=sectors)
    assert out.n_tracks > 0
