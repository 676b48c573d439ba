"""Pins of the oracle's cellular-automaton seeding and the pipeline invariants.

* Neighbour finding equals a brute force over all (down, up) pairs written
  independently here in numpy float32 (bit-exact), including duplicated
  clusters and exact ties.
* Cleaned links are reciprocal (a bijection), cleaning is idempotent, start
  hits are exactly the chain heads in (sector, row, id) order.
* Output tracks: at most one hit per pad row (at most 159 hits, one per
  row), every cluster in at most one track, canonical order.
"""
import json
import os
from types import SimpleNamespace

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import synth

F = np.float32
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def brute_links(x, y, z, row, sec, P, n_rows):
    n = len(x)
    up = np.full(n, -1); dn = np.full(n, -1)
    WY, WZ, IWY, IWZ, CUT = (F(P.win_y), F(P.win_z), F(P.inv_var_y), F(P.inv_var_z), F(P.link_cut))
    for i in range(n):
        r = row[i]
        if r < 1 or r > n_rows - 2:
            continue
        best = None
        for d in range(n):
            if sec[d] != sec[i] or row[d] != r - 1:
                continue
            if not (abs(F(y[d] - y[i])) <= WY and abs(F(z[d] - z[i])) <= WZ):
                continue
            for u in range(n):
                if sec[u] != sec[i] or row[u] != r + 1:
                    continue
                if not (abs(F(y[u] - y[i])) <= WY and abs(F(z[u] - z[i])) <= WZ):
                    continue
                w = F(F(x[i] - x[d]) / F(x[u] - x[d]))
                ey = F(y[i] - F(y[d] + F(F(y[u] - y[d]) * w)))
                ez = F(z[i] - F(z[d] + F(F(z[u] - z[d]) * w)))
                score = F(F(F(ey * ey) * IWY) + F(F(ez * ez) * IWZ))
                if score <= CUT:
                    cand = (score, u, d)
                    if best is None or cand < best:
                        best = cand
        if best is not None:
            up[i], dn[i] = best[1], best[2]
    return up, dn


def tiny_event(y, z, row, sec):
    geom = synth.default_geometry()
    x = geom.row_x[row].astype(np.float32)
    return SimpleNamespace(x=x, y=np.asarray(y, np.float32), z=np.asarray(z, np.float32),
                           row=np.asarray(row, np.int16), sector=np.asarray(sec, np.uint8),
                           geom=geom, n=len(x))


@settings(max_examples=60, deadline=None, derandomize=True)
@given(st.data())
def test_neighbours_equal_brute_force(orc, data):
    n = data.draw(st.integers(1, 60))
    rows = data.draw(st.lists(st.integers(0, 4), min_size=n, max_size=n))
    secs = data.draw(st.lists(st.integers(0, 1), min_size=n, max_size=n))
    grid = st.integers(-20, 20).map(lambda v: v * 0.125)       # coarse lattice: exact ties
    ys = data.draw(st.lists(grid, min_size=n, max_size=n))
    zs = data.draw(st.lists(grid, min_size=n, max_size=n))
    ndup = data.draw(st.integers(0, n))
    idx = data.draw(st.lists(st.integers(0, n - 1), min_size=ndup, max_size=ndup))
    ys += [ys[i] for i in idx]; zs += [zs[i] for i in idx]
    rows += [rows[i] for i in idx]; secs += [secs[i] for i in idx]
    ev = tiny_event(ys, zs, rows, secs)
    P = orc.default_params()
    r = orc.track(ev, precision=32)
    bu, bd = brute_links(ev.x, ev.y, ev.z, ev.row, ev.sector, P, 159)
    np.testing.assert_array_equal(r['up'], bu)
    np.testing.assert_array_equal(r['dn'], bd)


def test_neighbours_random_dense_rows(orc):
    rng = np.random.default_rng(5)
    n = 180
    rows = rng.integers(10, 14, n)
    ev = tiny_event(rng.uniform(-2, 2, n), rng.uniform(-2, 2, n), rows, np.zeros(n, int))
    r = orc.track(ev, precision=32)
    bu, bd = brute_links(ev.x, ev.y, ev.z, ev.row, ev.sector, orc.default_params(), 159)
    np.testing.assert_array_equal(r['up'], bu)
    np.testing.assert_array_equal(r['dn'], bd)
    assert (bu >= 0).sum() > 20


@pytest.fixture(scope="module")
def c1(orc):
    ev = synth.make_config('C1')
    return ev, orc.track(ev, precision=32)


@pytest.fixture(scope="module")
def c2(orc):
    ev = synth.make_config('C2')
    return ev, orc.track(ev, precision=32)


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_link_invariants(which, request):
    ev, r = request.getfixturevalue(which)
    up, dn, cup, cdn = r['up'], r['dn'], r['cup'], r['cdn']
    i = np.nonzero(cup >= 0)[0]
    np.testing.assert_array_equal(cdn[cup[i]], i)                 # reciprocal
    j = np.nonzero(cdn >= 0)[0]
    np.testing.assert_array_equal(cup[cdn[j]], j)
    assert np.all(ev.row[cup[i]] == ev.row[i] + 1)                # one row per link
    assert np.all(ev.sector[cup[i]] == ev.sector[i])
    # idempotence: cleaning the cleaned links changes nothing
    cup2 = np.where((cup >= 0) & (cdn[np.maximum(cup, 0)] == np.arange(len(cup))), cup, -1)
    np.testing.assert_array_equal(cup2, cup)
    # raw links: cleaned links are a subset
    assert np.all((cup < 0) | (cup == up)) and np.all((cdn < 0) | (cdn == dn))
    # start hits are the chain heads, in (sector, row, id) order
    heads = np.nonzero((cup >= 0) & (cdn < 0))[0]
    order = np.lexsort((heads, ev.row[heads], ev.sector[heads]))
    np.testing.assert_array_equal(r['starts'], heads[order])
    # number of chains = number of heads (every linked cluster reaches exactly one head)
    linked = np.nonzero((cup >= 0) | (cdn >= 0))[0]
    head_of = {}
    for h in heads:
        q = h
        while q >= 0:
            assert q not in head_of
            head_of[q] = h
            q = cup[q]
    assert set(head_of) == set(linked.tolist())


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_track_invariants(which, request, orc):
    ev, r = request.getfixturevalue(which)
    facts = json.load(open(GOLDEN))
    P = orc.default_params()
    off, ids = r['hit_off'], r['hit_ids']
    assert len(np.unique(ids)) == len(ids)                        # each cluster in <= 1 track
    for t in range(len(off) - 1):
        h = ids[off[t]:off[t + 1]]
        rows = ev.row[h]
        assert np.all(np.diff(rows) > 0)                          # <= 1 hit per row, ascending
        assert P.min_hits <= len(h) <= facts["max_clusters_per_track"]
        assert np.all(ev.sector[h] == r['sector'][t])
        assert r['ndf'][t] == 2 * len(h) - 5
    # canonical order of start hits
    st_ = r['seed_start'][r['trk_seed']]
    key = ev.sector[st_].astype(np.int64) * 10**12 + ev.row[st_].astype(np.int64) * 10**8 + st_
    assert np.all(np.diff(key) > 0)
    # seeds: chain heads with chain length >= min_seed_hits, seed hits one per row
    assert facts["seed_hits_low"] == P.min_seed_hits
    for k in range(len(r['seed_start'])):
        row_hits = r['seed_hits'][k]
        v = row_hits[row_hits >= 0]
        assert len(v) == r['seed_nhits'][k]
        assert np.all(ev.row[v] == np.nonzero(row_hits >= 0)[0])


def test_shuffle_invariance_c1(orc, c1):
    ev, r = c1
    rng = np.random.default_rng(99)
    perm = rng.permutation(ev.n)
    ev2 = SimpleNamespace(x=ev.x[perm], y=ev.y[perm], z=ev.z[perm], row=ev.row[perm],
                          sector=ev.sector[perm], geom=ev.geom, n=ev.n)
    r2 = orc.track(ev2, precision=32)

    def tracks(ev_, rr):
        out = set()
        for t in range(len(rr['hit_off']) - 1):
            h = rr['hit_ids'][rr['hit_off'][t]:rr['hit_off'][t + 1]]
            out.add(tuple(zip(ev_.x[h].tolist(), ev_.y[h].tolist(), ev_.z[h].tolist())))
        return out

    assert tracks(ev, r) == tracks(ev2, r2)


def test_empty_and_single_cluster(orc):
    for n in (0, 1):
        ev = tiny_event(np.zeros(n), np.zeros(n), np.full(n, 5), np.zeros(n, int))
        r = orc.track(ev, precision=32)
        assert len(r['starts']) == 0 and len(r['hit_off']) == 1
