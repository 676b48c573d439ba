"""Injected-truth physics metrics (efficiency, clones, fakes) for tests.

A truth segment is (track, sector); it is reconstructable if it holds at
least `min_hits` non-doubled clusters.  A reconstructed track matches a
segment if at least 90 % of its hits come from that truth track (doubled
clusters count).  Efficiency = matched reconstructable / reconstructable,
clones = extra matches, fakes = unmatched tracks.
"""
import numpy as np


def segment_table(ev, min_hits=10):
    m = (ev.truth_track >= 0) & ~ev.truth_double
    key = ev.truth_track[m].astype(np.int64) * 64 + ev.sector[m].astype(np.int64)
    keys, cnt = np.unique(key, return_counts=True)
    return keys[cnt >= min_hits]


def match_tracks(ev, hit_off, hit_ids, sectors, frac=0.9):
    """Return per-track matched segment key (or -1)."""
    out = np.full(len(hit_off) - 1, -1, dtype=np.int64)
    tt = ev.truth_track
    for t in range(len(hit_off) - 1):
        ids = hit_ids[hit_off[t]:hit_off[t + 1]]
        lab = tt[ids]
        lab = lab[lab >= 0]
        if lab.size == 0:
            continue
        v, c = np.unique(lab, return_counts=True)
        k = np.argmax(c)
        if c[k] >= frac * len(ids):
            out[t] = int(v[k]) * 64 + int(sectors[t])
    return out


def efficiency(ev, hit_off, hit_ids, sectors, min_hits=10, pt_min=None):
    seg = segment_table(ev, min_hits)
    if pt_min is not None:
        pt = ev.tracks['pt'][seg // 64]
        seg = seg[pt >= pt_min]
    m = match_tracks(ev, hit_off, hit_ids, sectors)
    matched = m[m >= 0]
    u, c = np.unique(matched, return_counts=True)
    found = np.isin(seg, u)
    eff = found.mean() if seg.size else 1.0
    clones = int((c - 1).sum())
    fakes = int((m < 0).sum())
    return dict(eff=float(eff), n_seg=int(seg.size), n_found=int(found.sum()), clones=clones,
                fakes=fakes, n_tracks=len(m), clone_rate=clones / max(1, len(m)),
                fake_rate=fakes / max(1, len(m)))
