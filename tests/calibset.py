"""Frozen calibration track subset built from a tracked event and its truth.

Truth-matched primaries with at least `min_hits` hits (the library's FP32
gradient is accurate to about 1e-4 from 40 hits on) and chi2/ndf <= 4 at the
default calibration, whatever pad row their segment starts on (optionally
only segments starting within the first `max_inner_row` + 1 rows).  Each
carries its q/pT prior (the tracklet's final q/pT), the external tan(lambda)
and the vertex flag.
"""
import numpy as np

import truth


def calib_subset(ev, hit_off, hit_ids, sectors, chi2, ndf, k_prior, min_hits=40, max_q=4.0,
                 max_tracks=None, max_inner_row=None):
    m = truth.match_tracks(ev, hit_off, hit_ids, sectors)
    keep = []
    for t in range(len(hit_off) - 1):
        n = hit_off[t + 1] - hit_off[t]
        if m[t] < 0 or n < min_hits or chi2[t] / ndf[t] > max_q:
            continue
        if max_inner_row is not None and ev.row[hit_ids[hit_off[t]]] > max_inner_row:
            continue
        if not ev.tracks['primary'][m[t] // 64]:
            continue
        keep.append(t)
        if max_tracks and len(keep) >= max_tracks:
            break
    keep = np.array(keep, dtype=np.int64)
    offs = [0]; ids = []
    for t in keep:
        h = hit_ids[hit_off[t]:hit_off[t + 1]]
        ids.append(h); offs.append(offs[-1] + len(h))
    ids = np.concatenate(ids) if ids else np.zeros(0, np.int64)
    lab = m[keep] // 64
    return dict(tracks=keep, hit_off=np.array(offs, np.int64), hit_ids=ids.astype(np.int64),
                k0=np.asarray(k_prior)[keep].astype(np.float64),
                ext_tgl=ev.tracks['tgl_ext'][lab].astype(np.float64),
                use_vertex=np.ones(len(keep), np.uint8), truth=lab)
