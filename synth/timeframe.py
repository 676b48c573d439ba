"""Synthetic continuous-readout time frames.

With continuous readout (the paper's Run-3 outlook, Sec. "Track
reconstruction in the TPC") the TPC delivers time frames of many
overlapping collisions instead of triggered events.  A cluster is then
known by its readout time, not by its z: a cluster created at z by a
collision at time t_c drifts to the end plate of its side and is read out
at t = t_c + (L - side z) / v_drift.  Everything here is in drift-length
units (cm): tau = v_drift t = c + (L - side z) with c = v_drift t_c, side =
+1 for A-side sectors (0-17) and -1 for C-side sectors (18-35).

A frame of length F holds M collisions at uniform times c in [0, F); each
collision is an event of the batching workload's lognormal multiplicity
(make_event with its seed); clusters with tau >= F belong to the next
frame and are dropped, as are clusters smeared to tau < 0.  The clusters
of all collisions are shuffled together.  No tracker arithmetic lives here: the frame is only input.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .events import Geometry, N_WEDGES, Z_MAX, default_geometry, make_event


@dataclass
class TimeFrame:
    x: np.ndarray             # float32 [n] sector-local x
    y: np.ndarray             # float32 [n]
    tau: np.ndarray           # float32 [n] readout time in drift-length units (cm)
    row: np.ndarray           # int16 [n]
    sector: np.ndarray        # uint8 [n]
    tau64: np.ndarray         # float64 values before the FP32 cast
    z64: np.ndarray           # float64 true z of the cluster (before smearing: the smeared z)
    truth_track: np.ndarray   # int32 [n] frame-wide particle index, -1 for noise
    truth_coll: np.ndarray    # int32 [n] collision index
    truth_double: np.ndarray  # bool [n]
    coll_c: np.ndarray        # float64 [M] collision times (cm of drift)
    tracks: dict              # per-particle truth (concatenated over collisions) + 'coll'
    length: float             # frame length F (cm of drift)
    geom: Geometry
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _multiplicity(rng, lo=50, hi=20000):
    mu, sd = np.log(1000.0), np.log(400.0) / 6.0
    while True:
        n = int(round(np.exp(rng.normal(mu, sd))))
        if lo <= n <= hi:
            return n


def make_timeframe(seed: int, n_collisions: int, length: float, noise: float = 0.02,
                   multiplicity=None, times=None, smear: bool = True, geom: Geometry = None,
                   **event_kw) -> TimeFrame:
    """A frame of `n_collisions` collisions over `length` cm of drift.
    multiplicity: None (lognormal, as the batching workload), an int, or a
    list of ints; times: None (uniform in [0, length)) or a list of c."""
    geom = geom or default_geometry()
    rng = np.random.Generator(np.random.PCG64(seed))
    if times is None:
        times = rng.uniform(0.0, length, n_collisions)
    times = np.asarray(times, dtype=np.float64)
    if multiplicity is None:
        mult = [_multiplicity(rng) for _ in range(n_collisions)]
    elif np.isscalar(multiplicity):
        mult = [int(multiplicity)] * n_collisions
    else:
        mult = [int(m) for m in multiplicity]
    L = float(geom.z_max)
    cols = {k: [] for k in ("x", "y", "tau", "row", "sector", "z", "trk", "coll", "dbl")}
    trk_all = {}
    base = 0
    for k in range(n_collisions):
        ev = make_event(seed=seed * 1000 + k + 1, n_primaries=mult[k], noise=noise, smear=smear,
                        geom=geom, shuffle=False, **event_kw)
        side = np.where(ev.sector.astype(np.int64) < N_WEDGES, 1.0, -1.0)
        tau = times[k] + (L - side * ev.z64)
        # inside [0, F) also after the FP32 cast (smearing can put a cluster
        # of a collision at c = 0 before the frame start)
        keep = (tau >= 0.0) & (tau < length) & (tau.astype(np.float32) < np.float32(length))
        cols["x"].append(ev.x64[keep]); cols["y"].append(ev.y64[keep]); cols["tau"].append(tau[keep])
        cols["row"].append(ev.row[keep]); cols["sector"].append(ev.sector[keep]); cols["z"].append(ev.z64[keep])
        t = ev.truth_track[keep]
        cols["trk"].append(np.where(t >= 0, t + base, -1).astype(np.int32))
        cols["coll"].append(np.full(int(keep.sum()), k, np.int32))
        cols["dbl"].append(ev.truth_double[keep])
        ntr = len(ev.tracks["q"])
        for key, v in ev.tracks.items():
            trk_all.setdefault(key, []).append(np.asarray(v))
        trk_all.setdefault("coll", []).append(np.full(ntr, k, np.int32))
        base += ntr
    cat = {k: np.concatenate(v) for k, v in cols.items()}
    tracks = {k: np.concatenate(v) for k, v in trk_all.items()}
    n = cat["x"].shape[0]
    perm = rng.permutation(n)
    tf = TimeFrame(x=cat["x"][perm].astype(np.float32), y=cat["y"][perm].astype(np.float32),
                   tau=cat["tau"][perm].astype(np.float32), row=cat["row"][perm].astype(np.int16),
                   sector=cat["sector"][perm].astype(np.uint8), tau64=cat["tau"][perm], z64=cat["z"][perm],
                   truth_track=cat["trk"][perm], truth_coll=cat["coll"][perm], truth_double=cat["dbl"][perm],
                   coll_c=times, tracks=tracks, length=float(length), geom=geom, seed=seed)
    tf.meta = dict(n_collisions=n_collisions, multiplicity=mult, noise=noise, smear=smear)
    return tf


# Time-frame workloads (lengths in cm of drift; L = 250 cm is one full drift):
#   TF-small: 6 collisions of 300 primaries over 3 drift lengths, sliced per
#             drift length (parity case, seconds in the oracle);
#   TF:       24 collisions of the batching workload's lognormal multiplicity
#             over 6 drift lengths (4 collisions per drift time), sliced per
#             drift length.
TF_CONFIGS = {
    "TF-small": dict(seed=1006001, n_collisions=6, length=3 * Z_MAX, multiplicity=300),
    "TF": dict(seed=1006002, n_collisions=24, length=6 * Z_MAX),
}
TF_SLICE = Z_MAX


def make_tf_config(name: str, **over) -> TimeFrame:
    kw = dict(TF_CONFIGS[name]); kw.update(over)
    return make_timeframe(**kw)
