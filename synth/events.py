"""Synthetic central-Pb-Pb-shaped TPC events.

The paper's tracking timings (Sec. "Track reconstruction in the TPC",
Table 1) were taken on real central Pb-Pb data that is not available here.
These seeded events stand in for it.  Everything is generated in FP64 with
``numpy.random.Generator(PCG64(seed))`` and cast once to the FP32 SoA that
the tracker consumes; the FP64 values are kept for exactness checks.

Detector model (all lengths in cm):
  * 18 azimuthal wedges of 20 deg, each split at z = 0 into an A-side (z >= 0,
    sectors 0-17) and a C-side sector (z < 0, sectors 18-35);
  * wedge w is centred at alpha_w = (w + 0.5) * 20 deg; its local frame is
    x = r cos(phi - alpha), y = r sin(phi - alpha), z global;
  * 159 pad-row planes x = X_r, X_r = 85 + r * 162 / 158, rounded once to FP32
    (the clusters of a row lie exactly on the FP32 plane);
  * acceptance |y| <= X_r tan(10 deg), |z| <= 250;
  * uniform solenoid B_z = 0.5 T, no material.

A helix produces one cluster per crossing of a row plane inside a sector's
acceptance, on its outgoing leg only (transverse turning angle <= pi).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

C_LIGHT = 2.99792458e-3          # GeV / (T cm): radius[cm] = pT / (C_LIGHT * B)
N_ROWS = 159
N_WEDGES = 18
N_SECTORS = 36
R_FIRST, R_LAST = 85.0, 247.0
Z_MAX = 250.0
SIGMA_Y, SIGMA_Z = 0.1, 0.15
SIGMA_TGL_EXT = 1e-3
MAP_NA, MAP_NB = 8, 8
BSPLINE_KNOTS = np.array([0, 0, 0, 0, 0.2, 0.4, 0.6, 0.8, 1, 1, 1, 1], dtype=np.float64)


@dataclass
class Geometry:
    row_x: np.ndarray                     # float32 [n_rows]
    tan_half_angle: np.float32
    z_max: np.float32
    bz: np.float32
    n_sectors: int = N_SECTORS
    n_rows: int = N_ROWS


def default_geometry() -> Geometry:
    rx = (R_FIRST + np.arange(N_ROWS, dtype=np.float64) * ((R_LAST - R_FIRST) / (N_ROWS - 1)))
    return Geometry(row_x=rx.astype(np.float32),
                    tan_half_angle=np.float32(np.tan(np.deg2rad(10.0))),
                    z_max=np.float32(Z_MAX), bz=np.float32(0.5))


@dataclass
class CalibTheta:
    """Calibration parameters: per-sector drift scale delta, time offset tau
    (cm) and a 36 x 8 x 8 radial displacement map (cm)."""
    drift_scale: np.ndarray   # float64 [36]
    time_offset: np.ndarray   # float64 [36]
    dmap: np.ndarray          # float64 [36, 8, 8]

    @staticmethod
    def zeros() -> "CalibTheta":
        return CalibTheta(np.zeros(N_SECTORS), np.zeros(N_SECTORS), np.zeros((N_SECTORS, MAP_NA, MAP_NB)))

    def flat(self) -> np.ndarray:
        return np.concatenate([self.drift_scale, self.time_offset, self.dmap.ravel()])


@dataclass
class Event:
    x: np.ndarray             # float32 [n]
    y: np.ndarray
    z: np.ndarray
    row: np.ndarray           # int16 [n]
    sector: np.ndarray        # uint8 [n]
    x64: np.ndarray           # float64 values before the FP32 cast
    y64: np.ndarray
    z64: np.ndarray
    truth_track: np.ndarray   # int32 [n], -1 for noise
    truth_double: np.ndarray  # bool [n], second cluster of a doubled crossing
    tracks: dict              # per-track truth arrays
    geom: Geometry
    seed: int
    theta: Optional[CalibTheta] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def bspline_basis(u: np.ndarray) -> np.ndarray:
    """The 8 clamped uniform cubic B-spline basis functions on [0, 1]
    (knots 0,0,0,0,1/5,2/5,3/5,4/5,1,1,1,1), by the Cox-de Boor recursion.
    Arguments outside [0, 1] are clamped."""
    t = BSPLINE_KNOTS
    u = np.clip(np.asarray(u, dtype=np.float64), 0.0, 1.0)
    n = u.shape[0]
    m = len(t) - 1
    # one row per basis function (contiguous), transposed at the end
    N = np.zeros((m, n))
    for i in range(m):
        N[i] = (t[i] <= u) & (u < t[i + 1])
    N[7, u >= 1.0] = 1.0           # right end belongs to the last non-empty span
    for p in range(1, 4):
        M = np.zeros((m - p, n))
        for i in range(m - p):
            a = (u - t[i]) / (t[i + p] - t[i]) if t[i + p] > t[i] else 0.0
            b = (t[i + p + 1] - u) / (t[i + p + 1] - t[i + 1]) if t[i + p + 1] > t[i + 1] else 0.0
            M[i] = a * N[i] + b * N[i + 1]
        N = M
    return np.ascontiguousarray(N[:8].T)


def draw_theta(seed: int = 1005999, sd_delta=2e-3, sd_tau=0.1, amp=0.3) -> CalibTheta:
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(0.0, sd_delta, N_SECTORS)
    tau = rng.normal(0.0, sd_tau, N_SECTORS)
    c = rng.uniform(-amp, amp, (N_SECTORS, MAP_NA, MAP_NB))
    return CalibTheta(d, tau, c)


def _side(sector: np.ndarray) -> np.ndarray:
    return np.where(sector < N_WEDGES, 1.0, -1.0)


def _radial_displacement(theta: CalibTheta, sector, x, y, tan_a):
    xh = (x - R_FIRST) / (R_LAST - R_FIRST)
    uh = (y / x + tan_a) / (2.0 * tan_a)
    Ba = bspline_basis(xh)
    Bb = bspline_basis(uh)
    c = theta.dmap[sector]                      # [n, 8, 8]
    return np.einsum('na,nab,nb->n', Ba, c, Bb)


def apply_inverse_calibration(theta: CalibTheta, sector, x, y, z, tan_a, zmax=Z_MAX):
    """Map true (smeared) cluster positions to the positions a default
    transformation would report under miscalibration theta, i.e. the inverse
    of the correction: drift (closed form) and radial map (fixed point, FP64)."""
    sector = np.asarray(sector, dtype=np.int64)
    side = _side(sector)
    dl, tau = theta.drift_scale[sector], theta.time_offset[sector]
    zd = side * (zmax - tau - (zmax - side * z) / (1.0 + dl))
    xd = x.copy()
    for _ in range(200):
        nx = x - _radial_displacement(theta, sector, xd, y, tan_a)
        done = np.max(np.abs(nx - xd)) if nx.size else 0.0
        xd = nx
        if done < 1e-12:
            break
    return xd, zd


def _helix_crossings(tr: dict, geom: Geometry, wedges, single_sector: bool):
    """All (track, wedge, row) crossings on the outgoing leg, in FP64."""
    X = geom.row_x.astype(np.float64)
    tan_a = float(np.float64(geom.tan_half_angle))
    kap = -C_LIGHT * float(geom.bz) * tr['q'] / tr['pt']        # signed curvature, ccw > 0
    tgl = np.sinh(tr['eta'])
    out = {k: [] for k in ('trk', 'sector', 'row', 'y', 'z', 'ell')}
    ntr = kap.shape[0]
    rows = np.arange(N_ROWS)
    for w in wedges:
        a = (w + 0.5) * np.deg2rad(20.0)
        ca, sa = np.cos(a), np.sin(a)
        xvl = tr['xv'] * ca + tr['yv'] * sa
        yvl = -tr['xv'] * sa + tr['yv'] * ca
        psi0 = tr['phi0'] - a
        k2 = kap[:, None]
        v = np.sin(psi0)[:, None] + k2 * (X[None, :] - xvl[:, None])
        okv = np.abs(v) <= 1.0
        vs = np.clip(v, -1.0, 1.0)
        base = np.arcsin(vs)
        for th in (base, np.pi - base):
            dpsi = np.where(k2 > 0, th - psi0[:, None], psi0[:, None] - th)
            dpsi = np.mod(dpsi, 2.0 * np.pi)
            ell = dpsi / np.abs(k2)
            ok = okv & (ell > 0) & (dpsi <= np.pi)
            yl = yvl[:, None] - (np.cos(th) - np.cos(psi0)[:, None]) / k2
            z = tr['zv'][:, None] + tgl[:, None] * ell
            ok &= (np.abs(yl) <= X[None, :] * tan_a) & (np.abs(z) <= float(geom.z_max))
            ti, ri = np.nonzero(ok)
            if ti.size == 0:
                continue
            zz = z[ti, ri]
            if single_sector:
                sec = np.zeros_like(ti)
            else:
                sec = w + N_WEDGES * (zz < 0)
            out['trk'].append(ti)
            out['sector'].append(sec)
            out['row'].append(rows[ri])
            out['y'].append(yl[ti, ri])
            out['z'].append(zz)
            out['ell'].append(ell[ti, ri])
    if not out['trk']:
        return {k: np.zeros(0, dtype=np.int64 if k in ('trk', 'sector', 'row') else np.float64) for k in out}
    res = {k: np.concatenate(v) for k, v in out.items()}
    # canonical generation order: by track, then arc length (outgoing leg order)
    order = np.lexsort((res['ell'], res['trk']))
    return {k: v[order] for k, v in res.items()}


def make_event(seed: int, n_primaries: int, n_secondaries: int = 0, noise: float = 0.0,
               doubling: float = 0.0, single_sector: bool = False, smear: bool = True,
               pt_range=(0.1, 10.0), eta_range=(-0.9, 0.9), phi_range=None,
               theta: Optional[CalibTheta] = None, geom: Optional[Geometry] = None,
               shuffle: bool = True) -> Event:
    geom = geom or default_geometry()
    rng = np.random.Generator(np.random.PCG64(seed))
    if phi_range is None:
        phi_range = (0.0, np.deg2rad(20.0)) if single_sector else (0.0, 2.0 * np.pi)

    def draw_kin(n):
        q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        pt = np.exp(rng.uniform(np.log(pt_range[0]), np.log(pt_range[1]), n))
        eta = rng.uniform(eta_range[0], eta_range[1], n)
        phi0 = rng.uniform(phi_range[0], phi_range[1], n)
        return q, pt, eta, phi0

    q, pt, eta, phi0 = draw_kin(n_primaries)
    xv = np.zeros(n_primaries); yv = np.zeros(n_primaries); zv = np.zeros(n_primaries)
    prim = np.ones(n_primaries, dtype=bool)
    if n_secondaries:
        rho = rng.uniform(0.0, 60.0, n_secondaries)
        az = rng.uniform(0.0, 2.0 * np.pi, n_secondaries)
        eta_p = rng.uniform(-0.9, 0.9, n_secondaries)
        q2, pt2, eta2, phi2 = draw_kin(n_secondaries)
        q = np.concatenate([q, q2]); pt = np.concatenate([pt, pt2])
        eta = np.concatenate([eta, eta2]); phi0 = np.concatenate([phi0, phi2])
        xv = np.concatenate([xv, rho * np.cos(az)]); yv = np.concatenate([yv, rho * np.sin(az)])
        zv = np.concatenate([zv, rho * np.sinh(eta_p)])
        prim = np.concatenate([prim, np.zeros(n_secondaries, dtype=bool)])
    tr = dict(q=q, pt=pt, eta=eta, phi0=phi0, xv=xv, yv=yv, zv=zv, primary=prim,
              tgl=np.sinh(eta))
    tr['tgl_ext'] = tr['tgl'] + rng.normal(0.0, SIGMA_TGL_EXT, q.shape[0])

    wedges = [0] if single_sector else list(range(N_WEDGES))
    cr = _helix_crossings(tr, geom, wedges, single_sector)
    nc = cr['trk'].shape[0]
    X = geom.row_x.astype(np.float64)
    cx = X[cr['row']]
    cy_true, cz_true = cr['y'], cr['z']
    if smear:
        cy = cy_true + rng.normal(0.0, SIGMA_Y, nc)
        cz = cz_true + rng.normal(0.0, SIGMA_Z, nc)
    else:
        cy, cz = cy_true.copy(), cz_true.copy()
    trk = cr['trk'].astype(np.int32)
    sec = cr['sector'].astype(np.int64)
    row = cr['row'].astype(np.int64)
    dbl = np.zeros(nc, dtype=bool)
    if doubling > 0.0 and nc:
        m = rng.random(nc) < doubling
        nd = int(m.sum())
        dy = cy_true[m] + (rng.normal(0.0, SIGMA_Y, nd) if smear else 0.0)
        dz = cz_true[m] + (rng.normal(0.0, SIGMA_Z, nd) if smear else 0.0)
        cx = np.concatenate([cx, cx[m]]); cy = np.concatenate([cy, dy]); cz = np.concatenate([cz, dz])
        trk = np.concatenate([trk, trk[m]]); sec = np.concatenate([sec, sec[m]])
        row = np.concatenate([row, row[m]]); dbl = np.concatenate([dbl, np.ones(nd, dtype=bool)])
    n_noise = int(round(noise * cx.shape[0]))
    if n_noise:
        if single_sector:
            ns = np.zeros(n_noise, dtype=np.int64)
        else:
            ns = rng.integers(0, N_SECTORS, n_noise)
        nr = rng.integers(0, N_ROWS, n_noise)
        nxr = X[nr]
        ymax = nxr * float(geom.tan_half_angle)
        ny = rng.uniform(-1.0, 1.0, n_noise) * ymax
        zu = rng.uniform(0.0, float(geom.z_max), n_noise)
        if single_sector:
            nz = rng.uniform(-float(geom.z_max), float(geom.z_max), n_noise)
        else:
            nz = np.where(ns < N_WEDGES, zu, -zu)
        cx = np.concatenate([cx, nxr]); cy = np.concatenate([cy, ny]); cz = np.concatenate([cz, nz])
        trk = np.concatenate([trk, -np.ones(n_noise, dtype=np.int32)])
        sec = np.concatenate([sec, ns]); row = np.concatenate([row, nr])
        dbl = np.concatenate([dbl, np.zeros(n_noise, dtype=bool)])
    if theta is not None:
        cx, cz = apply_inverse_calibration(theta, sec, cx, cy, cz, float(geom.tan_half_angle),
                                           float(geom.z_max))
    n = cx.shape[0]
    perm = rng.permutation(n) if shuffle else np.arange(n)
    ev = Event(x=cx[perm].astype(np.float32), y=cy[perm].astype(np.float32),
               z=cz[perm].astype(np.float32), row=row[perm].astype(np.int16),
               sector=sec[perm].astype(np.uint8), x64=cx[perm], y64=cy[perm], z64=cz[perm],
               truth_track=trk[perm], truth_double=dbl[perm], tracks=tr, geom=geom, seed=seed,
               theta=theta)
    ev.meta = dict(n_primaries=n_primaries, n_secondaries=n_secondaries, noise=noise,
                   doubling=doubling, single_sector=single_sector, smear=smear)
    return ev


def _c4_multiplicity(e: int) -> int:
    rng = np.random.Generator(np.random.PCG64(1004000 + e + 500000))
    mu, sd = np.log(1000.0), np.log(400.0) / 6.0
    while True:
        n = int(round(np.exp(rng.normal(mu, sd))))
        if 50 <= n <= 20000:
            return n


CONFIGS = {
    # one wedge spanning both z-sides, tracked as one unit (sector index 0)
    'C1': dict(seed=1001, n_primaries=200, noise=0.01, single_sector=True),
    # full 36-sector event, ~0.7 M clusters
    'C2': dict(seed=1002, n_primaries=5000, noise=0.02),
    # central-Pb-Pb-shaped event, ~3 M clusters
    'C3': dict(seed=1003, n_primaries=18000, n_secondaries=4000, noise=0.05, doubling=0.10),
}


def _make_indexed(args):
    name, index = args
    return make_config(name, index)


def make_configs(name: str, indices, workers: int = 8) -> list:
    """make_config(name, i) for every i of `indices`, in order, generated in
    up to `workers` worker processes (events are independent; a miscalibrated
    event costs seconds in the FP64 fixed-point inverse of the calibration).
    Workers use the 'spawn' start method, so they never inherit a GPU
    context; a script that calls this needs the usual __main__ guard."""
    import concurrent.futures
    import multiprocessing
    import os
    indices = list(indices)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(workers, avail, len(indices)))
    if workers == 1:
        return [make_config(name, i) for i in indices]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as pool:
        return list(pool.map(_make_indexed, [(name, i) for i in indices]))


def make_config(name: str, index: int = 0, **over) -> Event:
    """C1/C2/C3 events; C4 event `index` (0..63, lognormal multiplicity);
    C5 event `index` (C2-sized, miscalibrated with draw_theta())."""
    if name in CONFIGS:
        kw = dict(CONFIGS[name]); kw.update(over)
        return make_event(**kw)
    if name == 'C4':
        kw = dict(seed=1004000 + index, n_primaries=_c4_multiplicity(index), noise=0.02)
        kw.update(over)
        return make_event(**kw)
    if name == 'C5':
        kw = dict(seed=1005000 + index, n_primaries=5000, noise=0.02, theta=draw_theta())
        kw.update(over)
        return make_event(**kw)
    raise KeyError(name)
