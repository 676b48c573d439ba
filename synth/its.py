"""Synthetic events of an ITS-like six-layer silicon tracker.

The paper's fast ITS standalone tracking (Sec. "Fast ITS standalone
tracking") runs on the clusters of six silicon layers around the beam pipe
(two pixel layers, two drift layers, two strip layers) and uses a constant
solenoid field and the average material of each layer for multiple
scattering.  The real geometry and data are not available; this generator
stands in for them.  Everything is FP64 (numpy PCG64) cast once to the FP32
cluster SoA.

Detector model (lengths in cm):
  * layer l is a polygon of n_l flat staves around the beam axis: stave k
    lies in the plane at distance r_l from the axis whose normal points at
    alpha = (k + 1/2) 2 pi / n_l; its local frame is x = along the normal,
    y = across, z global; it covers |y| <= r_l tan(pi / n_l), |z| <= h_l;
  * r = 3.9, 7.6, 15.0, 23.9, 38.0, 43.0; n = 20, 40, 14, 22, 34, 38;
    h = 14.1, 14.1, 22.2, 29.7, 43.1, 48.9 (the Run-2 ITS layout);
  * resolution (y, z) = (12, 100), (35, 25), (20, 830) um for the pixel,
    drift and strip layers; material x/X0 = 1.14 %, 1.14 %, 1.13 %, 1.26 %,
    0.83 %, 0.86 % per layer;
  * uniform B_z = 0.5 T.
Particles start at a vertex drawn around the beam axis (transverse 50 um,
longitudinal 5 cm); at each layer crossing the direction receives a
Gaussian multiple-scattering kick of the Highland width (beta = 1, path
through the stave at the crossing angle) in two orthogonal planes.  A
particle leaves when it misses a layer's polygon in z, or curls before it.
Noise clusters are spread uniformly over the staves.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 2.99792458e-3


@dataclass
class ItsGeometry:
    radius: np.ndarray        # float32 [6] stave plane distance from the axis
    n_staves: np.ndarray      # int32 [6]
    half_z: np.ndarray        # float32 [6]
    x_over_x0: np.ndarray     # float32 [6]
    sigma_y: np.ndarray       # float32 [6]
    sigma_z: np.ndarray       # float32 [6]
    bz: float = 0.5

    @property
    def n_layers(self) -> int:
        return int(self.radius.shape[0])


def default_its_geometry() -> ItsGeometry:
    return ItsGeometry(
        radius=np.array([3.9, 7.6, 15.0, 23.9, 38.0, 43.0], np.float32),
        n_staves=np.array([20, 40, 14, 22, 34, 38], np.int32),
        half_z=np.array([14.1, 14.1, 22.2, 29.7, 43.1, 48.9], np.float32),
        x_over_x0=np.array([0.0114, 0.0114, 0.0113, 0.0126, 0.0083, 0.0086], np.float32),
        sigma_y=np.array([0.0012, 0.0012, 0.0035, 0.0035, 0.0020, 0.0020], np.float32),
        sigma_z=np.array([0.0100, 0.0100, 0.0025, 0.0025, 0.0830, 0.0830], np.float32))


@dataclass
class ItsEvent:
    x: np.ndarray             # float32 [n] stave-local x (the stave plane)
    y: np.ndarray
    z: np.ndarray
    layer: np.ndarray         # int8 [n]
    stave: np.ndarray         # int16 [n]
    y64: np.ndarray
    z64: np.ndarray
    truth_track: np.ndarray   # int32 [n], -1 for noise
    tracks: dict              # per-particle truth
    vertex: np.ndarray        # float64 [3]
    geom: ItsGeometry
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def highland(p, t):
    """Highland width (rad) for momentum p (GeV, beta = 1) through t radiation lengths."""
    return 0.0136 / p * np.sqrt(t) * (1.0 + 0.038 * np.log(t))


def make_its_event(seed: int, n_primaries: int, noise: float = 0.0, smear: bool = True, scatter: bool = True,
                   pt_range=(0.1, 10.0), eta_range=(-0.9, 0.9), vertex=None, geom: ItsGeometry = None,
                   shuffle: bool = True) -> ItsEvent:
    geom = geom or default_its_geometry()
    rng = np.random.Generator(np.random.PCG64(seed))
    if vertex is None:
        vertex = np.array([rng.normal(0.0, 0.005), rng.normal(0.0, 0.005), rng.normal(0.0, 5.0)])
    vertex = np.asarray(vertex, np.float64)
    n = n_primaries
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    pt = np.exp(rng.uniform(np.log(pt_range[0]), np.log(pt_range[1]), n))
    eta = rng.uniform(eta_range[0], eta_range[1], n)
    phi0 = rng.uniform(0.0, 2.0 * np.pi, n)
    tracks = dict(q=q, pt=pt, eta=eta, phi0=phi0, tgl=np.sinh(eta))
    # state per particle: global position, transverse direction angle psi,
    # tan(lambda), curvature (ccw > 0), alive flag
    X = np.full(n, vertex[0]); Y = np.full(n, vertex[1]); Z = np.full(n, vertex[2])
    psi = phi0.copy()
    tgl = np.sinh(eta)
    kap = -C_LIGHT * geom.bz * q / pt
    alive = np.ones(n, bool)
    out = {k: [] for k in ("trk", "layer", "stave", "y", "z")}
    for l in range(geom.n_layers):
        r = float(np.float64(geom.radius[l]))
        ns = int(geom.n_staves[l])
        w = r * np.tan(np.pi / ns)
        dk = 2.0 * np.pi / ns
        # stave guessed from the azimuth where the transverse circle reaches radius r
        # (then corrected by the exact plane crossing); the chord estimate is enough
        step = np.maximum(r - np.hypot(X, Y), 0.0)
        ang = np.arctan2(Y + step * np.sin(psi), X + step * np.cos(psi))
        k0 = np.floor(np.mod(ang, 2.0 * np.pi) / dk).astype(np.int64) % ns
        hit = np.zeros(n, bool)
        ky = np.zeros(n, np.int64); yy = np.zeros(n); zz = np.zeros(n); ell_b = np.full(n, np.inf)
        psi_b = np.zeros(n)
        for dkk in (0, -1, 1):
            k = (k0 + dkk) % ns
            a = (k + 0.5) * dk
            ca, sa = np.cos(a), np.sin(a)
            xl = X * ca + Y * sa
            yl = -X * sa + Y * ca
            p0 = psi - a
            with np.errstate(invalid="ignore", divide="ignore"):
                v = np.sin(p0) + kap * (r - xl)
                okv = np.abs(v) <= 1.0
                base = np.arcsin(np.clip(v, -1.0, 1.0))
                for th in (base, np.pi - base):
                    dpsi = np.where(kap > 0, th - p0, p0 - th)
                    dpsi = np.mod(dpsi, 2.0 * np.pi)
                    ell = dpsi / np.abs(kap)
                    y1 = yl - (np.cos(th) - np.cos(p0)) / kap
                    z1 = Z + tgl * ell
                    ok = alive & okv & (ell > 1e-9) & (dpsi <= np.pi) & (np.abs(y1) <= w) & (np.abs(z1) <= float(geom.half_z[l]))
                    better = ok & (ell < ell_b)
                    ell_b = np.where(better, ell, ell_b)
                    ky = np.where(better, k, ky)
                    yy = np.where(better, y1, yy)
                    zz = np.where(better, z1, zz)
                    psi_b = np.where(better, th + a, psi_b)
                    hit |= better
        alive &= hit
        idx = np.nonzero(alive)[0]
        a = (ky[idx] + 0.5) * dk
        out["trk"].append(idx); out["layer"].append(np.full(idx.size, l)); out["stave"].append(ky[idx])
        out["y"].append(yy[idx]); out["z"].append(zz[idx])
        # move to the crossing
        X[idx] = r * np.cos(a) - yy[idx] * np.sin(a)
        Y[idx] = r * np.sin(a) + yy[idx] * np.cos(a)
        Z[idx] = zz[idx]
        psi[idx] = psi_b[idx]
        if scatter and idx.size:
            lam = np.arctan(tgl[idx])
            p = (np.abs(C_LIGHT * geom.bz / kap[idx])) / np.cos(lam)
            cphi = np.abs(np.cos(psi[idx] - a))          # crossing angle against the stave normal
            t = float(geom.x_over_x0[l]) / (np.cos(lam) * np.maximum(cphi, 1e-3))
            th0 = highland(p, t)
            d1 = rng.normal(0.0, 1.0, idx.size) * th0
            d2 = rng.normal(0.0, 1.0, idx.size) * th0
            lam2 = lam + d2
            psi[idx] += d1 / np.cos(lam)
            kap[idx] = kap[idx] * np.cos(lam) / np.cos(lam2)
            tgl[idx] = np.tan(lam2)
    trk = np.concatenate(out["trk"]).astype(np.int32)
    lay = np.concatenate(out["layer"]).astype(np.int64)
    stv = np.concatenate(out["stave"]).astype(np.int64)
    cy = np.concatenate(out["y"]); cz = np.concatenate(out["z"])
    sy = geom.sigma_y.astype(np.float64)[lay]; sz = geom.sigma_z.astype(np.float64)[lay]
    if smear:
        cy = cy + rng.normal(0.0, 1.0, cy.size) * sy
        cz = cz + rng.normal(0.0, 1.0, cz.size) * sz
    n_noise = int(round(noise * trk.size))
    if n_noise:
        nl = rng.integers(0, geom.n_layers, n_noise)
        nst = np.array([rng.integers(0, int(geom.n_staves[l])) for l in nl], np.int64)
        rr = geom.radius.astype(np.float64)[nl]
        wn = rr * np.tan(np.pi / geom.n_staves.astype(np.float64)[nl])
        ny = rng.uniform(-1.0, 1.0, n_noise) * wn
        nz = rng.uniform(-1.0, 1.0, n_noise) * geom.half_z.astype(np.float64)[nl]
        trk = np.concatenate([trk, -np.ones(n_noise, np.int32)]); lay = np.concatenate([lay, nl])
        stv = np.concatenate([stv, nst]); cy = np.concatenate([cy, ny]); cz = np.concatenate([cz, nz])
    m = trk.size
    perm = rng.permutation(m) if shuffle else np.arange(m)
    xr = geom.radius[lay]
    ev = ItsEvent(x=xr[perm].astype(np.float32), y=cy[perm].astype(np.float32), z=cz[perm].astype(np.float32),
                  layer=lay[perm].astype(np.int8), stave=stv[perm].astype(np.int16), y64=cy[perm], z64=cz[perm],
                  truth_track=trk[perm], tracks=tracks, vertex=vertex, geom=geom, seed=seed)
    ev.meta = dict(n_primaries=n_primaries, noise=noise, smear=smear, scatter=scatter)
    return ev


# ITS workloads: a pp-like event (60 primaries), a minimum-bias-Pb-Pb-like
# event (600 primaries) and a central-Pb-Pb-like one (3,000 primaries within
# |eta| < 0.9, about 1,700 per unit of rapidity), 1 % noise.
ITS_CONFIGS = {
    "ITS-pp": dict(seed=1007001, n_primaries=60, noise=0.01),
    "ITS-mb": dict(seed=1007002, n_primaries=600, noise=0.01),
    "ITS-central": dict(seed=1007003, n_primaries=3000, noise=0.01),
}


def make_its_config(name: str, index: int = 0, **over) -> ItsEvent:
    kw = dict(ITS_CONFIGS[name]); kw["seed"] = kw["seed"] + 1000 * index; kw.update(over)
    return make_its_event(**kw)
