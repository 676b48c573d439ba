"""CPU oracle of the TPC CA + Kalman track finder -- TEST INFRASTRUCTURE.

Plain, slow, obviously-correct reference (``oracle.cpp``, built with g++
``-O2 -ffp-contract=off``).  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product path
never does.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpcca_oracle.so")
NPAR = 36 + 36 + 36 * 64


def build(force: bool = True) -> str:
    """Compile the oracle shared library with g++ (no contraction, no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", os.path.join(HERE, "oracle.cpp")]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Geometry(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("n_rows", C.c_int32), ("row_x", C.POINTER(C.c_float)),
                ("tan_half_angle", C.c_float), ("z_max", C.c_float), ("bz", C.c_float)]


class Params(C.Structure):
    _fields_ = [("win_y", C.c_float), ("win_z", C.c_float), ("inv_var_y", C.c_float),
                ("inv_var_z", C.c_float), ("link_cut", C.c_float), ("chi2_ext", C.c_float),
                ("max_gap", C.c_int32), ("min_seed_hits", C.c_int32), ("min_hits", C.c_int32),
                ("owned_num", C.c_int32), ("owned_den", C.c_int32), ("sin_max", C.c_float),
                ("sigma_y", C.c_float), ("sigma_z", C.c_float), ("sigma_vertex", C.c_float),
                ("sigma_tgl", C.c_float), ("chi2_merge", C.c_float), ("merge_dist", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ItsGeometry(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("radius", C.c_float * 6), ("half_z", C.c_float * 6),
                ("x_over_x0", C.c_float * 6), ("sigma_y", C.c_float * 6), ("sigma_z", C.c_float * 6),
                ("n_staves", C.c_int32 * 6), ("bz", C.c_float)]


class ItsParams(C.Structure):
    _fields_ = [("vtx_sin_phi", C.c_float), ("vtx_bin", C.c_float), ("vtx_range", C.c_float),
                ("trk_sin_phi", C.c_float), ("trk_dtgl", C.c_float), ("chi2_cut", C.c_float),
                ("sigma_vy", C.c_float), ("sigma_vz", C.c_float), ("sin_max", C.c_float),
                ("min_clusters", C.c_int32), ("tukey_c", C.c_float), ("fit_iters", C.c_int32),
                ("cov_scale_in", C.c_float)]


class Result(C.Structure):
    P64 = C.POINTER(C.c_int64)
    _fields_ = [("n", C.c_int64), ("up", P64), ("dn", P64), ("cup", P64), ("cdn", P64),
                ("n_starts", C.c_int64), ("starts", P64), ("n_seeds", C.c_int64),
                ("seed_start", P64), ("seed_nhits", C.POINTER(C.c_int32)),
                ("seed_key", C.POINTER(C.c_uint64)), ("seed_rlo", C.POINTER(C.c_int32)),
                ("seed_rhi", C.POINTER(C.c_int32)), ("seed_hits", P64),
                ("seed_state", C.POINTER(C.c_double)), ("n_tracks", C.c_int64),
                ("trk_seed", P64), ("trk_sector", C.POINTER(C.c_int32)),
                ("trk_xref", C.POINTER(C.c_double)), ("trk_p", C.POINTER(C.c_double)),
                ("trk_cov", C.POINTER(C.c_double)), ("trk_chi2", C.POINTER(C.c_double)),
                ("trk_ndf", C.POINTER(C.c_int32)), ("hit_off", P64), ("hit_ids", P64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_default_params.argtypes = [C.POINTER(Params)]
        L.orc_transport.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                    dp, dp, dp]
        L.orc_transport.restype = C.c_int
        L.orc_kf_update.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                    dp, dp, dp]
        L.orc_kf_update1.argtypes = [C.c_int, dp, dp, C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_fit_hits.argtypes = [C.c_int, C.POINTER(Geometry), C.POINTER(Params), C.c_int32, dp, dp,
                                   dp, C.c_double, dp, dp, dp]
        L.orc_fit_hits.restype = C.c_int
        L.orc_track.argtypes = [C.c_int, C.POINTER(Geometry), C.POINTER(Params), C.c_int64, dp, dp, dp,
                                C.POINTER(C.c_int16), C.POINTER(C.c_uint8), C.POINTER(C.c_uint8),
                                C.POINTER(C.POINTER(Result))]
        L.orc_result_free.argtypes = [C.POINTER(Result)]
        L.orc_calib_apply.argtypes = [C.POINTER(Geometry), C.c_int64, C.POINTER(C.c_uint8), dp, dp, dp,
                                      dp, dp, dp]
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        L.orc_rotate.argtypes = [C.c_int, C.c_double, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_rotate.restype = C.c_int
        L.orc_merge.argtypes = [C.POINTER(Geometry), C.POINTER(Params), C.c_int64, dp, dp, dp,
                                C.POINTER(C.c_int16), C.c_int64, i32p, dp, dp, dp, dp, i64p, i64p,
                                i32p, i32p, i32p, dp, dp, i32p, dp, dp, C.POINTER(C.POINTER(Result))]
        fp = C.POINTER(C.c_float)
        L.orc_its_default_params.argtypes = [C.POINTER(ItsParams)]
        L.orc_its_default_params.restype = None
        L.orc_its.argtypes = [C.POINTER(ItsGeometry), C.POINTER(ItsParams), C.c_int64, fp, fp, fp,
                              C.POINTER(C.c_int8), C.POINTER(C.c_int16), i64p, i64p, fp] + \
            [i32p, i32p, i32p, i32p, i32p, fp, i32p, i32p, fp, fp, fp, i32p, i32p, fp, fp, dp, i32p]
        L.orc_its_ms.argtypes = [C.POINTER(ItsGeometry), C.c_int, fp, fp]
        L.orc_calib_apply32.argtypes = [C.POINTER(Geometry), C.c_int64, C.POINTER(C.c_uint8), fp, fp, fp,
                                        fp, fp, fp]
        L.orc_calib_chi2.argtypes = [C.POINTER(Geometry), C.POINTER(Params), C.c_int64, dp, dp, dp,
                                     C.POINTER(C.c_uint8), C.c_int64, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), dp, dp, C.POINTER(C.c_uint8), dp, dp,
                                     C.POINTER(C.c_int64), dp, dp]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def default_params() -> Params:
    p = Params()
    lib().orc_default_params(C.byref(p))
    return p


def make_geometry(geom):
    """Geometry struct from a synth.Geometry; keeps the row table alive."""
    rx = np.ascontiguousarray(geom.row_x, dtype=np.float32)
    g = Geometry(geom.n_sectors, geom.n_rows, _ptr(rx, C.c_float), float(geom.tan_half_angle),
                 float(geom.z_max), float(geom.bz))
    g._keep = rx
    return g


def transport(p, cov, x0, x1, bz=0.5, sin_max=0.99, precision=64):
    p = np.ascontiguousarray(p, dtype=np.float64); cov = np.ascontiguousarray(cov, dtype=np.float64)
    op = np.zeros(5); oc = np.zeros(15); F = np.zeros(25)
    ok = lib().orc_transport(precision, _ptr(p, C.c_double), _ptr(cov, C.c_double), x0, x1, bz,
                             sin_max, _ptr(op, C.c_double), _ptr(oc, C.c_double), _ptr(F, C.c_double))
    return bool(ok), op, oc, F.reshape(5, 5)


def kf_update(p, cov, my, mz, vy, vz, precision=64):
    p = np.ascontiguousarray(p, dtype=np.float64); cov = np.ascontiguousarray(cov, dtype=np.float64)
    op = np.zeros(5); oc = np.zeros(15); c2 = C.c_double(0)
    lib().orc_kf_update(precision, _ptr(p, C.c_double), _ptr(cov, C.c_double), my, mz, vy, vz,
                        _ptr(op, C.c_double), _ptr(oc, C.c_double), C.byref(c2))
    return op, oc, c2.value


def kf_update1(p, cov, q, m, v, precision=64):
    """Scalar-measurement update of state component q (value m, variance v)."""
    p = np.ascontiguousarray(p, dtype=np.float64); cov = np.ascontiguousarray(cov, dtype=np.float64)
    op = np.zeros(5); oc = np.zeros(15); c2 = C.c_double(0)
    lib().orc_kf_update1(precision, _ptr(p, C.c_double), _ptr(cov, C.c_double), int(q), m, v,
                         _ptr(op, C.c_double), _ptr(oc, C.c_double), C.byref(c2))
    return op, oc, c2.value


def fit_hits(geom, x, y, z, k0, params=None, precision=64):
    g = make_geometry(geom)
    P = params or default_params()
    x = np.ascontiguousarray(x, dtype=np.float64); y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    p = np.zeros(5); cv = np.zeros(15); c2 = C.c_double(0)
    ok = lib().orc_fit_hits(precision, C.byref(g), C.byref(P), len(x), _ptr(x, C.c_double),
                            _ptr(y, C.c_double), _ptr(z, C.c_double), k0, _ptr(p, C.c_double),
                            _ptr(cv, C.c_double), C.byref(c2))
    return bool(ok), p, cv, c2.value


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def track(ev, precision=32, params=None, sector_mask=None, use64=False, theta=None):
    """Run the oracle pipeline on a synth.Event.  precision=32 rounds the
    coordinates to FP32 and computes in FP32 (decision parity); 64 computes
    in FP64 (from the FP64 coordinates if use64).  With a calibration theta
    (flat [drift scale, time offset, map]) the clusters are corrected first:
    in FP32 by calib_apply32 (the tracker's input correction) for
    precision=32, in FP64 by calib_apply otherwise."""
    g = make_geometry(ev.geom)
    P = params or default_params()
    if use64:
        x, y, z = ev.x64, ev.y64, ev.z64
    else:
        x, y, z = (ev.x.astype(np.float64), ev.y.astype(np.float64), ev.z.astype(np.float64))
    if theta is not None:
        if precision == 32:
            xf, zf = calib_apply32(ev.geom, ev.sector, x.astype(np.float32), y.astype(np.float32),
                                   z.astype(np.float32), theta)
            x, z = xf.astype(np.float64), zf.astype(np.float64)
        else:
            x, z = calib_apply(ev.geom, ev.sector, x, y, z, np.asarray(theta, np.float64))
    x = np.ascontiguousarray(x); y = np.ascontiguousarray(y); z = np.ascontiguousarray(z)
    row = np.ascontiguousarray(ev.row, dtype=np.int16)
    sec = np.ascontiguousarray(ev.sector, dtype=np.uint8)
    mask = None if sector_mask is None else np.ascontiguousarray(sector_mask, dtype=np.uint8)
    out = C.POINTER(Result)()
    lib().orc_track(precision, C.byref(g), C.byref(P), ev.n, _ptr(x, C.c_double), _ptr(y, C.c_double),
                    _ptr(z, C.c_double), _ptr(row, C.c_int16), _ptr(sec, C.c_uint8),
                    _ptr(mask, C.c_uint8) if mask is not None else None, C.byref(out))
    r = out.contents
    n, ns, nt, nr = r.n, r.n_seeds, r.n_tracks, ev.geom.n_rows
    res = dict(
        up=_arr(r.up, n, np.int64), dn=_arr(r.dn, n, np.int64),
        cup=_arr(r.cup, n, np.int64), cdn=_arr(r.cdn, n, np.int64),
        starts=_arr(r.starts, r.n_starts, np.int64),
        seed_start=_arr(r.seed_start, ns, np.int64), seed_nhits=_arr(r.seed_nhits, ns, np.int32),
        seed_key=_arr(r.seed_key, ns, np.uint64), seed_rlo=_arr(r.seed_rlo, ns, np.int32),
        seed_rhi=_arr(r.seed_rhi, ns, np.int32),
        seed_hits=_arr(r.seed_hits, ns * nr, np.int64).reshape(ns, nr),
        seed_state=_arr(r.seed_state, ns * 20, np.float64).reshape(ns, 20),
        trk_seed=_arr(r.trk_seed, nt, np.int64), sector=_arr(r.trk_sector, nt, np.int32),
        x_ref=_arr(r.trk_xref, nt, np.float64), p=_arr(r.trk_p, 5 * nt, np.float64).reshape(nt, 5),
        cov=_arr(r.trk_cov, 15 * nt, np.float64).reshape(nt, 15),
        chi2=_arr(r.trk_chi2, nt, np.float64), ndf=_arr(r.trk_ndf, nt, np.int32),
        hit_off=_arr(r.hit_off, nt + 1, np.int64), hit_ids=_arr(r.hit_ids, int(r.hit_off[nt]), np.int64),
    )
    lib().orc_result_free(out)
    return res


def rotate(x, p, cov, dalpha, bz=0.5, sin_max=0.99, precision=64):
    """State at plane x turned into a frame rotated by dalpha about z:
    (ok, new x, p, cov, Jacobian)."""
    p = np.ascontiguousarray(p, dtype=np.float64); cov = np.ascontiguousarray(cov, dtype=np.float64)
    ox = C.c_double(0); op = np.zeros(5); oc = np.zeros(15); J = np.zeros(25)
    ok = lib().orc_rotate(precision, float(x), _ptr(p, C.c_double), _ptr(cov, C.c_double), float(dalpha), bz,
                          sin_max, C.byref(ox), _ptr(op, C.c_double), _ptr(oc, C.c_double), _ptr(J, C.c_double))
    return bool(ok), ox.value, op, oc, J.reshape(5, 5)


def merge(ev, seg, params=None, slices=None):
    """The sector merger on the segments `seg` of event `ev` (a track()
    result: sector, x_ref, p, cov, chi2, hit_off, hit_ids).  Returns the
    links, the per-segment best candidates with their chi2 and second-best
    chi2, and the merged tracks (head = index of the innermost segment).
    `ev` needs geom, n, x, y, z (float32 or float64) and row.  slices: the
    time-frame slice of every segment (None for one event)."""
    g = make_geometry(ev.geom)
    P = params or default_params()
    x = np.ascontiguousarray(ev.x, dtype=np.float64); y = np.ascontiguousarray(ev.y, dtype=np.float64)
    z = np.ascontiguousarray(ev.z, dtype=np.float64)
    row = np.ascontiguousarray(ev.row, dtype=np.int16)
    ns = len(seg['x_ref'])
    sec = np.ascontiguousarray(seg['sector'], dtype=np.int32)
    xr = np.ascontiguousarray(seg['x_ref'], dtype=np.float64)
    sp = np.ascontiguousarray(seg['p'], dtype=np.float64)
    sc = np.ascontiguousarray(seg['cov'], dtype=np.float64)
    sx2 = np.ascontiguousarray(seg['chi2'], dtype=np.float64)
    so = np.ascontiguousarray(seg['hit_off'], dtype=np.int64)
    si = np.ascontiguousarray(seg['hit_ids'], dtype=np.int64)
    link = np.zeros(ns, np.int32); bi = np.zeros(ns, np.int32); bo = np.zeros(ns, np.int32)
    ci = np.zeros(ns); ci2 = np.zeros(ns); co = np.zeros(ns); co2 = np.zeros(ns)
    out = C.POINTER(Result)()
    i32 = lambda a: _ptr(a, C.c_int32)
    f64 = lambda a: _ptr(a, C.c_double)
    sl = None if slices is None else np.ascontiguousarray(slices, dtype=np.int32)
    lib().orc_merge(C.byref(g), C.byref(P), ev.n, f64(x), f64(y), f64(z), _ptr(row, C.c_int16), ns, i32(sec),
                    f64(xr), f64(sp), f64(sc), f64(sx2), _ptr(so, C.c_int64), _ptr(si, C.c_int64),
                    i32(sl) if sl is not None else None, i32(link),
                    i32(bi), f64(ci), f64(ci2), i32(bo), f64(co), f64(co2), C.byref(out))
    r = out.contents
    nt = r.n_tracks
    res = dict(link=link, best_in=bi, chi_in=ci, chi_in2=ci2, best_out=bo, chi_out=co, chi_out2=co2,
               head=_arr(r.trk_seed, nt, np.int64), sector=_arr(r.trk_sector, nt, np.int32),
               x_ref=_arr(r.trk_xref, nt, np.float64), p=_arr(r.trk_p, 5 * nt, np.float64).reshape(nt, 5),
               cov=_arr(r.trk_cov, 15 * nt, np.float64).reshape(nt, 15),
               chi2=_arr(r.trk_chi2, nt, np.float64), ndf=_arr(r.trk_ndf, nt, np.int32),
               hit_off=_arr(r.hit_off, nt + 1, np.int64), hit_ids=_arr(r.hit_ids, int(r.hit_off[nt]), np.int64))
    lib().orc_result_free(out)
    return res


class _Clusters:
    """Cluster arrays with a geometry, in the form track() and merge() read."""

    def __init__(self, geom, x, y, z, row, sector):
        self.geom, self.x, self.y, self.z, self.row, self.sector = geom, x, y, z, row, sector

    @property
    def n(self):
        return int(self.x.shape[0])


def timeframe_slices(geom, tau, sector, slice_len):
    """Slicing of a continuous-readout time frame (reading R-25): slice s =
    floor(tau / slice_len) with the quotient rounded to FP32, and the
    pseudo-coordinate z' = side (L - (tau - s slice_len)) evaluated in FP32
    in that order (side = +1 for the first half of the sectors, -1 for the
    second; L = z_max).  Returns (s int64, z' float32)."""
    L = np.float32(geom.z_max)
    D = np.float32(slice_len)
    tau = np.asarray(tau, dtype=np.float32)
    s = np.floor(tau / D).astype(np.int64)
    side = np.where(np.asarray(sector).astype(np.int64) < geom.n_sectors // 2, np.float32(1.0), np.float32(-1.0))
    zp = side * (L - (tau - s.astype(np.float32) * D))
    return s, zp.astype(np.float32)


def timeframe(tf, slice_len, n_slices, params=None):
    """Time-frame tracking (Sec. "Track reconstruction in the TPC": slices of
    the frame along the time axis tracked individually, their segments
    merged afterwards; reading R-25).
      1. every cluster gets its slice and pseudo-coordinate (timeframe_slices);
         0 <= slice < n_slices is required;
      2. each slice is tracked as one event (track(), FP32) on its clusters
         in ascending frame order (x, y, z', row, sector);
      3. the segments are taken into frame coordinates: hit ids to frame
         ids, the state's z shifted by -side s slice_len (FP64);
      4. the sector merger (FP64) runs on all segments with their slice
         indices, on the frame coordinates of the clusters, z = side (L - tau)
         (FP64 from the FP32 tau).
    Returns dict(seg=..., slice=..., merged=merge() result)."""
    geom = tf.geom
    P = params or default_params()
    s, zp = timeframe_slices(geom, tf.tau, tf.sector, slice_len)
    if s.size and (s.min() < 0 or s.max() >= n_slices):
        raise ValueError("cluster outside the slices")
    half = geom.n_sectors // 2
    keys = ("sector", "x_ref", "p", "cov", "chi2", "ndf")
    parts = {k: [] for k in keys}
    offs, ids, sl = [0], [], []
    for k in range(n_slices):
        idx = np.nonzero(s == k)[0]
        ev = _Clusters(geom, tf.x[idx], tf.y[idx], zp[idx], tf.row[idx], tf.sector[idx])
        r = track(ev, precision=32, params=P)
        nt = len(r["x_ref"])
        side = np.where(r["sector"] < half, 1.0, -1.0)
        p = r["p"].copy()
        p[:, 1] = p[:, 1] - side * (float(k) * float(np.float32(slice_len)))
        for key in keys:
            parts[key].append(p if key == "p" else r[key])
        for t in range(nt):
            h = idx[r["hit_ids"][r["hit_off"][t]:r["hit_off"][t + 1]]]
            ids.append(h)
            offs.append(offs[-1] + len(h))
        sl.append(np.full(nt, k, np.int32))
    seg = {key: np.concatenate(v) if v else np.zeros(0) for key, v in parts.items()}
    seg["hit_off"] = np.asarray(offs, np.int64)
    seg["hit_ids"] = np.concatenate(ids).astype(np.int64) if ids else np.zeros(0, np.int64)
    slices = np.concatenate(sl) if sl else np.zeros(0, np.int32)
    side_c = np.where(tf.sector.astype(np.int64) < half, 1.0, -1.0)
    ztf = side_c * (float(geom.z_max) - tf.tau.astype(np.float64))
    frame = _Clusters(geom, tf.x.astype(np.float64), tf.y.astype(np.float64), ztf, tf.row, tf.sector)
    merged = merge(frame, seg, params=P, slices=slices)
    return dict(seg=seg, slice=slices, merged=merged, z_tf=ztf)


def make_its_geometry(g):
    G = ItsGeometry()
    G.n_layers = g.n_layers
    for i in range(g.n_layers):
        G.radius[i] = float(g.radius[i]); G.half_z[i] = float(g.half_z[i])
        G.x_over_x0[i] = float(g.x_over_x0[i]); G.sigma_y[i] = float(g.sigma_y[i])
        G.sigma_z[i] = float(g.sigma_z[i]); G.n_staves[i] = int(g.n_staves[i])
    G.bz = float(g.bz)
    return G


def its_default_params() -> ItsParams:
    P = ItsParams()
    lib().orc_its_default_params(C.byref(P))
    return P


def its(ev, params=None):
    """ITS standalone tracking of one event (reading R-26): the SPD vertexer,
    tracklets, Kalman following and inward fit (FP32), the bi-square vertex
    fit (FP64).  Returns a dict of numpy arrays (per tracklet: tl0, tl1, ok,
    cls[6], ncls, chi2, outward layer/stave/x/p/cov, inward ok/stave/p/cov)
    and the vertexer and fit results."""
    G = make_its_geometry(ev.geom)
    P = params or its_default_params()
    n = ev.n
    x = np.ascontiguousarray(ev.x, np.float32); y = np.ascontiguousarray(ev.y, np.float32)
    z = np.ascontiguousarray(ev.z, np.float32)
    lay = np.ascontiguousarray(ev.layer, np.int8); stv = np.ascontiguousarray(ev.stave, np.int16)
    nb = int(round(2.0 * P.vtx_range / P.vtx_bin))
    cap = max(int((ev.layer == 0).sum()), 1)
    hist = np.zeros(nb, np.int64); meta = np.zeros(7, np.int64); vz = np.zeros(1, np.float32)
    i32 = lambda k=1: np.zeros(cap * k, np.int32)
    f32 = lambda k=1: np.zeros(cap * k, np.float32)
    o = dict(tl0=i32(), tl1=i32(), ok=i32(), cls=i32(6), ncls=i32(), chi2=f32(), olayer=i32(), ostave=i32(),
             ox=f32(), op=f32(5), oc=f32(15), iok=i32(), istave=i32(), ip=f32(5), ic=f32(15))
    vfit = np.zeros(4); vn = np.zeros(1, np.int32)
    fp = lambda a: _ptr(a, C.c_float)
    ip = lambda a: _ptr(a, C.c_int32)
    lib().orc_its(C.byref(G), C.byref(P), n, fp(x), fp(y), fp(z), _ptr(lay, C.c_int8), _ptr(stv, C.c_int16),
                  _ptr(hist, C.c_int64), _ptr(meta, C.c_int64), fp(vz), ip(o["tl0"]), ip(o["tl1"]), ip(o["ok"]),
                  ip(o["cls"]), ip(o["ncls"]), fp(o["chi2"]), ip(o["olayer"]), ip(o["ostave"]), fp(o["ox"]),
                  fp(o["op"]), fp(o["oc"]), ip(o["iok"]), ip(o["istave"]), fp(o["ip"]), fp(o["ic"]),
                  _ptr(vfit, C.c_double), ip(vn))
    T = int(meta[4])
    res = {k: v[:T * (len(v) // cap)] for k, v in o.items()}
    res["cls"] = res["cls"].reshape(T, 6)
    for k, w in (("op", 5), ("oc", 15), ("ip", 5), ("ic", 15)):
        res[k] = res[k].reshape(T, w)
    res.update(hist=hist, n_pairs=int(meta[0]), peak=int(meta[1]), vz_n=int(meta[2]), vz_qsum=int(meta[3]),
               vz=float(vz[0]), vz_ok=bool(meta[5]), vfit_ok=bool(meta[6]), vertex=vfit[:3].copy(),
               vfit_sumw=float(vfit[3]), vfit_n=int(vn[0]))
    return res


def its_ms(geom, layer, p, cov):
    """The multiple-scattering covariance increment of one layer (FP32)."""
    G = make_its_geometry(geom)
    p = np.ascontiguousarray(p, np.float32); c = np.ascontiguousarray(cov, np.float32).copy()
    lib().orc_its_ms(C.byref(G), int(layer), _ptr(p, C.c_float), _ptr(c, C.c_float))
    return c


def calib_apply(ev_or_geom, sector, x, y, z, theta):
    geom = getattr(ev_or_geom, 'geom', ev_or_geom)
    g = make_geometry(geom)
    sector = np.ascontiguousarray(sector, dtype=np.uint8)
    x = np.ascontiguousarray(x, dtype=np.float64); y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    xo = np.zeros_like(x); zo = np.zeros_like(z)
    lib().orc_calib_apply(C.byref(g), len(x), _ptr(sector, C.c_uint8), _ptr(x, C.c_double),
                          _ptr(y, C.c_double), _ptr(z, C.c_double), _ptr(th, C.c_double),
                          _ptr(xo, C.c_double), _ptr(zo, C.c_double))
    return xo, zo


def calib_apply32(ev_or_geom, sector, x, y, z, theta):
    """The FP32 input correction of the tracker (float32 in, float32 out)."""
    geom = getattr(ev_or_geom, 'geom', ev_or_geom)
    g = make_geometry(geom)
    sector = np.ascontiguousarray(sector, dtype=np.uint8)
    x = np.ascontiguousarray(x, dtype=np.float32); y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    th = np.ascontiguousarray(theta, dtype=np.float32)
    xo = np.zeros_like(x); zo = np.zeros_like(z)
    lib().orc_calib_apply32(C.byref(g), len(x), _ptr(sector, C.c_uint8), _ptr(x, C.c_float),
                            _ptr(y, C.c_float), _ptr(z, C.c_float), _ptr(th, C.c_float),
                            _ptr(xo, C.c_float), _ptr(zo, C.c_float))
    return xo, zo


def calib_chi2(geom, x, y, z, sector, hit_off, hit_ids, k0, theta, ext_tgl=None, use_vertex=None,
               params=None, grad=False):
    """Calibration objective chi2(theta) (and its exact FP64 gradient)."""
    g = make_geometry(geom)
    P = params or default_params()
    x = np.ascontiguousarray(x, dtype=np.float64); y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    sector = np.ascontiguousarray(sector, dtype=np.uint8)
    hit_off = np.ascontiguousarray(hit_off, dtype=np.int64)
    hit_ids = np.ascontiguousarray(hit_ids, dtype=np.int64)
    k0 = np.ascontiguousarray(k0, dtype=np.float64)
    nt = len(hit_off) - 1
    ext = None if ext_tgl is None else np.ascontiguousarray(ext_tgl, dtype=np.float64)
    uv = None if use_vertex is None else np.ascontiguousarray(use_vertex, dtype=np.uint8)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    c2 = C.c_double(0); ndf = C.c_int64(0)
    tc = np.zeros(nt)
    gr = np.zeros(NPAR) if grad else None
    lib().orc_calib_chi2(C.byref(g), C.byref(P), len(x), _ptr(x, C.c_double), _ptr(y, C.c_double),
                         _ptr(z, C.c_double), _ptr(sector, C.c_uint8), nt, _ptr(hit_off, C.c_int64),
                         _ptr(hit_ids, C.c_int64), _ptr(k0, C.c_double),
                         _ptr(ext, C.c_double) if ext is not None else None,
                         _ptr(uv, C.c_uint8) if uv is not None else None, _ptr(th, C.c_double),
                         C.byref(c2), C.byref(ndf), _ptr(tc, C.c_double),
                         _ptr(gr, C.c_double) if gr is not None else None)
    if grad:
        return c2.value, ndf.value, tc, gr
    return c2.value, ndf.value, tc
