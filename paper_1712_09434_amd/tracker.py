"""Python surface of libtpcca: the same calls as the C ABI, with torch
tensors for memory and streams.  Marshalling only; no arithmetic of the
method happens here."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A


def _check(L, ctx, rc):
    if rc != A.TPCCA_OK:
        msg = L.tpcca_last_error(ctx).decode() if ctx else ""
        raise A.TpccaError(rc, msg)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _mem(t: torch.Tensor) -> int:
    return A.TPCCA_MEM_DEVICE if t.is_cuda else A.TPCCA_MEM_HOST


def _stream_handle(device: torch.device):
    if device.type != "cuda":
        return None
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Tracks:
    """Tracks of one event (tensors on the input's device, already sliced to
    the counts)."""
    sector: torch.Tensor
    x_ref: torch.Tensor
    p: torch.Tensor
    cov: torch.Tensor
    chi2: torch.Tensor
    ndf: torch.Tensor
    k_prior: torch.Tensor
    hit_off: torch.Tensor
    hit_id: torch.Tensor
    taps: Optional[dict] = None

    @property
    def n_tracks(self) -> int:
        return int(self.x_ref.shape[0])


@dataclass
class FitTracks:
    """Fixed hit lists for tpcca_refit_grad: the clusters (default
    transformation), CSR hit lists in ascending pad row, the q/pT prior, the
    external tan(lambda) and the vertex flags (tensors on one device)."""
    clusters: tuple
    hit_off: torch.Tensor
    hit_id: torch.Tensor
    k_prior: torch.Tensor
    ext_tgl: Optional[torch.Tensor]
    use_vertex: Optional[torch.Tensor]

    @property
    def n_tracks(self) -> int:
        return int(self.hit_off.shape[0]) - 1


class Tracker:
    """tpcca_create / tpcca_track / tpcca_track_batch / tpcca_refit_grad."""

    def __init__(self, row_x, tan_half_angle: float, z_max: float, bz: float, n_sectors: int = 36,
                 params: Optional[A.tpcca_params] = None):
        self.L = A.load()
        self._rx = np.ascontiguousarray(row_x, dtype=np.float32)
        self.n_sectors, self.n_rows = int(n_sectors), int(self._rx.shape[0])
        g = A.tpcca_geometry(self.n_sectors, self.n_rows,
                             self._rx.ctypes.data_as(C.POINTER(C.c_float)),
                             float(tan_half_angle), float(z_max))
        f = A.tpcca_field(float(bz))
        ctx = C.c_void_p()
        _check(self.L, None, self.L.tpcca_create(C.byref(g), C.byref(f), C.byref(ctx)))
        self.ctx = ctx
        if params is not None:
            self.set_params(params)

    @classmethod
    def from_geometry(cls, geom, params=None):
        return cls(geom.row_x, float(geom.tan_half_angle), float(geom.z_max), float(geom.bz),
                   geom.n_sectors, params)

    def close(self):
        if getattr(self, "ctx", None):
            self.L.tpcca_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- params
    def set_params(self, p: A.tpcca_params):
        _check(self.L, self.ctx, self.L.tpcca_set_params(self.ctx, C.byref(p)))

    def get_params(self) -> A.tpcca_params:
        p = A.tpcca_params()
        _check(self.L, self.ctx, self.L.tpcca_get_params(self.ctx, C.byref(p)))
        return p

    # ----------------------------------------------------------- calibration
    def set_calib(self, theta: Optional[torch.Tensor]):
        """Install the calibration theta (flat float32 [drift_scale(S),
        time_offset(S), map(S*64)], host or device) as the correction of the
        tracking input, or remove it (None)."""
        if theta is None:
            _check(self.L, self.ctx, self.L.tpcca_set_calib(self.ctx, None))
            return
        S = self.n_sectors
        th = theta.detach().to(torch.float32).contiguous()
        if th.numel() != S * 66:
            raise ValueError(f"theta needs {S * 66} values")
        cal = A.tpcca_calib(_ptr(th), C.c_void_p(th.data_ptr() + 4 * S), C.c_void_p(th.data_ptr() + 8 * S),
                            _mem(th))
        _check(self.L, self.ctx, self.L.tpcca_set_calib(self.ctx, C.byref(cal)))

    # -------------------------------------------------------------- tracking
    @staticmethod
    def clusters_struct(x, y, z, row, sector) -> A.tpcca_clusters:
        for t in (x, y, z, row, sector):
            if not t.is_contiguous():
                raise ValueError("cluster arrays must be contiguous")
        assert x.dtype == torch.float32 and row.dtype == torch.int16 and sector.dtype == torch.uint8
        return A.tpcca_clusters(int(x.shape[0]), _ptr(x), _ptr(y), _ptr(z), _ptr(row), _ptr(sector),
                                _mem(x), _stream_handle(x.device))

    def _alloc_out(self, n: int, device, taps: bool, k_prior: bool = True, cap_tracks: int = 0):
        p = self.get_params()
        cap_t = cap_tracks or n // max(p.min_hits, 1) + 1
        cap_h = max(n, 1)
        f32 = dict(dtype=torch.float32, device=device)
        o = dict(sector=torch.empty(cap_t, dtype=torch.uint8, device=device),
                 x_ref=torch.empty(cap_t, **f32), p=torch.empty(cap_t, 5, **f32),
                 cov=torch.empty(cap_t, 15, **f32), chi2=torch.empty(cap_t, **f32),
                 ndf=torch.empty(cap_t, dtype=torch.int32, device=device),
                 k_prior=torch.empty(cap_t, **f32),
                 hit_off=torch.empty(cap_t + 1, dtype=torch.int32, device=device),
                 hit_id=torch.empty(cap_h, dtype=torch.int32, device=device))
        if taps:
            for k in ("dbg_up", "dbg_dn", "dbg_cup", "dbg_cdn", "dbg_start"):
                o[k] = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        st = A.tpcca_tracks()
        st.cap_tracks, st.cap_hits = cap_t, cap_h
        for k in ("sector", "x_ref", "p", "cov", "chi2", "ndf", "k_prior", "hit_off", "hit_id"):
            setattr(st, k, _ptr(o[k]))
        if taps:
            for k in ("dbg_up", "dbg_dn", "dbg_cup", "dbg_cdn", "dbg_start"):
                setattr(st, k, _ptr(o[k]))
        st.mem = A.TPCCA_MEM_DEVICE if torch.device(device).type == "cuda" else A.TPCCA_MEM_HOST
        return st, o

    @staticmethod
    def _slice(st: A.tpcca_tracks, o: dict, n: int) -> Tracks:
        nt, nh = int(st.n_tracks), int(st.n_hits)
        taps = None
        if "dbg_up" in o:
            taps = dict(up=o["dbg_up"][:n], dn=o["dbg_dn"][:n], cup=o["dbg_cup"][:n],
                        cdn=o["dbg_cdn"][:n], start=o["dbg_start"][:int(st.n_start)])
        return Tracks(sector=o["sector"][:nt], x_ref=o["x_ref"][:nt], p=o["p"][:nt], cov=o["cov"][:nt],
                      chi2=o["chi2"][:nt], ndf=o["ndf"][:nt], k_prior=o["k_prior"][:nt],
                      hit_off=o["hit_off"][:nt + 1], hit_id=o["hit_id"][:nh], taps=taps)

    def track(self, x, y, z, row, sector, taps: bool = False) -> Tracks:
        cl = self.clusters_struct(x, y, z, row, sector)
        st, o = self._alloc_out(int(x.shape[0]), x.device, taps)
        _check(self.L, self.ctx, self.L.tpcca_track(self.ctx, C.byref(cl), C.byref(st)))
        return self._slice(st, o, int(x.shape[0]))

    def merge(self, seg: Tracks, clusters: tuple, links: bool = False):
        """tpcca_merge: the sector merger on the tracks `seg` of one event
        (device tensors, as returned by track) whose hit ids index
        `clusters` (x, y, z, row, sector).  Returns the merged Tracks (their
        k_prior is not set), and with links=True also each segment's outer
        partner (int32, -1 for none)."""
        cl = self.clusters_struct(*clusters)
        T = seg.n_tracks
        dev = seg.x_ref.device
        st = A.tpcca_tracks()
        st.n_tracks = T
        keep = {k: getattr(seg, k).contiguous() for k in ("sector", "x_ref", "p", "cov", "chi2", "ndf",
                                                          "hit_off", "hit_id")}
        for k, v in keep.items():
            setattr(st, k, _ptr(v))
        st.clusters = C.pointer(cl)
        st.mem = _mem(seg.hit_off)
        H = int(seg.hit_id.numel())
        f32 = dict(dtype=torch.float32, device=dev)
        o = dict(sector=torch.empty(max(T, 1), dtype=torch.uint8, device=dev), x_ref=torch.empty(max(T, 1), **f32),
                 p=torch.empty(max(T, 1), 5, **f32), cov=torch.empty(max(T, 1), 15, **f32),
                 chi2=torch.empty(max(T, 1), **f32), ndf=torch.empty(max(T, 1), dtype=torch.int32, device=dev),
                 k_prior=torch.zeros(max(T, 1), **f32),
                 hit_off=torch.empty(T + 1, dtype=torch.int32, device=dev),
                 hit_id=torch.empty(max(H, 1), dtype=torch.int32, device=dev))
        out = A.tpcca_tracks()
        out.cap_tracks, out.cap_hits = T, H
        for k in ("sector", "x_ref", "p", "cov", "chi2", "ndf", "hit_off", "hit_id"):
            setattr(out, k, _ptr(o[k]))
        out.mem = _mem(o["hit_off"])
        lk = torch.empty(max(T, 1), dtype=torch.int32, device=dev) if links else None
        _check(self.L, self.ctx, self.L.tpcca_merge(self.ctx, C.byref(st), C.byref(out), _ptr(lk)))
        m = self._slice(out, o, 0)
        return (m, lk[:T]) if links else m

    def track_timeframe(self, x, y, tau, row, sector, slice_len: float, n_slices: int, segments: bool = False):
        """tpcca_track_timeframe: one continuous-readout time frame (device
        tensors; tau = readout time in cm of drift since the frame start)
        sliced every slice_len cm into n_slices slices, tracked and merged.
        Returns the merged Tracks in frame coordinates; with segments=True
        also (segment Tracks, their slices, their outer merge partners)."""
        cl = self.clusters_struct(x, y, tau, row, sector)
        n = int(x.shape[0])
        cap_t = n // max(self.get_params().min_hits, 1) + int(n_slices)
        m_st, m_o = self._alloc_out(n, x.device, False, cap_tracks=cap_t)
        m_st.k_prior = None                   # (not produced for frames)
        m_o["k_prior"].zero_()
        s_st = s_o = sl = lk = None
        if segments:
            s_st, s_o = self._alloc_out(n, x.device, False, cap_tracks=cap_t)
            s_st.k_prior = None
            s_o["k_prior"].zero_()
            sl = torch.empty(cap_t, dtype=torch.int32, device=x.device)
            lk = torch.empty(cap_t, dtype=torch.int32, device=x.device)
        _check(self.L, self.ctx, self.L.tpcca_track_timeframe(
            self.ctx, C.byref(cl), float(slice_len), int(n_slices), C.byref(m_st),
            C.byref(s_st) if segments else None, _ptr(sl), _ptr(lk)))
        merged = self._slice(m_st, m_o, n)
        if not segments:
            return merged
        seg = self._slice(s_st, s_o, n)
        T = seg.n_tracks
        return merged, seg, sl[:T], lk[:T]

    def track_batch(self, events: Sequence[tuple], taps: bool = False) -> List[Tracks]:
        E = len(events)
        cls = (A.tpcca_clusters * E)()
        sts = (A.tpcca_tracks * E)()
        outs = []
        for e, (x, y, z, row, sector) in enumerate(events):
            cls[e] = self.clusters_struct(x, y, z, row, sector)
            st, o = self._alloc_out(int(x.shape[0]), x.device, taps)
            sts[e] = st
            outs.append(o)
        _check(self.L, self.ctx, self.L.tpcca_track_batch(self.ctx, E, cls, sts))
        return [self._slice(sts[e], outs[e], int(events[e][0].shape[0])) for e in range(E)]

    # ----------------------------------------------------------- calibration
    def set_tuning(self, ckpt_every: int = 160, tracklet_grid: int = 0, use_graph: int = 0):
        t = A.tpcca_tuning(int(ckpt_every), int(tracklet_grid), int(use_graph))
        _check(self.L, self.ctx, self.L.tpcca_set_tuning(self.ctx, C.byref(t)))

    def refit_grad(self, fit: "FitTracks", theta: torch.Tensor, flags: bool = False):
        """Total chi2, ndf and d chi2/d theta (float64, flat layout
        [drift_scale(S), time_offset(S), map(S*64)]) of the fixed hit lists in
        `fit` under the calibration theta (flat float32, same layout).  With
        flags=True a fourth item holds the per-track status (int32,
        TPCCA_TRK_* bits)."""
        return self._refit_grad(self.L.tpcca_refit_grad, fit, theta, flags)

    def refit_grad_noalloc(self, fit: "FitTracks", theta: torch.Tensor, flags: bool = False):
        """refit_grad through tpcca_refit_grad_noalloc: the library allocates
        nothing (its scratch is a static device array); every tensor must be
        on the GPU.  The gradient tensor is allocated here, by the caller."""
        return self._refit_grad(self.L.tpcca_refit_grad_noalloc, fit, theta, flags)

    def _refit_grad(self, entry, fit: "FitTracks", theta: torch.Tensor, flags: bool = False):
        S = self.n_sectors
        th = theta.detach().to(torch.float32).contiguous()
        dev = th.device
        grad = torch.empty(S * 66, dtype=torch.float64, device=dev)
        tflag = torch.empty(max(fit.n_tracks, 1), dtype=torch.int32, device=dev) if flags else None
        cl = self.clusters_struct(*fit.clusters)
        st = A.tpcca_tracks()
        st.n_tracks = fit.n_tracks
        st.hit_off = _ptr(fit.hit_off)
        st.hit_id = _ptr(fit.hit_id)
        st.k_prior = _ptr(fit.k_prior)
        st.ext_tgl = _ptr(fit.ext_tgl)
        st.use_vertex = _ptr(fit.use_vertex)
        st.clusters = C.pointer(cl)
        st.mem = _mem(fit.hit_off)
        cal = A.tpcca_calib(_ptr(th), C.c_void_p(th.data_ptr() + 4 * S), C.c_void_p(th.data_ptr() + 8 * S),
                            _mem(th))
        g = A.tpcca_grad()
        g.d_drift_scale = _ptr(grad)
        g.d_time_offset = C.c_void_p(grad.data_ptr() + 8 * S)
        g.d_map = C.c_void_p(grad.data_ptr() + 16 * S)
        g.track_flag = _ptr(tflag)
        g.mem = _mem(grad)
        _check(self.L, self.ctx, entry(self.ctx, C.byref(st), C.byref(cal), C.byref(g)))
        if flags:
            return float(g.chi2), int(g.ndf), grad, tflag[:fit.n_tracks]
        return float(g.chi2), int(g.ndf), grad

    def get_tuning(self) -> A.tpcca_tuning:
        t = A.tpcca_tuning()
        _check(self.L, self.ctx, self.L.tpcca_get_tuning(self.ctx, C.byref(t)))
        return t

    def set_phase_timing(self, on: bool = True):
        _check(self.L, self.ctx, self.L.tpcca_set_phase_timing(self.ctx, 1 if on else 0))

    def phase_times(self) -> dict:
        """{phase: mean ms per timed call} since timing was enabled."""
        cap = 32
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        calls = C.c_int64(0)
        n = self.L.tpcca_phase_times(self.ctx, cap, names, ms, C.byref(calls))
        k = max(calls.value, 1)
        return {names[i].decode(): ms[i] / k for i in range(n)}, calls.value

    def debug_tracklets(self):
        n = C.c_int64(0)
        rc = self.L.tpcca_debug_tracklets(self.ctx, 0, C.byref(n), None, None, None, None)
        if rc not in (A.TPCCA_OK, A.TPCCA_E_CAPACITY):
            _check(self.L, self.ctx, rc)
        ns = n.value
        start = np.zeros(max(ns, 1), np.uint32); nh = np.zeros(max(ns, 1), np.int32)
        hits = np.zeros((max(ns, 1), self.n_rows), np.int32); state = np.zeros((max(ns, 1), 20), np.float32)
        _check(self.L, self.ctx, self.L.tpcca_debug_tracklets(
            self.ctx, ns, C.byref(n), start.ctypes.data_as(C.c_void_p), nh.ctypes.data_as(C.c_void_p),
            hits.ctypes.data_as(C.c_void_p), state.ctypes.data_as(C.c_void_p)))
        return dict(seed_start=start[:ns], seed_nhits=nh[:ns], seed_hits=hits[:ns], seed_state=state[:ns])
