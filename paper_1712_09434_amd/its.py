"""Binding of the ITS standalone tracker (tpcca_its_* in include/tpcca.h).

Argument marshalling only: every step (vertexer, tracklets, following,
inward fit, vertex fit) runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import torch

from . import _abi as A
from .tracker import _ptr, _stream_handle


def _check(L, ctx, rc):
    if rc != A.TPCCA_OK:
        msg = L.tpcca_its_last_error(ctx).decode() if ctx else ""
        raise A.TpccaError(rc, msg)


@dataclass
class ItsResult:
    """One event: per-tracklet tensors (device, sliced to the count) and the
    vertexer / vertex-fit scalars."""
    tl0: torch.Tensor
    tl1: torch.Tensor
    ok: torch.Tensor
    cls: torch.Tensor          # [T, 6]
    ncls: torch.Tensor
    chi2: torch.Tensor
    out_layer: torch.Tensor
    out_stave: torch.Tensor
    out_x: torch.Tensor
    out_p: torch.Tensor        # [T, 5]
    out_cov: torch.Tensor      # [T, 15]
    in_ok: torch.Tensor
    in_stave: torch.Tensor
    in_p: torch.Tensor         # [T, 5]
    in_cov: torch.Tensor       # [T, 15]
    hist: Optional[torch.Tensor]
    n_pairs: int
    peak: int
    vz_ok: bool
    vz: float
    vfit_ok: bool
    vfit_n: int
    vertex: tuple
    vfit_sumw: float


class ItsTracker:
    def __init__(self, geom, params: Optional[A.tpcca_its_params] = None):
        self.L = A.load()
        g = A.tpcca_its_geometry()
        g.n_layers = int(geom.n_layers)
        for i in range(g.n_layers):
            g.radius[i] = float(geom.radius[i]); g.half_z[i] = float(geom.half_z[i])
            g.x_over_x0[i] = float(geom.x_over_x0[i]); g.sigma_y[i] = float(geom.sigma_y[i])
            g.sigma_z[i] = float(geom.sigma_z[i]); g.n_staves[i] = int(geom.n_staves[i])
        g.bz = float(geom.bz)
        ctx = C.c_void_p()
        rc = self.L.tpcca_its_create(C.byref(g), C.byref(ctx))
        if rc != A.TPCCA_OK:
            raise A.TpccaError(rc, "tpcca_its_create")
        self.ctx = ctx
        self.nbins = 400
        if params is not None:
            self.set_params(params)

    @staticmethod
    def default_params() -> A.tpcca_its_params:
        p = A.tpcca_its_params()
        A.load().tpcca_its_default_params(C.byref(p))
        return p

    def set_params(self, p: A.tpcca_its_params):
        _check(self.L, self.ctx, self.L.tpcca_its_set_params(self.ctx, C.byref(p)))
        self.nbins = int(round(2.0 * p.vtx_range / p.vtx_bin))

    def _event(self, x, y, z, layer, stave, hist):
        """Marshals one event: the cluster struct, the output struct and the
        tensors behind both (kept alive by the caller until the call ends)."""
        dev = x.device
        cl = A.tpcca_its_clusters()
        cl.n = int(x.shape[0])
        keep = [t.contiguous() for t in (x, y, z, layer, stave)]
        cl.x, cl.y, cl.z, cl.layer, cl.stave = (_ptr(t) for t in keep)
        cl.stream = _stream_handle(dev)
        cap = max(int((layer == 0).sum().item()), 1)
        i32 = dict(dtype=torch.int32, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        o = dict(tl0=torch.empty(cap, **i32), tl1=torch.empty(cap, **i32), ok=torch.empty(cap, **i32),
                 cls=torch.empty(cap, 6, **i32), ncls=torch.empty(cap, **i32), chi2=torch.empty(cap, **f32),
                 out_layer=torch.empty(cap, **i32), out_stave=torch.empty(cap, **i32), out_x=torch.empty(cap, **f32),
                 out_p=torch.empty(cap, 5, **f32), out_cov=torch.empty(cap, 15, **f32),
                 in_ok=torch.empty(cap, **i32), in_stave=torch.empty(cap, **i32), in_p=torch.empty(cap, 5, **f32),
                 in_cov=torch.empty(cap, 15, **f32))
        h = torch.empty(self.nbins, dtype=torch.int32, device=dev) if hist else None
        st = A.tpcca_its_tracks()
        st.cap = cap
        for k in A.ITS_TRACK_ARRAYS:
            setattr(st, k, _ptr(o[k]))
        st.hist = _ptr(h)
        return cl, st, o, h, keep

    @staticmethod
    def _result(st, o, h) -> ItsResult:
        T = int(st.n_tracklets)
        sl = {k: v[:T] for k, v in o.items()}
        return ItsResult(**sl, hist=h, n_pairs=int(st.n_pairs), peak=int(st.peak), vz_ok=bool(st.vz_ok),
                         vz=float(st.vz), vfit_ok=bool(st.vfit_ok), vfit_n=int(st.vfit_n),
                         vertex=tuple(st.vertex), vfit_sumw=float(st.vfit_sumw))

    def track(self, x, y, z, layer, stave, hist: bool = False) -> ItsResult:
        cl, st, o, h, keep = self._event(x, y, z, layer, stave, hist)
        _check(self.L, self.ctx, self.L.tpcca_its_track(self.ctx, C.byref(cl), C.byref(st)))
        return self._result(st, o, h)

    def prepare_batch(self, events, hist: bool = False):
        """Marshals a batch once (output tensors, structs) and returns
        run(results=True): one tpcca_its_track_batch call on it, for repeated
        calls on the same inputs."""
        ev = [self._event(*e, hist) for e in events]
        n = len(ev)
        cls = (A.tpcca_its_clusters * max(n, 1))(*[e[0] for e in ev])
        sts = (A.tpcca_its_tracks * max(n, 1))(*[e[1] for e in ev])

        def run(results: bool = True):
            if n == 0:
                return []
            _check(self.L, self.ctx, self.L.tpcca_its_track_batch(self.ctx, n, cls, sts))
            return [self._result(sts[i], e[2], e[3]) for i, e in enumerate(ev)] if results else None
        return run

    def track_batch(self, events, hist: bool = False) -> list:
        """events: sequence of (x, y, z, layer, stave) device tensors, one
        tuple per event, all on one device and stream; one library call."""
        return self.prepare_batch(events, hist)()

    def close(self):
        if self.ctx:
            self.L.tpcca_its_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
