"""ctypes mirror of include/tpcca.h and the loader of libtpcca.so.

Argument marshalling only: every step of the path runs in the HIP library.
Importing this module does not need a GPU; calling into the library does.
The loader raises if the library has not been built -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpcca.so")

TPCCA_OK = 0
TPCCA_E_INVALID = -1
TPCCA_E_CAPACITY = -2
TPCCA_E_DEVICE = -3
TPCCA_E_NOMEM = -4
TPCCA_E_LIMIT = -5
TPCCA_MEM_HOST = 0
TPCCA_MEM_DEVICE = 1
TPCCA_MAX_ROW_CLUSTERS = 8192
TPCCA_NOALLOC_SCRATCH_BYTES = 128 << 20
TPCCA_TRK_NOT_FITTED, TPCCA_TRK_HITS, TPCCA_TRK_VERTEX, TPCCA_TRK_SHORT = 0, 1, 2, 4
TPCCA_GRAD_MIN_HITS = 40
TPCCA_GRAD_C2_UPDATES = 3
TPCCA_TF_MAX_SLICES = 1024
ERROR_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_CAPACITY", -3: "E_DEVICE", -4: "E_NOMEM", -5: "E_LIMIT"}

EXPORTED = ["tpcca_default_params", "tpcca_create", "tpcca_set_params", "tpcca_get_params",
            "tpcca_track", "tpcca_track_batch", "tpcca_refit_grad", "tpcca_debug_tracklets",
            "tpcca_set_tuning", "tpcca_get_tuning", "tpcca_set_phase_timing", "tpcca_phase_times",
            "tpcca_last_error", "tpcca_destroy", "tpcca_debug_fp32", "tpcca_refit_grad_noalloc",
            "tpcca_set_calib", "tpcca_merge", "tpcca_track_timeframe", "tpcca_its_default_params",
            "tpcca_its_create", "tpcca_its_set_params", "tpcca_its_track", "tpcca_its_track_batch",
            "tpcca_its_last_error",
            "tpcca_its_destroy"]


class tpcca_geometry(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("n_rows", C.c_int32), ("row_x", C.POINTER(C.c_float)),
                ("tan_half_angle", C.c_float), ("z_max", C.c_float)]


class tpcca_field(C.Structure):
    _fields_ = [("bz_tesla", C.c_float)]


class tpcca_params(C.Structure):
    _fields_ = [("win_y", C.c_float), ("win_z", C.c_float), ("inv_var_y", C.c_float),
                ("inv_var_z", C.c_float), ("link_cut", C.c_float), ("chi2_ext", C.c_float),
                ("max_gap", C.c_int32), ("min_seed_hits", C.c_int32), ("min_hits", C.c_int32),
                ("owned_num", C.c_int32), ("owned_den", C.c_int32), ("sin_max", C.c_float),
                ("sigma_y", C.c_float), ("sigma_z", C.c_float), ("sigma_vertex", C.c_float),
                ("sigma_tgl", C.c_float), ("chi2_merge", C.c_float), ("merge_dist", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class tpcca_tuning(C.Structure):
    _fields_ = [("ckpt_every", C.c_int32), ("tracklet_grid", C.c_int32), ("use_graph", C.c_int32)]


class tpcca_clusters(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("row", C.c_void_p), ("sector", C.c_void_p), ("mem", C.c_int32),
                ("stream", C.c_void_p)]


class tpcca_tracks(C.Structure):
    _fields_ = [("cap_tracks", C.c_int64), ("cap_hits", C.c_int64), ("n_tracks", C.c_int64),
                ("n_hits", C.c_int64), ("sector", C.c_void_p), ("x_ref", C.c_void_p),
                ("p", C.c_void_p), ("cov", C.c_void_p), ("chi2", C.c_void_p), ("ndf", C.c_void_p),
                ("k_prior", C.c_void_p), ("hit_off", C.c_void_p), ("hit_id", C.c_void_p),
                ("dbg_up", C.c_void_p), ("dbg_dn", C.c_void_p), ("dbg_cup", C.c_void_p),
                ("dbg_cdn", C.c_void_p), ("dbg_start", C.c_void_p), ("n_start", C.c_int64),
                ("clusters", C.POINTER(tpcca_clusters)), ("ext_tgl", C.c_void_p),
                ("use_vertex", C.c_void_p), ("mem", C.c_int32)]


class tpcca_its_geometry(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("radius", C.c_float * 6), ("half_z", C.c_float * 6),
                ("x_over_x0", C.c_float * 6), ("sigma_y", C.c_float * 6), ("sigma_z", C.c_float * 6),
                ("n_staves", C.c_int32 * 6), ("bz", C.c_float)]


class tpcca_its_params(C.Structure):
    _fields_ = [("vtx_sin_phi", C.c_float), ("vtx_bin", C.c_float), ("vtx_range", C.c_float),
                ("trk_sin_phi", C.c_float), ("trk_dtgl", C.c_float), ("chi2_cut", C.c_float),
                ("sigma_vy", C.c_float), ("sigma_vz", C.c_float), ("sin_max", C.c_float),
                ("min_clusters", C.c_int32), ("tukey_c", C.c_float), ("fit_iters", C.c_int32),
                ("cov_scale_in", C.c_float)]


class tpcca_its_clusters(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("layer", C.c_void_p), ("stave", C.c_void_p), ("stream", C.c_void_p)]


ITS_TRACK_ARRAYS = ("tl0", "tl1", "ok", "cls", "ncls", "chi2", "out_layer", "out_stave", "out_x", "out_p",
                    "out_cov", "in_ok", "in_stave", "in_p", "in_cov")


class tpcca_its_tracks(C.Structure):
    _fields_ = ([("cap", C.c_int64), ("n_tracklets", C.c_int64)] + [(k, C.c_void_p) for k in ITS_TRACK_ARRAYS]
                + [("hist", C.c_void_p), ("n_pairs", C.c_int64), ("peak", C.c_int32), ("vz_ok", C.c_int32),
                   ("vz", C.c_float), ("vfit_ok", C.c_int32), ("vfit_n", C.c_int32),
                   ("vertex", C.c_double * 3), ("vfit_sumw", C.c_double)])


class tpcca_calib(C.Structure):
    _fields_ = [("drift_scale", C.c_void_p), ("time_offset", C.c_void_p), ("map", C.c_void_p),
                ("mem", C.c_int32)]


class tpcca_grad(C.Structure):
    _fields_ = [("chi2", C.c_double), ("ndf", C.c_int64), ("d_drift_scale", C.c_void_p),
                ("d_time_offset", C.c_void_p), ("d_map", C.c_void_p), ("track_flag", C.c_void_p),
                ("mem", C.c_int32)]


_lib = None


class TpccaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libtpcca.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libtpcca.so not built ({path}); run __graft_entry__.build() or "
                           f"python -m paper_1712_09434_amd.build")
    L = C.CDLL(path)
    P = C.POINTER
    L.tpcca_default_params.argtypes = [P(tpcca_params)]
    L.tpcca_default_params.restype = None
    L.tpcca_create.argtypes = [P(tpcca_geometry), P(tpcca_field), P(C.c_void_p)]
    L.tpcca_set_params.argtypes = [C.c_void_p, P(tpcca_params)]
    L.tpcca_get_params.argtypes = [C.c_void_p, P(tpcca_params)]
    L.tpcca_track.argtypes = [C.c_void_p, P(tpcca_clusters), P(tpcca_tracks)]
    L.tpcca_merge.argtypes = [C.c_void_p, P(tpcca_tracks), P(tpcca_tracks), C.c_void_p]
    L.tpcca_merge.restype = C.c_int
    L.tpcca_track_timeframe.argtypes = [C.c_void_p, P(tpcca_clusters), C.c_float, C.c_int32, P(tpcca_tracks),
                                        P(tpcca_tracks), C.c_void_p, C.c_void_p]
    L.tpcca_track_timeframe.restype = C.c_int
    L.tpcca_its_default_params.argtypes = [P(tpcca_its_params)]
    L.tpcca_its_default_params.restype = None
    L.tpcca_its_create.argtypes = [P(tpcca_its_geometry), P(C.c_void_p)]
    L.tpcca_its_set_params.argtypes = [C.c_void_p, P(tpcca_its_params)]
    L.tpcca_its_track.argtypes = [C.c_void_p, P(tpcca_its_clusters), P(tpcca_its_tracks)]
    L.tpcca_its_track_batch.argtypes = [C.c_void_p, C.c_int32, P(tpcca_its_clusters), P(tpcca_its_tracks)]
    L.tpcca_its_last_error.argtypes = [C.c_void_p]
    L.tpcca_its_last_error.restype = C.c_char_p
    L.tpcca_its_destroy.argtypes = [C.c_void_p]
    L.tpcca_its_destroy.restype = None
    L.tpcca_set_calib.argtypes = [C.c_void_p, P(tpcca_calib)]
    L.tpcca_set_calib.restype = C.c_int
    L.tpcca_track_batch.argtypes = [C.c_void_p, C.c_int32, P(tpcca_clusters), P(tpcca_tracks)]
    L.tpcca_refit_grad.argtypes = [C.c_void_p, P(tpcca_tracks), P(tpcca_calib), P(tpcca_grad)]
    L.tpcca_refit_grad_noalloc.argtypes = [C.c_void_p, P(tpcca_tracks), P(tpcca_calib), P(tpcca_grad)]
    L.tpcca_debug_tracklets.argtypes = [C.c_void_p, C.c_int64, P(C.c_int64), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
    L.tpcca_set_tuning.argtypes = [C.c_void_p, P(tpcca_tuning)]
    L.tpcca_set_tuning.restype = C.c_int
    L.tpcca_get_tuning.argtypes = [C.c_void_p, P(tpcca_tuning)]
    L.tpcca_get_tuning.restype = C.c_int
    L.tpcca_set_phase_timing.argtypes = [C.c_void_p, C.c_int]
    L.tpcca_set_phase_timing.restype = C.c_int
    L.tpcca_phase_times.argtypes = [C.c_void_p, C.c_int32, P(C.c_char_p), P(C.c_double), P(C.c_int64)]
    L.tpcca_phase_times.restype = C.c_int
    L.tpcca_last_error.argtypes = [C.c_void_p]
    L.tpcca_last_error.restype = C.c_char_p
    L.tpcca_destroy.argtypes = [C.c_void_p]
    L.tpcca_destroy.restype = None
    L.tpcca_debug_fp32.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.tpcca_debug_fp32.restype = C.c_int
    for name in ("tpcca_create", "tpcca_set_params", "tpcca_get_params", "tpcca_track",
                 "tpcca_track_batch", "tpcca_refit_grad", "tpcca_refit_grad_noalloc",
                 "tpcca_debug_tracklets"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def default_params() -> tpcca_params:
    p = tpcca_params()
    load().tpcca_default_params(C.byref(p))
    return p
