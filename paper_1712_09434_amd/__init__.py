"""MI355X-native TPC cellular-automaton + Kalman track finder (libtpcca).

The hot path is the HIP library ``libtpcca.so`` (gfx950); this package only
loads it and marshals torch tensors into its C ABI (``include/tpcca.h``).
There is no CPU fallback: calls fail if the library is not built.
"""
from ._abi import TpccaError, default_params, load  # noqa: F401
from .tracker import FitTracks, Tracker, Tracks  # noqa: F401
from .calib import Chi2Refit, calibrate, calibrate_newton  # noqa: F401
