"""tpcca_refit_grad_noalloc against tpcca_refit_grad.

The allocation-free entry point runs the same kernels on a static device
scratch array instead of the context's workspace, choosing the largest
checkpoint stride whose workspace fits the array.  Results do not depend on
the stride, so the two entry points must agree bit for bit: chi2, ndf and
every gradient component.  Checked on two calls in a row (the second with
a smaller track set, so stale contents of the array from the first call
would show), on a set that fits only at a reduced stride, and for the
errors: a set too large for the array and host-memory arguments.
"""
import numpy as np
import pytest
import torch

import synth
from calibset import calib_subset

pytestmark = pytest.mark.gpu
S = 36


@pytest.fixture(scope="module")
def setup():
    from paper_1712_09434_amd import FitTracks, Tracker
    theta_star = synth.draw_theta(77)
    ev = synth.make_event(seed=31, n_primaries=600, noise=0.01, theta=theta_star)
    trk = Tracker.from_geometry(ev.geom)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    cl = (t(ev.x), t(ev.y), t(ev.z), t(ev.row), t(ev.sector))
    out = trk.track(*cl)
    off = out.hit_off.cpu().numpy().astype(np.int64)
    ids = out.hit_id.cpu().numpy().astype(np.int64)
    cs = calib_subset(ev, off, ids, out.sector.cpu().numpy(), out.chi2.cpu().numpy(),
                      out.ndf.cpu().numpy(), out.k_prior.cpu().numpy())
    print(f"[gpu] no-alloc gradient set: {len(cs['tracks'])} tracks, {len(cs['hit_ids'])} hits", flush=True)

    def fit_of(take, reps=1):
        """FitTracks of the calibration tracks `take`, the list repeated `reps` times."""
        take = np.tile(np.asarray(take, np.int64), reps)
        n = cs['hit_off'][take + 1] - cs['hit_off'][take]
        hoff = np.concatenate([[0], np.cumsum(n)])
        hid = np.concatenate([cs['hit_ids'][cs['hit_off'][i]:cs['hit_off'][i + 1]] for i in take])
        d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to("cuda:0")
        return FitTracks(clusters=cl, hit_off=d(hoff, np.int32), hit_id=d(hid, np.int32),
                         k_prior=d(cs['k0'][take], np.float32), ext_tgl=d(cs['ext_tgl'][take], np.float32),
                         use_vertex=d(cs['use_vertex'][take], np.uint8))

    yield trk, fit_of, len(cs['tracks']), theta_star
    trk.close()


def same(a, b):
    assert a[0] == b[0], (a[0], b[0])
    assert a[1] == b[1], (a[1], b[1])
    assert torch.equal(a[2], b[2]), float((a[2] - b[2]).abs().max())


def test_two_calls_in_a_row_match_the_allocating_entry(setup):
    trk, fit_of, nt, theta_star = setup
    th = torch.from_numpy((0.5 * theta_star.flat()).astype(np.float32)).cuda()
    big = fit_of(range(nt))
    small = fit_of(range(0, nt, 3))
    print(f"[gpu] no-alloc calls: {big.n_tracks} tracks, then {small.n_tracks}", flush=True)
    a1 = trk.refit_grad_noalloc(big, th)
    a2 = trk.refit_grad_noalloc(small, th)
    torch.cuda.synchronize()
    same(a1, trk.refit_grad(big, th))
    same(a2, trk.refit_grad(small, th))
    assert a2[0] < a1[0]


def test_reduced_stride_when_the_default_does_not_fit(setup):
    from paper_1712_09434_amd import _abi
    trk, fit_of, nt, theta_star = setup
    th = torch.from_numpy((0.3 * theta_star.flat()).astype(np.float32)).cuda()
    # at stride 160 every track keeps 348 states of 80 bytes: this set needs
    # more than the static scratch there and fits at a smaller stride
    reps = int(np.ceil(_abi.TPCCA_NOALLOC_SCRATCH_BYTES / (348 * 80 * nt))) + 1
    fit = fit_of(range(nt), reps)
    print(f"[gpu] no-alloc reduced stride: {fit.n_tracks} tracks", flush=True)
    same(trk.refit_grad_noalloc(fit, th), trk.refit_grad(fit, th))


def test_limits_and_memory_kinds(setup):
    from paper_1712_09434_amd import _abi, FitTracks, TpccaError
    trk, fit_of, nt, theta_star = setup
    th = torch.zeros(S * 66, device="cuda:0")
    # more than 128 MiB at every stride: at least 5.5 KB of states per track
    reps = int(np.ceil(_abi.TPCCA_NOALLOC_SCRATCH_BYTES / (5500 * nt))) + 1
    huge = fit_of(range(nt), reps)
    with pytest.raises(TpccaError) as e:
        trk.refit_grad_noalloc(huge, th)
    assert e.value.code == _abi.TPCCA_E_LIMIT
    fit = fit_of(range(nt))
    host = FitTracks(clusters=tuple(t.cpu() for t in fit.clusters), hit_off=fit.hit_off.cpu(),
                     hit_id=fit.hit_id.cpu(), k_prior=fit.k_prior.cpu(), ext_tgl=fit.ext_tgl.cpu(),
                     use_vertex=fit.use_vertex.cpu())
    with pytest.raises(TpccaError) as e:
        trk.refit_grad_noalloc(host, th.cpu())
    assert e.value.code == _abi.TPCCA_E_INVALID
    # still usable after the errors, and an empty set gives zeros
    empty = FitTracks(clusters=fit.clusters, hit_off=torch.zeros(1, dtype=torch.int32, device="cuda:0"),
                      hit_id=torch.zeros(1, dtype=torch.int32, device="cuda:0"),
                      k_prior=torch.zeros(1, device="cuda:0"), ext_tgl=None, use_vertex=None)
    c2, ndf, g = trk.refit_grad_noalloc(empty, th)
    assert c2 == 0.0 and ndf == 0 and torch.count_nonzero(g) == 0
    same(trk.refit_grad_noalloc(fit, th), trk.refit_grad(fit, th))
