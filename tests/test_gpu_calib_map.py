"""The calibration map in front of tracking (tpcca_set_calib), on the GPU.

With a calibration installed the library corrects every cluster inside
binning.  The oracle applies its own FP32 correction (calib_apply32, pinned
in test_oracle_calib32.py) to the same input clusters and tracks the result:
links, start hits, tracklets and final hit lists must agree bit for bit,
track parameters within 1e-4, on a miscalibrated full event with its
injected calibration installed.  Also: theta = 0 and a removed calibration
give the uncorrected result bit for bit; host and device theta agree; a
batch and a replayed graph see the installed calibration; a non-finite
theta is rejected.
"""
import numpy as np
import pytest
import torch

import synth
from test_gpu_track import compare, host, to_dev

pytestmark = pytest.mark.gpu
S = 36


@pytest.fixture(scope="module")
def tracker():
    from paper_1712_09434_amd import Tracker
    trk = Tracker.from_geometry(synth.default_geometry())
    yield trk
    trk.close()


@pytest.fixture(scope="module")
def miscal():
    print("[gpu] calibration map: generating a miscalibrated full event", flush=True)
    return synth.make_config("C5", 0), synth.draw_theta().flat().astype(np.float32)


def same_tracks(a, b):
    for k in ("hit_off", "hit_id", "sector", "x_ref", "p", "cov", "chi2", "ndf"):
        assert torch.equal(getattr(a, k).cpu(), getattr(b, k).cpu()), k


def test_parity_with_the_injected_calibration(tracker, orc, miscal):
    ev, th = miscal
    print(f"[gpu] parity with the calibration installed n={ev.n}", flush=True)
    tracker.set_calib(torch.from_numpy(th).cuda())
    try:
        out = host(tracker.track(*to_dev(ev), taps=True))
        tl = tracker.debug_tracklets()
    finally:
        tracker.set_calib(None)
    ref = orc.track(ev, precision=32, theta=th)
    compare(ev, out, tl, ref)
    raw = orc.track(ev, precision=32)
    # the correction really changed the input: some hit lists differ
    assert len(raw["hit_ids"]) != len(ref["hit_ids"]) or not np.array_equal(raw["hit_ids"], ref["hit_ids"])


def test_zero_and_removed_calibration_change_nothing(tracker, miscal):
    ev, th = miscal
    cl = to_dev(ev)
    base = tracker.track(*cl)
    tracker.set_calib(torch.zeros(S * 66, device="cuda:0"))
    zero = tracker.track(*cl)
    tracker.set_calib(torch.from_numpy(th).cuda())
    corr = tracker.track(*cl)
    tracker.set_calib(None)
    after = tracker.track(*cl)
    same_tracks(base, zero)
    same_tracks(base, after)
    assert not torch.equal(base.p.cpu()[:100], corr.p.cpu()[:100])


def test_host_theta_batch_and_graph(tracker, miscal):
    ev, th = miscal
    ev2 = synth.make_event(seed=6, n_primaries=300, noise=0.05)
    cl, cl2 = to_dev(ev), to_dev(ev2)
    tracker.set_calib(torch.from_numpy(th).cuda())
    dev_out = tracker.track(*cl)
    tracker.set_calib(torch.from_numpy(th))                 # host memory
    host_out = tracker.track(*cl)
    single2 = tracker.track(*cl2)
    batch = tracker.track_batch([cl, cl2])
    same_tracks(dev_out, host_out)
    same_tracks(dev_out, batch[0])
    same_tracks(single2, batch[1])
    # graph replay: capture with one calibration, replay after installing another
    s = torch.cuda.Stream()
    tracker.set_tuning(use_graph=1)
    try:
        with torch.cuda.stream(s):
            g1 = tracker.track(*cl)
            tracker.set_calib(torch.from_numpy(0.5 * th).cuda())
            g2 = tracker.track(*cl)
            tracker.set_tuning(use_graph=0)
            e2 = tracker.track(*cl)
        s.synchronize()
    finally:
        tracker.set_tuning(use_graph=0)
        tracker.set_calib(None)
    same_tracks(dev_out, g1)
    same_tracks(e2, g2)


def test_invalid_theta_rejected(tracker):
    from paper_1712_09434_amd import TpccaError
    bad = torch.zeros(S * 66)
    bad[5] = float("nan")
    with pytest.raises(TpccaError):
        tracker.set_calib(bad)
    with pytest.raises(ValueError):
        tracker.set_calib(torch.zeros(10))
