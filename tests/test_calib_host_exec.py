"""The library's calibration-gradient code executed on the host.

tests/host/calib_host.hip compiles tpcca_calib.hip for the CPU (the per-hit,
per-track and partials functions are host+device) and runs it with exact-size
buffers, also under AddressSanitizer; its FP32 gradient is compared with the
oracle's FP64 gradient on a small miscalibrated event.  This checks the
kernels' arithmetic and indexing without a GPU; the GPU tests check the
same on the device.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from calibset import calib_subset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "calib_host.hip")
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math"]

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    d = tmp_path_factory.mktemp("calib_host")
    plain = str(d / "calib_host")
    asan = str(d / "calib_host_asan")
    subprocess.run(["hipcc", *FLAGS, "-o", plain, SRC], check=True, capture_output=True)
    subprocess.run(["hipcc", *FLAGS, "-Xarch_host", "-fsanitize=address", "-o", asan, SRC], check=True,
                   capture_output=True)
    return plain, asan


@pytest.fixture(scope="module")
def data(orc, tmp_path_factory):
    theta_star = synth.draw_theta(77)
    ev = synth.make_event(seed=31, n_primaries=300, noise=0.01, theta=theta_star)
    r = orc.track(ev, precision=32)
    kp = r["seed_state"][r["trk_seed"], 4].astype(np.float32)
    cs = calib_subset(ev, r["hit_off"], r["hit_ids"], r["sector"], r["chi2"], r["ndf"], kp)
    cs["k0"] = cs["k0"].astype(np.float32).astype(np.float64)
    cs["ext_tgl"] = cs["ext_tgl"].astype(np.float32).astype(np.float64)
    d = tmp_path_factory.mktemp("calib_data")
    w = lambda n, a: np.ascontiguousarray(a).tofile(str(d / n))
    w("hit_off", cs["hit_off"].astype(np.int32)); w("hit_id", cs["hit_ids"].astype(np.uint32))
    w("k0", cs["k0"].astype(np.float32)); w("ext", cs["ext_tgl"].astype(np.float32))
    w("uv", cs["use_vertex"].astype(np.uint8)); w("x", ev.x); w("y", ev.y); w("z", ev.z)
    w("sec", ev.sector); w("row_x", ev.geom.row_x)
    return ev, cs, theta_star, str(d)


def run(binary, d, theta, K):
    np.asarray(theta, np.float32).tofile(os.path.join(d, "theta"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    subprocess.run([binary, d, str(K)], check=True, capture_output=True, env=env)
    g = np.fromfile(os.path.join(d, "out_grad"), np.float64)
    gs = g[:-1].reshape(36, 66)
    return g[-1], np.concatenate([gs[:, 0], gs[:, 1], gs[:, 2:].ravel()])


@pytest.mark.parametrize("where", ["zero", "half"])
def test_host_gradient_matches_oracle(binaries, data, orc, where):
    ev, cs, theta_star, d = data
    th = (np.zeros(36 * 66) if where == "zero" else 0.5 * theta_star.flat()).astype(np.float32)
    c2, g = run(binaries[0], d, th, 12)
    rc2, _, _, rg = orc.calib_chi2(ev.geom, ev.x.astype(float), ev.y.astype(float), ev.z.astype(float),
                                   ev.sector, cs["hit_off"], cs["hit_ids"], cs["k0"], th.astype(float),
                                   ext_tgl=cs["ext_tgl"], use_vertex=cs["use_vertex"], grad=True)
    assert abs(c2 - rc2) <= 1e-4 * rc2
    for sl in (slice(0, 36), slice(36, 72), slice(72, 36 * 66)):
        assert np.linalg.norm(g[sl] - rg[sl]) <= 1e-3 * np.linalg.norm(rg[sl])


def test_host_gradient_under_asan_all_strides(binaries, data):
    ev, cs, theta_star, d = data
    ref = None
    for K in (1, 7, 12, 160):
        c2, g = run(binaries[1], d, 0.3 * theta_star.flat(), K)
        if ref is None:
            ref = (c2, g)
        assert c2 == ref[0] and np.array_equal(g, ref[1]), K
