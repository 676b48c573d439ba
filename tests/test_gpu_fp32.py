"""Bitwise check of the device FP32 arithmetic the bit-exact contract rests on.

Neighbour links, hit choices and stop decisions are taken from FP32 values
that the CPU oracle reproduces only if the device's division and square roots
are correctly rounded (IEEE 754 round to nearest even), as the host's are.
Each operation is evaluated on the device through the library's test tap
(same compile flags as the tracking kernels) and compared bit for bit with
numpy float32 on the host:

* the cosine root sqrt_rn_normal on every float in [2^-24, 1] (its callers'
  arguments 1 - s^2 lie in [2^-23 - 2^-48, 1]), on 2^24 random floats over its
  whole stated domain [2^-96, max], and on the edges (+-0, negatives -> NaN,
  the domain limits, one ulp around powers of two);
* the reciprocal 1 / x on every float in [1/4, 4) and on 2^24 random floats of
  any magnitude (subnormal results included: denormals are kept);
* the quotient a / b on 2^24 random pairs of mixed magnitudes;
* sqrtf on 2^24 random non-negative floats (subnormals included).
"""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

CHUNK = 1 << 25


def _bits(lo, hi):
    return np.arange(lo, hi, dtype=np.uint32).view(np.float32)


def device_op(op, a, b=None):
    from paper_1712_09434_amd import _abi
    L = _abi.load()
    da = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to("cuda:0")
    db = torch.from_numpy(np.ascontiguousarray(b, np.float32)).to("cuda:0") if b is not None else None
    out = torch.empty_like(da)
    st = torch.cuda.current_stream().cuda_stream
    rc = L.tpcca_debug_fp32(op, da.numel(), C.c_void_p(da.data_ptr()),
                            C.c_void_p(db.data_ptr()) if db is not None else None,
                            C.c_void_p(out.data_ptr()), C.c_void_p(st))
    assert rc == 0
    return out.cpu().numpy()


def same_bits(got, want, what):
    g, w = got.view(np.uint32), want.view(np.uint32)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan), what + ": NaN pattern"
    bad = np.nonzero((g != w) & ~nan)[0]
    assert bad.size == 0, (what, bad.size, got[bad[:4]], want[bad[:4]])


def random_floats(rng, n, lo_exp, hi_exp, sign=False):
    """n floats with uniform random mantissas and exponents in [lo_exp, hi_exp]."""
    e = rng.integers(lo_exp + 127, hi_exp + 127 + 1, n).astype(np.uint32)
    m = rng.integers(0, 1 << 23, n, dtype=np.uint32)
    s = (rng.integers(0, 2, n).astype(np.uint32) << 31) if sign else np.uint32(0)
    return (s | (e << 23) | m).view(np.float32)


def test_cosine_root_every_float_in_callers_range():
    lo = np.float32(2.0 ** -24).view(np.uint32)
    hi = np.float32(1.0).view(np.uint32) + 1
    print(f"[gpu] sqrt_rn_normal over {hi - lo} floats", flush=True)
    for c0 in range(int(lo), int(hi), CHUNK):
        a = _bits(c0, min(c0 + CHUNK, int(hi)))
        same_bits(device_op(0, a), np.sqrt(a), f"sqrt_rn_normal chunk {c0:#x}")


def test_cosine_root_whole_domain_and_edges():
    rng = np.random.default_rng(6)
    a = random_floats(rng, 1 << 24, -96, 127)
    edges = [0.0, -0.0, -1.0, -1e-30, 2.0 ** -96, 2.0 ** -23 - 2.0 ** -48, 2.0 ** -23, 1.0,
             np.finfo(np.float32).max]
    for k in range(-96, 128):
        p = np.float32(2.0 ** k)
        edges += [p, np.nextafter(p, np.float32(0)), np.nextafter(p, np.float32(np.inf))]
    a = np.concatenate([a, np.array(edges, np.float32)])
    with np.errstate(invalid="ignore"):
        same_bits(device_op(0, a), np.sqrt(a), "sqrt_rn_normal domain")


def test_reciprocal():
    lo = np.float32(0.25).view(np.uint32)
    hi = np.float32(4.0).view(np.uint32)
    print(f"[gpu] 1/x over {hi - lo} floats", flush=True)
    for c0 in range(int(lo), int(hi), CHUNK):
        a = _bits(c0, min(c0 + CHUNK, int(hi)))
        same_bits(device_op(2, a), np.float32(1.0) / a, f"reciprocal chunk {c0:#x}")
    rng = np.random.default_rng(7)
    a = random_floats(rng, 1 << 24, -126, 127, sign=True)
    with np.errstate(over="ignore", under="ignore"):
        same_bits(device_op(2, a), np.float32(1.0) / a, "reciprocal random")


def test_division():
    rng = np.random.default_rng(8)
    n = 1 << 24
    a = random_floats(rng, n, -40, 40, sign=True)
    b = random_floats(rng, n, -40, 40, sign=True)
    # and quotients near the ends of the range (subnormal and huge results)
    a2 = random_floats(rng, 1 << 20, -126, -100)
    b2 = random_floats(rng, 1 << 20, 0, 30)
    a = np.concatenate([a, a2, b2]); b = np.concatenate([b, b2, a2])
    with np.errstate(over="ignore", under="ignore"):
        same_bits(device_op(1, a, b), a / b, "division")


def test_sqrtf():
    rng = np.random.default_rng(9)
    a = random_floats(rng, 1 << 24, -126, 127)
    sub = (rng.integers(1, 1 << 23, 1 << 16, dtype=np.uint32)).view(np.float32)   # subnormals
    a = np.concatenate([a, sub, np.array([0.0, -0.0], np.float32)])
    same_bits(device_op(3, a), np.sqrt(a), "sqrtf")
