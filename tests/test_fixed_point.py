"""The fixed-point terms of fusion's per-frame voxel sums (gsdf_fixed.hpp),
built for the host from the same header the kernel includes: exact for
non-negative and large negative terms, within 2^7 units for small negative
ones, including
the remainder that rounds up to 2^32 (the saturating conversion)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def fx(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fixed") / "libfixed.so")
    src = os.path.join(HERE, "native", "fixed_point_harness.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-o", out, src])
    lib = C.CDLL(out)
    lib.fixed_term_host.restype = C.c_uint64
    lib.fixed_term_host.argtypes = [C.c_float, C.c_float, C.c_float]
    lib.from_fixed_host.restype = C.c_float
    lib.from_fixed_host.argtypes = [C.c_uint64, C.c_double]
    return lib


def _term(lib, w, x, f):
    ws = np.float32(w) * np.float32(2.0 ** f)
    wh = ws * np.float32(2.0 ** -32)
    v = lib.fixed_term_host(float(ws), float(wh), float(np.float32(x)))
    v = v - (1 << 64) if v >= (1 << 63) else v
    s = float(np.float32(ws) * np.float32(x))   # the float32 product, in units of 2^-f
    return v, s


def test_non_negative_terms_are_exact(fx):
    rng = np.random.default_rng(0)
    for f in (24, 40, 52, 56):
        for _ in range(2000):
            w = np.float32(rng.uniform(0.0, 1.0))
            x = np.float32(rng.uniform(0.0, 1.0) * 10.0 ** rng.integers(-9, 1))
            v, s = _term(fx, w, x, f)
            assert v == int(s), (f, w, x, v, s)


def test_negative_terms_within_2_to_7_units(fx):
    rng = np.random.default_rng(1)
    for f in (24, 40, 52, 56):
        for _ in range(2000):
            w = np.float32(rng.uniform(0.0, 1.0))
            x = -np.float32(rng.uniform(0.0, 1.0) * 10.0 ** rng.integers(-12, 1))
            v, s = _term(fx, w, x, f)
            assert abs(v - s) <= 128, (f, w, x, v, s)
            if -s >= 2.0 ** 32:
                assert v == int(s), (f, w, x, v, s)


def test_remainder_that_rounds_to_2_pow_32(fx):
    """A negative term of |w x 2^f| < 128 leaves hi = -1 and a remainder
    2^32 - |w x 2^f| that rounds to 2^32 in float32; the conversion
    saturates, so the term reads -1 unit (not a wrapped value)."""
    for s_units in (1.0, 3.5, 100.0, 127.0):
        f = 52
        w = 1.0
        x = -s_units * 2.0 ** -f
        v, s = _term(fx, w, x, f)
        assert v == -1, (s_units, v)
    # just past the rounding point the remainder stays below 2^32
    v, s = _term(fx, 1.0, -200.0 * 2.0 ** -52, 52)
    assert abs(v - s) <= 128


def test_sum_of_terms_is_order_independent_and_close(fx):
    rng = np.random.default_rng(2)
    f = 52
    w = rng.uniform(0.0, 1.0, 500).astype(np.float32)
    x = rng.uniform(-0.05, 0.05, 500).astype(np.float32)
    terms = [_term(fx, wi, xi, f)[0] for wi, xi in zip(w, x)]
    a = sum(terms) % (1 << 64)
    b = sum(terms[::-1]) % (1 << 64)
    assert a == b
    total = fx.from_fixed_host(a, 2.0 ** -f)
    exact = float(np.sum(w.astype(np.float64) * x.astype(np.float64)))
    assert abs(total - exact) <= 1e-6 * np.sum(np.abs(w * x)) + 1e-12
