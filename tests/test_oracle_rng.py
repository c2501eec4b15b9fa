"""Pins of the oracle's random numbers against independent references.

* Philox4x32-10 against the installed rocRAND engine (its host-callable
  header, compiled and run here) -- an implementation that shares nothing
  with the oracle.
* The Box-Muller mapping against libm log/cos/sin on the same Philox words.
* The series log / sincos / Newton cube root against long-double libm.
* The normal deviates' moments and a Kolmogorov-Smirnov test.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    out = tmp_path_factory.mktemp("rocrand") / "philox_ref"
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-w",
                    os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", str(out)], check=True)
    return str(out)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(1)
    cases = [(0, 0, 0, 0, 0, 0), (2**32 - 1,) * 6, (5, 2**32 - 1, 1, 0, 7, 0), (123, 0, 0, 0, 0, 0),
             (0, 1, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0), (0, 0, 0, 1, 0, 0), (0, 0, 0, 0, 1, 0),
             (0, 0, 0, 0, 0, 1)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, 6)) for _ in range(200)]
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    res = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in res.strip().splitlines()], np.uint64)
    got = np.array([O.philox4x32_10(c[:4], c[4:]) for c in cases], np.uint64)
    assert ref.shape == got.shape
    np.testing.assert_array_equal(got, ref)


def _philox_words(seed, pid, step, ens):
    key = (seed & 0xFFFFFFFF, seed >> 32)
    return np.concatenate([O.philox4x32_10((pid, step, b, ens), key) for b in (0, 1)])


@pytest.mark.parametrize("f32", [False, True])
def test_box_muller_mapping_against_libm(f32):
    for seed, pid, step, ens in [(0, 0, 0, 0), (0, 17, 3, 0), (12345, 999, 2**32 - 1, 5), (2**40 + 3, 7, 42, 1)]:
        r = _philox_words(seed, pid, step, ens)
        if f32:
            u = ((r >> np.uint64(9)).astype(np.float64) * 2.0**-23 + 2.0**-24)
        else:
            u = r.astype(np.float64) * 2.0**-32 + 2.0**-33
        ref = []
        for p in range(4):
            rad = math.sqrt(-2.0 * math.log(u[2 * p]))
            ref += [rad * math.cos(2 * math.pi * u[2 * p + 1]), rad * math.sin(2 * math.pi * u[2 * p + 1])]
        got = O.normals(seed, pid, step, ens, f32)
        tol = 2e-6 if f32 else 1e-13
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("f32", [False, True])
def test_normal_moments_and_ks(f32):
    z = O.normals_batch(2024, 400_000, 7, 0, f32).reshape(-1)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 5 * math.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the five deviates a step uses are uncorrelated
    zz = O.normals_batch(2024, 200_000, 8, 0, f32)[:, :5]
    c = np.corrcoef(zz.T)
    assert np.abs(c - np.eye(5)).max() < 5 / math.sqrt(zz.shape[0])


def test_distinct_counters_give_distinct_streams():
    a = O.normals(0, 1, 2, 0, False)
    for other in [(0, 2, 2, 0), (0, 1, 3, 0), (0, 1, 2, 1), (1, 1, 2, 0)]:
        assert not np.allclose(a, O.normals(other[0], other[1], other[2], other[3], False))


def _ulp(x, dtype):
    return np.spacing(np.abs(x).astype(dtype)).astype(np.float64)


def test_series_log_accuracy():
    rng = np.random.default_rng(3)
    xs = np.exp(rng.uniform(-30.0, 12.0, 20000))
    xs = np.concatenate([xs, [1.0, 0.5, 2.0, 2.0**-33, 1 - 2.0**-33, 0.7071067811865476, 255.0]])
    ref = np.log(xs.astype(np.longdouble))
    got = np.array([O.log64(float(x)) for x in xs], dtype=np.longdouble)
    err = np.abs(got - ref) / np.maximum(_ulp(np.asarray(ref, np.float64), np.float64), 2.0**-1074)
    assert err.max() <= 4.0
    xf = xs.astype(np.float32)
    xf = xf[np.isfinite(xf) & (xf > 0)]
    reff = np.log(xf.astype(np.longdouble))
    gotf = np.array([O.log32(float(x)) for x in xf], dtype=np.longdouble)
    errf = np.abs(gotf - reff) / _ulp(np.asarray(reff, np.float32), np.float32)
    keep = np.abs(reff) > 1e-3  # relative ulps blow up only at log(1) = 0
    assert errf[keep].max() <= 4.0
    assert np.abs(gotf - reff)[~keep].max() <= 4 * 2.0**-24 * 1e-3


def test_series_sincos_accuracy():
    rng = np.random.default_rng(4)
    ts = np.concatenate([rng.uniform(0.0, 1.0, 20000), [2.0**-33, 0.125, 0.25, 0.375, 0.5, 0.875, 1 - 2.0**-33]])
    two_pi = np.longdouble("6.283185307179586476925286766559")
    arg = two_pi * ts.astype(np.longdouble)
    rs, rc = np.sin(arg), np.cos(arg)
    got = np.array([O.sincos2pi64(float(t)) for t in ts], dtype=np.longdouble)
    assert np.abs(got[:, 0] - rs).max() <= 4 * 2.0**-53
    assert np.abs(got[:, 1] - rc).max() <= 4 * 2.0**-53
    tf = ts.astype(np.float32)
    argf = two_pi * tf.astype(np.longdouble)
    gotf = np.array([O.sincos2pi32(float(t)) for t in tf], dtype=np.longdouble)
    assert np.abs(gotf[:, 0] - np.sin(argf)).max() <= 4 * 2.0**-24
    assert np.abs(gotf[:, 1] - np.cos(argf)).max() <= 4 * 2.0**-24


def test_newton_cbrt_accuracy():
    rng = np.random.default_rng(5)
    xs = np.exp(rng.uniform(-40.0, 20.0, 5000))
    ref = np.cbrt(xs)
    got = np.array([O.cbrt64(float(x)) for x in xs])
    assert (np.abs(got - ref) / np.spacing(ref)).max() <= 2.0
    assert O.cbrt64(27.0) == 3.0 and O.cbrt64(0.125) == 0.5
