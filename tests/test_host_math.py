"""The FP64 normal quantile and CDF of the FP64 loops and their logarithm and exponential (csrc/device_math_f64.h), built
for the host by g++, against the exact quantile computed here with 40-digit
arithmetic (mpmath): relative error within 1e-15 over q from the smallest
subnormal to 1 - 2^-53, both sides of 1/2, the pieces' edges included. The
same function runs on the GPU (test_gpu_device_math.py checks it there
against SciPy). Host code only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_15195_amd", "csrc")


def _exact_quantile(q):
    """Phi^{-1}(q) to about 35 digits: erfinv for moderate q, else Newton on
    log Phi(z) = log q (so tiny q keep their digits)."""
    mpmath.mp.dps = 40
    q = mpmath.mpf(q)
    if q > mpmath.mpf("0.5"):
        return -_exact_quantile(1 - q)
    if q > mpmath.mpf("1e-8"):
        return -mpmath.sqrt(2) * mpmath.erfinv(1 - 2 * q)
    z = -mpmath.sqrt(-2 * mpmath.log(q))
    for _ in range(200):
        dz = (mpmath.log(mpmath.ncdf(z)) - mpmath.log(q)) / (mpmath.npdf(z) / mpmath.ncdf(z))
        z -= dz
        if abs(dz) < mpmath.mpf(10) ** -36:
            break
    return z


def test_fp64_quantile_against_the_exact_quantile(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "ninv64_check")
    r = subprocess.run([gxx, "-std=c++17", "-O2", "-mfma", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host_sanitize", "ninv64_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host build unavailable: " + r.stderr[-300:])
    rng = np.random.default_rng(7)
    qs = np.concatenate([
        rng.uniform(0.0, 1.0, 1500),
        10.0 ** rng.uniform(-307.0, -0.3, 1500),
        1.0 - 10.0 ** rng.uniform(-15.9, -0.3, 800),
        [5e-324, 1e-320, 2.2250738585072014e-308, 1.4e-11, 0.0749999, 0.075, 0.0750001,
         0.5 - 2.0 ** -53, 0.5 + 2.0 ** -53, 0.925, 1.0 - 2.0 ** -53],
    ])
    qs = qs[(qs > 0.0) & (qs < 1.0)]
    text = "\n".join(repr(float(q)) for q in qs) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = [float(v) for v in out.stdout.split()]
    assert len(got) == len(qs)
    worst = 0.0
    for q, z in zip(qs, got):
        ref = _exact_quantile(float(q))
        if ref == 0:
            assert abs(z) < 1e-300
            continue
        rel = float(abs((mpmath.mpf(z) - ref) / ref))
        worst = max(worst, rel)
        assert rel <= 1e-15, (float(q), z, float(ref), rel)
    # the interval's ends and values outside it
    out = subprocess.run([exe], input="0\n1\n-0.5\n1.5\nnan\n", capture_output=True, text=True, timeout=60)
    ends = [float(v) for v in out.stdout.split()]
    assert ends[0] == -np.inf and ends[1] == np.inf and all(np.isnan(ends[2:]))
    # the symmetry z(1 - q) = -z(q) holds exactly where 1 - q is exact
    half = qs[qs < 0.5][:200]
    text = "\n".join(repr(float(q)) for q in np.concatenate([half, 1.0 - half])) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=120)
    vals = np.array([float(v) for v in out.stdout.split()])
    lo, hi = vals[:len(half)], vals[len(half):]
    exact = (1.0 - (1.0 - half)) == half
    assert np.array_equal(lo[exact], -hi[exact])
    print("FP64 quantile on the host: max relative error %.2e over %d points" % (worst, len(qs)))


def test_fp64_normal_cdf_against_the_exact_cdf(tmp_path):
    # phi64 (device_math_f64.h) on the host against mpmath's 40-digit normal
    # CDF: relative error within 2e-15 wherever Phi(t) is a normal double,
    # exact 0 / 1 at -inf / +inf, 0 below the smallest subnormal
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "phi64_check")
    r = subprocess.run([gxx, "-std=c++17", "-O2", "-mfma", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host_sanitize", "phi64_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host build unavailable: " + r.stderr[-300:])
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11)
    ts = np.concatenate([rng.uniform(-37.5, 9.0, 2500), rng.uniform(-3.0, 3.0, 1000),
                         [0.0, -0.0, 1e-300, -1e-300, -37.5, -38.4, 8.3, 38.5, -39.0, -1e6, np.inf, -np.inf]])
    text = "\n".join(repr(float(t)) for t in ts) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = [float(v) for v in out.stdout.split()]
    assert len(got) == len(ts)
    worst = 0.0
    for t, v in zip(ts, got):
        if t == -np.inf or t < -38.5:
            assert v == 0.0
            continue
        if t == np.inf:
            assert v == 1.0
            continue
        ref = mpmath.ncdf(mpmath.mpf(float(t)))
        if ref < mpmath.mpf("2.2250738585072014e-308"):
            continue
        rel = float(abs((mpmath.mpf(v) - ref) / ref))
        worst = max(worst, rel)
        assert rel <= 2e-15, (float(t), v, float(ref), rel)
    print("FP64 normal CDF on the host: max relative error %.2e" % worst)


def test_fp64_log_against_the_exact_log(tmp_path):
    # log64 (the quantile's logarithm, device_math_f64.h) on the host against
    # mpmath's 40-digit log: within one unit in the last place from the smallest
    # subnormal to the largest double, around 1 and around the reduction's
    # split at sqrt(1/2); exact at 1
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "log64_check")
    r = subprocess.run([gxx, "-std=c++17", "-O2", "-mfma", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host_sanitize", "log64_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host build unavailable: " + r.stderr[-300:])
    mpmath.mp.dps = 40
    rng = np.random.default_rng(3)
    split = 0.70710678118654752
    xs = np.concatenate([
        10.0 ** rng.uniform(-323.0, 308.0, 2000),
        rng.uniform(0.5, 2.0, 1500),
        1.0 + 10.0 ** rng.uniform(-16.0, -1.0, 400),
        1.0 - 10.0 ** rng.uniform(-16.0, -1.0, 400),
        split * (1.0 + rng.uniform(-1e-12, 1e-12, 200)),
        [5e-324, 1e-310, 2.2250738585072014e-308, 0.5, 2.0, 0.075, 1e308, 1.7976931348623157e308],
    ])
    text = "\n".join(repr(float(x)) for x in xs) + "\n"
    out = subprocess.run([exe], input=text + "1\n", capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = [float(v) for v in out.stdout.split()]
    assert len(got) == len(xs) + 1 and got[-1] == 0.0
    worst = 0.0
    for x, v in zip(xs, got):
        ref = mpmath.log(mpmath.mpf(float(x)))
        ulps = float(abs(mpmath.mpf(v) - ref)) / np.spacing(abs(float(ref)))
        worst = max(worst, ulps)
        assert ulps <= 1.0, (float(x), v, float(ref), ulps)
    print("FP64 log on the host: max error %.2f units in the last place" % worst)


def test_fp64_exp_against_the_exact_exp(tmp_path):
    # exp64 (the normal CDF's Gaussian factor, device_math_f64.h) on the host
    # against mpmath's 40-digit exp over its domain [-745, 0]: within one unit in
    # the last place (one subnormal step where the result is subnormal); exact at 0
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "exp64_check")
    r = subprocess.run([gxx, "-std=c++17", "-O2", "-mfma", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host_sanitize", "exp64_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host build unavailable: " + r.stderr[-300:])
    mpmath.mp.dps = 40
    rng = np.random.default_rng(5)
    ln2h = 0.34657359027997264
    xs = np.concatenate([
        rng.uniform(-745.0, 0.0, 3000),
        -(10.0 ** rng.uniform(-20.0, 2.8, 1500)),
        [-745.0, -744.4, -708.4, -708.39, -ln2h, -ln2h * (1 + 1e-15), -ln2h * 3, -1e-300],
    ])
    text = "\n".join(repr(float(x)) for x in xs) + "\n"
    out = subprocess.run([exe], input=text + "0\n", capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = [float(v) for v in out.stdout.split()]
    assert len(got) == len(xs) + 1 and got[-1] == 1.0
    worst = 0.0
    for x, v in zip(xs, got):
        ref = mpmath.exp(mpmath.mpf(float(x)))
        ulps = float(abs(mpmath.mpf(v) - ref)) / np.spacing(float(ref))
        worst = max(worst, ulps)
        assert ulps <= 1.0, (float(x), v, float(ref), ulps)
    print("FP64 exp on the host: max error %.2f units in the last place" % worst)
