"""Unit pins of the device pieces through the test hooks: the FP32 loop's
normal tail and quantile and the FP64 loop's normal CDF and quantile
(device_math_f64.h, fitted rationals; pinned on the CPU too, in
test_host_math.py) against
SciPy (ndtr, log_ndtr, ndtri, ndtri_exp) on a million points each, tails
included; and the lattice coordinates against the oracle's exact integer
definition, bit for bit (FP64 and FP32, both lattices of a term, the key
ranges' edges). The error figures are printed.

Bounds: the FP32 tail's relative error is the rational's (< 1.4e-6) plus the
rounding of the exponent -v^2 in FP32 (up to 2^-24 |v^2|, i.e. ln 2 v^2 2^-24
relative); the FP32 quantile's is the main rational's for s = sqrt(-log2 q) <= 34 and
the split path's second rational's beyond (q < 2^-1156, exponents to -2^20);
FP64 is HIP's library (relative errors of a few 1e-13 in the far lower
tail)."""
import math

import numpy as np
import pytest
from scipy.special import log_ndtr, ndtr, ndtri, ndtri_exp

from oracle import lattice
from tests.gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu

KAPPA = math.sqrt(1.0 / (2.0 * math.log(2.0)))
LN2 = math.log(2.0)


def _probe(V, torch, what, x_np):
    x = torch.tensor(x_np, dtype=torch.float64, device="cuda")
    out = torch.empty((len(x_np), 3), dtype=torch.float64, device="cuda")
    V.vecchia_probe_math(what, x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_fp32_normal_tail_main_and_split_paths():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    t = np.concatenate([np.linspace(-13.0, 13.0, 600_000), np.linspace(-1000.0, -9.0, 400_000)])
    o = _probe(V, torch, V.VECCHIA_PROBE_PHI_F32, t)
    v = (t * KAPPA).astype(np.float32).astype(np.float64)     # the FP32 argument the loop sees
    te = -np.abs(v) / KAPPA
    # exponent rounding: f = -v^2 in FP32 carries up to 2^-24 |f| absolute
    bound = 2.0e-6 + 2.0 * LN2 * v * v * 2.0 ** -24
    main = np.abs(v) <= 11.0                                   # 2^(-v^2) normal in FP32
    rel = np.abs(o[main, 0] / ndtr(te[main]) - 1.0)
    split = np.log(o[:, 1]) + o[:, 2] * LN2 - log_ndtr(te)
    print("FP32 tail: main path max rel %.2e, split path max |log err| %.2e" % (rel.max(), np.abs(split).max()))
    assert np.all(rel <= bound[main])
    assert np.all(np.abs(split) <= bound)


def test_fp32_quantile_from_q_and_from_its_log():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    q = np.concatenate([np.logspace(-37.5, math.log10(0.5), 900_000), np.linspace(0.3, 0.5, 100_000)])
    o = _probe(V, torch, V.VECCHIA_PROBE_NINV_F32, q)
    want = -ndtri(o[:, 1])                                     # at the FP32 q the loop sees
    err = np.abs(o[:, 0] - want)
    print("FP32 quantile: max abs err %.2e, max rel %.2e" % (err.max(), (err / np.maximum(want, 0.05)).max()))
    assert np.all(err <= 4e-6 * np.maximum(want, 0.05) + 1e-6)
    lq = -np.logspace(0.0, math.log10(1048576.0 + 126.0), 200_000)
    o = _probe(V, torch, V.VECCHIA_PROBE_NINV_LOG2_F32, lq)
    lqf = lq.astype(np.float32).astype(np.float64)
    want = -ndtri_exp(lqf * LN2)
    rel = np.abs(o[:, 0] - want) / np.maximum(want, 0.05)
    fit = -lqf <= 34.0 ** 2             # the main rational's range, s = sqrt(-log2 q) <= 34
    print("FP32 quantile from log2 q (split path): max rel %.2e for q >= 2^-1156, %.2e beyond (to 2^-1048702)"
          % (rel[fit].max(), rel[~fit].max()))
    assert np.all(rel[fit] <= 5e-6)
    assert np.all(rel[~fit] <= 1e-6)


def test_fp64_library_pieces():
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    x = np.linspace(-37.5, 8.2, 1_000_000)
    o = _probe(V, torch, V.VECCHIA_PROBE_PHI_F64, x)
    rel = np.abs(o[:, 0] / ndtr(x) - 1.0)
    print("FP64 normal CDF: max rel %.2e against SciPy's ndtr" % rel.max())
    # phi64 is within 1e-15 of the exact CDF (test_host_math.py); ndtr itself
    # is off by up to about 2e-13 in the far lower tail
    assert rel.max() <= 1e-12
    u = np.concatenate([np.logspace(-307, -1, 800_000), np.linspace(0.1, 1.0 - 2.0 ** -53, 200_000)])
    o = _probe(V, torch, V.VECCHIA_PROBE_NINV_F64, u)
    want = ndtri(u)
    err = np.abs(o[:, 0] - want) / np.maximum(np.abs(want), 1.0)
    print("FP64 quantile: max rel %.2e" % err.max())
    # both it and SciPy's ndtri are within about 6e-16 of the exact quantile
    assert err.max() <= 2e-15


def test_fp64_quantile_subnormal_and_edge_inputs():
    # the quantile's own logarithm splits p into mantissa and exponent on the
    # device (frexp); subnormal p, the smallest normal, 1/2 and the pieces'
    # edges against the quantile to 40 digits (mpmath, Newton on log Phi)
    mpmath = pytest.importorskip("mpmath")
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    u = np.array([5e-324, 1e-322, 1e-320, 3e-316, 1e-310, 2.2250738585072014e-308, 4.4501477170144028e-308,
                  1e-300, 1e-100, 1e-20, 0.0749999999, 0.075, 0.0750000001, 0.5, 1.0 - 0.075, 1.0 - 2.0 ** -53])
    o = _probe(V, torch, V.VECCHIA_PROBE_NINV_F64, u)
    mpmath.mp.dps = 40

    def exact(q):
        q = mpmath.mpf(float(q))
        if q > 0.5:
            return -exact(1 - q)
        if q > mpmath.mpf("1e-8"):
            return -mpmath.sqrt(2) * mpmath.erfinv(1 - 2 * q)
        z = -mpmath.sqrt(-2 * mpmath.log(q))
        for _ in range(200):
            dz = (mpmath.log(mpmath.ncdf(z)) - mpmath.log(q)) / (mpmath.npdf(z) / mpmath.ncdf(z))
            z -= dz
            if abs(dz) < mpmath.mpf(10) ** -36:
                break
        return z

    for q, z in zip(u, o[:, 0]):
        ref = exact(q)
        if ref == 0:
            assert z == 0.0
            continue
        assert abs(float((mpmath.mpf(float(z)) - ref) / ref)) <= 2e-15, (q, z, float(ref))


@pytest.mark.parametrize("seed,term,shift,dim,second", [
    (1, 0, 0, 0, False), (0x5EED5EED5EED, 12345, 7, 5, False), (2 ** 64 - 1, 2 ** 31 - 1, 65535, 31, False),
    (77, 3, 2, 32, False), (77, 3, 2, 62, False), (77, 3, 2, 1, True), (9, 2 ** 31 - 1, 65535, 62, True),
])
def test_lattice_coordinates_bit_for_bit(seed, term, shift, dim, second):
    torch = torch_cuda()
    from paper_2007_15195_amd import vecchia as V
    n = 1 << 18
    w64 = torch.empty(n, dtype=torch.float64, device="cuda")
    w32 = torch.empty(n, dtype=torch.float32, device="cuda")
    V.vecchia_probe_lattice(seed, term, shift, dim, second, n, w64, w32)
    torch.cuda.synchronize()
    S = lattice.shift(seed, term, shift, dim, second)
    assert np.array_equal(w64.cpu().numpy(), lattice.points(n, dim, S))
    assert np.array_equal(w32.cpu().numpy().astype(np.float64), lattice.points(n, dim, S, fp32=True))
