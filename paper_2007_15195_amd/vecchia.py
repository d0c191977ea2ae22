"""ctypes binding of libvecchia.so, with the C ABI's names (include/vecchia.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch CUDA tensors (float64); streams are torch.cuda
streams or raw hipStream_t integers. Host arrays are numpy arrays. A non-OK
status raises VecchiaError carrying the status and the library's message.
The library must have been built (python -m paper_2007_15195_amd.build); there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libvecchia.so")

VECCHIA_OK = 0
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_NOT_PD", 4: "E_HIP", 5: "E_BUSY",
                6: "E_NOT_READY", 7: "E_NONFINITE"}
VECCHIA_ORDER_GIVEN, VECCHIA_ORDER_COORD, VECCHIA_ORDER_MAXMIN = 0, 1, 2
VECCHIA_COV_EXPONENTIAL, VECCHIA_COV_MATERN = 0, 1
VECCHIA_FP64, VECCHIA_FP32_LOOP = 0, 1
VECCHIA_MAX_M = 63
VECCHIA_MAX_SHIFTS = 65536
VECCHIA_MAX_POINTS = 1 << 30
VECCHIA_QMC_INDEPENDENT = 1
VECCHIA_NOALLOC_SCRATCH_BYTES = 64 << 20
VECCHIA_PROFILE_FULL_SOV = -1   # vecchia_profile_read key of the full-dimension kernel

EXPORTED = [
    "vecchia_last_error", "vecchia_order", "vecchia_plan", "vecchia_plan_from_cov",
    "vecchia_replan", "vecchia_plan_info", "vecchia_plan_neighbours", "vecchia_logcdf", "vecchia_logcdf_noalloc",
    "vecchia_plan_status",
    "vecchia_plan_destroy", "vecchia_batch_create", "vecchia_batch_logcdf", "vecchia_batch_status",
    "vecchia_batch_destroy", "vecchia_server_create", "vecchia_submit", "vecchia_poll",
    "vecchia_server_destroy", "vecchia_profile_enable", "vecchia_profile_read", "vecchia_profile_reset",
    "vecchia_autotune", "vecchia_tuning_get", "vecchia_tuning_set", "vecchia_calibrate_valu",
    "vecchia_mixture_logcdf", "vecchia_mixture_rule", "vecchia_mixture_search",
    "vecchia_plan_censored", "vecchia_plan_from_cov_censored", "vecchia_plan_censoring",
    "vecchia_mixbatch_create", "vecchia_mixbatch_logcdf", "vecchia_mixbatch_status", "vecchia_mixbatch_destroy",
    "vecchia_map_anisotropic", "vecchia_plan_block", "vecchia_plan_block_terms", "vecchia_plan_from_cov_block",
    "vecchia_full_logcdf", "vecchia_probe_math", "vecchia_probe_lattice",
]


class VecchiaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class vecchia_cov(ctypes.Structure):
    _fields_ = [("family", c_int32), ("reserved", c_int32), ("nu", c_double), ("sigma2", c_double),
                ("range", c_double), ("nugget", c_double)]


class vecchia_mixture(ctypes.Structure):
    _fields_ = [("beta", c_double), ("gamma", c_double), ("n_nodes", c_int32), ("reserved", c_int32)]


class vecchia_qmc(ctypes.Structure):
    _fields_ = [("n_points", c_int32), ("n_shifts", c_int32), ("seed", c_uint64),
                ("precision", c_int32), ("flags", c_int32)]


_lib = None


def lib():
    """Load libvecchia.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_15195_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.vecchia_last_error.restype = ctypes.c_char_p
    sig = {
        "vecchia_order": [c_void_p, c_int64, c_int32, c_void_p, c_void_p],
        "vecchia_plan": [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int32, POINTER(vecchia_cov),
                         c_void_p, POINTER(c_void_p)],
        "vecchia_plan_from_cov": [c_void_p, c_int64, c_void_p, c_int32, c_void_p, POINTER(c_void_p)],
        "vecchia_plan_censored": [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                  POINTER(vecchia_cov), c_void_p, POINTER(c_void_p)],
        "vecchia_plan_from_cov_censored": [c_void_p, c_int64, c_void_p, c_int32, c_int64, c_void_p,
                                           POINTER(c_void_p)],
        "vecchia_plan_censoring": [c_void_p, POINTER(c_int64)],
        "vecchia_mixbatch_create": [c_void_p, c_int32, c_int32, POINTER(vecchia_qmc), POINTER(c_void_p)],
        "vecchia_mixbatch_logcdf": [c_void_p, c_void_p, POINTER(vecchia_mixture), c_void_p, c_void_p, c_void_p,
                                    c_void_p],
        "vecchia_mixbatch_status": [c_void_p, c_void_p],
        "vecchia_mixbatch_destroy": [c_void_p],
        "vecchia_map_anisotropic": [c_void_p, c_int64, c_double, c_double, c_void_p],
        "vecchia_plan_block": [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int32, c_int32, POINTER(vecchia_cov),
                               c_void_p, POINTER(c_void_p)],
        "vecchia_plan_block_terms": [c_void_p, POINTER(c_int64), c_void_p, c_void_p, c_void_p],
        "vecchia_plan_from_cov_block": [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                                        POINTER(c_void_p)],
        "vecchia_full_logcdf": [c_void_p, c_void_p, c_double, c_void_p, POINTER(vecchia_qmc), c_void_p, c_void_p],
        "vecchia_replan": [c_void_p, c_void_p, c_int32, c_void_p, c_void_p],
        "vecchia_plan_info": [c_void_p, POINTER(c_int64), POINTER(c_int32)],
        "vecchia_plan_neighbours": [c_void_p, c_void_p, c_void_p],
        "vecchia_logcdf": [c_void_p, c_void_p, c_double, c_void_p, POINTER(vecchia_qmc), c_void_p,
                           c_void_p, c_void_p],
        "vecchia_logcdf_noalloc": [c_void_p, c_void_p, c_double, c_void_p, POINTER(vecchia_qmc), c_void_p,
                                   c_void_p, c_void_p],
        "vecchia_plan_status": [c_void_p, POINTER(c_int64)],
        "vecchia_plan_destroy": [c_void_p],
        "vecchia_batch_create": [c_void_p, c_int32, c_void_p, POINTER(c_void_p)],
        "vecchia_batch_logcdf": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
        "vecchia_batch_status": [c_void_p, c_void_p],
        "vecchia_batch_destroy": [c_void_p],
        "vecchia_server_create": [c_size_t, c_int32, POINTER(c_void_p)],
        "vecchia_submit": [c_void_p, c_void_p, c_void_p, c_double, c_void_p, POINTER(vecchia_qmc),
                           POINTER(c_uint64)],
        "vecchia_poll": [c_void_p, c_uint64, POINTER(c_double), POINTER(c_double), POINTER(c_int32),
                         POINTER(c_double)],
        "vecchia_server_destroy": [c_void_p],
        "vecchia_profile_enable": [c_int32],
        "vecchia_profile_read": [c_int32, c_int32, POINTER(c_double), POINTER(c_int64), POINTER(c_int64)],
        "vecchia_profile_reset": [],
        "vecchia_autotune": [c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p],
        "vecchia_tuning_get": [c_int32, c_int32, POINTER(c_int32)],
        "vecchia_tuning_set": [c_int32, c_int32, c_int32],
        "vecchia_calibrate_valu": [c_void_p, c_void_p],
        "vecchia_probe_math": [c_int32, c_int64, c_void_p, c_void_p, c_void_p],
        "vecchia_probe_lattice": [c_uint64, c_int64, c_int32, c_int32, c_int32, c_int64, c_void_p, c_void_p,
                                  c_void_p],
        "vecchia_mixture_logcdf": [c_void_p, c_void_p, POINTER(vecchia_mixture), c_void_p, POINTER(vecchia_qmc),
                                   c_void_p, c_void_p, c_void_p],
        "vecchia_mixture_rule": [POINTER(vecchia_mixture), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
        "vecchia_mixture_search": [POINTER(vecchia_mixture), c_void_p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = c_int32
    _lib = L
    return L


def _check(status: int):
    if status != VECCHIA_OK:
        raise VecchiaError(status, lib().vecchia_last_error().decode())


def _stream_ptr(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, n: int | None = None, name: str = "tensor") -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} must hold at least {n} values")
    return t.data_ptr()


def make_cov(family=VECCHIA_COV_MATERN, nu=0.5, sigma2=1.0, range=0.1, nugget=0.0) -> vecchia_cov:
    return vecchia_cov(int(family), 0, float(nu), float(sigma2), float(range), float(nugget))


def make_qmc(n_points=1000, n_shifts=10, seed=1, precision=VECCHIA_FP64, independent=False) -> vecchia_qmc:
    """QMC settings; independent: separate point sets for each term's numerator
    and denominator (VECCHIA_QMC_INDEPENDENT)."""
    return vecchia_qmc(int(n_points), int(n_shifts), int(seed) & (2 ** 64 - 1), int(precision),
                       VECCHIA_QMC_INDEPENDENT if independent else 0)


def as_cov(c) -> vecchia_cov:
    if c is None or isinstance(c, vecchia_cov):
        return c
    return make_cov(c.family, c.nu, c.sigma2, c.range, c.nugget)


def as_qmc(q) -> vecchia_qmc:
    if isinstance(q, vecchia_qmc):
        return q
    return make_qmc(q.n_points, q.n_shifts, q.seed, q.precision, getattr(q, "independent", False))


# ----------------------------------------------------------------- entry points

def vecchia_last_error() -> str:
    return lib().vecchia_last_error().decode()


def vecchia_order(locs: np.ndarray, ordering: int, perm=None) -> np.ndarray:
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    D = locs.shape[0]
    out = np.empty(D, dtype=np.int64)
    pin = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    _check(lib().vecchia_order(locs.ctypes.data, D, int(ordering),
                               None if pin is None else pin.ctypes.data, out.ctypes.data))
    return out


def vecchia_plan(locs: np.ndarray, ordering: int, m: int, cov, perm=None, stream=None) -> int:
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    if locs.ndim != 2:
        raise ValueError("locs must be D x dim")
    pin = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    h = c_void_p()
    c = as_cov(cov)
    _check(lib().vecchia_plan(locs.ctypes.data, locs.shape[0], locs.shape[1], int(ordering),
                              None if pin is None else pin.ctypes.data, int(m), byref(c),
                              _stream_ptr(stream), byref(h)))
    return h.value


def _nbr_table(nbr, D: int, m: int):
    if nbr is None:
        return None
    nb = np.full((D, m), -1, dtype=np.int32)
    for i, row in enumerate(nbr):
        row = list(row)
        nb[i, :len(row)] = row
    return nb


def vecchia_plan_from_cov(Sigma: np.ndarray, m: int, nbr=None, stream=None) -> int:
    Sigma = np.ascontiguousarray(Sigma, dtype=np.float64)
    D = Sigma.shape[0]
    nb = _nbr_table(nbr, D, m)
    h = c_void_p()
    _check(lib().vecchia_plan_from_cov(Sigma.ctypes.data, D, None if nb is None else nb.ctypes.data,
                                       int(m), _stream_ptr(stream), byref(h)))
    return h.value


def vecchia_plan_censored(locs: np.ndarray, observed, ordering: int, m: int, cov, perm=None,
                          stream=None) -> int:
    """Censored plan of one replicate: observed[u] true where site u's value is
    observed (eq. (11)); those sites are ordered first."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    if locs.ndim != 2:
        raise ValueError("locs must be D x dim")
    obs = np.ascontiguousarray(np.asarray(observed, dtype=bool), dtype=np.uint8)
    if obs.shape != (locs.shape[0],):
        raise ValueError("observed must hold one flag per location")
    pin = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    h = c_void_p()
    c = as_cov(cov)
    _check(lib().vecchia_plan_censored(locs.ctypes.data, locs.shape[0], locs.shape[1], int(ordering),
                                       None if pin is None else pin.ctypes.data, obs.ctypes.data, int(m),
                                       byref(c), _stream_ptr(stream), byref(h)))
    return h.value


def vecchia_plan_from_cov_censored(Sigma: np.ndarray, m: int, n_observed: int, nbr=None, stream=None) -> int:
    Sigma = np.ascontiguousarray(Sigma, dtype=np.float64)
    D = Sigma.shape[0]
    nb = _nbr_table(nbr, D, m)
    h = c_void_p()
    _check(lib().vecchia_plan_from_cov_censored(Sigma.ctypes.data, D, None if nb is None else nb.ctypes.data,
                                                int(m), int(n_observed), _stream_ptr(stream), byref(h)))
    return h.value


def vecchia_plan_censoring(plan: int) -> int:
    n = c_int64()
    _check(lib().vecchia_plan_censoring(plan, byref(n)))
    return n.value


def vecchia_replan(plan: int, locs: np.ndarray, ordering: int, perm=None, stream=None) -> None:
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    pin = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    _check(lib().vecchia_replan(plan, locs.ctypes.data, int(ordering),
                                None if pin is None else pin.ctypes.data, _stream_ptr(stream)))


def vecchia_plan_info(plan: int):
    D = c_int64()
    m = c_int32()
    _check(lib().vecchia_plan_info(plan, byref(D), byref(m)))
    return D.value, m.value


def vecchia_plan_neighbours(plan: int):
    D, m = vecchia_plan_info(plan)
    perm = np.empty(D, dtype=np.int64)
    nbr = np.empty((D, max(m, 1)), dtype=np.int32)
    _check(lib().vecchia_plan_neighbours(plan, perm.ctypes.data, nbr.ctypes.data if m > 0 else None))
    return perm, nbr[:, :m]


def plan_n_terms(plan: int) -> int:
    """Terms of a plan: D, or the number of joint terms of a block plan."""
    D, _ = vecchia_plan_info(plan)
    n = c_int64()
    if lib().vecchia_plan_block_terms(plan, byref(n), None, None, None) == VECCHIA_OK:
        return n.value
    return D


def vecchia_logcdf(plan: int, x, qmc, out, scale: float = 1.0, cov_override=None, terms=None,
                   stream=None) -> None:
    D, _ = vecchia_plan_info(plan)
    q = as_qmc(qmc)
    c = as_cov(cov_override)
    _check(lib().vecchia_logcdf(plan, _dev_ptr(x, D, "x"), float(scale),
                                None if c is None else ctypes.addressof(c), byref(q),
                                _dev_ptr(out, 2, "out"),
                                None if terms is None else _dev_ptr(terms, 2 * plan_n_terms(plan), "terms"),
                                _stream_ptr(stream)))


def vecchia_logcdf_noalloc(plan: int, x, qmc, out, scale: float = 1.0, cov_override=None, terms=None,
                           stream=None) -> None:
    """vecchia_logcdf on the library's static per-GPU scratch array (no allocation)."""
    D, _ = vecchia_plan_info(plan)
    q = as_qmc(qmc)
    c = as_cov(cov_override)
    _check(lib().vecchia_logcdf_noalloc(plan, _dev_ptr(x, D, "x"), float(scale),
                                        None if c is None else ctypes.addressof(c), byref(q),
                                        _dev_ptr(out, 2, "out"),
                                        None if terms is None else _dev_ptr(terms, 2 * plan_n_terms(plan), "terms"),
                                        _stream_ptr(stream)))


def vecchia_plan_status(plan: int) -> int:
    bad = c_int64(-1)
    st = lib().vecchia_plan_status(plan, byref(bad))
    if st not in (VECCHIA_OK, 3):
        _check(st)
    return bad.value


def vecchia_plan_destroy(plan: int) -> None:
    _check(lib().vecchia_plan_destroy(plan))


def vecchia_batch_create(plans, qmcs) -> int:
    n = len(plans)
    arr = (c_void_p * n)(*plans)
    qa = (vecchia_qmc * n)(*[as_qmc(q) for q in qmcs])
    h = c_void_p()
    _check(lib().vecchia_batch_create(ctypes.addressof(arr), n, ctypes.addressof(qa), byref(h)))
    return h.value


def vecchia_batch_logcdf(batch: int, x, out, scales=None, covs=None, stream=None) -> None:
    sc = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
    ca = None if covs is None else (vecchia_cov * len(covs))(*[as_cov(c) for c in covs])
    _check(lib().vecchia_batch_logcdf(batch, _dev_ptr(x, None, "x"),
                                      None if sc is None else sc.ctypes.data,
                                      None if ca is None else ctypes.addressof(ca),
                                      _dev_ptr(out, None, "out"), _stream_ptr(stream)))


def vecchia_batch_status(batch: int, n: int) -> np.ndarray:
    bad = np.empty(n, dtype=np.int64)
    st = lib().vecchia_batch_status(batch, bad.ctypes.data)
    if st not in (VECCHIA_OK, 3):
        _check(st)
    return bad


def vecchia_batch_destroy(batch: int) -> None:
    _check(lib().vecchia_batch_destroy(batch))


def vecchia_server_create(hbm_budget_bytes: int, max_slots: int) -> int:
    h = c_void_p()
    _check(lib().vecchia_server_create(int(hbm_budget_bytes), int(max_slots), byref(h)))
    return h.value


def vecchia_submit(server: int, plan: int, x, qmc, scale: float = 1.0, cov_override=None) -> int:
    D, _ = vecchia_plan_info(plan)
    q = as_qmc(qmc)
    c = as_cov(cov_override)
    t = c_uint64()
    _check(lib().vecchia_submit(server, plan, _dev_ptr(x, D, "x"), float(scale),
                                None if c is None else ctypes.addressof(c), byref(q), byref(t)))
    return t.value


def vecchia_poll(server: int, ticket: int):
    """Returns None while running, else (logF, se, latency_s)."""
    lf, se, lat = c_double(), c_double(), c_double()
    done = c_int32()
    _check(lib().vecchia_poll(server, ticket, byref(lf), byref(se), byref(done), byref(lat)))
    return (lf.value, se.value, lat.value) if done.value else None


def vecchia_server_destroy(server: int) -> None:
    _check(lib().vecchia_server_destroy(server))


def vecchia_profile_enable(on: int) -> None:
    _check(lib().vecchia_profile_enable(int(on)))


def vecchia_profile_read(K: int, precision: int):
    """(total_ms, launches, sov_steps) of the recorded QMC launches of size K."""
    ms, nl, st = c_double(), c_int64(), c_int64()
    _check(lib().vecchia_profile_read(int(K), int(precision), byref(ms), byref(nl), byref(st)))
    return ms.value, nl.value, st.value


def vecchia_profile_reset() -> None:
    _check(lib().vecchia_profile_reset())


def vecchia_autotune(precision: int, n_points: int, n_shifts: int, ms, stream=None):
    """Tune the chunk size for each K in ms; returns (chunks, median_ms) lists."""
    ms = [int(v) for v in ms]
    arr = (c_int32 * max(1, len(ms)))(*ms)
    chunks = (c_int32 * max(1, len(ms)))()
    t = (ctypes.c_float * max(1, len(ms)))()
    _check(lib().vecchia_autotune(int(precision), int(n_points), int(n_shifts), ctypes.cast(arr, c_void_p),
                                  len(ms), _stream_ptr(stream), ctypes.cast(chunks, c_void_p),
                                  ctypes.cast(t, c_void_p)))
    return list(chunks)[:len(ms)], list(t)[:len(ms)]


def vecchia_tuning_get(precision: int, m: int) -> int:
    v = c_int32()
    _check(lib().vecchia_tuning_get(int(precision), int(m), byref(v)))
    return v.value


def vecchia_tuning_set(precision: int, m: int, chunk_points: int) -> None:
    _check(lib().vecchia_tuning_set(int(precision), int(m), int(chunk_points)))


def vecchia_calibrate_valu(stream=None) -> dict:
    """Measured wave64 instructions per CU per ns: fma, exp, log, rcp, sqrt."""
    r = (c_double * 5)()
    _check(lib().vecchia_calibrate_valu(_stream_ptr(stream), ctypes.cast(r, c_void_p)))
    return dict(zip(("fma", "exp", "log", "rcp", "sqrt"), list(r)))


VECCHIA_PROBE_PHI_F32, VECCHIA_PROBE_NINV_F32, VECCHIA_PROBE_NINV_LOG2_F32 = 0, 1, 2
VECCHIA_PROBE_PHI_F64, VECCHIA_PROBE_NINV_F64 = 3, 4


def vecchia_probe_math(what: int, x, out, stream=None) -> None:
    """Device normal CDF / quantile pieces at x (float64 CUDA tensor); out: n x 3."""
    n = x.numel()
    _check(lib().vecchia_probe_math(int(what), n, _dev_ptr(x, n, "x"), _dev_ptr(out, 3 * n, "out"),
                                    _stream_ptr(stream)))


def vecchia_probe_lattice(seed: int, term: int, shift: int, dim: int, second: bool, n: int, w64=None, w32=None,
                          stream=None) -> None:
    """Lattice coordinates p = 1..n as the kernels form them (FP64 into w64, FP32 into w32)."""
    import torch
    p64 = None if w64 is None else _dev_ptr(w64, n, "w64")
    p32 = None
    if w32 is not None:
        if not (isinstance(w32, torch.Tensor) and w32.is_cuda and w32.dtype == torch.float32 and
                w32.is_contiguous() and w32.numel() >= n):
            raise ValueError("w32 must be a contiguous float32 CUDA tensor of n values")
        p32 = w32.data_ptr()
    _check(lib().vecchia_probe_lattice(int(seed) & (2 ** 64 - 1), int(term), int(shift), int(dim),
                                       1 if second else 0, int(n), p64, p32, _stream_ptr(stream)))


MIX_SEARCH_NODES = 24


def make_mixture(beta: float = 0.0, gamma: float = 2.0, n_nodes: int = 48) -> vecchia_mixture:
    return vecchia_mixture(float(beta), float(gamma), int(n_nodes), 0)


def vecchia_mixture_search(mix: vecchia_mixture):
    """Scales of the first (search) pass (host only)."""
    sc = np.empty(MIX_SEARCH_NODES, dtype=np.float64)
    _check(lib().vecchia_mixture_search(byref(mix), sc.ctypes.data))
    return sc


def vecchia_mixture_rule(mix: vecchia_mixture, search_logh):
    """(window, v, scales, log weights) of the second-pass rule for given search
    values log h(v_j) (host only)."""
    h = np.ascontiguousarray(search_logh, dtype=np.float64)
    if h.shape != (MIX_SEARCH_NODES,):
        raise ValueError(f"need {MIX_SEARCH_NODES} search values")
    n = max(1, int(mix.n_nodes))
    win = np.empty(2, dtype=np.float64)
    v = np.empty(n, dtype=np.float64)
    sc = np.empty(n, dtype=np.float64)
    lw = np.empty(n, dtype=np.float64)
    _check(lib().vecchia_mixture_rule(byref(mix), h.ctypes.data, win.ctypes.data, v.ctypes.data, sc.ctypes.data,
                                      lw.ctypes.data))
    n = int(mix.n_nodes)
    return (float(win[0]), float(win[1])), v[:n], sc[:n], lw[:n]


def vecchia_mixture_logcdf(plan: int, x, mix: vecchia_mixture, qmc, out, nodes=None, cov_override=None,
                           stream=None) -> None:
    D, _ = vecchia_plan_info(plan)
    q = as_qmc(qmc)
    c = as_cov(cov_override)
    _check(lib().vecchia_mixture_logcdf(plan, _dev_ptr(x, D, "x"), byref(mix),
                                        None if c is None else ctypes.addressof(c), byref(q),
                                        _dev_ptr(out, 2, "out"),
                                        None if nodes is None else _dev_ptr(nodes, 2 * int(mix.n_nodes), "nodes"),
                                        _stream_ptr(stream)))


def vecchia_mixbatch_create(plans, n_nodes: int, qmc) -> int:
    n = len(plans)
    arr = (c_void_p * n)(*plans)
    q = as_qmc(qmc)
    h = c_void_p()
    _check(lib().vecchia_mixbatch_create(ctypes.addressof(arr), n, int(n_nodes), byref(q), byref(h)))
    return h.value


def vecchia_mixbatch_logcdf(mb: int, x, mix: vecchia_mixture, out, total=None, cov_override=None,
                            stream=None) -> None:
    c = as_cov(cov_override)
    _check(lib().vecchia_mixbatch_logcdf(mb, _dev_ptr(x, None, "x"), byref(mix),
                                         None if c is None else ctypes.addressof(c), _dev_ptr(out, None, "out"),
                                         None if total is None else _dev_ptr(total, 2, "total"),
                                         _stream_ptr(stream)))


def vecchia_mixbatch_status(mb: int, n: int):
    bad = np.empty(n, dtype=np.int64)
    st = lib().vecchia_mixbatch_status(mb, bad.ctypes.data)
    if st not in (VECCHIA_OK, 3):
        _check(st)
    return bad


def vecchia_mixbatch_destroy(mb: int) -> None:
    _check(lib().vecchia_mixbatch_destroy(mb))


def vecchia_map_anisotropic(locs: np.ndarray, phi: float, A: float) -> np.ndarray:
    """Coordinates whose Euclidean distances are Section 4.1's anisotropic distances."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    out = np.empty_like(locs)
    _check(lib().vecchia_map_anisotropic(locs.ctypes.data, locs.shape[0], float(phi), float(A), out.ctypes.data))
    return out


def vecchia_plan_block(locs: np.ndarray, ordering: int, m: int, p: int, cov, perm=None, stream=None) -> int:
    """Joint block plan: groups of p consecutive plan positions (Section 3.2)."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    if locs.ndim != 2:
        raise ValueError("locs must be D x dim")
    pin = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    h = c_void_p()
    c = as_cov(cov)
    _check(lib().vecchia_plan_block(locs.ctypes.data, locs.shape[0], locs.shape[1], int(ordering),
                                    None if pin is None else pin.ctypes.data, int(m), int(p), byref(c),
                                    _stream_ptr(stream), byref(h)))
    return h.value


def vecchia_plan_block_terms(plan: int):
    """(var_off, vars, split) of a block plan."""
    n = c_int64()
    _check(lib().vecchia_plan_block_terms(plan, byref(n), None, None, None))
    off = np.empty(n.value + 1, dtype=np.int32)
    split = np.empty(n.value, dtype=np.int32)
    _check(lib().vecchia_plan_block_terms(plan, byref(n), off.ctypes.data, None, split.ctypes.data))
    var = np.empty(max(1, int(off[-1])), dtype=np.int32)
    _check(lib().vecchia_plan_block_terms(plan, byref(n), None, var.ctypes.data, None))
    return off, var[:int(off[-1])], split


def vecchia_plan_from_cov_block(Sigma: np.ndarray, terms, stream=None) -> int:
    """terms: list of (variables, split) pairs over an explicit covariance."""
    Sigma = np.ascontiguousarray(Sigma, dtype=np.float64)
    off = np.zeros(len(terms) + 1, dtype=np.int32)
    for g, (v, _) in enumerate(terms):
        off[g + 1] = off[g] + len(v)
    var = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.int32) for v, _ in terms]), dtype=np.int32)
    split = np.array([sp for _, sp in terms], dtype=np.int32)
    h = c_void_p()
    _check(lib().vecchia_plan_from_cov_block(Sigma.ctypes.data, Sigma.shape[0], off.ctypes.data, var.ctypes.data,
                                             split.ctypes.data, len(terms), _stream_ptr(stream), byref(h)))
    return h.value


def vecchia_full_logcdf(plan: int, x, qmc, out, scale: float = 1.0, cov_override=None, stream=None) -> None:
    """Full-dimension SOV log Phi_D(x / scale) on the plan's ordering (FP64)."""
    D, _ = vecchia_plan_info(plan)
    q = as_qmc(qmc)
    c = as_cov(cov_override)
    _check(lib().vecchia_full_logcdf(plan, _dev_ptr(x, D, "x"), float(scale),
                                     None if c is None else ctypes.addressof(c), byref(q),
                                     _dev_ptr(out, 2, "out"), _stream_ptr(stream)))

