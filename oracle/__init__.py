"""ctypes front end of the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  It shares no code with the HIP library and
the product path never imports it.

Every function mirrors one step of the method of Honkonen & Honkonen
(arXiv:1803.07560); the C source names the section or equation each follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class Lattice(C.Structure):
    """Parameters of Eq. Gen2: nx space sites (M), nt time slices (L), nu, D, a, tau,
    plus the test knobs g (nonlinear coupling, 1 in the paper) and m2 (mass term, 0),
    the observable behind C(r): 0 anchored at the first site, 1 averaged over
    all anchors, and antithetic: 1 makes every sample index a pair of points (the
    point of its words and of the complemented words) whose means the records sum."""

    _fields_ = [("nx", C.c_int32), ("nt", C.c_int32), ("nu", C.c_double), ("D", C.c_double),
                ("a", C.c_double), ("tau", C.c_double), ("g", C.c_double), ("m2", C.c_double),
                ("observable", C.c_int32), ("antithetic", C.c_int32)]

    @property
    def d(self) -> int:
        return int(self.nx) * int(self.nt)


OBS_ANCHOR, OBS_AVERAGED = 0, 1


def lattice(nx, nt, nu=1.0, D=1.0, a=1.0, tau=1.0, g=1.0, m2=0.0, observable=0,
            antithetic=0) -> Lattice:
    return Lattice(int(nx), int(nt), float(nu), float(D), float(a), float(tau), float(g), float(m2),
                   int(observable), int(antithetic))


def sums_len(nx: int) -> int:
    return 3 + 3 * nx


def result_len(nx: int) -> int:
    return 5 + 2 * nx


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = C.CDLL(_LIB_PATH)
        u32p, u64p, dp = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_double)
        latp = C.POINTER(Lattice)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_words.argtypes = [C.c_int32, C.c_uint64, C.c_uint64, C.c_uint64, u32p]
        L.oracle_words.restype = None
        L.oracle_point.argtypes = [C.c_int32, C.c_uint64, C.c_uint64, dp, dp, C.c_uint64, dp]
        L.oracle_point.restype = None
        L.oracle_residual.argtypes = [latp, dp, dp]
        L.oracle_residual.restype = C.c_int
        L.oracle_action.argtypes = [latp, dp]
        L.oracle_action.restype = C.c_double
        L.oracle_action_batch.argtypes = [latp, C.c_size_t, dp, dp]
        L.oracle_action_batch.restype = C.c_int
        L.oracle_observable.argtypes = [latp, dp, dp]
        L.oracle_observable.restype = C.c_int
        for name in ("oracle_sums", "oracle_split_sums", "oracle_sums_l1", "oracle_sums_shifted",
                     "oracle_sums_shifted_l1"):
            f = getattr(L, name)
            f.argtypes = [latp, C.c_uint64, C.c_size_t, u64p, dp, dp, u64p, u64p, dp, C.c_int32]
            f.restype = C.c_int
        for name in ("oracle_finalize", "oracle_finalize_shifted"):
            f = getattr(L, name)
            f.argtypes = [C.c_int32, C.c_int32, C.c_size_t, dp, dp, dp, dp]
            f.restype = C.c_int
        L.oracle_plan_uniform.argtypes = [C.c_int32, dp, dp, C.c_int32, u64p, dp, dp]
        L.oracle_plan_uniform.restype = C.c_int
        L.oracle_nsphere.argtypes = [C.c_int32, C.c_uint64, C.c_uint64, dp, dp, C.c_uint64, dp]
        L.oracle_nsphere.restype = C.c_int
        i32p = C.POINTER(C.c_int32)
        L.oracle_is_basis.argtypes = [C.c_int32, C.c_int32, dp]
        L.oracle_is_basis.restype = C.c_int
        L.oracle_is_modes.argtypes = [latp, dp, dp, dp, i32p, dp, dp]
        L.oracle_is_modes.restype = C.c_int
        L.oracle_is_point.argtypes = [latp, dp, dp, C.c_uint64, C.c_uint64, C.c_uint64, dp, dp]
        L.oracle_is_point.restype = C.c_int
        L.oracle_is_sums.argtypes = [latp, C.c_uint64, dp, dp, C.c_double, C.c_size_t, u64p, u64p,
                                     u64p, dp, C.c_int32]
        L.oracle_is_sums.restype = C.c_int
        L.oracle_sph_volume.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.oracle_sph_volume.restype = C.c_double
        L.oracle_sph_point.argtypes = [C.c_int32, C.c_uint64, C.c_uint64, C.c_double, C.c_double,
                                       C.c_uint64, dp]
        L.oracle_sph_point.restype = C.c_int
        L.oracle_sph_sums.argtypes = [latp, C.c_uint64, C.c_double, C.c_size_t, u64p, dp, dp,
                                      u64p, u64p, dp]
        L.oracle_sph_sums.restype = C.c_int
        _lib = L
    return _lib


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def words(d: int, seed: int, sub_id: int, index: int) -> np.ndarray:
    out = np.zeros(d, dtype=np.uint32)
    lib().oracle_words(d, seed, sub_id, index, _ptr(out, C.c_uint32))
    return out


def point(d: int, seed: int, sub_id: int, lo, hi, index: int) -> np.ndarray:
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    out = np.zeros(d, dtype=np.float64)
    lib().oracle_point(d, seed, sub_id, _ptr(lo, C.c_double), _ptr(hi, C.c_double), index,
                       _ptr(out, C.c_double))
    return out


def points(d: int, seed: int, sub_id: int, lo, hi, indices) -> np.ndarray:
    return np.stack([point(d, seed, sub_id, lo, hi, int(i)) for i in indices])


def residual(lat: Lattice, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(lat.d, dtype=np.float64)
    if lib().oracle_residual(C.byref(lat), _ptr(u, C.c_double), _ptr(out, C.c_double)) != 0:
        raise ValueError("oracle_residual: invalid arguments")
    return out


def action(lat: Lattice, u) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    return float(lib().oracle_action(C.byref(lat), _ptr(u, C.c_double)))


def observable(lat: Lattice, u) -> np.ndarray:
    """p_r, r = 0 .. nx-1, of one configuration (anchored or averaged per lat.observable)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(lat.nx, dtype=np.float64)
    if lib().oracle_observable(C.byref(lat), _ptr(u, C.c_double), _ptr(out, C.c_double)) != 0:
        raise ValueError("oracle_observable: invalid arguments")
    return out


def action_batch(lat: Lattice, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, lat.d)
    out = np.zeros(u.shape[0], dtype=np.float64)
    if lib().oracle_action_batch(C.byref(lat), u.shape[0], _ptr(u, C.c_double),
                                 _ptr(out, C.c_double)) != 0:
        raise ValueError("oracle_action_batch: invalid arguments")
    return out


def _subvol_args(lat, ids, lo, hi, n, offset):
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    ns = ids.shape[0]
    lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(ns, lat.d)
    hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(ns, lat.d)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, dtype=np.uint64), (ns,)))
    offset = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, dtype=np.uint64), (ns,)))
    return ids, lo, hi, n, offset


def sums(lat: Lattice, seed: int, ids, lo, hi, n, offset=0, nthreads: int | None = None):
    """Per-subvolume sums records (nsub x (3 + 3 nx))."""
    ids, lo, hi, n, offset = _subvol_args(lat, ids, lo, hi, n, offset)
    out = np.zeros((ids.shape[0], sums_len(lat.nx)), dtype=np.float64)
    nt = nthreads or os.cpu_count() or 1
    rc = lib().oracle_sums(C.byref(lat), seed, ids.shape[0], _ptr(ids, C.c_uint64),
                           _ptr(lo, C.c_double), _ptr(hi, C.c_double), _ptr(n, C.c_uint64),
                           _ptr(offset, C.c_uint64), _ptr(out, C.c_double), nt)
    if rc != 0:
        raise ValueError(f"oracle_sums failed ({rc})")
    return out


def _sums_call(name, width, lat, seed, ids, lo, hi, n, offset, nthreads):
    ids, lo, hi, n, offset = _subvol_args(lat, ids, lo, hi, n, offset)
    out = np.zeros((ids.shape[0], width), dtype=np.float64)
    nt = nthreads or os.cpu_count() or 1
    rc = getattr(lib(), name)(C.byref(lat), seed, ids.shape[0], _ptr(ids, C.c_uint64),
                              _ptr(lo, C.c_double), _ptr(hi, C.c_double), _ptr(n, C.c_uint64),
                              _ptr(offset, C.c_uint64), _ptr(out, C.c_double), nt)
    if rc != 0:
        raise ValueError(f"{name} failed ({rc})")
    return out


def sums_l1(lat: Lattice, seed: int, ids, lo, hi, n, offset=0, nthreads: int | None = None):
    """Sums records with nx more fields, sum |p_r w| per r (nsub x (3 + 4 nx))."""
    return _sums_call("oracle_sums_l1", sums_len(lat.nx) + lat.nx, lat, seed, ids, lo, hi, n,
                      offset, nthreads)


def sums_shifted(lat: Lattice, seed: int, ids, lo, hi, n, offset=0,
                 nthreads: int | None = None):
    """Shifted records [n, sigma, sum w, ...] with w = exp(sigma - S), sigma the
    smallest action of the subvolume's samples (nsub x (4 + 3 nx))."""
    return _sums_call("oracle_sums_shifted", sums_len(lat.nx) + 1, lat, seed, ids, lo, hi, n,
                      offset, nthreads)


def sums_shifted_l1(lat: Lattice, seed: int, ids, lo, hi, n, offset=0,
                    nthreads: int | None = None):
    """Shifted records with nx more fields, sum |p_r w| of the shifted weights
    (nsub x (4 + 4 nx))."""
    return _sums_call("oracle_sums_shifted_l1", sums_len(lat.nx) + 1 + lat.nx, lat, seed, ids, lo,
                      hi, n, offset, nthreads)


def split_sums(lat: Lattice, seed: int, ids, lo, hi, n, offset=0, nthreads: int | None = None):
    """Upper-half sums of w and w^2 per dimension (nsub x 2d)."""
    ids, lo, hi, n, offset = _subvol_args(lat, ids, lo, hi, n, offset)
    out = np.zeros((ids.shape[0], 2 * lat.d), dtype=np.float64)
    nt = nthreads or os.cpu_count() or 1
    rc = lib().oracle_split_sums(C.byref(lat), seed, ids.shape[0], _ptr(ids, C.c_uint64),
                                 _ptr(lo, C.c_double), _ptr(hi, C.c_double), _ptr(n, C.c_uint64),
                                 _ptr(offset, C.c_uint64), _ptr(out, C.c_double), nt)
    if rc != 0:
        raise ValueError(f"oracle_split_sums failed ({rc})")
    return out


def finalize(nx: int, d: int, lo, hi, sums_records, evals_per_sample: int = 1) -> dict:
    """Z, C(r) and their errors; n_evals counts evals_per_sample integrand
    evaluations per record sample (2 for antithetic pairs)."""
    s = np.ascontiguousarray(sums_records, dtype=np.float64).reshape(-1, sums_len(nx))
    ns = s.shape[0]
    lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(ns, d)
    hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(ns, d)
    out = np.zeros(result_len(nx), dtype=np.float64)
    rc = lib().oracle_finalize(nx, d, ns, _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                               _ptr(s, C.c_double), _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError(f"oracle_finalize failed ({rc})")
    return {"Z": out[0], "Z_err": out[1], "log_Z": out[2], "ess": out[3],
            "n_evals": out[4] * evals_per_sample,
            "C": out[5:5 + nx].copy(), "C_err": out[5 + nx:5 + 2 * nx].copy()}


def finalize_shifted(nx: int, d: int, lo, hi, shifted_records, evals_per_sample: int = 1) -> dict:
    """finalize over shifted records: log_Z stays finite where Z underflows."""
    s = np.ascontiguousarray(shifted_records, dtype=np.float64).reshape(-1, sums_len(nx) + 1)
    ns = s.shape[0]
    lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(ns, d)
    hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(ns, d)
    out = np.zeros(result_len(nx), dtype=np.float64)
    rc = lib().oracle_finalize_shifted(nx, d, ns, _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                                       _ptr(s, C.c_double), _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError(f"oracle_finalize_shifted failed ({rc})")
    return {"Z": out[0], "Z_err": out[1], "log_Z": out[2], "ess": out[3],
            "n_evals": out[4] * evals_per_sample,
            "C": out[5:5 + nx].copy(), "C_err": out[5 + nx:5 + 2 * nx].copy()}


def plan_uniform(d: int, box_lo, box_hi, k: int):
    box_lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, dtype=np.float64), (d,)))
    box_hi = np.ascontiguousarray(np.broadcast_to(np.asarray(box_hi, dtype=np.float64), (d,)))
    cnt = 1 << k
    ids = np.zeros(cnt, dtype=np.uint64)
    lo = np.zeros((cnt, d), dtype=np.float64)
    hi = np.zeros((cnt, d), dtype=np.float64)
    if lib().oracle_plan_uniform(d, _ptr(box_lo, C.c_double), _ptr(box_hi, C.c_double), k,
                                 _ptr(ids, C.c_uint64), _ptr(lo, C.c_double),
                                 _ptr(hi, C.c_double)) != 0:
        raise ValueError("oracle_plan_uniform: invalid arguments")
    return ids, lo, hi


def budget_split(budget: int, count: int) -> np.ndarray:
    """Samples per subvolume for a total budget over `count` subvolumes in id order:
    floor(B/count) each, plus one for the first B mod count."""
    base, extra = divmod(int(budget), int(count))
    n = np.full(count, base, dtype=np.uint64)
    n[:extra] += 1
    return n


def integrate_uniform(lat: Lattice, seed: int, box_lo, box_hi, k: int, budget: int,
                      nthreads: int | None = None) -> dict:
    """Oracle of the uniform-split convenience entry: plan, sums, finalize.  The
    budget counts integrand evaluations: with antithetic pairs, budget // 2 pairs
    are split over the subvolumes."""
    ids, lo, hi = plan_uniform(lat.d, box_lo, box_hi, k)
    per = 2 if lat.antithetic else 1
    n = budget_split(budget // per, len(ids))
    s = sums(lat, seed, ids, lo, hi, n, 0, nthreads)
    res = finalize(lat.nx, lat.d, lo, hi, s, per)
    res["sums"] = s
    return res


def nsphere(dim: int, seed: int, lo, hi, n: int, sub_id: int = 1) -> dict:
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, dtype=np.float64), (dim,)))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, dtype=np.float64), (dim,)))
    out = np.zeros(5, dtype=np.float64)
    if lib().oracle_nsphere(dim, seed, sub_id, _ptr(lo, C.c_double), _ptr(hi, C.c_double), n,
                            _ptr(out, C.c_double)) != 0:
        raise ValueError("oracle_nsphere: invalid arguments")
    return {"n": out[0], "sum_f": out[1], "sum_f2": out[2], "result": out[3], "abserr": out[4]}


# ------------------------------------------------ Gaussian-proposal sampling

def _is_box(d, lo, hi):
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, dtype=np.float64), (d,)))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, dtype=np.float64), (d,)))
    return lo, hi


def is_basis(nx: int, nt: int) -> np.ndarray:
    """d x d orthonormal real Fourier basis (rows: lattice variables, columns: modes)."""
    E = np.zeros((nx * nt, nx * nt))
    if lib().oracle_is_basis(nx, nt, _ptr(E, C.c_double)) != 0:
        raise ValueError("oracle_is_basis: invalid arguments")
    return E


def is_modes(lat: Lattice, lo, hi) -> dict:
    d = lat.d
    lo, hi = _is_box(d, lo, hi)
    lam, scale = np.zeros(d), np.zeros(d)
    uni = np.zeros(d, dtype=np.int32)
    lk = C.c_double()
    if lib().oracle_is_modes(C.byref(lat), _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                             _ptr(lam, C.c_double), _ptr(uni, C.c_int32),
                             _ptr(scale, C.c_double), C.byref(lk)) != 0:
        raise ValueError("oracle_is_modes: invalid arguments")
    return {"lambda": lam, "uniform": uni.astype(bool), "scale": scale, "log_k": lk.value}


def is_point(lat: Lattice, lo, hi, seed: int, stream: int, index: int):
    """(u, sum z^2/2) of one sample of the Gaussian proposal."""
    d = lat.d
    lo, hi = _is_box(d, lo, hi)
    u = np.zeros(d)
    hz = C.c_double()
    if lib().oracle_is_point(C.byref(lat), _ptr(lo, C.c_double), _ptr(hi, C.c_double), seed,
                             stream, index, _ptr(u, C.c_double), C.byref(hz)) != 0:
        raise ValueError("oracle_is_point: invalid arguments")
    return u, hz.value


IS_UNIFORM_STREAM = 1 << 63


def is_sums(lat: Lattice, seed: int, lo, hi, ids, n, offset=0, gaussian_fraction=0.9,
            nthreads: int | None = None):
    """Per-stream sums records of the mixture weight W/K (streams with bit 63 of
    the id set draw from the box's uniform density, the others from the Gaussian)."""
    d = lat.d
    lo, hi = _is_box(d, lo, hi)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, dtype=np.uint64), ids.shape))
    offset = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, dtype=np.uint64), ids.shape))
    out = np.zeros((ids.shape[0], sums_len(lat.nx)))
    nt = nthreads or os.cpu_count() or 1
    if lib().oracle_is_sums(C.byref(lat), seed, _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                            float(gaussian_fraction), ids.shape[0], _ptr(ids, C.c_uint64),
                            _ptr(n, C.c_uint64),
                            _ptr(offset, C.c_uint64), _ptr(out, C.c_double), nt) != 0:
        raise ValueError("oracle_is_sums: invalid arguments")
    return out


def is_plan(budget: int, n_streams: int, gaussian_fraction: float):
    """Streams and sample counts of one run: round(alpha * budget) samples over
    Gaussian streams 1..n_streams and the rest over uniform streams
    2^63 + 1 .. 2^63 + n_streams, each share split as budget_split does
    (a component with no samples has no streams)."""
    n_g = int(round(gaussian_fraction * budget))
    ids, n = [], []
    for base, total in ((0, n_g), (IS_UNIFORM_STREAM, budget - n_g)):
        if total == 0:
            continue
        ids += [base + 1 + i for i in range(n_streams)]
        n += list(budget_split(total, n_streams))
    return np.array(ids, dtype=np.uint64), np.array(n, dtype=np.uint64)


def integrate_is(lat: Lattice, seed: int, lo, hi, n_streams: int, budget: int,
                 gaussian_fraction: float = 0.9, nthreads: int | None = None) -> dict:
    """Z and C(r) by the defensive Gaussian-proposal sampler: Z = K sum W/K / N
    over all N = budget samples, i.e. finalize with 'volumes' K n_s / N (each
    stream's mean weighted by its share of the samples; the two components
    count as strata of the variance)."""
    m = is_modes(lat, lo, hi)
    ids, n = is_plan(budget, n_streams, gaussian_fraction)
    s = is_sums(lat, seed, lo, hi, ids, n, 0, gaussian_fraction, nthreads)
    d = lat.d
    vlo = np.zeros((len(ids), d))
    vhi = np.ones((len(ids), d))
    vhi[:, 0] = np.exp(m["log_k"]) * n / float(budget)
    res = finalize(lat.nx, d, vlo, vhi, s)
    res["sums"] = s
    res["log_k"] = m["log_k"]
    return res


# ------------------------------------------------ spherical coordinates

def sph_volume(d: int, rho_lo: float, rho_hi: float) -> float:
    v = lib().oracle_sph_volume(d, float(rho_lo), float(rho_hi))
    if v < 0:
        raise ValueError("oracle_sph_volume: invalid arguments")
    return v


def sph_point(d: int, seed: int, stream: int, rho_lo: float, rho_hi: float, index: int):
    u = np.zeros(d)
    if lib().oracle_sph_point(d, seed, stream, float(rho_lo), float(rho_hi), index,
                              _ptr(u, C.c_double)) != 0:
        raise ValueError("oracle_sph_point: invalid arguments")
    return u


def sph_sums(lat: Lattice, seed: int, box: float, ids, rho_lo, rho_hi, n, offset=0):
    """Per-shell sums records of exp(-S) inside the cube [-box, box]^d."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    m = ids.shape[0]
    rl = np.ascontiguousarray(np.broadcast_to(np.asarray(rho_lo, dtype=np.float64), (m,)))
    rh = np.ascontiguousarray(np.broadcast_to(np.asarray(rho_hi, dtype=np.float64), (m,)))
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, dtype=np.uint64), (m,)))
    offset = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, dtype=np.uint64), (m,)))
    out = np.zeros((m, sums_len(lat.nx)))
    if lib().oracle_sph_sums(C.byref(lat), seed, float(box), m, _ptr(ids, C.c_uint64),
                             _ptr(rl, C.c_double), _ptr(rh, C.c_double), _ptr(n, C.c_uint64),
                             _ptr(offset, C.c_uint64), _ptr(out, C.c_double)) != 0:
        raise ValueError("oracle_sph_sums: invalid arguments")
    return out


def sph_finalize(nx: int, d: int, rho_lo, rho_hi, sums_records) -> dict:
    """finalize with shell volumes: each shell is passed as a 1-D 'box' of
    length V (the finalize multiplies extents), padded with unit extents."""
    rl, rh = np.atleast_1d(rho_lo), np.atleast_1d(rho_hi)
    vol = np.array([sph_volume(d, a, b) for a, b in zip(rl, rh)])
    lo = np.zeros((len(vol), d))
    hi = np.ones((len(vol), d))
    hi[:, 0] = vol
    return finalize(nx, d, lo, hi, sums_records)
