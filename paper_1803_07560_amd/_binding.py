"""ctypes binding of ``libbfi.so`` (declared in ``include/bfi.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  There is no fallback -- if the library is missing, loading raises.
Functions carry the names of the C entry points.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BFI_LIBRARY may name another build of the same ABI (e.g. an installed copy)
LIB_PATH = os.environ.get("BFI_LIBRARY") or os.path.join(_HERE, "libbfi.so")

BFI_FP64 = 0
BFI_FP32_SHIFTED = 1
BFI_FP64_SHIFTED = 2
BFI_OBS_ANCHOR = 0
BFI_OBS_AVERAGED = 1
PRECISIONS = {"fp64": BFI_FP64, "fp32": BFI_FP32_SHIFTED, "fp64s": BFI_FP64_SHIFTED,
              BFI_FP64: BFI_FP64, BFI_FP32_SHIFTED: BFI_FP32_SHIFTED,
              BFI_FP64_SHIFTED: BFI_FP64_SHIFTED}

STATUS = {0: "BFI_OK", -1: "BFI_EINVAL", -2: "BFI_ENOMEM", -3: "BFI_EDEVICE",
          -4: "BFI_EUNSUPPORTED", -5: "BFI_EBUSY", -6: "BFI_ECANCELLED", -7: "BFI_EBUDGET",
          -8: "BFI_ENOTFOUND"}
MAX_NX = 64
MAX_D = 64


class BfiError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))
        self.message = message


class bfi_lattice(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nt", C.c_int32), ("nu", C.c_double), ("D", C.c_double),
                ("a", C.c_double), ("tau", C.c_double), ("g", C.c_double), ("m2", C.c_double),
                ("observable", C.c_int32), ("antithetic", C.c_int32)]

    @property
    def d(self) -> int:
        return int(self.nx) * int(self.nt)


class bfi_subvolumes(C.Structure):
    _fields_ = [("count", C.c_size_t), ("id", C.POINTER(C.c_uint64)),
                ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double)),
                ("n", C.POINTER(C.c_uint64)), ("offset", C.POINTER(C.c_uint64))]


class bfi_launch(C.Structure):
    _fields_ = [("samples_per_thread", C.c_int32), ("block", C.c_int32),
                ("persistent", C.c_int32), ("use_graph", C.c_int32)]


class bfi_result(C.Structure):
    _fields_ = [("Z", C.c_double), ("Z_err", C.c_double), ("log_Z", C.c_double),
                ("ess", C.c_double), ("n_evals", C.c_double), ("nx", C.c_int32),
                ("C", C.c_double * MAX_NX), ("C_err", C.c_double * MAX_NX)]

    def to_dict(self) -> dict:
        n = int(self.nx)
        return {"Z": self.Z, "Z_err": self.Z_err, "log_Z": self.log_Z, "ess": self.ess,
                "n_evals": self.n_evals, "C": np.array(self.C[:n]),
                "C_err": np.array(self.C_err[:n])}


class bfi_adaptive_progress(C.Structure):
    _fields_ = [("round", C.c_int32), ("holdout_checks", C.c_int32), ("leaves", C.c_uint64),
                ("evals", C.c_uint64), ("rel_err", C.c_double), ("holdout_rel_err", C.c_double)]


ADAPTIVE_PROGRESS_FN = C.CFUNCTYPE(None, C.POINTER(bfi_adaptive_progress), C.c_void_p)


class bfi_adaptive_config(C.Structure):
    _fields_ = [("target_rel_err", C.c_double), ("max_evals", C.c_uint64),
                ("n_min", C.c_uint64), ("n_max", C.c_uint64), ("split_log2", C.c_int32),
                ("max_rounds", C.c_int32), ("refine_fraction", C.c_double),
                ("round_evals", C.c_uint64), ("min_ess", C.c_double),
                ("split_samples", C.c_uint64), ("holdout", C.c_int32),
                ("progress", ADAPTIVE_PROGRESS_FN), ("progress_user", C.c_void_p)]


class bfi_adaptive_stats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("leaves", C.c_uint64), ("evals", C.c_uint64),
                ("rel_err", C.c_double), ("holdout_checks", C.c_int32),
                ("holdout_used", C.c_int32), ("holdout_seed", C.c_uint64),
                ("holdout_rel_err", C.c_double), ("device_seconds", C.c_double),
                ("graph_instantiations", C.c_int32), ("graph_updates", C.c_int32)]


class bfi_shells(C.Structure):
    _fields_ = [("count", C.c_size_t), ("id", C.POINTER(C.c_uint64)),
                ("rho_lo", C.POINTER(C.c_double)), ("rho_hi", C.POINTER(C.c_double)),
                ("n", C.POINTER(C.c_uint64)), ("offset", C.POINTER(C.c_uint64))]


class bfi_server_config(C.Structure):
    _fields_ = [("memory_budget", C.c_uint64), ("max_requests", C.c_int32),
                ("chunks_per_step", C.c_int32), ("max_pending", C.c_int32),
                ("step_evals", C.c_uint64), ("max_samples_per_thread", C.c_int32)]


class bfi_request(C.Structure):
    _fields_ = [("lat", bfi_lattice), ("prec", C.c_int32), ("seed", C.c_uint64),
                ("box", C.c_double), ("split_log2", C.c_int32), ("budget", C.c_uint64)]


class bfi_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("cancelled", C.c_uint64),
                ("rejected", C.c_uint64), ("steps", C.c_uint64), ("evals", C.c_uint64),
                ("busy_seconds", C.c_double)]


BFI_INTEGRAND_NSPHERE = 0
BFI_INTEGRAND_BURGERS_Z = 1
BFI_INTEGRAND_BURGERS_N = 2


class bfi_integrand(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("lat", bfi_lattice),
                ("prec", C.c_int32), ("distance", C.c_int32)]

    @property
    def d(self) -> int:
        return int(self.dim) if self.kind == BFI_INTEGRAND_NSPHERE else self.lat.d


class bfi_hdi_config(C.Structure):
    _fields_ = [("n_initial", C.c_uint64), ("sample_factor", C.c_double),
                ("rel_diff", C.c_double), ("abs_diff", C.c_double), ("max_abs", C.c_double),
                ("split_log2", C.c_int32), ("max_depth", C.c_int32), ("max_evals", C.c_uint64)]


class bfi_hdi_stats(C.Structure):
    _fields_ = [("evals", C.c_uint64), ("accepted", C.c_uint64), ("unconverged", C.c_uint64),
                ("generations", C.c_int32), ("depth", C.c_int32)]


def partial_len(nx: int) -> int:
    return 4 + 3 * nx


def split_len(d: int) -> int:
    return 1 + 2 * d


_P = C.POINTER
_vp = C.c_void_p
_SIGNATURES = {
    "bfi_status_string": ([C.c_int], C.c_char_p),
    "bfi_last_error": ([], C.c_char_p),
    "bfi_shape_supported": ([C.c_int32, C.c_int32], C.c_int),
    "bfi_supported_shapes": ([_P(C.c_int32), C.c_int32, _P(C.c_int32)], C.c_int),
    "bfi_context_create": ([C.c_int32, _P(_vp)], C.c_int),
    "bfi_context_destroy": ([_vp], C.c_int),
    "bfi_eval": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, _P(bfi_subvolumes), _P(bfi_launch),
                  _P(C.c_double), _P(C.c_double)], C.c_int),
    "bfi_eval_noalloc": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, _P(bfi_subvolumes),
                          _P(bfi_launch), _P(C.c_double), _P(C.c_double)], C.c_int),
    "bfi_plan_create": ([_vp, _P(bfi_lattice), C.c_int, _P(bfi_subvolumes), _P(bfi_launch),
                         _P(_vp)], C.c_int),
    "bfi_plan_run": ([_vp, C.c_uint64, _vp, _vp], C.c_int),
    "bfi_plan_partials": ([_vp, _P(C.c_double)], C.c_int),
    "bfi_plan_info": ([_vp, _P(C.c_uint64), _P(C.c_uint64), _P(bfi_launch)], C.c_int),
    "bfi_plan_kernel_ms": ([_vp, _P(C.c_double)], C.c_int),
    "bfi_plan_destroy": ([_vp], C.c_int),
    "bfi_partials_merge": ([C.c_int32, C.c_size_t, _P(C.c_double), _P(C.c_double)], C.c_int),
    "bfi_finalize": ([_P(bfi_lattice), _P(bfi_subvolumes), _P(C.c_double), _P(bfi_result)],
                     C.c_int),
    "bfi_integrate": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, _P(C.c_double), _P(C.c_double),
                       C.c_int32, C.c_uint64, _P(bfi_launch), _P(bfi_result)], C.c_int),
    "bfi_integrate_adaptive": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, _P(C.c_double),
                                _P(C.c_double), _P(bfi_adaptive_config), _P(bfi_launch),
                                _P(bfi_result), _P(bfi_adaptive_stats), _P(C.c_uint64),
                                _P(C.c_double), _P(C.c_double), _P(C.c_uint64), _P(C.c_uint64),
                                C.c_size_t, _P(C.c_size_t)], C.c_int),
    "bfi_adaptive_decide": ([_P(bfi_lattice), _P(bfi_subvolumes), _P(C.c_double), _P(C.c_double),
                             _P(C.c_double), _P(bfi_adaptive_config), _P(C.c_int32)], C.c_int),
    "bfi_integrand_eval": ([_vp, _P(bfi_integrand), C.c_uint64, _P(bfi_subvolumes),
                            _P(bfi_launch), _P(C.c_double), _P(C.c_double), _P(C.c_int32)],
                           C.c_int),
    "bfi_integrate_hdi": ([_vp, _P(bfi_integrand), C.c_uint64, _P(C.c_double), _P(C.c_double),
                           _P(bfi_hdi_config), _P(bfi_launch), _P(C.c_double), _P(C.c_double),
                           _P(bfi_hdi_stats)], C.c_int),
    "bfi_is_modes": ([_P(bfi_lattice), C.c_double, C.c_double, _P(C.c_double), _P(C.c_int32),
                      _P(C.c_double), _P(C.c_double)], C.c_int),
    "bfi_is_eval": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, C.c_double, C.c_double,
                     C.c_double, C.c_size_t, _P(C.c_uint64), _P(C.c_uint64), _P(C.c_uint64),
                     _P(bfi_launch), _P(C.c_double)], C.c_int),
    "bfi_integrate_is": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, C.c_double, C.c_double,
                          C.c_double, C.c_uint32, C.c_uint64, _P(bfi_launch), _P(bfi_result)],
                         C.c_int),
    "bfi_debug_is_points": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, C.c_double, C.c_double,
                             C.c_uint64, _P(C.c_uint64), C.c_uint64, _P(C.c_double),
                             _P(C.c_double)], C.c_int),
    "bfi_sph_eval": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, C.c_double, _P(bfi_shells),
                      _P(bfi_launch), _P(C.c_double)], C.c_int),
    "bfi_sph_finalize": ([_P(bfi_lattice), _P(bfi_shells), _P(C.c_double), _P(bfi_result)],
                         C.c_int),
    "bfi_integrate_sph": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, C.c_double, C.c_int32,
                           C.c_uint64, C.c_double, _P(bfi_launch), _P(bfi_result)], C.c_int),
    "bfi_debug_sph_points": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, C.c_uint64, C.c_double,
                              C.c_double, C.c_uint64, _P(C.c_uint64), _P(C.c_double)], C.c_int),
    "bfi_server_create": ([_vp, _P(bfi_server_config), _P(_vp)], C.c_int),
    "bfi_server_submit": ([_vp, _P(bfi_request), _P(C.c_uint64)], C.c_int),
    "bfi_server_poll": ([_vp, C.c_uint64, _P(bfi_result), _P(C.c_int32), _P(C.c_double)], C.c_int),
    "bfi_server_wait": ([_vp, C.c_uint64, C.c_double, _P(bfi_result), _P(C.c_int32),
                         _P(C.c_double)], C.c_int),
    "bfi_server_cancel": ([_vp, C.c_uint64], C.c_int),
    "bfi_server_stats_get": ([_vp, _P(bfi_server_stats)], C.c_int),
    "bfi_server_destroy": ([_vp], C.c_int),
    "bfi_autotune": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, _P(bfi_launch), _P(C.c_double)],
                     C.c_int),
    "bfi_tune_save": ([_vp, C.c_char_p], C.c_int),
    "bfi_tune_load": ([_vp, C.c_char_p], C.c_int),
    "bfi_debug_points": ([_vp, C.c_int32, C.c_int, C.c_uint64, C.c_uint64, _P(C.c_double),
                          _P(C.c_double), _P(C.c_uint64), C.c_uint64, _P(C.c_double)], C.c_int),
    "bfi_debug_action": ([_vp, _P(bfi_lattice), C.c_int, C.c_uint64, _P(C.c_double),
                          _P(C.c_double)], C.c_int),
}
EXPORTED = tuple(_SIGNATURES)

_lib = None


def load():
    """Load libbfi.so; raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1803_07560_amd/build.py` (or __graft_entry__.build())")
        # PyTorch ships its own HIP runtime (same soname as ROCm's).  Loading it
        # first makes libbfi.so bind to that copy, so torch tensors, streams and
        # this library share one runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _check(status: int, where: str):
    if status != 0:
        msg = load().bfi_last_error()
        raise BfiError(status, where, msg.decode() if msg else "")


def _dp(a):
    return a.ctypes.data_as(_P(C.c_double))


def _u64p(a):
    return a.ctypes.data_as(_P(C.c_uint64))


def _prec(p) -> int:
    return PRECISIONS[p]


def lattice(nx, nt, nu=1.0, D=1.0, a=1.0, tau=1.0, g=1.0, m2=0.0,
            observable="anchor", antithetic=False) -> bfi_lattice:
    """observable: "anchor" (u_{0,0} u_{0,r}, the paper's) or "averaged" (over all anchors);
    antithetic: each sample index gives a pair of points (see bfi_lattice)."""
    obs = {"anchor": BFI_OBS_ANCHOR, "averaged": BFI_OBS_AVERAGED}.get(observable, observable)
    return bfi_lattice(int(nx), int(nt), float(nu), float(D), float(a), float(tau), float(g),
                       float(m2), int(obs), int(antithetic))


def launch(samples_per_thread=0, block=0, persistent=-1, use_graph=0) -> bfi_launch:
    return bfi_launch(int(samples_per_thread), int(block), int(persistent), int(use_graph))


class Subvolumes:
    """Owns contiguous arrays for a bfi_subvolumes view (ids, lo/hi n x d, n, offset)."""

    def __init__(self, ids, lo, hi, n, offset, d: int):
        self.ids = np.ascontiguousarray(ids, dtype=np.uint64)
        cnt = self.ids.shape[0]
        self.lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(cnt, d)
        self.hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(cnt, d)
        self.n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, np.uint64), (cnt,)))
        self.offset = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, np.uint64), (cnt,)))
        self.view = bfi_subvolumes(cnt, _u64p(self.ids), _dp(self.lo), _dp(self.hi), _u64p(self.n),
                                   _u64p(self.offset))

    @classmethod
    def of(cls, obj, d: int) -> "Subvolumes":
        if isinstance(obj, cls):
            return obj
        return cls(obj.ids, obj.lo, obj.hi, obj.n, obj.offset, d)

    def __len__(self):
        return int(self.ids.shape[0])


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(getattr(stream, "cuda_stream", stream))


def _dev_ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


# ----------------------------------------------------------------------- API

def bfi_shape_supported(nx: int, nt: int) -> bool:
    return load().bfi_shape_supported(nx, nt) == 0


def bfi_supported_shapes() -> list[tuple[int, int]]:
    buf = (C.c_int32 * 256)()
    cnt = C.c_int32()
    _check(load().bfi_supported_shapes(buf, 128, C.byref(cnt)), "bfi_supported_shapes")
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(cnt.value)]


def bfi_context_create(device: int = 0):
    h = C.c_void_p()
    _check(load().bfi_context_create(device, C.byref(h)), "bfi_context_create")
    return h


def bfi_context_destroy(ctx):
    _check(load().bfi_context_destroy(ctx), "bfi_context_destroy")


def bfi_eval(ctx, lat, prec, seed, subs, launch_=None, split=False):
    sv = Subvolumes.of(subs, lat.d)
    part = np.zeros((len(sv), partial_len(lat.nx)), dtype=np.float64)
    spl = np.zeros((len(sv), split_len(lat.d)), dtype=np.float64) if split else None
    _check(load().bfi_eval(ctx, C.byref(lat), _prec(prec), int(seed), C.byref(sv.view),
                           C.byref(launch_) if launch_ is not None else None, _dp(part),
                           _dp(spl) if spl is not None else None), "bfi_eval")
    return (part, spl) if split else part


def bfi_eval_noalloc(ctx, lat, prec, seed, subs, launch_=None, split=False):
    """bfi_eval through the allocation-free entry point (static device scratch)."""
    sv = Subvolumes.of(subs, lat.d)
    part = np.zeros((len(sv), partial_len(lat.nx)), dtype=np.float64)
    spl = np.zeros((len(sv), split_len(lat.d)), dtype=np.float64) if split else None
    _check(load().bfi_eval_noalloc(ctx, C.byref(lat), _prec(prec), int(seed), C.byref(sv.view),
                                   C.byref(launch_) if launch_ is not None else None, _dp(part),
                                   _dp(spl) if spl is not None else None), "bfi_eval_noalloc")
    return (part, spl) if split else part


def bfi_plan_create(ctx, lat, prec, subs, launch_=None):
    sv = Subvolumes.of(subs, lat.d)
    h = C.c_void_p()
    _check(load().bfi_plan_create(ctx, C.byref(lat), _prec(prec), C.byref(sv.view),
                                  C.byref(launch_) if launch_ is not None else None, C.byref(h)),
           "bfi_plan_create")
    return h


def bfi_plan_run(plan, seed, partials_dev=None, stream=None):
    _check(load().bfi_plan_run(plan, int(seed), _dev_ptr(partials_dev), _stream_handle(stream)),
           "bfi_plan_run")


def bfi_plan_info(plan) -> dict:
    ni, ne, l = C.c_uint64(), C.c_uint64(), bfi_launch()
    _check(load().bfi_plan_info(plan, C.byref(ni), C.byref(ne), C.byref(l)), "bfi_plan_info")
    return {"n_items": ni.value, "n_evals": ne.value, "samples_per_thread": l.samples_per_thread,
            "block": l.block, "persistent": l.persistent, "use_graph": l.use_graph}


def bfi_plan_partials(plan, count: int, nx: int, out: np.ndarray | None = None) -> np.ndarray:
    """Per-subvolume records of the last run; `out` (count x (4 + 3 nx), float64,
    C-contiguous) is filled in place when given."""
    if out is None:
        out = np.zeros((count, partial_len(nx)), dtype=np.float64)
    elif out.shape != (count, partial_len(nx)) or out.dtype != np.float64 or \
            not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous float64 array of shape "
                         f"({count}, {partial_len(nx)})")
    _check(load().bfi_plan_partials(plan, _dp(out)), "bfi_plan_partials")
    return out


def bfi_plan_kernel_ms(plan) -> float:
    ms = C.c_double()
    _check(load().bfi_plan_kernel_ms(plan, C.byref(ms)), "bfi_plan_kernel_ms")
    return ms.value


def bfi_plan_destroy(plan):
    _check(load().bfi_plan_destroy(plan), "bfi_plan_destroy")


def bfi_partials_merge(nx: int, acc, more) -> np.ndarray:
    """Merged copy of two record arrays of disjoint sample ranges (count x
    (4 + 3 nx))."""
    a = np.array(acc, dtype=np.float64, order="C", copy=True)
    b = np.ascontiguousarray(more, dtype=np.float64)
    if a.shape != b.shape or a.ndim != 2 or a.shape[1] != partial_len(nx):
        raise ValueError(f"record arrays must both be count x {partial_len(nx)}")
    _check(load().bfi_partials_merge(int(nx), a.shape[0], _dp(a), _dp(b)), "bfi_partials_merge")
    return a


def bfi_finalize(lat, subs, partials) -> dict:
    sv = Subvolumes.of(subs, lat.d)
    p = np.ascontiguousarray(partials, dtype=np.float64)
    res = bfi_result()
    _check(load().bfi_finalize(C.byref(lat), C.byref(sv.view), _dp(p), C.byref(res)),
           "bfi_finalize")
    return res.to_dict()


def _box(d, box_lo, box_hi):
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, np.float64), (d,)))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(box_hi, np.float64), (d,)))
    return lo, hi


def bfi_integrate(ctx, lat, prec, seed, box_lo, box_hi, split_log2, budget, launch_=None) -> dict:
    lo, hi = _box(lat.d, box_lo, box_hi)
    res = bfi_result()
    _check(load().bfi_integrate(ctx, C.byref(lat), _prec(prec), int(seed), _dp(lo), _dp(hi),
                                int(split_log2), int(budget),
                                C.byref(launch_) if launch_ is not None else None, C.byref(res)),
           "bfi_integrate")
    return res.to_dict()


def adaptive_config(target_rel_err=1e-3, max_evals=1 << 34, n_min=1 << 12, n_max=1 << 22,
                    split_log2=10, max_rounds=64, refine_fraction=0.5,
                    round_evals=0, min_ess=0.0, split_samples=1 << 16,
                    holdout=False, progress=None) -> bfi_adaptive_config:
    """progress: optional callable taking a dict (round, holdout_checks, leaves,
    evals, rel_err, holdout_rel_err), called once per round and per holdout pass."""
    cfg = bfi_adaptive_config(float(target_rel_err), int(max_evals), int(n_min), int(n_max),
                              int(split_log2), int(max_rounds), float(refine_fraction),
                              int(round_evals), float(min_ess), int(split_samples),
                              int(bool(holdout)))
    if progress is not None:
        def _cb(p, _user):
            progress({f: getattr(p.contents, f) for f, _ in bfi_adaptive_progress._fields_})
        cfg.progress = ADAPTIVE_PROGRESS_FN(_cb)
        cfg._keep = cfg.progress  # the C function pointer lives as long as the config
    return cfg


def bfi_integrate_adaptive(ctx, lat, prec, seed, box_lo, box_hi, cfg, launch_=None,
                           leaf_capacity: int = 1 << 20) -> dict:
    """Returns the estimate, the run statistics, the status name (BFI_OK or
    BFI_EBUDGET) and the final partition (ids, lo, hi, n, offset)."""
    lo, hi = _box(lat.d, box_lo, box_hi)
    res, st = bfi_result(), bfi_adaptive_stats()
    cap = int(leaf_capacity)
    ids = np.zeros(cap, np.uint64)
    llo = np.zeros((cap, lat.d))
    lhi = np.zeros((cap, lat.d))
    ln = np.zeros(cap, np.uint64)
    loff = np.zeros(cap, np.uint64)
    nl = C.c_size_t()
    s = load().bfi_integrate_adaptive(ctx, C.byref(lat), _prec(prec), int(seed), _dp(lo), _dp(hi),
                                      C.byref(cfg),
                                      C.byref(launch_) if launch_ is not None else None,
                                      C.byref(res), C.byref(st), _u64p(ids), _dp(llo), _dp(lhi),
                                      _u64p(ln), _u64p(loff), cap, C.byref(nl))
    if s not in (0, -7):
        _check(s, "bfi_integrate_adaptive")
    k = nl.value
    out = res.to_dict()
    out.update({"status": STATUS[s], "rounds": st.rounds, "leaves": st.leaves, "evals": st.evals,
                "rel_err": st.rel_err, "holdout_checks": st.holdout_checks,
                "holdout_used": bool(st.holdout_used), "holdout_seed": st.holdout_seed,
                "holdout_rel_err": st.holdout_rel_err, "device_seconds": st.device_seconds,
                "graph_instantiations": st.graph_instantiations,
                "graph_updates": st.graph_updates,
                "partition": Subvolumes(ids[:k], llo[:k], lhi[:k], ln[:k], loff[:k], lat.d)})
    return out


def bfi_adaptive_decide(lat, leaves, partials, split, cfg, split_base=None) -> np.ndarray:
    """split_base: records of the samples the split statistics cover (None: the
    same samples as `partials`)."""
    sv = Subvolumes.of(leaves, lat.d)
    p = np.ascontiguousarray(partials, dtype=np.float64)
    s = np.ascontiguousarray(split, dtype=np.float64)
    b = None if split_base is None else np.ascontiguousarray(split_base, dtype=np.float64)
    if b is not None and b.shape != p.shape:
        raise ValueError("split_base must have the shape of partials")
    act = np.zeros(len(sv), dtype=np.int32)
    _check(load().bfi_adaptive_decide(C.byref(lat), C.byref(sv.view), _dp(p), _dp(s),
                                      None if b is None else _dp(b), C.byref(cfg),
                                      act.ctypes.data_as(_P(C.c_int32))),
           "bfi_adaptive_decide")
    return act


def integrand_nsphere(dim: int) -> bfi_integrand:
    return bfi_integrand(BFI_INTEGRAND_NSPHERE, int(dim), bfi_lattice(), BFI_FP64, 0)


def integrand_burgers(lat, prec="fp64", distance=None) -> bfi_integrand:
    """exp(-S) (distance None: the normalisation) or u_{0,0} u_{0,r} exp(-S)."""
    if distance is None:
        return bfi_integrand(BFI_INTEGRAND_BURGERS_Z, 0, lat, _prec(prec), 0)
    return bfi_integrand(BFI_INTEGRAND_BURGERS_N, 0, lat, _prec(prec), int(distance))


def bfi_integrand_eval(ctx, f, seed, subs, launch_=None):
    """(result, abserr, split_dim) arrays, one entry per subvolume."""
    sv = Subvolumes.of(subs, f.d)
    res = np.zeros(len(sv))
    err = np.zeros(len(sv))
    dim = np.zeros(len(sv), dtype=np.int32)
    _check(load().bfi_integrand_eval(ctx, C.byref(f), int(seed), C.byref(sv.view),
                                     C.byref(launch_) if launch_ is not None else None, _dp(res),
                                     _dp(err), dim.ctypes.data_as(_P(C.c_int32))),
           "bfi_integrand_eval")
    return res, err, dim


def hdi_config(n_initial=1_000_000, sample_factor=2.0, rel_diff=1.025, abs_diff=0.0,
               max_abs=0.0, split_log2=0, max_depth=20, max_evals=1 << 34) -> bfi_hdi_config:
    return bfi_hdi_config(int(n_initial), float(sample_factor), float(rel_diff), float(abs_diff),
                          float(max_abs), int(split_log2), int(max_depth), int(max_evals))


def bfi_integrate_hdi(ctx, f, seed, box_lo, box_hi, cfg, launch_=None) -> dict:
    lo, hi = _box(f.d, box_lo, box_hi)
    res, err, st = C.c_double(), C.c_double(), bfi_hdi_stats()
    s = load().bfi_integrate_hdi(ctx, C.byref(f), int(seed), _dp(lo), _dp(hi), C.byref(cfg),
                                 C.byref(launch_) if launch_ is not None else None,
                                 C.byref(res), C.byref(err), C.byref(st))
    if s not in (0, -7):
        _check(s, "bfi_integrate_hdi")
    return {"result": res.value, "abserr": err.value, "status": STATUS[s],
            **{k: getattr(st, k) for k, _ in bfi_hdi_stats._fields_}}


IS_UNIFORM_STREAM = 1 << 63


def bfi_is_modes(lat, box_lo, box_hi) -> dict:
    """Mode table of the Gaussian-proposal sampler over the cube [box_lo, box_hi]^d."""
    d = lat.d
    lam, scale = np.zeros(d), np.zeros(d)
    uni = np.zeros(d, dtype=np.int32)
    lk = C.c_double()
    _check(load().bfi_is_modes(C.byref(lat), float(box_lo), float(box_hi), _dp(lam),
                               uni.ctypes.data_as(_P(C.c_int32)), _dp(scale), C.byref(lk)),
           "bfi_is_modes")
    return {"lambda": lam, "uniform": uni.astype(bool), "scale": scale, "log_k": lk.value}


def bfi_is_eval(ctx, lat, prec, seed, box_lo, box_hi, gaussian_fraction, ids, n, offset=0,
                launch_=None) -> np.ndarray:
    """Partial records of W/K per stream (bit 63 of the id: uniform component)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, dtype=np.uint64), ids.shape))
    offset = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, dtype=np.uint64), ids.shape))
    out = np.zeros((ids.shape[0], 4 + 3 * lat.nx))
    _check(load().bfi_is_eval(ctx, C.byref(lat), _prec(prec), int(seed), float(box_lo),
                              float(box_hi), float(gaussian_fraction), ids.shape[0], _u64p(ids),
                              _u64p(n), _u64p(offset),
                              C.byref(launch_) if launch_ is not None else None, _dp(out)),
           "bfi_is_eval")
    return out


def bfi_integrate_is(ctx, lat, prec, seed, box_lo, box_hi, budget, gaussian_fraction=0.9,
                     streams=64, launch_=None) -> dict:
    res = bfi_result()
    _check(load().bfi_integrate_is(ctx, C.byref(lat), _prec(prec), int(seed), float(box_lo),
                                   float(box_hi), float(gaussian_fraction), int(streams),
                                   int(budget), C.byref(launch_) if launch_ is not None else None,
                                   C.byref(res)), "bfi_integrate_is")
    return res.to_dict()


def bfi_debug_is_points(ctx, lat, prec, seed, box_lo, box_hi, stream, index):
    """(points n x d, sum z^2/2 per point) of one sampler stream."""
    idx = np.ascontiguousarray(index, dtype=np.uint64)
    u = np.zeros((idx.shape[0], lat.d))
    hz = np.zeros(idx.shape[0])
    _check(load().bfi_debug_is_points(ctx, C.byref(lat), _prec(prec), int(seed), float(box_lo),
                                      float(box_hi), int(stream), _u64p(idx), idx.shape[0],
                                      _dp(u), _dp(hz)), "bfi_debug_is_points")
    return u, hz


class Shells:
    """Owns contiguous arrays for a bfi_shells view (ids, radii, n, offset)."""

    def __init__(self, ids, rho_lo, rho_hi, n, offset=0):
        self.ids = np.ascontiguousarray(ids, dtype=np.uint64)
        m = self.ids.shape[0]
        bc = lambda a, t: np.ascontiguousarray(np.broadcast_to(np.asarray(a, t), (m,)))  # noqa: E731
        self.rho_lo, self.rho_hi = bc(rho_lo, np.float64), bc(rho_hi, np.float64)
        self.n, self.offset = bc(n, np.uint64), bc(offset, np.uint64)
        self.view = bfi_shells(m, _u64p(self.ids), _dp(self.rho_lo), _dp(self.rho_hi),
                               _u64p(self.n), _u64p(self.offset))

    def __len__(self):
        return int(self.ids.shape[0])


def bfi_sph_eval(ctx, lat, prec, seed, box, shells, launch_=None) -> np.ndarray:
    sh = shells if isinstance(shells, Shells) else Shells(*shells)
    part = np.zeros((len(sh), partial_len(lat.nx)))
    _check(load().bfi_sph_eval(ctx, C.byref(lat), _prec(prec), int(seed), float(box),
                               C.byref(sh.view), C.byref(launch_) if launch_ is not None else None,
                               _dp(part)), "bfi_sph_eval")
    return part


def bfi_sph_finalize(lat, shells, partials) -> dict:
    sh = shells if isinstance(shells, Shells) else Shells(*shells)
    p = np.ascontiguousarray(partials, dtype=np.float64)
    res = bfi_result()
    _check(load().bfi_sph_finalize(C.byref(lat), C.byref(sh.view), _dp(p), C.byref(res)),
           "bfi_sph_finalize")
    return res.to_dict()


def bfi_integrate_sph(ctx, lat, prec, seed, box, nshells, budget, pilot_fraction=0.125,
                      launch_=None) -> dict:
    res = bfi_result()
    _check(load().bfi_integrate_sph(ctx, C.byref(lat), _prec(prec), int(seed), float(box),
                                    int(nshells), int(budget), float(pilot_fraction),
                                    C.byref(launch_) if launch_ is not None else None,
                                    C.byref(res)), "bfi_integrate_sph")
    return res.to_dict()


def bfi_debug_sph_points(ctx, lat, prec, seed, sid, rho_lo, rho_hi, index) -> np.ndarray:
    idx = np.ascontiguousarray(index, dtype=np.uint64)
    out = np.zeros((idx.shape[0], lat.d))
    _check(load().bfi_debug_sph_points(ctx, C.byref(lat), _prec(prec), int(seed), int(sid),
                                       float(rho_lo), float(rho_hi), idx.shape[0], _u64p(idx),
                                       _dp(out)), "bfi_debug_sph_points")
    return out


def server_config(memory_budget=1 << 30, max_requests=256, chunks_per_step=4,
                  max_pending=100000, step_evals=1 << 25,
                  max_samples_per_thread=0) -> bfi_server_config:
    return bfi_server_config(int(memory_budget), int(max_requests), int(chunks_per_step),
                             int(max_pending), int(step_evals), int(max_samples_per_thread))


def request(lat, prec, seed, box, split_log2, budget) -> bfi_request:
    return bfi_request(lat, _prec(prec), int(seed), float(box), int(split_log2), int(budget))


def bfi_server_create(ctx, cfg):
    h = C.c_void_p()
    _check(load().bfi_server_create(ctx, C.byref(cfg), C.byref(h)), "bfi_server_create")
    return h


def bfi_server_submit(srv, req) -> int:
    t = C.c_uint64()
    _check(load().bfi_server_submit(srv, C.byref(req), C.byref(t)), "bfi_server_submit")
    return t.value


def bfi_server_poll(srv, ticket):
    res, done, lat = bfi_result(), C.c_int32(), C.c_double()
    _check(load().bfi_server_poll(srv, int(ticket), C.byref(res), C.byref(done), C.byref(lat)),
           "bfi_server_poll")
    return (res.to_dict(), lat.value) if done.value else None


def bfi_server_wait(srv, ticket, timeout_s=60.0):
    res, done, lat = bfi_result(), C.c_int32(), C.c_double()
    _check(load().bfi_server_wait(srv, int(ticket), float(timeout_s), C.byref(res), C.byref(done),
                                  C.byref(lat)), "bfi_server_wait")
    return (res.to_dict(), lat.value) if done.value else None


def bfi_server_cancel(srv, ticket):
    _check(load().bfi_server_cancel(srv, int(ticket)), "bfi_server_cancel")


def bfi_server_stats_get(srv) -> dict:
    st = bfi_server_stats()
    _check(load().bfi_server_stats_get(srv, C.byref(st)), "bfi_server_stats_get")
    return {f: getattr(st, f) for f, _ in bfi_server_stats._fields_}


def bfi_server_destroy(srv):
    _check(load().bfi_server_destroy(srv), "bfi_server_destroy")


def bfi_autotune(ctx, lat, prec, evals_per_trial=1 << 26):
    best, rate = bfi_launch(), C.c_double()
    _check(load().bfi_autotune(ctx, C.byref(lat), _prec(prec), int(evals_per_trial),
                               C.byref(best), C.byref(rate)), "bfi_autotune")
    return {"samples_per_thread": best.samples_per_thread, "block": best.block,
            "persistent": best.persistent, "evals_per_s": rate.value}


def bfi_tune_save(ctx, path: str):
    _check(load().bfi_tune_save(ctx, path.encode()), "bfi_tune_save")


def bfi_tune_load(ctx, path: str):
    _check(load().bfi_tune_load(ctx, path.encode()), "bfi_tune_load")


def bfi_debug_points(ctx, d, prec, seed, sub_id, lo, hi, index) -> np.ndarray:
    lo, hi = _box(d, lo, hi)
    idx = np.ascontiguousarray(index, dtype=np.uint64)
    out = np.zeros((idx.shape[0], d), dtype=np.float64)
    _check(load().bfi_debug_points(ctx, int(d), _prec(prec), int(seed), int(sub_id), _dp(lo),
                                   _dp(hi), _u64p(idx), idx.shape[0], _dp(out)),
           "bfi_debug_points")
    return out


def bfi_debug_action(ctx, lat, prec, points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, lat.d)
    out = np.zeros(p.shape[0], dtype=np.float64)
    _check(load().bfi_debug_action(ctx, C.byref(lat), _prec(prec), p.shape[0], _dp(p), _dp(out)),
           "bfi_debug_action")
    return out
