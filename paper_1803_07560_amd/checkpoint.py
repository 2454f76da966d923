"""Checkpoint and resume of a Monte Carlo run over a fixed subvolume list.

Every point is addressed by (seed, subvolume id, sample index) through the
counter-based Philox stream, so the whole state of a run (paper section 3: each
subvolume's integral is estimated from its own samples) is
  * the lattice (the parameters of Eq. Gen2, the observable and the sampler:
    single points or antithetic pairs), the precision and the seed,
  * the subvolume list (ids, boxes) with the range of sample indices evaluated
    so far, [offset, offset + n) per subvolume,
  * the partial records of those samples.
Resuming evaluates the next indices of every subvolume and merges the records
(``bfi_partials_merge``); nothing else is needed to continue exactly where the
run stopped.  The state is written as JSON with every double as a hexadecimal
float, so a reload is bit-identical.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

from . import _binding as _b

FORMAT = "bfi-checkpoint-1"
_LATTICE_FIELDS = ("nx", "nt", "nu", "D", "a", "tau", "g", "m2", "observable", "antithetic")


@dataclass
class RunState:
    lat: _b.bfi_lattice
    prec: str                # "fp64" or "fp32"
    seed: int
    subs: _b.Subvolumes      # n = samples evaluated, offset = first index evaluated
    partials: np.ndarray     # count x (4 + 3 nx)

    @property
    def evals(self) -> int:
        return int(self.subs.n.sum()) * (2 if self.lat.antithetic else 1)


def _prec_name(prec) -> str:
    code = _b._prec(prec)
    return "fp64" if code == _b.BFI_FP64 else "fp32"


def start(ctx, lat, prec, seed, subs, launch=None) -> RunState:
    """Evaluate the subvolumes as given (their n samples from their offsets)."""
    sv = _b.Subvolumes.of(subs, lat.d)
    sv = _b.Subvolumes(sv.ids, sv.lo, sv.hi, sv.n, sv.offset, lat.d)  # own copy
    part = _b.bfi_eval(ctx, lat, prec, seed, sv, launch)
    return RunState(lat, _prec_name(prec), int(seed), sv, part)


def advance(ctx, state: RunState, n_more, launch=None) -> RunState:
    """Evaluate the next n_more samples (scalar or per subvolume) of every
    subvolume and merge them into a new state; `state` is left unchanged."""
    sv = state.subs
    d = state.lat.d
    more = np.ascontiguousarray(np.broadcast_to(np.asarray(n_more, np.uint64), (len(sv),)))
    nxt = _b.Subvolumes(sv.ids, sv.lo, sv.hi, more, sv.offset + sv.n, d)
    part = _b.bfi_eval(ctx, state.lat, state.prec, state.seed, nxt, launch)
    merged = _b.bfi_partials_merge(state.lat.nx, state.partials, part)
    subs = _b.Subvolumes(sv.ids, sv.lo, sv.hi, sv.n + more, sv.offset, d)
    return RunState(state.lat, state.prec, state.seed, subs, merged)


def result(state: RunState) -> dict:
    """Z, C(r) and their errors from the samples evaluated so far."""
    return _b.bfi_finalize(state.lat, state.subs, state.partials)


def _hex(a) -> list:
    return [float(x).hex() for x in np.asarray(a, np.float64).ravel()]


def _unhex(xs, shape) -> np.ndarray:
    return np.array([float.fromhex(x) for x in xs], np.float64).reshape(shape)


def to_json(state: RunState) -> str:
    lat = {f: getattr(state.lat, f) for f in _LATTICE_FIELDS}
    for f in ("nu", "D", "a", "tau", "g", "m2"):
        lat[f] = float(lat[f]).hex()
    sv = state.subs
    doc = {
        "format": FORMAT,
        "lattice": lat,
        "precision": state.prec,
        "seed": str(state.seed),
        "count": len(sv),
        "id": [str(int(x)) for x in sv.ids],
        "lo": _hex(sv.lo),
        "hi": _hex(sv.hi),
        "n": [str(int(x)) for x in sv.n],
        "offset": [str(int(x)) for x in sv.offset],
        "partials": _hex(state.partials),
    }
    return json.dumps(doc)


def from_json(text: str) -> RunState:
    doc = json.loads(text)
    if doc.get("format") != FORMAT:
        raise ValueError(f"not a {FORMAT} document")
    L = doc["lattice"]
    lat = _b.bfi_lattice(int(L["nx"]), int(L["nt"]),
                         *(float.fromhex(L[f]) for f in ("nu", "D", "a", "tau", "g", "m2")),
                         int(L["observable"]), int(L.get("antithetic", 0)))
    cnt, d, nx = int(doc["count"]), lat.d, lat.nx
    sizes = {"id": cnt, "lo": cnt * d, "hi": cnt * d, "n": cnt, "offset": cnt,
             "partials": cnt * _b.partial_len(nx)}
    for k, want in sizes.items():
        if len(doc[k]) != want:
            raise ValueError(f"checkpoint field {k!r}: {len(doc[k])} entries, expected {want}")
    u64 = lambda xs: np.array([int(x) for x in xs], np.uint64)
    subs = _b.Subvolumes(u64(doc["id"]), _unhex(doc["lo"], (cnt, d)), _unhex(doc["hi"], (cnt, d)),
                         u64(doc["n"]), u64(doc["offset"]), d)
    part = _unhex(doc["partials"], (cnt, _b.partial_len(nx)))
    if doc["precision"] not in ("fp64", "fp32"):
        raise ValueError(f"unknown precision {doc['precision']!r}")
    return RunState(lat, doc["precision"], int(doc["seed"]), subs, part)


def save(state: RunState, path: str) -> None:
    """Write the state atomically (a temporary file renamed over `path`)."""
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(to_json(state))
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def load(path: str) -> RunState:
    with open(path) as f:
        return from_json(f.read())
