"""Comparison helpers of the GPU parity tests: GPU records against the oracle's
records on the same points, with tolerances taken against each sum's L1 scale.

Layouts: the library's partial record is [n, sigma, w, w^2, p_r w (nx),
(p_r w)^2 (nx), p_r w^2 (nx)] with the sums scaled by exp(sigma) (first order)
or exp(2 sigma) (second order); the oracle's plain record is [n, w, w^2, ...]
(+ nx fields sum |p_r w| from oracle.sums_l1), its shifted record
[n, sigma, w, ...] (+ the same L1 fields from oracle.sums_shifted_l1)."""
import numpy as np


def move_shift(part, nx, sigma):
    """Library records moved to the per-record shifts `sigma`, in the oracle's
    layout [n, w, w^2, p_r w, (p_r w)^2, p_r w^2] (sigma = 0: plain sums)."""
    f1 = np.exp(np.asarray(sigma, dtype=np.float64) - part[:, 1])
    f2 = f1 * f1
    out = np.zeros((part.shape[0], 3 + 3 * nx))
    out[:, 0] = part[:, 0]
    out[:, 1] = part[:, 2] * f1
    out[:, 2] = part[:, 3] * f2
    out[:, 3:3 + nx] = part[:, 4:4 + nx] * f1[:, None]
    out[:, 3 + nx:3 + 3 * nx] = part[:, 4 + nx:4 + 3 * nx] * f2[:, None]
    return out


def assert_records_close(got, want, l1, nx, rtol):
    """got/want in the oracle's plain layout (same shift), l1 = sum |p_r w| on
    that shift.  Bars: w, w^2, (p_r w)^2 against themselves (positive sums);
    p_r w against sum |p_r w|; p_r w^2 against sqrt(sum (p_r w)^2 sum w^2)
    (Cauchy-Schwarz).  Returns the largest scaled error."""
    assert np.array_equal(got[:, 0], want[:, 0])
    pw2 = want[:, 3 + nx:3 + 2 * nx]
    scale = np.concatenate([want[:, 1:3], l1, pw2, np.sqrt(pw2) * np.sqrt(want[:, 2:3])], axis=1)
    err = np.abs(got[:, 1:] - want[:, 1:])
    bad = err > rtol * scale + 1e-300
    worst = float((err / (scale + 1e-300)).max())
    assert not bad.any(), (np.argwhere(bad)[:5], worst)
    return worst


def volumes(lo, hi):
    return np.prod(np.asarray(hi) - np.asarray(lo), axis=1)


def c_scale(lo, hi, plain, l1):
    """L1 scale of C(r) = N(r)/Z: sum_s V_s/n_s sum |p_r w|_s over Z (both on
    the same shift), the size of the terms whose rounding C(r) inherits."""
    v = volumes(lo, hi) / plain[:, 0]
    z = np.sum(v * plain[:, 1])
    return np.sum(v[:, None] * l1, axis=0) / z


def assert_result_close(got, want, cscale, tol):
    """Z (through log Z) within tol relative; C(r) within tol of its L1 scale
    plus |C(r)| (the ratio also inherits Z's relative error); C_err within
    tol relative plus tol of the C(r) scale (its own rounding).  Returns the
    largest scaled errors."""
    dz = abs(got["log_Z"] - want["log_Z"])
    assert dz <= tol, (got["log_Z"], want["log_Z"])
    bar = tol * (cscale + np.abs(want["C"]))
    dc = np.abs(got["C"] - want["C"])
    assert np.all(dc <= bar), (got["C"], want["C"], dc / bar)
    de = np.abs(got["C_err"] - want["C_err"])
    assert np.all(de <= tol * np.abs(want["C_err"]) + tol * cscale), (got["C_err"], want["C_err"])
    return {"log_Z": float(dz), "C_over_scale": float(np.max(dc / (cscale + np.abs(want["C"]))))}
