"""Pins for the oracle's two observables behind C(r) (section 4's equal-time
correlation): the product anchored at the first site, and the same product
averaged over all nx*nt anchors.

Per configuration (exact):
  * a constant field c gives p_r = c^2 for every r;
  * a plane wave A_l cos(2 pi k m / nx + phi_l), 0 < k < nx/2, gives the
    trigonometric-sum closed form p_r = mean_l(A_l^2) cos(2 pi k r / nx) / 2;
  * the averaged product equals the anchored one averaged over the nx*nt
    periodic translations of the configuration (the group the action of
    Eq. Gen2 is invariant under), and is itself invariant under them, under the
    mirror x -> -x and under u -> -u; it is symmetric in r <-> nx - r.
In expectation:
  * uniform weights: C(0) = B^2/3 and C(r > 0) = 0, with the textbook errors of
    a mean over d independent sites (which fixes the 1/(nx nt) normalisation);
  * the regulated Gaussian (3x2): C(r) = (P^-1)_{0r} with a smaller error bar than
    the anchored estimator on the same points;
  * tiny nonlinear lattices: the anchored quadrature value."""
import math

import numpy as np
import pytest

import oracle
import workloads


def rand_config(nx, nt, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(-2, 2, nx * nt)


@pytest.mark.parametrize("obs", [0, 1])
def test_constant_field(oracle_lib, obs):
    lat = oracle.lattice(5, 3, observable=obs)
    np.testing.assert_array_equal(oracle.observable(lat, np.full(15, -1.5)), np.full(5, 2.25))


@pytest.mark.parametrize("nx,nt,k", [(5, 1, 1), (8, 2, 3), (10, 2, 2), (16, 4, 5)])
def test_plane_wave_closed_form(oracle_lib, nx, nt, k):
    lat = oracle.lattice(nx, nt, observable=1)
    A = 1.0 + 0.25 * np.arange(nt)
    phi = 0.3 + 0.7 * np.arange(nt)
    m = np.arange(nx)
    u = np.concatenate([A[l] * np.cos(2 * np.pi * k * m / nx + phi[l]) for l in range(nt)])
    want = np.mean(A ** 2) * np.cos(2 * np.pi * k * np.arange(nx) / nx) / 2
    np.testing.assert_allclose(oracle.observable(lat, u), want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("nx,nt", [(4, 2), (5, 3), (10, 2), (16, 4), (1, 3), (2, 1)])
def test_averaged_is_group_average_of_anchored(oracle_lib, nx, nt):
    anch = oracle.lattice(nx, nt, observable=0)
    avg = oracle.lattice(nx, nt, observable=1)
    u = rand_config(nx, nt, nx * 100 + nt)
    grid = u.reshape(nt, nx)
    shifted = [np.roll(np.roll(grid, -l, axis=0), -m, axis=1).ravel()
               for l in range(nt) for m in range(nx)]
    want = np.mean([oracle.observable(anch, v) for v in shifted], axis=0)
    got = oracle.observable(avg, u)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)
    # invariances of the averaged product
    for v in shifted[1:]:
        np.testing.assert_allclose(oracle.observable(avg, v), got, rtol=1e-13, atol=1e-15)
    mirror = np.roll(grid[:, ::-1], 1, axis=1).ravel()  # u(t, x) -> u(t, -x)
    np.testing.assert_allclose(oracle.observable(avg, mirror), got, rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(oracle.observable(avg, -u), got)
    for r in range(1, nx):
        assert got[r] == pytest.approx(got[nx - r], rel=1e-13, abs=1e-15)
    # the anchored product is not translation invariant (a plausible mix-up)
    if nx * nt > 1:
        assert not np.allclose(oracle.observable(anch, shifted[1]), oracle.observable(anch, u))


def test_sums_record_bruteforce_averaged(oracle_lib):
    nx, nt = 4, 2
    lat = oracle.lattice(nx, nt, nu=0.7, observable=1)
    sv = workloads.uniform_partition(8, 2.0, 2, per_sub=150, offset=3)
    got = oracle.sums(lat, 5, sv.ids, sv.lo, sv.hi, sv.n, sv.offset, nthreads=2)
    for s in range(len(sv)):
        U = oracle.points(8, 5, int(sv.ids[s]), sv.lo[s], sv.hi[s], range(3, 153))
        w = np.exp(-oracle.action_batch(lat, U))
        G = U.reshape(-1, nt, nx)
        p = np.stack([(G * np.roll(G, -r, axis=2)).mean(axis=(1, 2)) for r in range(nx)], 1)
        pw = p * w[:, None]
        want = np.concatenate([[150, w.sum(), (w * w).sum()], pw.sum(0), (pw ** 2).sum(0),
                               (pw * w[:, None]).sum(0)])
        np.testing.assert_allclose(got[s], want, rtol=1e-12, atol=1e-300)


def test_uniform_weights_textbook_errors(oracle_lib):
    """w == 1: p_0 is the mean of d independent u^2 (variance 4B^4/45/d) and,
    for 0 < r < nx/2, p_r the mean of d uncorrelated products of variance
    (B^2/3)^2; at r = nx/2 every product appears twice."""
    B, nx, nt, n = 2.0, 6, 2, 60000
    d = nx * nt
    lat = oracle.lattice(nx, nt, D=1e32, observable=1)
    one = workloads.uniform_partition(d, B, 0, per_sub=n)
    res = oracle.finalize(nx, d, one.lo, one.hi,
                          oracle.sums(lat, 4, one.ids, one.lo, one.hi, one.n, one.offset))
    s0 = B * B * math.sqrt(4 / 45) / math.sqrt(n * d)
    sr = (B * B / 3) / math.sqrt(n * d)
    assert res["C_err"][0] == pytest.approx(s0, rel=0.03)
    assert abs(res["C"][0] - B * B / 3) < 4 * s0
    for r in range(1, nx):
        want = sr * (math.sqrt(2) if r == nx // 2 else 1.0)
        assert res["C_err"][r] == pytest.approx(want, rel=0.03)
        assert abs(res["C"][r]) < 4 * want


def test_regulated_gaussian_averaged(oracle_lib):
    """g = 0, m2 = 1 on 3x2 over [-5, 5]^6 (every mode's width is at most 1):
    both observables estimate (P^-1)_{0r}; the averaged one on the same points
    has a smaller error bar."""
    nx, nt, nu, m2 = 3, 2, 0.5, 1.0
    d = nx * nt
    sh = lambda n: np.roll(np.eye(n), 1, axis=1)
    Tt, Sx = np.kron(sh(nt), np.eye(nx)), np.kron(np.eye(nt), sh(nx))
    A = (Tt - np.eye(d)) - nu * (Sx + Sx.T - 2 * np.eye(d))
    cov = np.linalg.inv(A.T @ A + m2 * np.eye(d))
    out = {}
    for obs in (0, 1):
        lat = oracle.lattice(nx, nt, nu=nu, g=0.0, m2=m2, observable=obs)
        out[obs] = oracle.integrate_uniform(lat, 7, -5.0, 5.0, 4, 1 << 22)
    for r in range(nx):
        for obs in (0, 1):
            assert abs(out[obs]["C"][r] - cov[0, r]) < 4 * out[obs]["C_err"][r]
        assert out[1]["C_err"][r] < 0.8 * out[0]["C_err"][r]
    assert out[0]["Z"] == out[1]["Z"]


@pytest.mark.parametrize("nx,nt,B,nu", [(3, 1, 2.0, 1.0), (2, 2, 2.0, 0.5)])
def test_nonlinear_tiny_lattice_averaged(oracle_lib, nx, nt, B, nu):
    from test_oracle_estimator import _gauss_legendre_box
    Zq, Cq = _gauss_legendre_box(oracle.lattice(nx, nt, nu=nu), B, 8)
    res = oracle.integrate_uniform(oracle.lattice(nx, nt, nu=nu, observable=1), 2, -B, B, 4,
                                   1 << 20)
    assert abs(res["Z"] - Zq) < 4 * res["Z_err"]
    for r in range(nx):
        assert abs(res["C"][r] - Cq[r]) < 4 * res["C_err"][r]


def test_observable_rejects_unknown_kind(oracle_lib):
    with pytest.raises(ValueError):
        oracle.observable(oracle.lattice(3, 1, observable=2), np.zeros(3))
