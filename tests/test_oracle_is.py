"""Pins for the oracle's Gaussian-proposal importance sampler (the quadratic
part of the action of Eq. Gen2 as proposal, near-flat modes uniform over the
box).  Nothing here comes from the sampler itself:

  * the basis is orthonormal and diagonalises P = A^T A/(D tau) + m2 I built
    from periodic shift matrices, with the eigenvalues the mode table reports;
  * coefficients along Gaussian modes have variance min(1/lambda, R^2), along
    the uniform constant mode R^2/3; Box-Muller normals pass a Kolmogorov-Smirnov test; the
    reported sum z^2/2 equals sum lambda a^2/2 over the Gaussian modes;
  * g = 0 with every mode Gaussian: every in-box weight is exp(0) = 1, and Z is
    the Gaussian integral (2 pi)^(d/2) / sqrt(det P) with C(r) = (P^-1)_{0r};
  * g = 1: Z and C(r) agree with tensor-product quadrature on tiny lattices and
    with the plain uniform estimator on 4x2 (also at nu = 1/2, where the
    checkerboard mode of an even lattice has lambda = 0 and gets the box's width);
  * on the 10x2 workload box the effective sample size per point is far above
    the uniform sampler's."""
import math

import numpy as np
import pytest

import oracle


def shift_P(nx, nt, nu=1.0, D=1.0, a=1.0, tau=1.0, m2=0.0):
    d = nx * nt
    sh = lambda n: np.roll(np.eye(n), 1, axis=1)
    Tt, Sx = np.kron(sh(nt), np.eye(nx)), np.kron(np.eye(nt), sh(nx))
    A = (Tt - np.eye(d)) - nu * tau / a**2 * (Sx + Sx.T - 2 * np.eye(d))
    return A.T @ A / (D * tau) + m2 * np.eye(d)


@pytest.mark.parametrize("nx,nt", [(1, 1), (2, 1), (3, 2), (4, 2), (5, 3), (10, 2), (16, 4)])
def test_basis_diagonalises_the_quadratic_form(oracle_lib, nx, nt):
    E = oracle.is_basis(nx, nt)
    d = nx * nt
    np.testing.assert_allclose(E.T @ E, np.eye(d), atol=1e-13)
    for nu, m2 in [(1.0, 0.0), (0.37, 0.5), (0.5, 0.0)]:
        lat = oracle.lattice(nx, nt, nu=nu, D=1.3, tau=0.8, a=1.1, m2=m2)
        P = shift_P(nx, nt, nu, 1.3, 1.1, 0.8, m2)
        lam = oracle.is_modes(lat, -2.0, 2.0)["lambda"]
        np.testing.assert_allclose(P @ E, E * lam[None, :], atol=1e-12 * max(1, lam.max()))
        np.testing.assert_allclose(np.sort(lam), np.linalg.eigvalsh(P), atol=1e-11)
        assert lam[0] == pytest.approx(m2, abs=1e-14)     # the constant mode


def test_mode_table(oracle_lib):
    lat = oracle.lattice(10, 2)
    B = 4.0
    m = oracle.is_modes(lat, -B, B)
    R = B * math.sqrt(20)
    lam = m["lambda"]
    assert m["uniform"][0] and m["uniform"].sum() == 1       # only the constant mode
    g = ~m["uniform"]
    np.testing.assert_allclose(m["scale"][g], np.minimum(1 / np.sqrt(lam[g]), R))
    assert m["scale"][0] == R
    assert m["log_k"] == pytest.approx(np.log(2 * R) + np.sum(np.log(np.sqrt(2 * np.pi) *
                                                                     m["scale"][g])))
    # nu = 1/2 on an even lattice: the checkerboard (-1)^(l+m) is a null mode
    # too; it stays Gaussian with the box's width
    m2 = oracle.is_modes(oracle.lattice(4, 2, nu=0.5), -2.0, 2.0)
    j = 1 * 4 + 3                     # time Nyquist x space Nyquist
    assert m2["lambda"][j] == pytest.approx(0.0, abs=1e-14) and not m2["uniform"][j]
    assert m2["scale"][j] == pytest.approx(2.0 * math.sqrt(8))
    # m2 > 0 with a wide box: the constant mode is Gaussian as well
    m3 = oracle.is_modes(oracle.lattice(3, 2, m2=1.0), -6.0, 6.0)
    assert not m3["uniform"].any()


def test_sampler_moments_and_normality(oracle_lib):
    from scipy import stats
    nx, nt, B = 4, 2, 3.0
    lat = oracle.lattice(nx, nt, nu=0.8)
    m = oracle.is_modes(lat, -B, B)
    E = oracle.is_basis(nx, nt)
    N = 6000
    U = np.zeros((N, 8))
    HZ = np.zeros(N)
    for i in range(N):
        U[i], HZ[i] = oracle.is_point(lat, -B, B, 5, 3, i)
    A = U @ E                                 # coefficients along the modes
    g = ~m["uniform"]
    var = A.var(axis=0)
    np.testing.assert_allclose(var[g], m["scale"][g] ** 2, rtol=0.08)
    R = B * math.sqrt(8)
    np.testing.assert_allclose(var[~g], R * R / 3, rtol=0.08)
    assert np.all(np.abs(A[:, ~g]) <= R)
    np.testing.assert_allclose(HZ, 0.5 * (A[:, g] ** 2 / m["scale"][g] ** 2).sum(1), rtol=1e-10)
    Z = A[:, g] / m["scale"][g]
    for j in range(Z.shape[1]):
        assert stats.kstest(Z[:, j], "norm").pvalue > 1e-3
    c = np.corrcoef(Z.T)
    assert np.max(np.abs(c - np.eye(c.shape[0]))) < 0.06


def test_gaussian_weights_are_one_and_z_is_the_gaussian_integral(oracle_lib):
    nx, nt, nu, m2, B = 3, 2, 0.5, 1.0, 6.0
    d = nx * nt
    lat = oracle.lattice(nx, nt, nu=nu, g=0.0, m2=m2)
    m = oracle.is_modes(lat, -B, B)
    assert not m["uniform"].any()
    s = oracle.is_sums(lat, 2, -B, B, np.array([1, 2], np.uint64), 50_000, gaussian_fraction=1.0)
    # w in {0, 1}: sum w = sum w^2 = number of points inside the box
    np.testing.assert_allclose(s[:, 1], s[:, 2], rtol=1e-10)
    assert np.all(s[:, 1] <= s[:, 0] * (1 + 1e-9)) and np.all(s[:, 1] >= 0.999 * s[:, 0])
    res = oracle.integrate_is(lat, 2, -B, B, 8, 1 << 18, gaussian_fraction=1.0)
    P = shift_P(nx, nt, nu, m2=m2)
    Zexact = (2 * np.pi) ** (d / 2) / math.sqrt(np.linalg.det(P))
    assert abs(res["Z"] - Zexact) < 4 * res["Z_err"] + 1e-9 * Zexact
    assert res["Z_err"] < 1e-3 * Zexact
    cov = np.linalg.inv(P)
    for r in range(nx):
        assert abs(res["C"][r] - cov[0, r]) < 4 * res["C_err"][r]


@pytest.mark.parametrize("nx,nt,B,nu", [(3, 1, 2.0, 1.0), (2, 2, 2.0, 0.5), (3, 1, 4.0, 0.5)])
def test_nonlinear_tiny_lattice_against_quadrature(oracle_lib, nx, nt, B, nu):
    from test_oracle_estimator import _gauss_legendre_box
    Zq, Cq = _gauss_legendre_box(oracle.lattice(nx, nt, nu=nu), B, 8)
    res = oracle.integrate_is(oracle.lattice(nx, nt, nu=nu), 4, -B, B, 8, 1 << 19)
    assert abs(res["Z"] - Zq) < 4 * res["Z_err"]
    for r in range(nx):
        assert abs(res["C"][r] - Cq[r]) < 4 * res["C_err"][r]


@pytest.mark.parametrize("nu,obs", [(1.0, 0), (0.5, 0), (0.7, 1)])
def test_agrees_with_the_uniform_sampler(oracle_lib, nu, obs):
    lat = oracle.lattice(4, 2, nu=nu, observable=obs)
    B = 2.0
    u = oracle.integrate_uniform(lat, 1, -B, B, 4, 1 << 20)
    g = oracle.integrate_is(lat, 2, -B, B, 8, 1 << 19)
    assert abs(u["Z"] - g["Z"]) < 4 * math.hypot(u["Z_err"], g["Z_err"])
    for r in range(4):
        assert abs(u["C"][r] - g["C"][r]) < 4 * math.hypot(u["C_err"][r], g["C_err"][r])


def test_effective_sample_size_on_the_workload_box(oracle_lib):
    lat = oracle.lattice(10, 2)
    g = oracle.integrate_is(lat, 1, -4.0, 4.0, 8, 1 << 18)
    u = oracle.integrate_uniform(lat, 1, -4.0, 4.0, 3, 1 << 18)
    assert g["ess"] > 50 and g["ess"] > 20 * u["ess"]


def test_rejects_bad_boxes(oracle_lib):
    with pytest.raises(ValueError):
        oracle.is_modes(oracle.lattice(3, 1), np.array([0.0, 1.0, 1.0]), np.array([1.0, 1.0, 2.0]))
    with pytest.raises(ValueError):
        oracle.is_point(oracle.lattice(3, 1, observable=5), -1, 1, 1, 1, 0)


def test_mixture_pins(oracle_lib):
    """alpha = 0 is the plain uniform sampler on the same points; alpha < 1
    bounds the weights by V/(1 - alpha) (so sum W^2 <= bound * sum W), and the
    mixture matches quadrature on 3x1, nu = 1/2, box [-4, 4], where the nonlinear
    term can cancel the residual and the Gaussian alone has heavy-tailed weights
    (depending on the seed, a biased Z or an error bar blown up by one sample)."""
    from test_oracle_estimator import _gauss_legendre_box
    nx, nt, B, nu = 3, 1, 4.0, 0.5
    d = nx * nt
    lat = oracle.lattice(nx, nt, nu=nu)
    # alpha = 0, one stream: Z = V mean(exp(-S)) over the uniform points of that id
    sid = oracle.IS_UNIFORM_STREAM + 1
    g0 = oracle.integrate_is(lat, 6, -B, B, 1, 40_000, gaussian_fraction=0.0)
    plain = oracle.sums(lat, 6, np.array([sid], np.uint64), np.full((1, d), -B),
                        np.full((1, d), B), np.array([40_000], np.uint64))
    res = oracle.finalize(nx, d, np.full((1, d), -B), np.full((1, d), B), plain)
    assert g0["Z"] == pytest.approx(res["Z"], rel=1e-12)
    np.testing.assert_allclose(g0["C"], res["C"], rtol=1e-11, atol=1e-14)
    # bounded weights
    alpha = 0.9
    m = oracle.is_modes(lat, -B, B)
    bound = (2 * B) ** d / (1 - alpha) / np.exp(m["log_k"])      # for W/K
    ids, n = oracle.is_plan(1 << 16, 4, alpha)
    s = oracle.is_sums(lat, 6, -B, B, ids, n, 0, alpha)
    assert np.all(s[:, 2] <= bound * s[:, 1] * (1 + 1e-12))
    Zq, _ = _gauss_legendre_box(lat, B, 8)
    for seed in (4, 5):
        mixed = oracle.integrate_is(lat, seed, -B, B, 8, 1 << 19, gaussian_fraction=alpha)
        assert abs(mixed["Z"] - Zq) < 4 * mixed["Z_err"]
        assert mixed["Z_err"] < 0.02 * Zq
