"""Pins for the oracle's discretised action (paper section 2, Eq. Gen2).

Each test states a fact fixed by the mathematics rather than by retyping the
oracle's loop:
  * a constant field has zero action (every difference vanishes);
  * with the nonlinear term dropped (g = 0) the action is the quadratic form
    |A u|^2 / (2 D tau) with A = (T_t - 1) - (nu tau / a^2)(S_x + S_x^-1 - 2),
    built from periodic shift matrices;
  * the residual vanishes on one explicit-Euler step of Burgers' equation
    v_t + v v_x = nu v_xx (central differences), which fixes the sign and size of
    the advection and viscous terms against the time difference;
  * a time-independent plane wave has a closed-form action from trigonometric
    sums (fixes the 1/(2a), nu/a^2 and 1/(2 D tau) factors and the periodic wrap);
  * one space site reduces to a random walk, sum (u_{l+1} - u_l)^2 / (2 D tau);
    two sites and one time slice reduce to 4 nu^2 tau (u_1 - u_0)^2 / (D a^4);
  * translations in l and m and the parity u_{l,m} -> -u_{l,-m} leave S unchanged.
"""
import math

import numpy as np
import pytest

import oracle

SHAPES = [(1, 1), (1, 3), (2, 1), (2, 2), (3, 1), (3, 2), (4, 2), (5, 3), (8, 2), (10, 2), (16, 4)]


def _rand_params(rng):
    return dict(nu=float(rng.uniform(0.05, 2.0)), D=float(rng.uniform(0.3, 3.0)),
                a=float(rng.uniform(0.5, 2.0)), tau=float(rng.uniform(0.2, 1.5)))


@pytest.mark.parametrize("nx,nt", SHAPES)
def test_constant_field_has_zero_action(oracle_lib, nx, nt):
    rng = np.random.Generator(np.random.PCG64(nx * 100 + nt))
    lat = oracle.lattice(nx, nt, **_rand_params(rng))
    for c in (0.0, 0.37, -3.999, 1e3):
        assert oracle.action(lat, np.full(nx * nt, c)) == 0.0


def _shift(n):
    """(P u)_i = u_{i+1 mod n}."""
    return np.roll(np.eye(n), 1, axis=1)


def _linear_operator(nx, nt, nu, a, tau):
    It, Ix = np.eye(nt), np.eye(nx)
    Tt = np.kron(_shift(nt), Ix)                  # u_{l,m} -> u_{l+1,m}
    Sx = np.kron(It, _shift(nx))                  # u_{l,m} -> u_{l,m+1}
    lap = Sx + Sx.T - 2.0 * np.eye(nx * nt)
    return (Tt - np.eye(nx * nt)) - (nu * tau / a**2) * lap


@pytest.mark.parametrize("nx,nt", SHAPES)
def test_gaussian_case_is_quadratic_form(oracle_lib, nx, nt):
    rng = np.random.Generator(np.random.PCG64(31 + nx * nt))
    for _ in range(5):
        p = _rand_params(rng)
        m2 = float(rng.choice([0.0, 0.7]))
        lat = oracle.lattice(nx, nt, g=0.0, m2=m2, **p)
        A = _linear_operator(nx, nt, p["nu"], p["a"], p["tau"])
        P = A.T @ A / (p["D"] * p["tau"]) + m2 * np.eye(nx * nt)
        u = rng.uniform(-4, 4, size=nx * nt)
        want = 0.5 * u @ P @ u
        assert oracle.action(lat, u) == pytest.approx(want, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("nx", [3, 4, 5, 10, 16])
def test_residual_vanishes_on_euler_step(oracle_lib, nx):
    """R_{0,m} = 0 when u_1 is one forward-Euler step of v_t = -v v_x + nu v_xx."""
    rng = np.random.Generator(np.random.PCG64(5 + nx))
    for _ in range(5):
        p = _rand_params(rng)
        a, tau, nu = p["a"], p["tau"], p["nu"]
        u0 = rng.uniform(-2, 2, size=nx)
        ux = (np.roll(u0, -1) - np.roll(u0, 1)) / (2 * a)
        uxx = (np.roll(u0, -1) - 2 * u0 + np.roll(u0, 1)) / a**2
        u1 = u0 + tau * (-u0 * ux + nu * uxx)
        lat = oracle.lattice(nx, 2, **p)
        R = oracle.residual(lat, np.concatenate([u0, u1]))
        scale = np.abs(u0).max() + tau * (np.abs(u0 * ux).max() + nu * np.abs(uxx).max())
        assert np.all(np.abs(R[:nx]) <= 1e-13 * scale)
        # the second time slice does not vanish in general
        assert np.abs(R[nx:]).max() > 1e-6


@pytest.mark.parametrize("nx,nt", [(5, 1), (5, 3), (8, 2), (10, 2), (16, 4), (7, 2)])
def test_plane_wave_closed_form(oracle_lib, nx, nt):
    """u_{l,m} = A cos(k m + phi), k = 2 pi / nx, the same at every time slice:
    R = tau (alpha c s + beta c) with c, s the cosine and sine at site m,
    alpha = -g A^2 sin(k)/a, beta = 4 nu A sin^2(k/2)/a^2; summing the squares
    over a full period (nx >= 5) gives S = nt tau nx (alpha^2/8 + beta^2/2)/(2D)."""
    rng = np.random.Generator(np.random.PCG64(77 + nx))
    for _ in range(5):
        p = _rand_params(rng)
        A = float(rng.uniform(0.2, 3.0))
        phi = float(rng.uniform(0, 2 * math.pi))
        k = 2 * math.pi / nx
        row = A * np.cos(k * np.arange(nx) + phi)
        u = np.tile(row, nt)
        alpha = -A**2 * math.sin(k) / p["a"]
        beta = 4 * p["nu"] * A * math.sin(k / 2) ** 2 / p["a"] ** 2
        want = nt * p["tau"] * nx * (alpha**2 / 8 + beta**2 / 2) / (2 * p["D"])
        assert oracle.action(oracle.lattice(nx, nt, **p), u) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("nt", [1, 2, 3, 5])
def test_single_site_is_random_walk(oracle_lib, nt):
    rng = np.random.Generator(np.random.PCG64(9 + nt))
    p = _rand_params(rng)
    u = rng.uniform(-3, 3, size=nt)
    want = sum((u[(l + 1) % nt] - u[l]) ** 2 for l in range(nt)) / (2 * p["D"] * p["tau"])
    assert oracle.action(oracle.lattice(1, nt, **p), u) == pytest.approx(want, rel=1e-13, abs=0)


def test_two_sites_one_slice_closed_form(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(10):
        p = _rand_params(rng)
        u = rng.uniform(-3, 3, size=2)
        want = 4 * p["nu"] ** 2 * p["tau"] * (u[1] - u[0]) ** 2 / (p["D"] * p["a"] ** 4)
        assert oracle.action(oracle.lattice(2, 1, **p), u) == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("nx,nt", [(3, 2), (4, 2), (5, 3), (10, 2), (16, 4)])
def test_translation_and_parity_invariance(oracle_lib, nx, nt):
    rng = np.random.Generator(np.random.PCG64(3 + nx * nt))
    p = _rand_params(rng)
    lat = oracle.lattice(nx, nt, **p)
    for _ in range(5):
        u = rng.uniform(-4, 4, size=(nt, nx))
        S = oracle.action(lat, u.ravel())
        for sl in range(nt):
            for sm in range(nx):
                v = np.roll(np.roll(u, sl, axis=0), sm, axis=1)
                assert oracle.action(lat, v.ravel()) == pytest.approx(S, rel=1e-13)
        parity = -u[:, (-np.arange(nx)) % nx]
        assert oracle.action(lat, parity.ravel()) == pytest.approx(S, rel=1e-13)
        # neither u -> -u nor x -> -x alone is a symmetry once the advection term acts
        if nx >= 3:
            assert oracle.action(lat, (-u).ravel()) != pytest.approx(S, rel=1e-9)
            assert oracle.action(lat, u[:, (-np.arange(nx)) % nx].ravel()) != \
                pytest.approx(S, rel=1e-9)


def test_sign_of_coupling_is_a_reflection(oracle_lib):
    """S_g(u) = S_{-g}(-u): the sign of g only reverses the x direction, so Z and
    C(r) over a symmetric box do not depend on it."""
    rng = np.random.Generator(np.random.PCG64(21))
    for nx, nt in [(4, 2), (10, 2)]:
        u = rng.uniform(-4, 4, size=nx * nt)
        assert oracle.action(oracle.lattice(nx, nt, g=1.0), u) == pytest.approx(
            oracle.action(oracle.lattice(nx, nt, g=-1.0), -u), rel=1e-14)


def test_mass_term(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(12))
    u = rng.uniform(-4, 4, size=20)
    s0 = oracle.action(oracle.lattice(10, 2), u)
    s1 = oracle.action(oracle.lattice(10, 2, m2=0.3), u)
    assert s1 - s0 == pytest.approx(0.15 * np.sum(u * u), rel=1e-12)


def test_batch_matches_single(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(13))
    lat = oracle.lattice(10, 2)
    U = rng.uniform(-4, 4, size=(50, 20))
    S = oracle.action_batch(lat, U)
    assert np.array_equal(S, [oracle.action(lat, u) for u in U])


def test_invalid_parameters_are_rejected(oracle_lib):
    u = np.zeros(8)
    for bad in (dict(D=0.0), dict(D=-1.0), dict(a=0.0), dict(tau=0.0), dict(nu=float("nan")),
                dict(D=float("inf"))):
        assert math.isnan(oracle.action(oracle.lattice(4, 2, **bad), u))
    with pytest.raises(ValueError):
        oracle.residual(oracle.lattice(0, 2), u)
