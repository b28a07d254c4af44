"""Pins of the oracle's variable conversions, fluxes, wave speeds and inversion."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import covariant as cov

GAM = 4.0 / 3.0


def ks():
    return I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=I.SPIN)


def sample(seed, n, wmax=10.0, smax=100.0):
    rng = np.random.default_rng(seed)
    x_lo, x_hi = I.ks_domain()
    out = []
    for _ in range(n):
        x1 = rng.uniform(x_lo[0], x_hi[0])
        x2 = rng.uniform(x_lo[1], x_hi[1])
        m = O.metric(ks(), x1, x2)
        out.append((x1, x2, m, cov.random_prim(rng, wmax, smax, m["g"])))
    return out


@pytest.mark.parametrize("x1,x2,m,P", sample(1, 20))
def test_prim2con_equals_stress_energy_projection(x1, x2, m, P):
    U = O.p2c(ks(), x1, x2, P)
    Uc = cov.conserved(m, P, GAM)
    scale = np.abs(Uc[:5]).max()
    assert np.allclose(U[:5], Uc[:5], rtol=1e-12, atol=1e-12 * scale)
    assert np.allclose(U[5:], Uc[5:], rtol=1e-13, atol=0)


@pytest.mark.parametrize("x1,x2,m,P", sample(2, 12))
@pytest.mark.parametrize("d", [0, 1, 2])
def test_flux_equals_covariant_flux(x1, x2, m, P, d):
    U, F, lam = O.phys_flux(ks(), x1, x2, P, d)
    Fc = cov.fluxes(m, P, GAM, d)
    scale = np.abs(Fc).max()
    mask = np.ones(9, bool)
    mask[5 + d] = False     # normal field and psi fluxes are set by the GLM solve
    mask[8] = False
    assert np.allclose(F[mask], Fc[mask], rtol=1e-11, atol=1e-12 * scale)
    assert F[5 + d] == 0.0 and F[8] == 0.0
    assert lam[0] <= lam[1]


@pytest.mark.parametrize("v", [-0.9, -0.3, 0.0, 0.4, 0.95])
@pytest.mark.parametrize("p", [1e-3, 0.1, 10.0])
def test_flat_hydro_speeds_are_relativistic_velocity_addition(v, p):
    """B = 0, flow along x in flat space: lambda = (v -+ c_s)/(1 -+ v c_s)."""
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    rho = 0.7
    W = 1 / math.sqrt(1 - v * v)
    P = [rho, W * v, 0, 0, p, 0, 0, 0, 0]
    _, _, lam = O.phys_flux(par, 0.0, 0.0, P, 0)
    h = 1 + GAM / (GAM - 1) * p / rho
    cs = math.sqrt(GAM * p / (rho * h))
    assert lam[0] == pytest.approx((v - cs) / (1 - v * cs), rel=1e-13, abs=1e-15)
    assert lam[1] == pytest.approx((v + cs) / (1 + v * cs), rel=1e-13, abs=1e-15)


def test_flat_alfven_limit_speed():
    """Cold, strongly magnetised plasma at rest: the fast bound tends to the Alfven speed
    c_a^2 = b^2 / (rho h + b^2) along and across the field."""
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    P = [1.0, 0, 0, 0, 1e-12, 2.0, 0, 0, 0]
    _, _, lam = O.phys_flux(par, 0.0, 0.0, P, 0)
    assert lam[1] == pytest.approx(math.sqrt(4.0 / 5.0), rel=1e-9)
    assert lam[0] == pytest.approx(-math.sqrt(4.0 / 5.0), rel=1e-9)


@pytest.mark.parametrize("x1,x2,m,P", sample(3, 40))
def test_con2prim_round_trip(x1, x2, m, P):
    U = O.p2c(ks(), x1, x2, P)
    guess = P.copy()
    guess[0] *= 1.3
    guess[4] *= 0.6
    guess[1:4] *= 0.8
    Pr, info = O.c2p(ks(), x1, x2, U, guess)
    assert info["fail"] == 0 and info["floored"] == 0
    assert info["iters"] <= 50
    assert np.allclose(Pr[[0, 4]], P[[0, 4]], rtol=1e-9)
    W = math.sqrt(1 + P[1:4] @ m["g"] @ P[1:4])
    assert np.allclose(Pr[1:4], P[1:4], rtol=1e-9, atol=1e-10 * W)
    assert np.array_equal(Pr[5:8], U[5:8] / m["sqrtg"]) and Pr[8] == P[8]


@pytest.mark.parametrize("x1,x2,m,P", sample(4, 20, wmax=3.0, smax=1.0))
def test_con2prim_round_trip_tight(x1, x2, m, P):
    """Moderate states converge to round-off (the tolerance is 1e-13 plus one more step)."""
    U = O.p2c(ks(), x1, x2, P)
    Pr, info = O.c2p(ks(), x1, x2, U, P)
    assert info["fail"] == 0
    assert np.allclose(Pr[[0, 4]], P[[0, 4]], rtol=1e-12)
    assert np.allclose(Pr[1:4], P[1:4], rtol=1e-11, atol=1e-13)


def test_con2prim_zero_momentum_closed_form():
    """S_i = 0: v = 0, so xi = Gamma (tau + D - B^2/2) - (Gamma - 1) D and p = (Gamma-1)(tau - B^2/2)."""
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    D, tau, B = 0.8, 2.5, np.array([0.3, -0.4, 0.5])
    B2 = B @ B
    U = np.concatenate([[D], [0, 0, 0], [tau], B, [0.0]])
    Pr, info = O.c2p(par, 0, 0, U, [1.0, 0.1, 0.1, 0.1, 1.0, 0, 0, 0, 0])
    assert info["fail"] == 0
    assert Pr[0] == pytest.approx(D, rel=1e-14)
    assert Pr[4] == pytest.approx((GAM - 1) * (tau - 0.5 * B2), rel=1e-13)
    assert np.allclose(Pr[1:4], 0, atol=1e-15)


def test_con2prim_reduces_to_hydro_when_unmagnetised():
    """B = 0 in flat space: compare with an independent root of the hydro pressure equation
    p = (Gamma-1)(E - S v - D/W) ... solved with brentq on p (a textbook SR-hydro inversion)."""
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    P = np.array([0.3, 2.0, -1.0, 0.5, 0.9, 0, 0, 0, 0])
    U = O.p2c(par, 0, 0, P)
    D, S, E = U[0], np.linalg.norm(U[1:4]), U[4] + U[0]

    def resid(p):
        v = S / (E + p)
        W = 1 / math.sqrt(1 - v * v)
        rho = D / W
        eps = (E + p - D * W - p * W * W) / (D * W)   # specific internal energy from the energy equation
        return (GAM - 1) * rho * eps - p
    p_root = optimize.brentq(resid, 1e-8, 100.0, xtol=1e-15, rtol=1e-15)
    Pr, info = O.c2p(par, 0, 0, U, P * 1.1)
    assert info["fail"] == 0
    assert Pr[4] == pytest.approx(p_root, rel=1e-12)


@pytest.mark.parametrize("x1,x2,m,P", sample(5, 10, wmax=5.0, smax=10.0))
def test_con2prim_against_brute_force_root(x1, x2, m, P):
    """Solve prim2con_covariant(P) = U for the 5 fluid unknowns with a generic root finder,
    using the 4-tensor construction (not the oracle's inversion formulas)."""
    U = O.p2c(ks(), x1, x2, P)
    Pr, info = O.c2p(ks(), x1, x2, U, P)
    assert info["fail"] == 0

    def resid(y):
        Q = P.copy()
        Q[0] = math.exp(y[0])
        Q[1:4] = y[1:4]
        Q[4] = math.exp(y[4])
        Uc = cov.conserved(m, Q, GAM)
        return (Uc[:5] - U[:5]) / np.abs(U[:5]).max()
    y0 = np.concatenate([[math.log(P[0] * 1.05)], P[1:4] * 0.97, [math.log(P[4] * 0.95)]])
    sol = optimize.root(resid, y0, method="hybr", tol=1e-14)
    assert np.abs(resid(sol.x)).max() < 1e-11
    assert math.exp(sol.x[0]) == pytest.approx(Pr[0], rel=1e-8)
    assert math.exp(sol.x[4]) == pytest.approx(Pr[4], rel=1e-7)


def test_con2prim_failures_keep_the_guess():
    par = ks()
    x1, x2 = math.log(6.0), 1.0
    guess = np.array([0.5, 0.1, 0.0, 0.02, 0.05, 0.01, 0.0, 0.0, 0.0])
    bad_D = O.p2c(par, x1, x2, guess)
    bad_D[0] = -1.0
    nan_U = O.p2c(par, x1, x2, guess)
    nan_U[4] = float("nan")
    # momentum far above the energy: no physical root with v < 1
    superluminal = O.p2c(par, x1, x2, guess)
    superluminal[1] = 50.0 * superluminal[4]
    for U in (bad_D, nan_U, superluminal):
        Pr, info = O.c2p(par, x1, x2, U, guess)
        assert info["fail"] == 1
        assert np.array_equal(Pr, guess)


def test_con2prim_floors():
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART, rho_floor=1e-4, p_floor=1e-6, w_max=5.0)
    lowrho = np.array([1e-6, 0.1, 0, 0, 1e-3, 0, 0, 0, 0])
    Pr, info = O.c2p(par, 0, 0, O.p2c(par, 0, 0, lowrho), lowrho)
    assert info["fail"] == 0 and info["floored"] == 1 and Pr[0] == 1e-4
    fast = np.array([1.0, 20.0, 0, 0, 1.0, 0, 0, 0, 0])   # W = sqrt(401) > 5
    Pr, info = O.c2p(par, 0, 0, O.p2c(par, 0, 0, fast), fast)
    assert info["floored"] == 1
    assert math.sqrt(1 + Pr[1] ** 2) == pytest.approx(5.0, rel=1e-13)
