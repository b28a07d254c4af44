"""Pins of the oracle's two-unknown Newton backup of the inversion (unknowns xi =
rho h W^2 and q = W^2 - 1; momentum and energy relations solved together).

* Both relations vanish at the (xi, W^2 - 1) of the state that generated U (computed
  here from the primitives and the 3-metric, not by the oracle's inversion).
* The analytic Jacobian equals central differences of the residuals.
* From perturbed guesses the iteration alone recovers the generating primitives.
* Without momentum the energy relation has the closed-form root
  xi = Gamma (tau + D - B^2 / 2) - (Gamma - 1) D.
* As a backup it does not invent a state where none exists (injected cells whose
  energy is below what their density needs), and where it does rescue a cell the
  1-D iteration gave up on, the result is a root of both relations.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import covariant as cov

GAM = 4.0 / 3.0


def ks(**kw):
    return I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=I.SPIN, **kw)


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


def xi_q(m, P):
    q = P[1:4] @ m["g"] @ P[1:4]           # W^2 - 1 = gamma_ij u~^i u~^j
    h = 1.0 + GAM / (GAM - 1.0) * P[4] / P[0]
    return P[0] * h * (1.0 + q), q


@pytest.mark.parametrize("x1,x2,m,P", sample(31, 20))
def test_relations_vanish_at_the_generating_state(x1, x2, m, P):
    U = O.p2c(ks(), x1, x2, P)
    xi, q = xi_q(m, P)
    F, _ = O.c2p_2d_residual(ks(), x1, x2, U, xi, q)
    sg = m["sqrtg"]
    scale = max(abs(U[4] / sg) + abs(U[0] / sg), xi) * max(xi, 1.0)
    assert abs(F[0]) <= 1e-11 * scale * xi and abs(F[1]) <= 1e-11 * scale, F


@pytest.mark.parametrize("x1,x2,m,P", sample(32, 12))
def test_jacobian_equals_central_differences(x1, x2, m, P):
    U = O.p2c(ks(), x1, x2, P)
    xi, q = xi_q(m, P)
    xi, q = 1.1 * xi, 0.9 * q          # away from the root
    _, J = O.c2p_2d_residual(ks(), x1, x2, U, xi, q)
    hx, hq = 1e-6 * xi, 1e-6 * max(q, 1e-3)
    Fpx, _ = O.c2p_2d_residual(ks(), x1, x2, U, xi + hx, q)
    Fmx, _ = O.c2p_2d_residual(ks(), x1, x2, U, xi - hx, q)
    Fpq, _ = O.c2p_2d_residual(ks(), x1, x2, U, xi, q + hq)
    Fmq, _ = O.c2p_2d_residual(ks(), x1, x2, U, xi, q - hq)
    Jfd = np.stack([(Fpx - Fmx) / (2 * hx), (Fpq - Fmq) / (2 * hq)], axis=1)
    assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-8 * np.abs(Jfd).max()), (J, Jfd)


@pytest.mark.parametrize("x1,x2,m,P", sample(33, 30))
def test_iteration_recovers_the_state_from_perturbed_guesses(x1, x2, m, P):
    U = O.p2c(ks(), x1, x2, P)
    guess = np.array(P, dtype=float)
    guess[0] *= 1.2
    guess[4] *= 0.8
    guess[1:4] *= 0.9
    got, nit = O.c2p_2d(ks(), x1, x2, U, guess)
    assert got is not None and nit <= 50
    assert np.allclose(got[:5], P[:5], rtol=1e-9, atol=1e-12 * np.abs(P[1:4]).max()), (got, P)
    assert np.array_equal(got[5:8], np.asarray(P[5:8])) or np.allclose(got[5:8], P[5:8], rtol=1e-14)


def test_no_momentum_closed_form():
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    P = np.array([0.7, 0.0, 0.0, 0.0, 0.3, 0.4, -0.2, 0.1, 0.0])
    U = O.p2c(par, 0.0, 0.0, P)
    B2 = P[5:8] @ P[5:8]
    xi = GAM * (U[4] + U[0] - 0.5 * B2) - (GAM - 1.0) * U[0]
    F, _ = O.c2p_2d_residual(par, 0.0, 0.0, U, xi, 0.0)
    assert abs(F[0]) <= 1e-15 and abs(F[1]) <= 1e-14 * xi
    got, _ = O.c2p_2d(par, 0.0, 0.0, U, P * np.array([1.3, 1, 1, 1, 0.5, 1, 1, 1, 1]))
    assert np.allclose(got[:5], P[:5], rtol=1e-12, atol=1e-14)


def test_backup_does_not_invent_states():
    """Energy below what the density needs (tau = -D/2): neither iteration has a root;
    with the backup enabled the cell still fails and keeps its guess."""
    for x1, x2, m, P in sample(34, 15):
        par = ks(c2p_2d=1)
        U = O.p2c(par, x1, x2, P)
        U[4] = -0.5 * U[0]
        out, info = O.c2p(par, x1, x2, U, P)
        assert info["fail"] == 1 and info["backup"] == 0
        assert np.array_equal(out[:9], np.asarray(P[:9], dtype=float))


def extreme_cases(seed=35, n=600):
    """Strongly magnetised, fast states with guesses off by large factors: the regime
    where the one-unknown iteration gives up."""
    rng = np.random.default_rng(seed)
    x_lo, x_hi = I.ks_domain()
    out = []
    for _ in range(n):
        x1 = rng.uniform(x_lo[0], x_hi[0])
        x2 = rng.uniform(x_lo[1], x_hi[1])
        m = O.metric(ks(), x1, x2)
        P = cov.random_prim(rng, 40.0, 1e4, m["g"])
        P[4] = P[0] * 10 ** rng.uniform(-5, -2)
        g = np.array(P, dtype=float)
        g[0] *= 10 ** rng.uniform(-2, 2)
        g[4] *= 10 ** rng.uniform(-2, 2)
        g[1:4] *= rng.uniform(0.0, 1.0)
        out.append((x1, x2, m, P, g))
    return out


def test_backup_rescues_are_roots_of_both_relations():
    one_fail = rescued = close = 0
    for x1, x2, m, P, g in extreme_cases():
        par1 = ks(c2p_maxit=50)
        U = O.p2c(par1, x1, x2, P)
        _, info1 = O.c2p(par1, x1, x2, U, g)
        if not info1["fail"]:
            continue
        one_fail += 1
        par2 = ks(c2p_maxit=50, c2p_2d=1)
        out, info2 = O.c2p(par2, x1, x2, U, g)
        if info2["fail"]:
            assert np.array_equal(out[:9], g[:9])
            continue
        rescued += 1
        assert info2["backup"] == 1
        # the rescued state is a root of both relations (unfloored cells)
        if not info2["floored"]:
            xi, q = xi_q(m, out)
            F, _ = O.c2p_2d_residual(par2, x1, x2, U, xi, q)
            sg = m["sqrtg"]
            scale = (abs(U[4]) + abs(U[0])) / sg + xi
            assert abs(F[1]) <= 1e-8 * scale and abs(F[0]) <= 1e-8 * scale * scale
        if np.allclose(out[:5], P[:5], rtol=1e-6, atol=1e-10):
            close += 1
    print(f"\nextreme states: 1-D iteration failed on {one_fail}; the 2-D backup rescued {rescued}, "
          f"{close} of them within 1e-6 of the generating state")
    assert one_fail > 0
