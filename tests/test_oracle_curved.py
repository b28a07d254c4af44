"""Pins of the oracle in curved spacetime and of its time-step rule, each against
something the oracle does not compute itself:

* the wave-speed bounds lambda+- along each direction in Kerr-Schild are the roots of
  the covariant isotropic dispersion relation omega^2 = c_e^2 (k.k + omega^2) with
  omega = k_mu u^mu for the covector k = (-lambda, e_d) (the fast-speed estimate of
  the HARM family of codes), built from the 4-metric and u^mu; in the limit
  c_e -> 1 they are the light cone -beta^d +- alpha sqrt(gamma^dd);
* the time step, c_h and kappa of a uniform flat state in closed form, with the
  speeds from a Lorentz boost of the rest-frame sound (or fast) wave;
* the curved-space finite-volume assembly (face-metric positions, flux divergence
  against the geometric sources): Michel's stationary accretion flow onto a
  Schwarzschild hole (a = 0 in Kerr-Schild coordinates) with a split-monopole radial
  field, which leaves the flow stationary, from scipy root-finding of the mass and
  Bernoulli constants; the one-substep residual (U(dt) - U_exact) / dt converges to
  zero at second order.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import covariant as cov

GAM = 4.0 / 3.0
NG = GAM / (GAM - 1.0)


def ks():
    return I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=I.SPIN)


def dispersion_roots(m, P, d):
    """Roots lambda of (1 - c^2) omega^2 - c^2 k.k = 0, omega = k_mu u^mu, k = (-lambda, e_d)."""
    f = cov.fluid(m, P, GAM)
    u, Gi = f["u"], f["Gi"]
    rhoh = f["rho"] * f["h"]
    cs2 = GAM * f["p"] / rhoh
    ca2 = f["b2"] / (rhoh + f["b2"])
    c2 = cs2 + ca2 - cs2 * ca2
    i = d + 1
    A = (1 - c2) * u[0] ** 2 - c2 * Gi[0, 0]
    Bq = -2 * (1 - c2) * u[0] * u[i] + 2 * c2 * Gi[0, i]
    Cq = (1 - c2) * u[i] ** 2 - c2 * Gi[i, i]
    disc = math.sqrt(Bq * Bq - 4 * A * Cq)
    r = sorted([(-Bq - disc) / (2 * A), (-Bq + disc) / (2 * A)])
    return np.array(r)


def ks_sample(seed, n, wmax=10.0, smax=100.0):
    rng = np.random.default_rng(seed)
    x_lo, x_hi = I.ks_domain()
    out = []
    for _ in range(n):
        x1 = rng.uniform(x_lo[0], x_hi[0])
        x2 = rng.uniform(x_lo[1], x_hi[1])
        m = O.metric(ks(), x1, x2)
        out.append((x1, x2, m, cov.random_prim(rng, wmax, smax, m["g"])))
    return out


@pytest.mark.parametrize("x1,x2,m,P", ks_sample(21, 30))
@pytest.mark.parametrize("d", [0, 1, 2])
def test_ks_speeds_are_roots_of_the_covariant_dispersion_relation(x1, x2, m, P, d):
    _, _, lam = O.phys_flux(ks(), x1, x2, P, d)
    ref = dispersion_roots(m, P, d)
    scale = max(abs(ref).max(), 1e-3)
    assert np.allclose(lam, ref, rtol=1e-10, atol=1e-12 * scale), (lam, ref)


@pytest.mark.parametrize("x1,x2,m,P", ks_sample(22, 12))
@pytest.mark.parametrize("d", [0, 1, 2])
def test_ks_speeds_tend_to_the_light_cone(x1, x2, m, P, d):
    """A cold, extremely magnetised state (c_e -> 1): the bounds approach the light
    cone of the 4-metric along d, -beta^d +- alpha sqrt(gamma^dd)."""
    P = np.array(P, dtype=float)
    P[4] = 1e-14 * P[0]
    P[5:8] *= 1e7 / math.sqrt(abs(P[5:8] @ m["g"] @ P[5:8]) / P[0] + 1e-300)
    _, _, lam = O.phys_flux(ks(), x1, x2, P, d)
    cone = -m["beta"][d] + np.array([-1.0, 1.0]) * m["alpha"] * math.sqrt(m["gi"][d, d])
    assert np.allclose(lam, cone, rtol=1e-6, atol=1e-6 * abs(cone).max()), (lam, cone)


# ----------------------------------------------------------------------------------
# Time step, c_h and kappa (uniform flat state)
# ----------------------------------------------------------------------------------
def boosted_speeds(v, c):
    """Largest |lambda| along the flow (relativistic velocity addition of v and c) and
    across it (Lorentz boost of a rest-frame wave of phase speed c whose lab wave
    vector is perpendicular to the flow)."""
    along = (abs(v) + c) / (1.0 + abs(v) * c)
    across = c * math.sqrt(1.0 - v * v) / math.sqrt(1.0 - v * v * c * c)
    return along, across


def flat_uniform(v, Bx, levels=(0,)):
    """3-D periodic flat box [0,1]x[0,2]x[0,0.5], level-0 cells 16x16x8, blocks of 8^3
    (one block per level listed), a uniform state moving along x."""
    params = I.base_params(metric=I.METRIC_MINKOWSKI_CART, ndim=3, nghost=3, x_lo=[0.0, 0.0, 0.0],
                           x_hi=[1.0, 2.0, 0.5], ncell0=[16, 16, 8], bc=[[I.BC_PERIODIC] * 2] * 3)
    blocks = np.array([[lv, 8, 8, 8, 0, 0, 0] for lv in levels], dtype=np.int32)
    rho, p = 1.3, 0.4
    W = 1.0 / math.sqrt(1.0 - v * v)
    n = 8 ** 3 * len(levels)
    prim = np.zeros((9, n))
    prim[0], prim[1], prim[4], prim[5] = rho, W * v, p, Bx
    return params, blocks, prim


@pytest.mark.parametrize("v", [0.0, 0.35, -0.8])
@pytest.mark.parametrize("Bx", [0.0, 0.9])
@pytest.mark.parametrize("levels", [(0,), (0, 1)])
def test_time_step_rule_closed_form(v, Bx, levels):
    params, blocks, prim = flat_uniform(v, Bx, levels)
    rho, p = prim[0, 0], prim[4, 0]
    h = 1.0 + NG * p / rho
    cs2 = GAM * p / (rho * h)
    # field along the flow: b^2 = B^2 / W^2 + (B.v)^2 = B^2 (1 - v^2 + v^2) = B^2
    b2 = Bx * Bx
    ca2 = b2 / (rho * h + b2)
    c = math.sqrt(cs2 + ca2 - cs2 * ca2)
    along, across = boosted_speeds(v, c)
    fine = max(levels)
    dx = np.array([1.0 / 16, 2.0 / 16, 0.5 / 8]) / 2 ** fine
    C = params["cfl"]
    dt = C / (along / dx[0] + across / dx[1] + across / dx[2])
    ch = C / (dt * (1 / dx).sum())
    kappa = params["glm_alpha"] * ch / dx.min()

    Og = O.OracleGrid(params, blocks)
    U, P = Og.init(prim)
    assert Og.state.dt_next == pytest.approx(dt, rel=1e-13)
    U1, P1 = np.zeros_like(U), np.zeros_like(P)
    Og.fill_ghosts(P)
    Og.substep(U, U, P, U1, P1, 0.0, 1.0)
    st = Og.stats()
    assert st["dt"] == pytest.approx(dt, rel=1e-13)
    assert st["ch"] == pytest.approx(ch, rel=1e-13)
    assert st["kappa"] == pytest.approx(kappa, rel=1e-13)
    # the face speeds of the uniform state are the cell speeds: the next step's dt
    # follows the same closed form
    assert st["dt_next"] == pytest.approx(dt, rel=1e-13)
    assert tuple(Og.state.lam) == pytest.approx((along, across, across), rel=1e-13)
    # the uniform state itself is preserved (the step changes nothing)
    idx = Og.interior_index()
    assert np.array_equal(U1[:, idx], U[:, idx])
    assert np.allclose(P1[:, idx], P[:, idx], rtol=1e-13, atol=1e-15)


def test_fixed_time_step_sets_ch_and_kappa():
    params, blocks, prim = flat_uniform(0.2, 0.0)
    Og = O.OracleGrid(params, blocks)
    U, P = Og.init(prim)
    Og.set_dt(1e-3)
    U1, P1 = np.zeros_like(U), np.zeros_like(P)
    Og.fill_ghosts(P)
    Og.substep(U, U, P, U1, P1, 0.0, 1.0)
    dx = np.array([1.0 / 16, 2.0 / 16, 0.5 / 8])
    st = Og.stats()
    assert st["dt"] == 1e-3 and st["dt_next"] == 1e-3
    assert st["ch"] == pytest.approx(params["cfl"] / (1e-3 * (1 / dx).sum()), rel=1e-14)
    assert st["kappa"] == pytest.approx(params["glm_alpha"] * st["ch"] / dx.min(), rel=1e-14)


# ----------------------------------------------------------------------------------
# Michel accretion with a split-monopole field in Kerr-Schild coordinates (a = 0)
# ----------------------------------------------------------------------------------
class Michel:
    """Polytropic (p = K rho^Gamma) transonic radial inflow onto a Schwarzschild hole,
    M = 1, sonic radius rc, rho(rc) = 1. Conserved along the flow: the mass flux
    rho u^r r^2 and the Bernoulli constant h^2 (1 - 2/r + (u^r)^2); at the sonic point
    (u^r)^2 = 1 / (2 rc) and c_s^2 = (u^r)^2 / (1 - 3 (u^r)^2)."""

    def __init__(self, rc=8.0):
        self.rc = rc
        uc2 = 1.0 / (2.0 * rc)
        cs2 = uc2 / (1.0 - 3.0 * uc2)
        theta = cs2 / (GAM - cs2 * NG)          # p / rho at the sonic point
        self.K = theta
        self.mdot = -math.sqrt(uc2) * rc * rc
        self.E = (1.0 + NG * theta) ** 2 * (1.0 - 2.0 / rc + uc2)

    def _f(self, lrho, r):
        rho = math.exp(lrho)
        h = 1.0 + NG * self.K * rho ** (GAM - 1.0)
        ur = self.mdot / (rho * r * r)
        return h * h * (1.0 - 2.0 / r + ur * ur) - self.E

    def at(self, r):
        """(rho, u^r) at radius r on the transonic branch (supersonic inside rc)."""
        lm = optimize.minimize_scalar(lambda lr: self._f(lr, r), bounds=(-20.0, 10.0), method="bounded",
                                      options=dict(xatol=1e-12)).x
        if r < self.rc:
            lr = optimize.brentq(self._f, -30.0, lm, args=(r,), xtol=1e-15, rtol=1e-15)
        else:
            lr = optimize.brentq(self._f, lm, 20.0, args=(r,), xtol=1e-15, rtol=1e-15)
        rho = math.exp(lr)
        return rho, self.mdot / (rho * r * r)


def michel_grid(N, B0=0.3, r0=2.5, r1=6.0, dth=0.5):
    x_lo = [math.log(r0), math.pi / 2 - dth, 0.0]
    x_hi = [math.log(r1), math.pi / 2 + dth, 2 * math.pi]
    params = I.base_params(ndim=2, spin=0.0, x_lo=x_lo, x_hi=x_hi, ncell0=[N, N, 1])
    blocks = np.array([[0, N, N, 1, 0, 0, 0]], dtype=np.int32)
    fl = Michel()
    dx = [(x_hi[e] - x_lo[e]) / N for e in range(2)]
    prim = np.zeros((9, N * N))
    radial = [fl.at(math.exp(x_lo[0] + (i + 0.5) * dx[0])) for i in range(N)]
    for j in range(N):
        x2 = x_lo[1] + (j + 0.5) * dx[1]
        for i in range(N):
            x1 = x_lo[0] + (i + 0.5) * dx[0]
            r = math.exp(x1)
            rho, ur = radial[i]
            m = O.metric(params, x1, x2)
            # u^t: Schwarzschild normalisation, then t_KS = t_BL + 2 ln(r/2 - 1)
            ut = math.sqrt(1.0 - 2.0 / r + ur * ur) / (1.0 - 2.0 / r) + 2.0 / (r - 2.0) * ur
            u1 = ur / r                                   # x1 = ln r
            ut1 = u1 + ut * m["beta"][0]                  # Eulerian W v^1
            W = math.sqrt(1.0 + m["g"][0, 0] * ut1 * ut1)
            assert abs(W - m["alpha"] * ut) <= 1e-12 * W  # the same 4-velocity
            # split monopole: sqrt(gamma) B^1 = B0 sin(theta), divergence-free
            prim[:, j * N + i] = [rho, ut1, 0.0, 0.0, fl.K * rho ** GAM, B0 * math.sin(x2) / m["sqrtg"], 0, 0, 0]
    return params, blocks, prim, x_lo, x_hi


def michel_residual(N, ncoarse=32):
    params, blocks, prim, x_lo, x_hi = michel_grid(N)
    Og = O.OracleGrid(params, blocks)
    U, P = Og.init(prim)
    dt = Og.state.dt_next
    U1, P1 = np.zeros_like(U), np.zeros_like(P)
    Og.substep(U, U, P, U1, P1, 0.0, 1.0)
    assert Og.stats()["c2p_fail"] == 0 and Og.stats()["floor_hits"] == 0
    idx = Og.interior_index()
    R = (U1[:, idx] - U[:, idx]) / dt
    Ui = U[:, idx]
    # a fixed physical region: 3 cells of the coarsest grid away from every boundary
    # (at least 3 cells at every resolution, so no stencil reaches a ghost cell)
    c1 = x_lo[0] + (np.arange(N) + 0.5) * (x_hi[0] - x_lo[0]) / N
    c2 = x_lo[1] + (np.arange(N) + 0.5) * (x_hi[1] - x_lo[1]) / N
    X1, X2 = [a.ravel() for a in np.meshgrid(c1, c2, indexing="xy")]
    b1, b2 = 3 * (x_hi[0] - x_lo[0]) / ncoarse, 3 * (x_hi[1] - x_lo[1]) / ncoarse
    sel = (X1 > x_lo[0] + b1) & (X1 < x_hi[0] - b1) & (X2 > x_lo[1] + b2) & (X2 < x_hi[1] - b2)
    scale = np.abs(Ui[:, sel]).mean(axis=1)
    # S_theta, S_phi, B^theta, B^phi and psi vanish in the exact state: measured
    # against |S_r| and |B~^r|
    scale[2] = scale[3] = scale[1]
    scale[6] = scale[7] = scale[8] = scale[5]
    return np.abs(R[:, sel]).mean(axis=1) / scale


@pytest.fixture(scope="module")
def michel_errors():
    return np.array([michel_residual(N) for N in (32, 64, 128)])


def test_michel_flow_residual_converges_at_second_order(michel_errors):
    e = michel_errors
    print("Michel residual (D, S1, S2, S3, tau, B1, B2, B3, psi) per resolution:\n", e)
    for q in (0, 1, 2, 4, 8):          # D, S_r, S_theta, tau, psi
        rates = np.log2(e[:-1, q] / e[1:, q])
        assert (rates >= 1.8).all(), (q, rates, e[:, q])
    # no phi momentum, no theta or phi field: those residuals vanish identically
    assert (e[:, [3, 6, 7]] == 0.0).all()
    # the radial field is transported exactly by the discrete scheme
    assert (e[:, 5] <= 1e-12).all()


def test_michel_state_is_the_flow_of_the_constants():
    """The root-found state keeps both constants along the radius (scipy's roots, not
    the oracle, are what the residual test measures against)."""
    fl = Michel()
    for r in (2.5, 4.0, 6.0, 12.0):
        rho, ur = fl.at(r)
        h = 1.0 + NG * fl.K * rho ** (GAM - 1.0)
        assert rho * ur * r * r == pytest.approx(fl.mdot, rel=1e-13)
        assert h * h * (1.0 - 2.0 / r + ur * ur) == pytest.approx(fl.E, rel=1e-13)
        assert (abs(ur) > math.sqrt(GAM * fl.K * rho ** (GAM - 1) / h)) == (r < fl.rc) or r == fl.rc
