"""Pins of reconstruction, the Riemann/GLM face flux and the geometric sources."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import covariant as cov

GAM = 4.0 / 3.0
MC, PPM = I.RECON_MC, I.RECON_PPM


# --- reconstruction -------------------------------------------------------------------
@pytest.mark.parametrize("method", [MC, PPM])
@pytest.mark.parametrize("a,b", [(1.0, 0.5), (-3.0, 2.0), (0.2, -0.7)])
def test_exact_on_linear_data(method, a, b):
    q = a + b * np.arange(6)               # cells i-3..i+2, face at i-1/2 = position 2.5
    qL, qR = O.recon_face(method, q)
    assert qL == pytest.approx(a + 2.5 * b, rel=1e-14)
    assert qR == pytest.approx(a + 2.5 * b, rel=1e-14)


def test_ppm_interface_exact_for_cubic_cell_averages():
    """Unlimited PPM interface value (7/12, -1/12 stencil) is exact for cell averages of a cubic."""
    f = lambda x: 1.0 + x + 0.1 * x * x + 0.02 * x ** 3
    F = lambda x: x + x * x / 2 + 0.1 * x ** 3 / 3 + 0.02 * x ** 4 / 4
    h = 0.1
    x0 = 0.3
    edges = x0 + h * np.arange(7)
    avg = (F(edges[1:]) - F(edges[:-1])) / h     # cells i-3..i+2
    qL, qR = O.recon_face(PPM, avg)
    face = edges[3]
    assert qL == pytest.approx(f(face), rel=1e-13)
    assert qR == pytest.approx(f(face), rel=1e-13)


@pytest.mark.parametrize("method", [MC, PPM])
def test_face_values_are_bounded_by_neighbours(method):
    rng = np.random.default_rng(11)
    for _ in range(2000):
        q = rng.standard_normal(6) * rng.choice([1e-3, 1.0, 1e3])
        qL, qR = O.recon_face(method, q)
        # left state belongs to cell i-1 (index 2), right state to cell i (index 3)
        lo_l, hi_l = min(q[1:4]), max(q[1:4])
        lo_r, hi_r = min(q[2:5]), max(q[2:5])
        tol = 1e-14 * np.abs(q).max()
        assert lo_l - tol <= qL <= hi_l + tol
        assert lo_r - tol <= qR <= hi_r + tol
        if method == MC:
            lo, hi = min(q[2], q[3]), max(q[2], q[3])
            assert lo - tol <= qL <= hi + tol and lo - tol <= qR <= hi + tol


def test_extremum_is_flattened():
    q = np.array([0.0, 1.0, 3.0, 1.0, 0.5, 0.2])   # cell i-1 (=3.0) is a local maximum
    qL, _ = O.recon_face(PPM, q)
    assert qL == 3.0
    qL, _ = O.recon_face(MC, q)
    assert qL == 3.0


# --- Riemann + GLM --------------------------------------------------------------------
def ks():
    return I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=I.SPIN)


@pytest.mark.parametrize("flux", [I.FLUX_HLL, I.FLUX_TVDLF])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_consistency_equal_states(flux, d):
    rng = np.random.default_rng(20 + d)
    par = I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=I.SPIN, flux=flux)
    x1, x2 = 1.3, 0.9
    m = O.metric(par, x1, x2)
    P = cov.random_prim(rng, 4.0, 5.0, m["g"])
    ch = 0.7
    F, lam = O.riemann(par, x1, x2, d, P, P, ch)
    U, Fp, lm = O.phys_flux(par, x1, x2, P, d)
    mask = np.ones(9, bool)
    mask[[5 + d, 8]] = False
    assert np.allclose(F[mask], Fp[mask], rtol=1e-14, atol=1e-15 * np.abs(Fp).max())
    assert F[5 + d] == pytest.approx(P[8], rel=1e-15)
    assert F[8] == pytest.approx(ch * ch * m["sqrtg"] * P[5 + d], rel=1e-14)
    assert lam == pytest.approx(max(abs(lm[0]), abs(lm[1])), rel=0)


def test_hll_supersonic_upwinds():
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART, flux=I.FLUX_HLL)
    W = 1 / math.sqrt(1 - 0.95 ** 2)
    PL = [1.0, W * 0.95, 0, 0, 1e-3, 0.0, 0.1, 0, 0]
    PR = [0.5, W * 0.95, 0, 0, 2e-3, 0.0, 0.2, 0, 0]
    F, _ = O.riemann(par, 0, 0, 0, PL, PR, 1.0)
    _, FL, lamL = O.phys_flux(par, 0, 0, PL, 0)
    _, _, lamR = O.phys_flux(par, 0, 0, PR, 0)
    assert lamL[0] > 0 and lamR[0] > 0
    assert np.allclose(F[:5], FL[:5], rtol=1e-14, atol=0)
    assert np.allclose(F[6:8], FL[6:8], rtol=1e-14, atol=0)


def test_glm_exact_solve_satisfies_characteristics():
    """psi + c_h B~ is carried right, psi - c_h B~ is carried left at speed c_h."""
    par = ks()
    x1, x2, d, ch = 0.8, 1.4, 1, 0.63
    m = O.metric(par, x1, x2)
    PL = np.array([1.0, 0.1, 0.02, 0.01, 0.3, 0.2, 0.11, -0.3, 0.05])
    PR = np.array([1.0, 0.1, 0.02, 0.01, 0.3, 0.2, -0.07, -0.3, -0.02])
    F, _ = O.riemann(par, x1, x2, d, PL, PR, ch)
    psi_s, b_s = F[5 + d], F[8] / ch ** 2
    sg = m["sqrtg"]
    assert psi_s + ch * b_s == pytest.approx(PL[8] + ch * sg * PL[5 + d], rel=1e-13)
    assert psi_s - ch * b_s == pytest.approx(PR[8] - ch * sg * PR[5 + d], rel=1e-13)


def test_tvdlf_mirror_symmetry():
    """Reflecting x -> -x maps the flux of a mirrored problem to minus the mirrored flux."""
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART, flux=I.FLUX_TVDLF)
    PL = np.array([1.0, 0.3, 0.1, 0.0, 1.0, 0.5, 0.2, 0.1, 0.01])
    PR = np.array([0.2, -0.1, 0.4, 0.2, 0.3, 0.5, -0.2, 0.3, -0.02])
    mir = lambda P: P * np.array([1, -1, 1, 1, 1, -1, 1, 1, 1])   # psi is a scalar
    F, _ = O.riemann(par, 0, 0, 0, PL, PR, 1.0)
    Fm, _ = O.riemann(par, 0, 0, 0, mir(PR), mir(PL), 1.0)
    sgn = np.array([-1, 1, -1, -1, -1, 1, -1, -1, -1])   # odd/even parity of each flux component
    assert np.allclose(Fm, sgn * F, rtol=1e-13, atol=1e-15)


# --- sources --------------------------------------------------------------------------
def christoffel0(Gi, dG):
    """Gamma^0_{mu nu} from the inverse metric and d_lambda g_{mu nu} (dG[lambda])."""
    out = np.zeros((4, 4))
    for mu in range(4):
        for nu in range(4):
            out[mu, nu] = 0.5 * sum(Gi[0, l] * (dG[mu][l, nu] + dG[nu][l, mu] - dG[l][mu, nu])
                                    for l in range(4))
    return out


@pytest.mark.parametrize("seed", range(8))
def test_sources_equal_covariant_christoffel_form(seed):
    rng = np.random.default_rng(100 + seed)
    par = ks()
    x_lo, x_hi = I.ks_domain()
    x1 = rng.uniform(x_lo[0], 2.5)
    x2 = rng.uniform(x_lo[1], x_hi[1])
    m = O.metric(par, x1, x2)
    P = cov.random_prim(rng, 3.0, 3.0, m["g"])
    U = O.p2c(par, x1, x2, P)
    S = O.sources(par, x1, x2, P, U, 0.37)
    f = cov.fluid(m, P, GAM)
    dG = cov.metric_derivs_fd(lambda a, b: O.metric(par, a, b), x1, x2)
    sqrt_mg = m["alpha"] * cov.sqrt_gamma(m)
    T = f["T"]
    mom = np.array([0.5 * sqrt_mg * np.sum(T * dG[1 + j]) for j in range(3)])
    dalpha = np.array([0.0, m["da"][0], m["da"][1], 0.0])
    # alpha derivatives by differences too, to keep the check independent
    h = 1e-4
    for ax in (0, 1):
        e = (h, 0) if ax == 0 else (0, h)
        dalpha[1 + ax] = (O.metric(par, x1 + e[0], x2 + e[1])["alpha"]
                          - O.metric(par, x1 - e[0], x2 - e[1])["alpha"]) / (2 * h)
    G0 = christoffel0(f["Gi"], dG)
    en = sqrt_mg * (T[:, 0] @ dalpha - m["alpha"] * np.sum(T * G0))
    scale = np.abs(np.concatenate([mom, [en]])).max()
    assert np.allclose(S[1:4], mom, rtol=1e-7, atol=1e-8 * scale)
    assert S[4] == pytest.approx(en, rel=1e-7, abs=1e-8 * scale)
    assert S[0] == 0 and not S[5:8].any()
    assert S[8] == -0.37 * U[8]


def test_flat_space_has_only_glm_damping():
    par = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    P = np.array([1.0, 0.3, 0.1, 0.2, 0.5, 0.1, 0.2, 0.3, 0.4])
    U = O.p2c(par, 0, 0, P)
    S = O.sources(par, 0.1, 0.2, P, U, 2.0)
    assert not S[:8].any() and S[8] == -0.8
