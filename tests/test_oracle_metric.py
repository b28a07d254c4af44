"""Pins of the oracle's spacetime metric (Kerr-Schild, x1 = ln r) against closed forms."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import covariant as cov

A = I.SPIN


def ks_params(spin=A):
    return I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=spin)


def points():
    rng = np.random.default_rng(7)
    x_lo, x_hi = I.ks_domain()
    for _ in range(25):
        yield rng.uniform(x_lo[0], x_hi[0]), rng.uniform(x_lo[1], x_hi[1])


@pytest.mark.parametrize("x1,x2", list(points()))
def test_determinant_and_lapse(x1, x2):
    m = O.metric(ks_params(), x1, x2)
    r, th = math.exp(x1), x2
    sig = r * r + A * A * math.cos(th) ** 2
    sqrt_minus_g = r * sig * math.sin(th)          # sqrt(-g) of Kerr-Schild times dr/dx1 = r
    G = cov.g4(m)
    assert np.linalg.det(G) == pytest.approx(-sqrt_minus_g ** 2, rel=1e-12)
    assert m["alpha"] * m["sqrtg"] == pytest.approx(sqrt_minus_g, rel=1e-13)
    assert m["sqrtg"] == pytest.approx(math.sqrt(np.linalg.det(m["g"])), rel=1e-12)
    assert np.allclose(m["gi"] @ m["g"], np.eye(3), atol=1e-12)


@pytest.mark.parametrize("x1,x2", list(points())[:10])
def test_inverse_four_metric_closed_form(x1, x2):
    """Kerr-Schild inverse metric: g^tt = -(1+z), g^tr = z, g^rr = Delta/Sigma, g^r phi = a/Sigma,
    g^theta theta = 1/Sigma, g^phi phi = 1/(Sigma sin^2), others 0; x1 = ln r rescales r by 1/r."""
    m = O.metric(ks_params(), x1, x2)
    Gi = np.linalg.inv(cov.g4(m))
    r, th = math.exp(x1), x2
    sig = r * r + A * A * math.cos(th) ** 2
    z = 2 * r / sig
    delta = r * r - 2 * r + A * A
    exp = np.zeros((4, 4))
    exp[0, 0] = -(1 + z)
    exp[0, 1] = exp[1, 0] = z / r
    exp[1, 1] = delta / sig / r ** 2
    exp[1, 3] = exp[3, 1] = A / sig / r
    exp[2, 2] = 1 / sig
    exp[3, 3] = 1 / (sig * math.sin(th) ** 2)
    assert np.allclose(Gi, exp, rtol=1e-11, atol=1e-12)
    # 3+1 relations for the inverse
    assert Gi[0, 0] == pytest.approx(-1 / m["alpha"] ** 2, rel=1e-12)
    assert np.allclose(Gi[0, 1:], m["beta"] / m["alpha"] ** 2, atol=1e-12)
    assert np.allclose(Gi[1:, 1:], m["gi"] - np.outer(m["beta"], m["beta"]) / m["alpha"] ** 2, atol=1e-11)


def test_schwarzschild_limit():
    x1, x2 = math.log(3.7), 1.1
    m = O.metric(ks_params(0.0), x1, x2)
    r = 3.7
    assert m["alpha"] == pytest.approx(1 / math.sqrt(1 + 2 / r), rel=1e-14)
    assert m["beta"][0] * r == pytest.approx((2 / r) / (1 + 2 / r), rel=1e-14)
    assert m["g"][0, 0] / r ** 2 == pytest.approx(1 + 2 / r, rel=1e-14)
    assert m["g"][1, 1] == pytest.approx(r * r, rel=1e-14)
    assert m["g"][2, 2] == pytest.approx(r * r * math.sin(x2) ** 2, rel=1e-14)
    assert m["g"][0, 2] == 0.0


def test_minkowski():
    p = I.base_params(metric=I.METRIC_MINKOWSKI_CART)
    m = O.metric(p, 0.3, 0.4)
    assert m["alpha"] == 1.0 and m["sqrtg"] == 1.0
    assert np.array_equal(m["g"], np.eye(3)) and not m["dg"].any() and not m["da"].any()


@pytest.mark.parametrize("x1,x2", list(points())[:12])
def test_derivatives_against_finite_differences(x1, x2):
    p = ks_params()
    fn = lambda a, b: O.metric(p, a, b)
    m = fn(x1, x2)
    for j, axis in ((0, 0), (1, 1)):
        h = 1e-3
        def d(hh, q):
            e = (hh, 0.0) if axis == 0 else (0.0, hh)
            return (q(fn(x1 + e[0], x2 + e[1])) - q(fn(x1 - e[0], x2 - e[1]))) / (2 * hh)
        def rich(q):
            return (4 * d(h / 2, q) - d(h, q)) / 3
        assert m["da"][j] == pytest.approx(rich(lambda mm: mm["alpha"]), rel=1e-8, abs=1e-11)
        assert np.allclose(m["db"][j], rich(lambda mm: mm["beta"]), rtol=1e-8, atol=1e-11)
        assert np.allclose(m["dg"][j], rich(lambda mm: mm["g"]), rtol=1e-8, atol=1e-9)
    assert not m["dg"][2].any() and not m["db"][2].any() and m["da"][2] == 0.0
