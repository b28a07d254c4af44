"""Pins of the oracle's entropy field and entropy-based inversion backup."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import covariant as cov
from tests.test_oracle_integration import wave_case

GAM = 4.0 / 3.0


def ks(**kw):
    return I.base_params(metric=I.METRIC_KS_SPH_LOGR, spin=I.SPIN, entropy=1, **kw)


def with_k(P):
    return np.concatenate([P, [P[4] / P[0] ** GAM]])


def sample(seed, n, wmax, smax, pmin=-3):
    rng = np.random.default_rng(seed)
    x_lo, x_hi = I.ks_domain()
    out = []
    for _ in range(n):
        x1 = rng.uniform(x_lo[0], x_hi[0])
        x2 = rng.uniform(x_lo[1], x_hi[1])
        m = O.metric(ks(), x1, x2)
        P = cov.random_prim(rng, wmax, smax, m["g"])
        P[4] = P[0] * 10 ** rng.uniform(pmin, 1)
        out.append((x1, x2, m, with_k(P)))
    return out


@pytest.mark.parametrize("x1,x2,m,P", sample(11, 30, wmax=40.0, smax=1e4, pmin=-6))
def test_entropy_inversion_recovers_the_state(x1, x2, m, P):
    """prim2con (a separate computation) then the entropy root gives the state back,
    also at high Lorentz factor, magnetisation up to 1e4 and p/rho down to 1e-6."""
    U = O.p2c(ks(), x1, x2, P)
    assert U[9] == U[0] * P[9]
    Pr = O.c2p_entropy(ks(), x1, x2, U, Wguess=1.0)
    assert Pr is not None
    W = math.sqrt(1 + P[1:4] @ m["g"] @ P[1:4])
    assert Pr[0] == pytest.approx(P[0], rel=1e-9)
    assert Pr[4] == pytest.approx(P[4], rel=1e-8)
    assert np.allclose(Pr[1:4], P[1:4], rtol=1e-8, atol=1e-9 * W)
    assert Pr[9] == U[9] / U[0]


@pytest.mark.parametrize("x1,x2,m,P", sample(12, 8, wmax=10.0, smax=100.0))
def test_entropy_root_satisfies_the_conserved_relations(x1, x2, m, P):
    """The backup's state reproduces D, S_i and B through the covariant stress-energy
    construction and has p = K rho^gamma: exactly what it is defined to satisfy."""
    U = O.p2c(ks(), x1, x2, P)
    U[9] *= 1.3                                  # a different entropy than the state's
    Pr = O.c2p_entropy(ks(), x1, x2, U, Wguess=2.0)
    assert Pr is not None
    Uc = cov.conserved(m, Pr[:9], GAM)
    for q in (0, 1, 2, 3):
        assert Uc[q] == pytest.approx(U[q], rel=1e-10, abs=1e-12 * np.abs(U[1:4]).max())
    assert np.allclose(Uc[5:8], U[5:8], rtol=1e-13)
    assert Pr[4] == pytest.approx(U[9] / U[0] * Pr[0] ** GAM, rel=1e-13)


def test_entropy_root_is_unique_and_bracketed():
    """The residual changes sign once on [1, inf): a dense scan of W through the
    covariant construction finds one sign change, at the backup's root."""
    x1, x2 = math.log(8.0), 1.1
    m = O.metric(ks(), x1, x2)
    P = with_k(np.array([0.2, 0.15, 0.02, -0.3, 0.05, 0.4, 0.01, 0.2, 0.0]))
    U = O.p2c(ks(), x1, x2, P)
    Pr = O.c2p_entropy(ks(), x1, x2, U)
    K = U[9] / U[0]
    sg = m["sqrtg"]
    D, S = U[0] / sg, U[1:4] / sg
    Sn = math.sqrt(S @ m["gi"] @ S)

    def resid(W):
        # momentum magnitude of the state with this W, rho = D/W, p = K rho^gamma and
        # the velocity direction of the true state, from the stress-energy construction
        rho = D / W
        Q = P[:9].copy()
        Q[0], Q[4] = rho, K * rho ** GAM
        Q[1:4] = P[1:4] * math.sqrt((W * W - 1) / (P[1:4] @ m["g"] @ P[1:4]))
        Uc = cov.conserved(m, Q, GAM)
        return math.sqrt(Uc[1:4] @ m["gi"] @ Uc[1:4]) / sg - Sn
    Ws = np.linspace(1.0, 10.0, 2001)
    r = np.array([resid(w) for w in Ws])
    changes = np.nonzero(np.diff(np.sign(r)))[0]
    assert len(changes) == 1
    Wtrue = math.sqrt(1 + P[1:4] @ m["g"] @ P[1:4])
    assert Ws[changes[0]] <= Wtrue <= Ws[changes[0] + 1]
    assert math.sqrt(1 + Pr[1:4] @ m["g"] @ Pr[1:4]) == pytest.approx(Wtrue, rel=1e-10)


def test_backup_engages_only_when_the_energy_inversion_fails():
    x1, x2 = math.log(6.0), 1.0
    P = with_k(np.array([0.5, 0.1, 0.0, 0.02, 0.05, 0.01, 0.0, 0.0, 0.0]))
    U = O.p2c(ks(), x1, x2, P)
    guess = P * 1.1
    # consistent state: the energy inversion succeeds, the backup is not used
    Pr, info = O.c2p(ks(), x1, x2, U, guess)
    assert info == dict(fail=0, iters=info["iters"], floored=0, backup=0)
    # energy far below what the density and momentum need: no root of the energy
    # relation with p >= 0, so the entropy root is taken
    Ub = U.copy()
    Ub[4] = -0.5 * U[0]
    Pr, info = O.c2p(ks(), x1, x2, Ub, guess)
    assert info["fail"] == 0 and info["backup"] == 1
    assert np.allclose(Pr, P, rtol=1e-9, atol=1e-12)
    # without the entropy field the same state fails and keeps the guess
    Pr0, info0 = O.c2p(dict(ks(), entropy=0), x1, x2, Ub[:9], guess[:9])
    assert info0["fail"] == 1 and np.array_equal(Pr0, guess[:9])
    # a non-positive entropy leaves nothing to invert
    Ub[9] = -1.0
    Pr, info = O.c2p(ks(), x1, x2, Ub, guess)
    assert info["fail"] == 1 and info["backup"] == 0 and np.array_equal(Pr, guess)


def test_entropy_field_is_passive():
    """With no cell needing the backup, carrying the entropy field changes none of the
    nine GRMHD rows by a single bit."""
    c = I.case_torus(2, n=(32, 16, 16), bs=8)
    ce = I.with_entropy(c)
    G0, G1 = O.OracleGrid(c.params, c.blocks), O.OracleGrid(ce.params, ce.blocks)
    U0, P0 = G0.run(c.prim, 3)
    U1, P1 = G1.run(ce.prim, 3)
    assert G1.stats()["c2p_backup"] == 0 and G1.stats()["c2p_fail"] == G0.stats()["c2p_fail"]
    idx = G0.interior_index()
    assert np.array_equal(U0[:, idx], U1[:9, idx])
    assert np.array_equal(P0[:, idx], P1[:9, idx])
    assert np.isfinite(P1[9, idx]).all() and (P1[9, idx] > 0).all()


def test_entropy_is_conserved_with_periodic_boundaries():
    c = I.with_entropy(I.case1(n=32))
    G = O.OracleGrid(c.params, c.blocks)
    U0, _ = G.init(c.prim)
    U, P = G.run(c.prim, 10)
    idx = G.interior_index()
    before, after = math.fsum(U0[9, idx]), math.fsum(U[9, idx])
    assert abs(after - before) <= 1e-13 * math.fsum(np.abs(U0[9, idx]))
    assert after != 0.0


def test_uniform_entropy_ratio_is_kept():
    """K uniform: the entropy flux is K times the mass flux at every face, so U[9] / U[0]
    stays K to rounding while the flow itself is not uniform."""
    c = I.with_entropy(I.case1(n=32))
    c.prim[9] = 0.37
    G = O.OracleGrid(c.params, c.blocks)
    U, P = G.run(c.prim, 10)
    idx = G.interior_index()
    assert np.abs(U[9, idx] / U[0, idx] - 0.37).max() <= 1e-14
    assert np.ptp(U[0, idx]) > 0.05


@pytest.mark.parametrize("recon,order", [(I.RECON_MC, 1.8), (I.RECON_PPM, 1.85)])
def test_entropy_converges_on_advected_wave(recon, order):
    """Contact wave with uniform p: K = p / rho^gamma translates with the flow; the
    evolved field converges to it at second order."""
    errs = []
    T = 0.4
    for n in (32, 64, 128):
        params, blocks, prim, v = wave_case(n, recon)
        params = dict(params, entropy=1)
        prim = np.vstack([prim, (prim[4] / prim[0] ** GAM)[None, :]])
        G = O.OracleGrid(params, blocks)
        U, P = G.init(prim)
        dt = 0.25 / n
        nsteps = int(round(T / dt))
        G.set_dt(dt)
        U1, P1 = np.zeros_like(U), np.zeros_like(P)
        for _ in range(nsteps):
            G.rk2_step(U, P, U1, P1)
        K = G.unpack(P)[9].reshape(2, 4, n // 2).transpose(1, 0, 2).reshape(4, n)[0]
        x = (np.arange(n) + 0.5) / n
        exact = 1.0 / (1.0 + 0.2 * np.sin(2 * math.pi * (x - v * nsteps * dt))) ** GAM
        errs.append(np.abs(K - exact).mean())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= order, (errs, rates)


def test_entropy_grid_restrictions():
    c = I.with_entropy(I.case_tree(n0=32, bs=8, levels=2))
    with pytest.raises(ValueError):
        O.OracleGrid(c.params, c.blocks)
    u = I.with_entropy(I.case1(n=32))
    with pytest.raises(ValueError):
        O.OracleGrid(dict(u.params, gamma_ad=2.5), u.blocks)
