"""Covariant (4-tensor) re-derivations used to pin the oracle's 3+1 formulas.

Everything here is built from the 4-metric and the stress-energy tensor
T^{mu nu} = (rho h + b^2) u^mu u^nu + (p + b^2/2) g^{mu nu} - b^mu b^nu of ideal MHD,
a different route from the oracle's Valencia expressions.
"""
import numpy as np


def g4(m):
    a, bu, g = m["alpha"], m["beta"], m["g"]
    bd = g @ bu
    G = np.zeros((4, 4))
    G[0, 0] = -a * a + bu @ bd
    G[0, 1:] = bd
    G[1:, 0] = bd
    G[1:, 1:] = g
    return G


def sqrt_gamma(m):
    return float(np.sqrt(np.linalg.det(m["g"])))


def fluid(m, P, gam):
    """u^mu, b^mu, T^{mu nu} for primitive vector P at a point with 3+1 metric m."""
    G = g4(m)
    Gi = np.linalg.inv(G)
    rho, ut, p, B = P[0], np.asarray(P[1:4]), P[4], np.asarray(P[5:8])
    W = np.sqrt(1.0 + ut @ m["g"] @ ut)
    u = np.concatenate([[W / m["alpha"]], ut - m["beta"] * W / m["alpha"]])
    ud = G @ u
    Bmu = np.concatenate([[0.0], B])
    b = (Bmu + (Bmu @ ud) * u) / W
    b2 = b @ G @ b
    h = 1.0 + gam / (gam - 1.0) * p / rho
    T = (rho * h + b2) * np.outer(u, u) + (p + 0.5 * b2) * Gi - np.outer(b, b)
    return dict(G=G, Gi=Gi, u=u, b=b, b2=b2, T=T, W=W, rho=rho, p=p, h=h)


def conserved(m, P, gam):
    """sqrt(gamma) (D, S_j, tau, B^i), psi from n_mu n_nu T^{mu nu} and -n_mu T^mu_j."""
    f = fluid(m, P, gam)
    al = m["alpha"]
    sg = sqrt_gamma(m)
    D = f["rho"] * al * f["u"][0]
    Tmix = f["T"] @ f["G"]           # T^mu_nu
    S = al * Tmix[0, 1:]
    tau = al * al * f["T"][0, 0] - D
    return np.concatenate([[sg * D], sg * S, [sg * tau], sg * np.asarray(P[5:8]), [P[8]]])


def fluxes(m, P, gam, d):
    """Coordinate fluxes along d: sqrt(-g) (rho u^d, T^d_j, alpha T^{0d} - rho u^d, b^j u^d - b^d u^j)."""
    f = fluid(m, P, gam)
    al = m["alpha"]
    sg = sqrt_gamma(m)
    sgg = al * sg
    i = d + 1
    Tmix = f["T"] @ f["G"]
    out = np.zeros(9)
    out[0] = sgg * f["rho"] * f["u"][i]
    out[1:4] = sgg * Tmix[i, 1:]
    out[4] = sgg * (al * f["T"][0, i] - f["rho"] * f["u"][i])
    for j in range(3):
        out[5 + j] = sgg * (f["b"][1 + j] * f["u"][i] - f["b"][i] * f["u"][1 + j])
    return out


def metric_derivs_fd(metric_fn, x1, x2, h=1e-3):
    """Richardson-extrapolated central differences of the 4-metric in x1 and x2 (x3: 0)."""
    def dfun(axis, hh):
        e = np.array([hh, 0.0]) if axis == 0 else np.array([0.0, hh])
        gp = g4(metric_fn(x1 + e[0], x2 + e[1]))
        gm = g4(metric_fn(x1 - e[0], x2 - e[1]))
        return (gp - gm) / (2 * hh)
    out = np.zeros((4, 4, 4))  # out[mu] = d_mu g
    for axis in (0, 1):
        out[1 + axis] = (4 * dfun(axis, h / 2) - dfun(axis, h)) / 3
    return out


def random_prim(rng, wmax=10.0, sigma_max=100.0, g=None):
    """A physical primitive state with Lorentz factor up to wmax and magnetisation up to sigma_max."""
    rho = 10 ** rng.uniform(-3, 0)
    p = rho * 10 ** rng.uniform(-3, 1)
    W = 1.0 + (wmax - 1.0) * rng.uniform() ** 2
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    g = np.eye(3) if g is None else g
    # scale the direction so that gamma_ij u~^i u~^j = W^2 - 1
    ut = n * np.sqrt((W * W - 1.0) / (n @ g @ n))
    bdir = rng.standard_normal(3)
    bdir /= np.sqrt(bdir @ g @ bdir)
    sigma = 10 ** rng.uniform(-3, np.log10(sigma_max))
    Bmag = np.sqrt(sigma * rho)
    P = np.zeros(9)
    P[0], P[1:4], P[4], P[5:8] = rho, ut, p, Bmag * bdir
    P[8] = rng.standard_normal() * 0.01
    return P
