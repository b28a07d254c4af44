"""Seeded synthetic inputs for the GRMHD substep (shared by the HIP path and the oracle).

This module draws random numbers and evaluates coordinate geometry only. It
holds none of the method's arithmetic: no spacetime metric, no equation of
state, no conversion between primitive and conserved variables, no flux. That
is what lets the HIP path and the independent CPU oracle start from the very
same bytes without sharing any code that computes the method.

Workloads
---------
The paper's scaling runs use an unspecified uniform-grid GRMHD setup with a
fixed number of cells per core (Section 3). The cases below are the
synthetic stand-ins: a 2-D special-relativistic MHD block, a magnetised torus
around a Kerr black hole on uniform 16^3 blocks, and an AMR-like list of
blocks of mixed size and level. Every draw comes from
``numpy.random.default_rng(12240 + k)`` for case k, in a fixed order.

Data layout handed to both sides
--------------------------------
``Case.prim`` is float64 ``[9][ncell_interior]``: the interior cells of block
0, then block 1, ..., each block x-fastest (axis 0 fastest, axis 2 slowest).
Variable order: rho, u~1, u~2, u~3 (Eulerian velocity times Lorentz factor,
contravariant), p, B1, B2, B3 (Eulerian field, contravariant), psi (GLM scalar).
``Case.blocks`` is int32 ``[nb][7]`` = (level, size0, size1, size2, origin0,
origin1, origin2), origins in level-l cells.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NVAR = 9
RHO, U1, U2, U3, PRS, B1, B2, B3, PSI = range(NVAR)

METRIC_MINKOWSKI_CART = 0
METRIC_KS_SPH_LOGR = 1
BC_PERIODIC, BC_OUTFLOW = 0, 1
RECON_MC, RECON_PPM = 0, 1
FLUX_HLL, FLUX_TVDLF = 0, 1
PREC_FP64, PREC_MIXED = 0, 1

SPIN = 0.9375
R_OUT = 50.0
TH_CUT = 0.1
TORUS_R0, TORUS_W = 12.0, 4.0
RHO_ATM, P_ATM = 1.0e-4, 1.0e-6


@dataclass
class Case:
    name: str
    params: dict
    blocks: np.ndarray
    prim: np.ndarray
    ioff: np.ndarray
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def nblocks(self) -> int:
        return int(self.blocks.shape[0])

    @property
    def ncell_interior(self) -> int:
        return int(self.ioff[-1])


def base_params(**kw) -> dict:
    p = dict(ndim=3, nghost=3, metric=METRIC_KS_SPH_LOGR, spin=SPIN, gamma_ad=4.0 / 3.0,
             x_lo=[0.0, 0.0, 0.0], x_hi=[1.0, 1.0, 1.0], ncell0=[1, 1, 1],
             bc=[[BC_OUTFLOW, BC_OUTFLOW], [BC_OUTFLOW, BC_OUTFLOW], [BC_PERIODIC, BC_PERIODIC]],
             recon=RECON_PPM, flux=FLUX_HLL, precision=PREC_FP64, fused=0,
             cfl=0.4, rho_floor=RHO_ATM, p_floor=P_ATM, w_max=50.0, glm_alpha=0.1,
             c2p_tol=1.0e-13, c2p_maxit=50, amr=0, entropy=0)
    p.update(kw)
    return p


def _ioff(blocks: np.ndarray) -> np.ndarray:
    n = blocks[:, 1].astype(np.int64) * blocks[:, 2] * blocks[:, 3]
    return np.concatenate([[0], np.cumsum(n)]).astype(np.int64)


def _block_cells(blk):
    """Global level-l indices (g0, g1, g2) of a block's interior cells, x fastest."""
    _, s0, s1, s2, o0, o1, o2 = (int(v) for v in blk)
    k, j, i = np.meshgrid(np.arange(s2), np.arange(s1), np.arange(s0), indexing="ij")
    return (o0 + i).ravel(), (o1 + j).ravel(), (o2 + k).ravel()


# ----------------------------------------------------------------------------------
# Case 1: 2-D special-relativistic MHD, one 64x64 periodic block.
# ----------------------------------------------------------------------------------
def case1(n: int = 64, seed: int = 12241) -> Case:
    rng = np.random.default_rng(seed)
    kx, ky = (int(v) for v in rng.integers(1, 4, size=2))
    phi0 = float(rng.uniform(0.0, 2.0 * math.pi))
    cm = rng.standard_normal(4)
    pm = rng.integers(1, 4, size=4)
    qm = rng.integers(1, 4, size=4)
    chi = rng.uniform(0.0, 2.0 * math.pi, size=4)
    u1 = rng.uniform(size=(n, n))          # [j][i]
    u2 = rng.uniform(size=(n, n))

    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xc, xc, indexing="xy")  # X[j][i] = x_i
    prim = np.zeros((NVAR, n, n))
    prim[RHO] = 1.0 + 0.1 * np.sin(2 * math.pi * (kx * X + ky * Y) + phi0)
    prim[PRS] = 1.0
    # |u~| <= 1/sqrt(3) is the same as |v| <= 1/2 for a unit spatial metric
    umag = math.sqrt(1.0 / 3.0) * np.sqrt(u1)
    ang = 2.0 * math.pi * u2
    prim[U1] = umag * np.cos(ang)
    prim[U2] = umag * np.sin(ang)

    # field: uniform 0.5 x-hat plus the central-difference curl of a corner potential
    xf = np.arange(n + 1) * h
    XF, YF = np.meshgrid(xf, xf, indexing="xy")
    A = np.zeros_like(XF)
    for m in range(4):
        A += cm[m] * np.sin(2 * math.pi * (pm[m] * XF + qm[m] * YF) + chi[m])
    A *= 0.05 / (2 * math.pi)
    # corners (j, i) .. (j+1, i+1) surround cell (j, i)
    a00, a01, a10, a11 = A[:-1, :-1], A[:-1, 1:], A[1:, :-1], A[1:, 1:]
    prim[B1] = 0.5 + ((a10 + a11) - (a00 + a01)) / (2 * h)
    prim[B2] = -((a01 + a11) - (a00 + a10)) / (2 * h)

    blocks = np.array([[0, n, n, 1, 0, 0, 0]], dtype=np.int32)
    params = base_params(ndim=2, nghost=2, metric=METRIC_MINKOWSKI_CART, spin=0.0,
                         x_lo=[0.0, 0.0, 0.0], x_hi=[1.0, 1.0, 1.0], ncell0=[n, n, 1],
                         bc=[[BC_PERIODIC] * 2, [BC_PERIODIC] * 2, [BC_PERIODIC] * 2],
                         recon=RECON_MC, flux=FLUX_TVDLF, rho_floor=1.0e-4, p_floor=1.0e-6)
    return Case(f"case1_srmhd2d_{n}", params, blocks, prim.reshape(NVAR, n * n).copy(),
                _ioff(blocks), steps=10, meta=dict(kx=kx, ky=ky))


# ----------------------------------------------------------------------------------
# Kerr-Schild torus cases (2, 3, 5 uniform; 4 AMR-like).
# ----------------------------------------------------------------------------------
def ks_domain(spin: float = SPIN):
    """Logarithmic-radius spherical domain: r in [0.8 r_H, 50], theta in [0.1, pi-0.1], phi in [0, 2pi)."""
    r_h = 1.0 + math.sqrt(1.0 - spin * spin)
    x_lo = [math.log(0.8 * r_h), TH_CUT, 0.0]
    x_hi = [math.log(R_OUT), math.pi - TH_CUT, 2.0 * math.pi]
    return x_lo, x_hi


def _torus_density(r, th):
    w = r * np.sin(th)
    zz = r * np.cos(th)
    d2 = (w - TORUS_R0) ** 2 + zz ** 2
    return np.maximum(0.0, 1.0 - d2 / TORUS_W ** 2) ** 3


def _torus_cells(params, level, g0, g1, g2, noise_u):
    """Primitive state of the synthetic torus at level-l cells (g0, g1, g2).

    Coordinate geometry only: the orbital velocity, the field normalisation and
    the volume factor use flat-space expressions in (ln r, theta, phi), so no
    part of the spacetime metric enters the inputs.
    """
    x_lo, x_hi, n0 = params["x_lo"], params["x_hi"], params["ncell0"]
    dx = [(x_hi[d] - x_lo[d]) / (n0[d] * 2 ** level) for d in range(3)]
    x1 = x_lo[0] + (g0 + 0.5) * dx[0]
    th = x_lo[1] + (g1 + 0.5) * dx[1]
    r = np.exp(x1)
    rho_t = _torus_density(r, th)
    prim = np.zeros((NVAR, g0.size))
    prim[RHO] = np.maximum(rho_t, RHO_ATM)
    p = np.maximum(0.01 * rho_t ** (4.0 / 3.0), P_ATM)
    inside = rho_t > 0.0
    p = np.where(inside, p * (1.0 + 0.02 * (2.0 * noise_u - 1.0)), p)
    prim[PRS] = p
    w = r * np.sin(th)
    omega = 1.0 / (w ** 1.5 + params["spin"])
    prim[U3] = np.where(inside, omega, 0.0)
    # poloidal field from A_phi = max(rho_t - 0.2, 0) at cell corners
    def a_phi(c0, c1):
        rr = np.exp(x_lo[0] + c0 * dx[0])
        tt = x_lo[1] + c1 * dx[1]
        return np.maximum(_torus_density(rr, tt) - 0.2, 0.0)
    a00 = a_phi(g0, g1)
    a10 = a_phi(g0 + 1, g1)
    a01 = a_phi(g0, g1 + 1)
    a11 = a_phi(g0 + 1, g1 + 1)
    dA_dth = ((a01 + a11) - (a00 + a10)) / (2 * dx[1])
    dA_dx1 = ((a10 + a11) - (a00 + a01)) / (2 * dx[0])
    vol = r ** 3 * np.sin(th)
    prim[B1] = dA_dth / vol
    prim[B2] = -dA_dx1 / vol
    return prim, r, th


def _uniform_blocks(n, bs):
    nb = [n[d] // bs for d in range(3)]
    out = []
    for b0 in range(nb[0]):
        for b1 in range(nb[1]):
            for b2 in range(nb[2]):          # phi-block index fastest
                out.append([0, bs, bs, bs, b0 * bs, b1 * bs, b2 * bs])
    return np.array(out, dtype=np.int32)


def _field_scale(prim, r):
    # field normalisation: max p / max(|B|^2/2) = 100 with the flat spatial metric
    bsq = (r * prim[B1]) ** 2 + (r * prim[B2]) ** 2
    bmax = float(bsq.max())
    return math.sqrt(float(prim[PRS].max()) / (100.0 * 0.5 * bmax)) if bmax > 0.0 else 1.0


def _finish_torus(prim, r):
    scale = _field_scale(prim, r)
    prim[B1] *= scale
    prim[B2] *= scale
    return prim


def case_torus(cfg: int, n=128, bs: int = 16, precision=None, fused=None, phi_slabs: int = 1) -> Case:
    """Cases 2 (128^3, FP64 plain), 3 (192^3, mixed) and 5 (384^3, mixed + turbulence).
    phi_slabs > 1: only the first of that many equal phi-slabs of the domain (one
    GPU's share of a run sharded along phi), n giving its own cell counts; its phi
    ends are joined periodically in place of the neighbouring slabs."""
    if isinstance(n, int):
        n = (n, n, n)
    assert all(v % bs == 0 for v in n)
    rng = np.random.default_rng(12240 + cfg)
    x_lo, x_hi = ks_domain()
    x_hi = [x_hi[0], x_hi[1], x_lo[2] + (x_hi[2] - x_lo[2]) / phi_slabs]
    prec = {2: PREC_FP64, 3: PREC_MIXED, 5: PREC_MIXED}[cfg] if precision is None else precision
    fus = {2: 0, 3: 0, 5: 1}[cfg] if fused is None else fused
    params = base_params(x_lo=x_lo, x_hi=x_hi, ncell0=list(n), precision=prec, fused=fus)
    blocks = _uniform_blocks(n, bs)
    ioff = _ioff(blocks)
    noise = rng.uniform(size=int(ioff[-1]))
    g = [np.concatenate(v) for v in zip(*(_block_cells(b) for b in blocks))]
    prim, r, th = _torus_cells(params, 0, g[0], g[1], g[2], noise)
    prim = _finish_torus(prim, r)
    if cfg == 5:
        _add_turbulence(params, prim, r, th, g, n, rng)
    steps = 100 if cfg == 5 else 10
    return Case(f"case{cfg}_ks_torus_{n[0]}x{n[1]}x{n[2]}", params, blocks, prim, ioff, steps)


def torus_with_face_field(case: Case):
    """A uniform-grid torus case (case_torus, case_torus_2d) for constrained
    transport: params with ct = 1 and the face field phi^d = sqrt(gamma) B^d as the
    discrete curl of the azimuthal potential A_phi = max(rho_t - 0.2, 0) that gives
    the cell-centred field, with the same normalisation (so phi^1 = dA/dtheta and
    phi^2 = -dA/dx1 on the faces, and the cell field follows from them)."""
    params = dict(case.params, ct=1)
    g = [np.concatenate(v) for v in zip(*(_block_cells(b) for b in case.blocks))]
    raw, r, _ = _torus_cells(case.params, 0, g[0], g[1], g[2], np.full(g[0].size, 0.5))
    raw[PRS] = case.prim[PRS]
    scale = _field_scale(raw, r)

    def potential(e, x1, x2, x3):
        if e != 2:
            return np.zeros_like(x1)
        return scale * np.maximum(_torus_density(np.exp(x1), x2) - 0.2, 0.0)

    phi = face_field_from_potential(params, case.blocks, potential)
    return Case(case.name + "_ct", params, case.blocks, case.prim, case.ioff, case.steps), phi


def case_torus_2d(n=(64, 64), bs: int = 16, precision=PREC_FP64, seed: int = 12250) -> Case:
    """The synthetic torus on an axisymmetric (ln r, theta) grid: ndim = 2 in the
    Kerr-Schild metric, n[0] x n[1] cells in blocks of bs x bs (phi is not resolved)."""
    assert n[0] % bs == 0 and n[1] % bs == 0
    rng = np.random.default_rng(seed)
    x_lo, x_hi = ks_domain()
    params = base_params(ndim=2, x_lo=x_lo, x_hi=x_hi, ncell0=[n[0], n[1], 1], precision=precision,
                         bc=[[BC_OUTFLOW, BC_OUTFLOW], [BC_OUTFLOW, BC_OUTFLOW], [BC_PERIODIC, BC_PERIODIC]])
    blocks = np.array([[0, bs, bs, 1, b0 * bs, b1 * bs, 0] for b0 in range(n[0] // bs)
                       for b1 in range(n[1] // bs)], dtype=np.int32)
    ioff = _ioff(blocks)
    noise = rng.uniform(size=int(ioff[-1]))
    g = [np.concatenate(v) for v in zip(*(_block_cells(b) for b in blocks))]
    prim, r, th = _torus_cells(params, 0, g[0], g[1], g[2], noise)
    prim = _finish_torus(prim, r)
    return Case(f"ks_torus_2d_{n[0]}x{n[1]}", params, blocks, prim, ioff, steps=10)


def _add_turbulence(params, prim, r, th, g, n, rng):
    """Seeded velocity field at Mach 0.3 of the Newtonian sound speed, torus cells only."""
    nm = 32
    kvec = rng.integers(-4, 5, size=(3, nm, 3))
    amp = rng.standard_normal((3, nm))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(3, nm))
    inside = np.flatnonzero(prim[U3] != 0.0)
    if inside.size == 0:
        return
    gam = params["gamma_ad"]
    cs = np.sqrt(gam * prim[PRS, inside] / prim[RHO, inside])
    ri, ti = r[inside], th[inside]
    scale = [ri, ri, ri * np.sin(ti)]
    gx = [g[0][inside] / n[0], g[1][inside] / n[1], g[2][inside] / n[2]]
    for comp in range(3):
        field_ = np.zeros(inside.size)
        for m in range(nm):
            arg = 2 * math.pi * (kvec[comp, m, 0] * gx[0] + kvec[comp, m, 1] * gx[1]
                                 + kvec[comp, m, 2] * gx[2]) + ph[comp, m]
            field_ += amp[comp, m] * np.sin(arg)
        rms = math.sqrt(float(np.mean(field_ ** 2)))
        prim[U1 + comp, inside] += 0.3 * cs * field_ / max(rms, 1e-300) / scale[comp]


def case4(nblocks: int = 4096, n0: int = 96, levels: int = 3, precision=PREC_MIXED, fused=1) -> Case:
    """AMR-like list: independent same-level patches of mixed size and level."""
    rng = np.random.default_rng(12244)
    x_lo, x_hi = ks_domain()
    params = base_params(x_lo=x_lo, x_hi=x_hi, ncell0=[n0, n0, n0], precision=precision, fused=fused)
    lev_p = np.array([2.0 ** l for l in range(levels)])
    lev_p /= lev_p.sum()
    lev = rng.choice(levels, size=nblocks, p=lev_p)
    size = rng.choice(np.array([8, 12, 16]), size=nblocks, p=[0.5, 0.3, 0.2])
    taken = {}
    out = []
    for b in range(nblocks):
        l, s = int(lev[b]), int(size[b])
        nslot = n0 * 2 ** l // s
        used = taken.setdefault((l, s), set())
        cap = nslot ** 3
        if len(used) >= cap:
            raise ValueError("lattice full")
        while True:
            slot = tuple(int(v) for v in rng.integers(0, nslot, size=3))
            if slot not in used:
                used.add(slot)
                break
        out.append([l, s, s, s, slot[0] * s, slot[1] * s, slot[2] * s])
    blocks = np.array(out, dtype=np.int32)
    ioff = _ioff(blocks)
    noise = rng.uniform(size=int(ioff[-1]))
    prim = np.zeros((NVAR, int(ioff[-1])))
    rr = np.zeros(int(ioff[-1]))
    tt = np.zeros(int(ioff[-1]))
    for b in range(nblocks):
        g0, g1, g2 = _block_cells(blocks[b])
        sl = slice(int(ioff[b]), int(ioff[b + 1]))
        prim[:, sl], rr[sl], tt[sl] = _torus_cells(params, int(blocks[b, 0]), g0, g1, g2, noise[sl])
    prim = _finish_torus(prim, rr)
    return Case(f"case4_amrlike_{nblocks}", params, blocks, prim, ioff, steps=10)


def _tree_leaves(params, bs, levels, thresholds):
    """Leaves (level, i, j, k) of a 2:1-balanced tree of bs^ndim blocks over the level-0
    lattice: a block is refined while the synthetic torus density sampled at its
    cells exceeds the threshold of its level, then coarse leaves next to leaves two
    levels finer (across faces, edges or corners) are refined until none is."""
    n0 = params["ncell0"]
    nd = int(params["ndim"])
    per = [params["bc"][d][0] == BC_PERIODIC for d in range(3)]
    nsl0 = [n0[d] // bs if d < nd else 1 for d in range(3)]
    leaves = {(0, i, j, k) for i in range(nsl0[0]) for j in range(nsl0[1]) for k in range(nsl0[2])}

    def rho_max(lf):
        l, i, j, _ = lf
        x_lo, x_hi = params["x_lo"], params["x_hi"]
        dx = [(x_hi[d] - x_lo[d]) / (n0[d] * 2 ** l) for d in range(2)]
        g0 = i * bs + np.arange(bs) + 0.5
        g1 = j * bs + np.arange(bs) + 0.5
        r = np.exp(x_lo[0] + g0 * dx[0])[:, None]
        th = (x_lo[1] + g1 * dx[1])[None, :]
        return float(_torus_density(r, th).max())

    def refine(lf):
        l, i, j, k = lf
        leaves.remove(lf)
        for a in range(2):
            for b in range(2):
                for c in range(2 if nd == 3 else 1):
                    leaves.add((l + 1, 2 * i + a, 2 * j + b, (2 * k + c) if nd == 3 else 0))

    def covering(l, idx):
        for m in range(l, -1, -1):
            key = (m,) + tuple(v >> (l - m) for v in idx)
            if key in leaves:
                return key
        return None

    def balance():
        changed = True
        while changed:
            changed = False
            for lf in sorted(leaves, reverse=True):
                if lf not in leaves or lf[0] < 2:
                    continue
                l = lf[0]
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for dk in ((-1, 0, 1) if nd == 3 else (0,)):
                            idx = [lf[1] + di, lf[2] + dj, lf[3] + dk]
                            ok = True
                            for d in range(nd):
                                n = nsl0[d] << l
                                if per[d]:
                                    idx[d] %= n
                                elif not 0 <= idx[d] < n:
                                    ok = False
                            cov = covering(l, idx) if ok else None
                            if cov is not None and cov[0] < l - 1:
                                refine(cov)
                                changed = True

    for l in range(levels - 1):
        for lf in sorted(lf for lf in leaves if lf[0] == l):
            if rho_max(lf) > thresholds[l]:
                refine(lf)
        balance()
    return sorted(leaves)


def case_tree_2d(n0: int = 64, bs: int = 16, levels: int = 3, precision=PREC_MIXED, seed: int = 12247) -> Case:
    """The block tree on the axisymmetric (ln r, theta) grid: ndim = 2, bs x bs
    blocks refined around the torus as in case_tree."""
    rng = np.random.default_rng(seed)
    x_lo, x_hi = ks_domain()
    params = base_params(ndim=2, x_lo=x_lo, x_hi=x_hi, ncell0=[n0, n0, 1], precision=precision, fused=0, amr=1,
                         bc=[[BC_OUTFLOW, BC_OUTFLOW], [BC_OUTFLOW, BC_OUTFLOW], [BC_PERIODIC, BC_PERIODIC]])
    leaves = _tree_leaves(params, bs, levels, thresholds=[0.0, 0.3] + [0.6] * max(0, levels - 3))
    blocks = np.array([[l, bs, bs, 1, i * bs, j * bs, 0] for (l, i, j, k) in leaves], dtype=np.int32)
    ioff = _ioff(blocks)
    noise = rng.uniform(size=int(ioff[-1]))
    prim = np.zeros((NVAR, int(ioff[-1])))
    rr = np.zeros(int(ioff[-1]))
    for b in range(len(blocks)):
        g0, g1, g2 = _block_cells(blocks[b])
        sl = slice(int(ioff[b]), int(ioff[b + 1]))
        prim[:, sl], rr[sl], _ = _torus_cells(params, int(blocks[b, 0]), g0, g1, g2, noise[sl])
    prim = _finish_torus(prim, rr)
    return Case(f"tree2d_{n0}_{bs}_{levels}", params, blocks, prim, ioff, steps=10)


def case_tree(n0: int = 64, bs: int = 16, levels: int = 3, precision=PREC_MIXED, seed: int = 12246) -> Case:
    """Block tree: equal-size blocks refined around the synthetic torus (level 1
    where it is present, level 2 where its density exceeds 0.3), 2:1 balanced,
    with the cross-level ghost rule (params amr = 1). Blocks are listed by level,
    phi-fastest; each is sampled at its own level's resolution."""
    rng = np.random.default_rng(seed)
    x_lo, x_hi = ks_domain()
    params = base_params(x_lo=x_lo, x_hi=x_hi, ncell0=[n0, n0, n0], precision=precision, fused=0, amr=1)
    leaves = _tree_leaves(params, bs, levels, thresholds=[0.0, 0.3] + [0.6] * max(0, levels - 3))
    blocks = np.array([[l, bs, bs, bs, i * bs, j * bs, k * bs] for (l, i, j, k) in leaves], dtype=np.int32)
    ioff = _ioff(blocks)
    noise = rng.uniform(size=int(ioff[-1]))
    prim = np.zeros((NVAR, int(ioff[-1])))
    rr = np.zeros(int(ioff[-1]))
    for b in range(len(blocks)):
        g0, g1, g2 = _block_cells(blocks[b])
        sl = slice(int(ioff[b]), int(ioff[b + 1]))
        prim[:, sl], rr[sl], _ = _torus_cells(params, int(blocks[b, 0]), g0, g1, g2, noise[sl])
    prim = _finish_torus(prim, rr)
    return Case(f"tree_{n0}_{bs}_{levels}", params, blocks, prim, ioff, steps=10)


def with_entropy(case: Case) -> Case:
    """The same case carrying the entropy field (entropy = 1): the primitives gain
    a tenth row, the entropy function K = p / rho^gamma of the initial state."""
    gam = float(case.params["gamma_ad"])
    K = case.prim[PRS] / case.prim[RHO] ** gam
    prim = np.vstack([case.prim, K[None, :]])
    return Case(case.name + "_entropy", dict(case.params, entropy=1), case.blocks, prim, case.ioff, case.steps,
                dict(case.meta))


def make_case(cfg: int, **kw) -> Case:
    if cfg == 1:
        return case1(**kw)
    if cfg in (2, 3, 5):
        return case_torus(cfg, **kw)
    if cfg == "slab":
        return case_torus(5, n=kw.get("n", (384, 384, 48)), phi_slabs=kw.get("phi_slabs", 8))
    if cfg == 4:
        return case4(**kw)
    if cfg == "tree":
        return case_tree(**kw)
    raise ValueError(cfg)


def uniform_state(n=(16, 16, 16), bs=(16, 16, 16), ndim=3, prim_value=None, bc=BC_PERIODIC,
                  metric=METRIC_MINKOWSKI_CART, recon=RECON_PPM, flux=FLUX_HLL) -> Case:
    """A spatially uniform state on a periodic Cartesian grid (any block tiling)."""
    if prim_value is None:
        prim_value = [1.0, 0.3, -0.2, 0.1, 0.7, 0.4, -0.3, 0.2, 0.0]
    nb = [n[d] // bs[d] for d in range(3)]
    blocks = []
    for b0 in range(nb[0]):
        for b1 in range(nb[1]):
            for b2 in range(nb[2]):
                blocks.append([0, bs[0], bs[1], bs[2], b0 * bs[0], b1 * bs[1], b2 * bs[2]])
    blocks = np.array(blocks, dtype=np.int32)
    ioff = _ioff(blocks)
    prim = np.repeat(np.asarray(prim_value, dtype=np.float64)[:, None], int(ioff[-1]), axis=1)
    g = 3 if recon == RECON_PPM else 2
    params = base_params(ndim=ndim, nghost=g, metric=metric, spin=0.0,
                         x_lo=[0.0, 0.0, 0.0], x_hi=[1.0, 1.0, 1.0], ncell0=list(n),
                         bc=[[bc] * 2] * 3, recon=recon, flux=flux)
    return Case("uniform", params, blocks, prim, ioff, steps=10)


# ----------------------------------------------------------------------------------
# Staggered face field (constrained transport) from a vector potential.
# ----------------------------------------------------------------------------------
def face_counts(params: dict, blocks: np.ndarray):
    """Faces per direction (totals over the blocks, every block holding all faces of
    its cells) and each block's first face per direction."""
    nd = int(params["ndim"])
    offs, tot = [], []
    for d in range(3):
        n = np.array([int((b[1] + (d == 0)) * (b[2] + (d == 1)) * (b[3] + (d == 2))) if d < nd else 0
                      for b in np.asarray(blocks)], dtype=np.int64)
        offs.append(np.concatenate([[0], np.cumsum(n)]).astype(np.int64))
        tot.append(int(offs[-1][-1]))
    return tot, offs


def face_field_from_potential(params: dict, blocks: np.ndarray, A) -> np.ndarray:
    """The magnetic flux density through every face, phi^d = sqrt(gamma) B^d, as the
    circulation of an edge-centred vector potential around the face over the face's
    coordinate area: with (d, j, k) cyclic,
      phi^d = (A_k(j + 1/2) - A_k(j - 1/2)) / dx_j - (A_j(k + 1/2) - A_j(k - 1/2)) / dx_k,
    each A_e taken at the centre of an edge along e (the k term only where axis k is
    resolved). A(e, x1, x2, x3) returns the covariant component along axis e at the
    given coordinate arrays. Layout: the resolved directions' face arrays one after
    another, each block's faces x fastest."""
    nd = int(params["ndim"])
    x_lo = np.asarray(params["x_lo"], dtype=np.float64)
    x_hi = np.asarray(params["x_hi"], dtype=np.float64)
    n0 = np.asarray(params["ncell0"], dtype=np.int64)
    out = []
    for d in range(nd):
        dj, dk = (d + 1) % 3, (d + 2) % 3
        parts = []
        for blk in np.asarray(blocks):
            lev, size, org = int(blk[0]), blk[1:4].astype(np.int64), blk[4:7].astype(np.int64)
            dx = (x_hi - x_lo) / (n0 * 2 ** lev)
            fs = size + (np.arange(3) == d)
            k, j, i = np.meshgrid(np.arange(fs[2]), np.arange(fs[1]), np.arange(fs[0]), indexing="ij")
            idx = [i.ravel(), j.ravel(), k.ravel()]

            def coord(e, shift):
                # position along e: face coordinate on axis d, cell centres elsewhere,
                # moved by `shift` half cells
                base = org[e] + idx[e] + (0.0 if e == d else 0.5)
                return x_lo[e] + (base + shift) * dx[e]

            def edge(axis, e_off, off):
                # A along `axis` at the edge beside the face, offset by off half cells on e_off
                x = [coord(e, off if e == e_off else 0.0) for e in range(3)]
                return A(axis, x[0], x[1], x[2])

            phi = np.zeros(idx[0].size)
            if dj < nd:
                phi += (edge(dk, dj, 0.5) - edge(dk, dj, -0.5)) / dx[dj]
            if dk < nd:
                phi -= (edge(dj, dk, 0.5) - edge(dj, dk, -0.5)) / dx[dk]
            parts.append(phi)
        out.append(np.concatenate(parts))
    return np.concatenate(out)
