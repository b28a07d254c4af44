"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this
module. It loads ``oracle/liboracle.so`` (built from ``oracle/oracle.c`` with gcc,
``-O2 -ffp-contract=off``, OpenMP over blocks, one thread unless ``set_threads``
asks for more, with bit-identical results) and shares nothing with the HIP library
or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
NV = 9


def nvar(params: dict) -> int:
    """Rows of P and U: nine GRMHD variables, plus the entropy field if carried."""
    return NV + (1 if int(params.get("entropy", 0)) else 0)


def build(force: bool = True) -> str:
    """Compile the oracle with plain IEEE FP64 semantics (no contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nghost", C.c_int), ("metric", C.c_int),
                ("spin", C.c_double), ("gamma_ad", C.c_double),
                ("x_lo", C.c_double * 3), ("x_hi", C.c_double * 3),
                ("ncell0", C.c_int * 3), ("bc", (C.c_int * 2) * 3),
                ("recon", C.c_int), ("flux", C.c_int),
                ("cfl", C.c_double), ("rho_floor", C.c_double), ("p_floor", C.c_double),
                ("w_max", C.c_double), ("glm_alpha", C.c_double), ("c2p_tol", C.c_double),
                ("c2p_maxit", C.c_int), ("amr", C.c_int), ("entropy", C.c_int), ("c2p_2d", C.c_int),
                ("ct", C.c_int)]


class Block(C.Structure):
    _fields_ = [("level", C.c_int), ("size", C.c_int * 3), ("origin", C.c_int * 3)]


class State(C.Structure):
    _fields_ = [("dt_next", C.c_double), ("dt", C.c_double), ("ch", C.c_double),
                ("kappa", C.c_double), ("lam", C.c_double * 3), ("dt_fixed", C.c_double),
                ("have_dt", C.c_int), ("c2p_fail", C.c_int64), ("floor_hits", C.c_int64),
                ("max_iter", C.c_int), ("c2p_backup", C.c_int64)]


_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def load(path: str):
    """Load an oracle build (the plain one, or the op-count build of opcount.py, which
    exports the same entry points) and declare its signatures."""
    L = C.CDLL(path)
    L.orc_grid_new.restype = C.c_void_p
    L.orc_grid_new.argtypes = [C.POINTER(Params), C.POINTER(Block), C.c_int64]
    L.orc_grid_free.argtypes = [C.c_void_p]
    L.orc_grid_layout.argtypes = [C.c_void_p, _I64, _I64]
    L.orc_fill_ghosts.argtypes = [C.c_void_p, _D, _I64, C.c_int64]
    L.orc_prim2con.argtypes = [C.c_void_p, _D, _D, _I64, C.c_int64]
    L.orc_con2prim.argtypes = [C.c_void_p, _D, _D, C.POINTER(C.c_int8), C.POINTER(State), _I64, C.c_int64]
    L.orc_compute_dt.argtypes = [C.c_void_p, _D, C.POINTER(State)]
    L.orc_set_dt.argtypes = [C.POINTER(State), C.c_double]
    L.orc_substep.restype = C.c_int
    L.orc_substep.argtypes = [C.c_void_p, _D, _D, _D, _D, _D, C.c_double, C.c_double,
                              C.POINTER(State), _I64, C.c_int64]
    L.orc_metric.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D]
    L.orc_p2c_point.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, _D]
    L.orc_c2p_point.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, _D, _D,
                                C.POINTER(C.c_int)]
    L.orc_phys_flux.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, C.c_int, _D, _D, _D]
    L.orc_riemann.restype = C.c_double
    L.orc_riemann.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_int, _D, _D,
                              C.c_double, _D]
    L.orc_recon_face.argtypes = [C.c_int, _D, _D]
    L.orc_c2p_entropy_point.restype = C.c_int
    L.orc_c2p_entropy_point.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, C.c_double, _D]
    L.orc_sources.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, _D, C.c_double, _D]
    L.orc_c2p_2d_point.restype = C.c_int
    L.orc_c2p_2d_point.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, _D, _D, C.POINTER(C.c_int)]
    L.orc_c2p_2d_residual.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _D, C.c_double, C.c_double,
                                      _D, _D]
    L.orc_substep_ct.restype = C.c_int
    L.orc_substep_ct.argtypes = [C.c_void_p, _D, _D, _D, _D, _D, _D, _D, _D, C.c_double, C.c_double,
                                 C.POINTER(State), _I64, C.c_int64]
    L.orc_face_count.argtypes = [C.c_void_p, _I64]
    L.orc_ct_center.argtypes = [C.c_void_p, _D, _D]
    L.orc_ct_divergence.argtypes = [C.c_void_p, _D, _D]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_get_threads.restype = C.c_int
    return L


def set_threads(n: int) -> None:
    """Threads of the oracle's block loops (1 = single-threaded, the default)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def make_params(d: dict) -> Params:
    p = Params()
    for k in ("ndim", "nghost", "metric", "recon", "flux", "c2p_maxit"):
        setattr(p, k, int(d[k]))
    p.amr = int(d.get("amr", 0))
    p.entropy = int(d.get("entropy", 0))
    p.c2p_2d = int(d.get("c2p_2d", 0))
    p.ct = int(d.get("ct", 0))
    for k in ("spin", "gamma_ad", "cfl", "rho_floor", "p_floor", "w_max", "glm_alpha", "c2p_tol"):
        setattr(p, k, float(d[k]))
    for e in range(3):
        p.x_lo[e] = float(d["x_lo"][e])
        p.x_hi[e] = float(d["x_hi"][e])
        p.ncell0[e] = int(d["ncell0"][e])
        for s in range(2):
            p.bc[e][s] = int(d["bc"][e][s])
    return p


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _sel(blocks):
    if blocks is None:
        return None, 0
    arr = np.ascontiguousarray(blocks, dtype=np.int64)
    return arr, arr.size


class OracleGrid:
    """A block list with the oracle's own padded layout and dt state."""

    def __init__(self, params: dict, blocks: np.ndarray):
        self.params = dict(params)
        self._p = make_params(params)
        nb = int(blocks.shape[0])
        arr = (Block * nb)()
        for b in range(nb):
            arr[b].level = int(blocks[b, 0])
            for e in range(3):
                arr[b].size[e] = int(blocks[b, 1 + e])
                arr[b].origin[e] = int(blocks[b, 4 + e])
        self._blocks = arr
        self.blocks = np.asarray(blocks, dtype=np.int32)
        h = lib().orc_grid_new(C.byref(self._p), arr, nb)
        if not h:
            raise ValueError("oracle rejected the block list")
        self._h = C.c_void_p(h)
        self.nb = nb
        self.nv = nvar(params)
        self.off = np.zeros(nb + 1, dtype=np.int64)
        self.ioff = np.zeros(nb + 1, dtype=np.int64)
        lib().orc_grid_layout(self._h, self.off.ctypes.data_as(_I64), self.ioff.ctypes.data_as(_I64))
        self.ncp = int(self.off[-1])
        self.nci = int(self.ioff[-1])
        self.state = State()
        self._pidx = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().orc_grid_free(self._h)
                self._h = None
        except Exception:
            pass

    # --- data marshalling ------------------------------------------------------------
    def interior_index(self) -> np.ndarray:
        """Index in P of every interior cell, in interior-packed order (each block's
        interior cells lead its region, x fastest)."""
        if self._pidx is None:
            parts = [self.off[b] + np.arange(int(np.prod(self.blocks[b, 1:4])), dtype=np.int64)
                     for b in range(self.nb)]
            self._pidx = np.concatenate(parts).astype(np.int64)
        return self._pidx

    def pack(self, interior: np.ndarray) -> np.ndarray:
        out = np.zeros((interior.shape[0], self.ncp), dtype=np.float64)
        out[:, self.interior_index()] = interior
        return out

    def unpack(self, padded: np.ndarray) -> np.ndarray:
        return np.ascontiguousarray(padded[:, self.interior_index()])

    # --- method calls ----------------------------------------------------------------
    def fill_ghosts(self, P, blocks=None):
        s, n = _sel(blocks)
        lib().orc_fill_ghosts(self._h, _dp(P), None if s is None else s.ctypes.data_as(_I64), n)

    def prim2con(self, P, U=None, blocks=None):
        if U is None:
            U = np.zeros_like(P)
        s, n = _sel(blocks)
        lib().orc_prim2con(self._h, _dp(P), _dp(U), None if s is None else s.ctypes.data_as(_I64), n)
        return U

    def con2prim(self, U, P, fail=None, blocks=None):
        s, n = _sel(blocks)
        fp = None if fail is None else fail.ctypes.data_as(C.POINTER(C.c_int8))
        lib().orc_con2prim(self._h, _dp(U), _dp(P), fp, C.byref(self.state),
                           None if s is None else s.ctypes.data_as(_I64), n)

    def compute_dt(self, P):
        lib().orc_compute_dt(self._h, _dp(P), C.byref(self.state))
        return self.state.dt_next

    def set_dt(self, dt):
        lib().orc_set_dt(C.byref(self.state), float(dt))

    def substep(self, Ub, Us, Ps, Uo, Po, a, b, blocks=None):
        s, n = _sel(blocks)
        rc = lib().orc_substep(self._h, _dp(Ub), _dp(Us), _dp(Ps), _dp(Uo), _dp(Po), float(a), float(b),
                               C.byref(self.state), None if s is None else s.ctypes.data_as(_I64), n)
        if rc != 0:
            raise RuntimeError("oracle substep: dt not initialised")

    # --- staggered face field (constrained transport) -------------------------------
    def face_count(self):
        n = np.zeros(3, dtype=np.int64)
        lib().orc_face_count(self._h, n.ctypes.data_as(_I64))
        return n

    def substep_ct(self, Ub, Us, Ps, Phib, Phis, Uo, Po, Phio, a, b, blocks=None):
        s, n = _sel(blocks)
        rc = lib().orc_substep_ct(self._h, _dp(Ub), _dp(Us), _dp(Ps), _dp(Phib), _dp(Phis), _dp(Uo), _dp(Po),
                                  _dp(Phio), float(a), float(b), C.byref(self.state),
                                  None if s is None else s.ctypes.data_as(_I64), n)
        if rc != 0:
            raise RuntimeError("oracle CT substep: dt not initialised or constrained transport not enabled")

    def ct_center(self, Phi, P):
        lib().orc_ct_center(self._h, _dp(Phi), _dp(P))

    def ct_divergence(self, Phi):
        div = np.zeros(self.nci)
        lib().orc_ct_divergence(self._h, _dp(Phi), _dp(div))
        return div

    def init_ct(self, prim_interior, Phi):
        """Padded P with the cell-centred field from the face field, ghosts filled,
        U = prim2con(P), dt from the centred reduction."""
        P = self.pack(np.asarray(prim_interior, dtype=np.float64))
        self.ct_center(Phi, P)
        self.fill_ghosts(P)
        U = self.prim2con(P)
        self.compute_dt(P)
        return U, P

    def rk2_step_ct(self, U, P, Phi, U1=None, P1=None, Phi1=None):
        """One SSP-RK2 step in place on (U, P, Phi)."""
        U1 = np.zeros_like(U) if U1 is None else U1
        P1 = np.zeros_like(P) if P1 is None else P1
        Phi1 = np.zeros_like(Phi) if Phi1 is None else Phi1
        self.fill_ghosts(P)
        self.substep_ct(U, U, P, Phi, Phi, U1, P1, Phi1, 0.0, 1.0)
        self.fill_ghosts(P1)
        self.substep_ct(U, U1, P1, Phi, Phi1, U, P, Phi, 0.5, 0.5)
        return U, P, Phi

    def stats(self):
        st = self.state
        return dict(c2p_fail=int(st.c2p_fail), floor_hits=int(st.floor_hits), max_iter=int(st.max_iter),
                    c2p_backup=int(st.c2p_backup),
                    dt=float(st.dt), dt_next=float(st.dt_next), ch=float(st.ch), kappa=float(st.kappa))

    # --- drivers ---------------------------------------------------------------------
    def init(self, prim_interior):
        """Padded P with ghosts filled, U = prim2con(P), dt from the centred reduction."""
        P = self.pack(np.asarray(prim_interior, dtype=np.float64))
        self.fill_ghosts(P)
        U = self.prim2con(P)
        self.compute_dt(P)
        return U, P

    def rk2_step(self, U, P, U1=None, P1=None):
        """One SSP-RK2 step in place on (U, P): stage (0, 1) then (1/2, 1/2)."""
        U1 = np.zeros_like(U) if U1 is None else U1
        P1 = np.zeros_like(P) if P1 is None else P1
        self.fill_ghosts(P)
        self.substep(U, U, P, U1, P1, 0.0, 1.0)
        self.fill_ghosts(P1)
        self.substep(U, U1, P1, U, P, 0.5, 0.5)
        return U, P

    def run(self, prim_interior, steps):
        U, P = self.init(prim_interior)
        U1 = np.zeros_like(U)
        P1 = np.zeros_like(P)
        for _ in range(steps):
            self.rk2_step(U, P, U1, P1)
        return U, P


# --- pointwise helpers for unit pins -------------------------------------------------
def _vec(x, n=NV):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))


def metric(params, x1, x2):
    out = np.zeros(62)
    lib().orc_metric(C.byref(make_params(params)), float(x1), float(x2), _dp(out))
    return dict(alpha=out[0], beta=out[1:4].copy(), g=out[4:13].reshape(3, 3).copy(),
                gi=out[13:22].reshape(3, 3).copy(), sqrtg=out[22], da=out[23:26].copy(),
                db=out[26:35].reshape(3, 3).copy(), dg=out[35:62].reshape(3, 3, 3).copy())


def p2c(params, x1, x2, P):
    n = nvar(params)
    U = np.zeros(n)
    lib().orc_p2c_point(C.byref(make_params(params)), float(x1), float(x2), _dp(_vec(P, n)), _dp(U))
    return U


def c2p(params, x1, x2, U, Pguess):
    n = nvar(params)
    P = np.zeros(n)
    info = (C.c_int * 4)()
    lib().orc_c2p_point(C.byref(make_params(params)), float(x1), float(x2), _dp(_vec(U, n)),
                        _dp(_vec(Pguess, n)), _dp(P), info)
    return P, dict(fail=info[0], iters=info[1], floored=info[2], backup=info[3])


def c2p_entropy(params, x1, x2, U, Wguess=1.0):
    """The entropy inversion alone (U has 10 entries); returns P or None."""
    P = np.zeros(NV + 1)
    rc = lib().orc_c2p_entropy_point(C.byref(make_params(params)), float(x1), float(x2),
                                     _dp(_vec(U, NV + 1)), float(Wguess), _dp(P))
    return None if rc else P


def c2p_2d(params, x1, x2, U, Pguess):
    """The two-unknown Newton iteration alone: (P or None, steps)."""
    P = np.zeros(NV)
    nit = C.c_int()
    rc = lib().orc_c2p_2d_point(C.byref(make_params(params)), float(x1), float(x2), _dp(_vec(U)),
                                _dp(_vec(Pguess)), _dp(P), C.byref(nit))
    return (None if rc else P), nit.value


def c2p_2d_residual(params, x1, x2, U, xi, z):
    F, J = np.zeros(2), np.zeros(4)
    lib().orc_c2p_2d_residual(C.byref(make_params(params)), float(x1), float(x2), _dp(_vec(U)), float(xi),
                              float(z), _dp(F), _dp(J))
    return F, J.reshape(2, 2)


def phys_flux(params, x1, x2, P, d):
    U, F, lam = np.zeros(NV), np.zeros(NV), np.zeros(2)
    lib().orc_phys_flux(C.byref(make_params(params)), float(x1), float(x2), _dp(_vec(P)), int(d),
                        _dp(U), _dp(F), _dp(lam))
    return U, F, lam


def riemann(params, x1, x2, d, PL, PR, ch):
    F = np.zeros(NV)
    lam = lib().orc_riemann(C.byref(make_params(params)), float(x1), float(x2), int(d), _dp(_vec(PL)),
                            _dp(_vec(PR)), float(ch), _dp(F))
    return F, lam


def recon_face(method, q6):
    out = np.zeros(2)
    lib().orc_recon_face(int(method), _dp(_vec(q6, 6)), _dp(out))
    return out[0], out[1]


def sources(params, x1, x2, P, U, kappa):
    S = np.zeros(NV)
    lib().orc_sources(C.byref(make_params(params)), float(x1), float(x2), _dp(_vec(P)), _dp(_vec(U)),
                      float(kappa), _dp(S))
    return S
