"""Python binding of the HIP library ``libbhac.so`` (argument marshalling only).

Each ``bhac_*`` function here forwards to the C entry point of the same name
(declared in ``include/bhac.h``). Device arrays are torch tensors on a ROCm device;
their raw pointers and the current HIP stream are passed through. Every step of
the method runs in the library's kernels; nothing here computes the method.

The library must have been built (``paper_2108_12240_amd/build.py``); loading
fails loudly otherwise, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbhac.so")
NVAR = 9

BHAC_OK, BHAC_EINVAL, BHAC_ENOMEM, BHAC_EDEVICE, BHAC_EALIAS, BHAC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5


class BhacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bhac error {code}: {msg}")
        self.code = code


class bhac_schedule(C.Structure):
    _fields_ = [("set", C.c_int), ("march_mask", C.c_int), ("march_faces", C.c_int), ("x1_staged", C.c_int)]


class bhac_params(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nghost", C.c_int), ("metric", C.c_int), ("spin", C.c_double),
                ("gamma_ad", C.c_double), ("x_lo", C.c_double * 3), ("x_hi", C.c_double * 3),
                ("ncell0", C.c_int * 3), ("bc", (C.c_int * 2) * 3), ("recon", C.c_int), ("flux", C.c_int),
                ("precision", C.c_int), ("fused", C.c_int), ("cfl", C.c_double), ("rho_floor", C.c_double),
                ("p_floor", C.c_double), ("w_max", C.c_double), ("glm_alpha", C.c_double),
                ("c2p_tol", C.c_double), ("c2p_maxit", C.c_int), ("amr", C.c_int), ("entropy", C.c_int),
                ("sched", bhac_schedule), ("ct", C.c_int)]


class bhac_block_desc(C.Structure):
    _fields_ = [("level", C.c_int), ("size", C.c_int * 3), ("origin", C.c_int * 3)]


class bhac_layout(C.Structure):
    _fields_ = [("ncell_padded", C.c_int64), ("ncell_interior", C.c_int64), ("nvar", C.c_int),
                ("nghost", C.c_int), ("block_offset", C.POINTER(C.c_int64)),
                ("block_interior_offset", C.POINTER(C.c_int64))]


class bhac_timestep(C.Structure):
    _fields_ = [("dt", C.c_double), ("dt_next", C.c_double), ("ch", C.c_double), ("kappa", C.c_double),
                ("lam", C.c_double * 3)]


class bhac_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib = None
_VP = C.c_void_p


def lib():
    """Load libbhac.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run paper_2108_12240_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        sig = {
            "bhac_alloc_blocks": [C.POINTER(bhac_params), C.POINTER(bhac_block_desc), C.c_int64,
                                  C.POINTER(_VP), C.POINTER(bhac_layout)],
            "bhac_free_blocks": [_VP],
            "bhac_fill_ghosts": [_VP, _VP, _VP],
            "bhac_fill_ghost_faces": [_VP, _VP, _VP],
            "bhac_prim2con": [_VP, _VP, _VP, _VP],
            "bhac_con2prim": [_VP, _VP, _VP, _VP, _VP],
            "bhac_substep": [_VP, _VP, _VP, _VP, _VP, _VP, C.c_double, C.c_double, _VP],
            "bhac_substep_noalloc": [_VP, _VP, _VP, _VP, _VP, _VP, C.c_double, C.c_double, _VP],
            "bhac_substep_ct": [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, C.c_double, C.c_double, _VP],
            "bhac_face_count": [_VP, C.POINTER(C.c_int64)],
            "bhac_ct_center": [_VP, _VP, _VP, _VP],
            "bhac_ct_divergence": [_VP, _VP, _VP, _VP],
            "bhac_compute_dt": [_VP, _VP, _VP],
            "bhac_set_dt": [_VP, C.c_double, _VP],
            "bhac_get_dt": [_VP, C.POINTER(C.c_double)],
            "bhac_get_timestep": [_VP, C.POINTER(bhac_timestep)],
            "bhac_get_stats": [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int),
                               C.POINTER(C.c_int64)],
            "bhac_reset_stats": [_VP, _VP],
            "bhac_get_schedule": [_VP, C.POINTER(bhac_schedule)],
            "bhac_set_timing": [_VP, C.c_int],
            "bhac_capture_rk2_step": [_VP, _VP, _VP, _VP, _VP],
            "bhac_capture_rk2_step_ct": [_VP, _VP, _VP, _VP, _VP, _VP, _VP],
            "bhac_launch_rk2_step": [_VP, _VP],
            "bhac_get_timing": [_VP, C.POINTER(bhac_kernel_time), C.c_int, C.POINTER(C.c_int)],
            "bhac_plan_ghosts": [C.POINTER(bhac_params), C.POINTER(bhac_block_desc), C.c_int64,
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.bhac_last_error.argtypes = []
        L.bhac_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != BHAC_OK:
        raise BhacError(rc, lib().bhac_last_error().decode())


def make_params(d: dict) -> bhac_params:
    p = bhac_params()
    for k in ("ndim", "nghost", "metric", "recon", "flux", "precision", "fused", "c2p_maxit"):
        setattr(p, k, int(d[k]))
    p.amr = int(d.get("amr", 0))
    p.ct = int(d.get("ct", 0))
    p.entropy = int(d.get("entropy", 0))
    sched = d.get("sched")
    if sched is not None:
        p.sched.set = 1
        p.sched.march_mask = int(sched["march_mask"])
        p.sched.march_faces = int(sched["march_faces"])
        p.sched.x1_staged = int(sched["x1_staged"])
    for k in ("spin", "gamma_ad", "cfl", "rho_floor", "p_floor", "w_max", "glm_alpha", "c2p_tol"):
        setattr(p, k, float(d[k]))
    for e in range(3):
        p.x_lo[e] = float(d["x_lo"][e])
        p.x_hi[e] = float(d["x_hi"][e])
        p.ncell0[e] = int(d["ncell0"][e])
        for s in range(2):
            p.bc[e][s] = int(d["bc"][e][s])
    return p


def make_blocks(blocks: np.ndarray):
    nb = int(blocks.shape[0])
    arr = (bhac_block_desc * nb)()
    for b in range(nb):
        arr[b].level = int(blocks[b, 0])
        for e in range(3):
            arr[b].size[e] = int(blocks[b, 1 + e])
            arr[b].origin[e] = int(blocks[b, 4 + e])
    return arr


# --- C entry points with the same names ----------------------------------------------
def bhac_plan_ghosts(params: dict, blocks: np.ndarray):
    """Host-only: (block_offset[nb+1], dst[n], src[n]) of the ghost gather map."""
    p, arr = make_params(params), make_blocks(blocks)
    nb = len(arr)
    off = np.zeros(nb + 1, dtype=np.int64)
    n = C.c_int64(0)
    _check(lib().bhac_plan_ghosts(C.byref(p), arr, nb, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(n),
                                  None, None))
    dst = np.zeros(n.value, dtype=np.int32)
    src = np.zeros(n.value, dtype=np.int32)
    _check(lib().bhac_plan_ghosts(C.byref(p), arr, nb, None, None, dst.ctypes.data_as(C.POINTER(C.c_int32)),
                                  src.ctypes.data_as(C.POINTER(C.c_int32))))
    return off, dst, src


def bhac_alloc_blocks(params: dict, blocks: np.ndarray):
    p, arr = make_params(params), make_blocks(blocks)
    h = _VP()
    lay = bhac_layout()
    _check(lib().bhac_alloc_blocks(C.byref(p), arr, len(arr), C.byref(h), C.byref(lay)))
    off = np.ctypeslib.as_array(lay.block_offset, shape=(len(arr) + 1,)).copy()
    ioff = np.ctypeslib.as_array(lay.block_interior_offset, shape=(len(arr) + 1,)).copy()
    return h, dict(ncell_padded=int(lay.ncell_padded), ncell_interior=int(lay.ncell_interior),
                   nvar=int(lay.nvar), nghost=int(lay.nghost), block_offset=off, block_interior_offset=ioff)


def bhac_free_blocks(h):
    _check(lib().bhac_free_blocks(h))


def _ptr(t):
    return None if t is None else _VP(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return _VP(stream.cuda_stream)


def bhac_fill_ghosts(h, prim, stream=None):
    _check(lib().bhac_fill_ghosts(h, _ptr(prim), _stream(stream)))


def bhac_fill_ghost_faces(h, prim, stream=None):
    _check(lib().bhac_fill_ghost_faces(h, _ptr(prim), _stream(stream)))


def bhac_prim2con(h, prim, cons, stream=None):
    _check(lib().bhac_prim2con(h, _ptr(prim), _ptr(cons), _stream(stream)))


def bhac_con2prim(h, cons, prim, fail=None, stream=None):
    _check(lib().bhac_con2prim(h, _ptr(cons), _ptr(prim), _ptr(fail), _stream(stream)))


def bhac_substep(h, U_base, U_stage, P_stage, U_out, P_out, a, b, stream=None):
    _check(lib().bhac_substep(h, _ptr(U_base), _ptr(U_stage), _ptr(P_stage), _ptr(U_out), _ptr(P_out),
                              float(a), float(b), _stream(stream)))


def bhac_substep_noalloc(h, U_base, U_stage, P_stage, U_out, P_out, a, b, stream=None):
    _check(lib().bhac_substep_noalloc(h, _ptr(U_base), _ptr(U_stage), _ptr(P_stage), _ptr(U_out), _ptr(P_out),
                                      float(a), float(b), _stream(stream)))


def bhac_substep_ct(h, U_base, U_stage, P_stage, phi_base, phi_stage, U_out, P_out, phi_out, a, b, stream=None):
    _check(lib().bhac_substep_ct(h, _ptr(U_base), _ptr(U_stage), _ptr(P_stage), _ptr(phi_base), _ptr(phi_stage),
                                 _ptr(U_out), _ptr(P_out), _ptr(phi_out), float(a), float(b), _stream(stream)))


def bhac_face_count(h):
    n = (C.c_int64 * 3)()
    _check(lib().bhac_face_count(h, n))
    return [int(x) for x in n]


def bhac_ct_center(h, phi, prim, stream=None):
    _check(lib().bhac_ct_center(h, _ptr(phi), _ptr(prim), _stream(stream)))


def bhac_ct_divergence(h, phi, div, stream=None):
    _check(lib().bhac_ct_divergence(h, _ptr(phi), _ptr(div), _stream(stream)))


def bhac_compute_dt(h, prim, stream=None):
    _check(lib().bhac_compute_dt(h, _ptr(prim), _stream(stream)))


def bhac_set_dt(h, dt, stream=None):
    _check(lib().bhac_set_dt(h, float(dt), _stream(stream)))


def bhac_get_dt(h) -> float:
    v = C.c_double()
    _check(lib().bhac_get_dt(h, C.byref(v)))
    return v.value


def bhac_get_timestep(h) -> dict:
    t = bhac_timestep()
    _check(lib().bhac_get_timestep(h, C.byref(t)))
    return dict(dt=t.dt, dt_next=t.dt_next, ch=t.ch, kappa=t.kappa, lam=list(t.lam))


def bhac_get_stats(h) -> dict:
    f, fl, it, bk = C.c_int64(), C.c_int64(), C.c_int(), C.c_int64()
    _check(lib().bhac_get_stats(h, C.byref(f), C.byref(fl), C.byref(it), C.byref(bk)))
    return dict(c2p_fail=f.value, floor_hits=fl.value, max_iter=it.value, c2p_backup=bk.value)


def bhac_get_schedule(h) -> dict:
    o = bhac_schedule()
    _check(lib().bhac_get_schedule(h, C.byref(o)))
    return dict(march_mask=o.march_mask, march_faces=o.march_faces, x1_staged=o.x1_staged)


def bhac_reset_stats(h, stream=None):
    _check(lib().bhac_reset_stats(h, _stream(stream)))


def bhac_capture_rk2_step(h, U, P, U1, P1):
    _check(lib().bhac_capture_rk2_step(h, _ptr(U), _ptr(P), _ptr(U1), _ptr(P1)))


def bhac_capture_rk2_step_ct(h, U, P, U1, P1, phi, phi1):
    _check(lib().bhac_capture_rk2_step_ct(h, _ptr(U), _ptr(P), _ptr(U1), _ptr(P1), _ptr(phi), _ptr(phi1)))


def bhac_launch_rk2_step(h, stream=None):
    _check(lib().bhac_launch_rk2_step(h, _stream(stream)))


def bhac_set_timing(h, enable: bool):
    _check(lib().bhac_set_timing(h, 1 if enable else 0))


def bhac_get_timing(h) -> dict:
    """{kernel family: (launches, total_ms)} since the last call (synchronises)."""
    arr = (bhac_kernel_time * 32)()
    n = C.c_int(0)
    _check(lib().bhac_get_timing(h, arr, 32, C.byref(n)))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(n.value, 32))}


# --- convenience wrapper around one grid ---------------------------------------------
class Grid:
    """A grid on the current ROCm device plus helpers to move states in and out."""

    def __init__(self, params: dict, blocks: np.ndarray, device="cuda"):
        import torch
        self.torch = torch
        self.params = dict(params)
        self.blocks = np.asarray(blocks, dtype=np.int32)
        self.device = torch.device(device)
        self.h, lay = bhac_alloc_blocks(params, self.blocks)
        self.ncp = lay["ncell_padded"]
        self.nci = lay["ncell_interior"]
        self.off = lay["block_offset"]
        self.ioff = lay["block_interior_offset"]
        self.nvar = lay["nvar"]
        self.pdtype = torch.float32 if int(params["precision"]) == 1 else torch.float64
        self._pidx = None

    def close(self):
        if self.h:
            bhac_free_blocks(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def interior_index(self) -> np.ndarray:
        """Index in P of every interior cell, interior-packed order (block-major, x
        fastest): each block's interior cells lead its region of P."""
        if self._pidx is None:
            parts = [self.off[b] + np.arange(int(np.prod(blk[1:4])), dtype=np.int64)
                     for b, blk in enumerate(self.blocks)]
            self._pidx = np.concatenate(parts).astype(np.int64)
        return self._pidx

    def new_state(self, kind="P"):
        """Primitive state [nvar][ncell_padded] (float or double) or conserved [nvar][ncell_interior]."""
        if kind == "P":
            return self.torch.zeros((self.nvar, self.ncp), dtype=self.pdtype, device=self.device)
        return self.torch.zeros((self.nvar, self.nci), dtype=self.torch.float64, device=self.device)

    def pack(self, prim_interior: np.ndarray):
        """Interior-packed primitives -> padded device array (ghost slots zero)."""
        out = np.zeros((self.nvar, self.ncp), dtype=np.float64)
        out[:, self.interior_index()] = prim_interior
        return self.torch.from_numpy(out).to(device=self.device, dtype=self.pdtype)

    def unpack(self, t) -> np.ndarray:
        """Device state -> interior-packed float64 host array (P or U)."""
        a = t.detach().to("cpu", self.torch.float64).numpy()
        if a.shape[1] == self.nci and self.nci != self.ncp:
            return np.ascontiguousarray(a)
        return np.ascontiguousarray(a[:, self.interior_index()])

    def fill_ghosts(self, P):
        bhac_fill_ghosts(self.h, P)

    def fill_ghost_faces(self, P):
        bhac_fill_ghost_faces(self.h, P)

    def prim2con(self, P, U):
        bhac_prim2con(self.h, P, U)

    def con2prim(self, U, P, fail=None):
        bhac_con2prim(self.h, U, P, fail)

    def compute_dt(self, P):
        bhac_compute_dt(self.h, P)

    def set_dt(self, dt):
        bhac_set_dt(self.h, dt)

    def substep(self, Ub, Us, Ps, Uo, Po, a, b):
        bhac_substep(self.h, Ub, Us, Ps, Uo, Po, a, b)

    def substep_noalloc(self, Ub, Us, Ps, Uo, Po, a, b):
        bhac_substep_noalloc(self.h, Ub, Us, Ps, Uo, Po, a, b)

    # --- staggered face field (constrained transport, params ct = 1) -----------------
    def face_count(self):
        return bhac_face_count(self.h)

    def new_faces(self):
        return self.torch.zeros(sum(self.face_count()), dtype=self.torch.float64, device=self.device)

    def substep_ct(self, Ub, Us, Ps, Phib, Phis, Uo, Po, Phio, a, b):
        bhac_substep_ct(self.h, Ub, Us, Ps, Phib, Phis, Uo, Po, Phio, a, b)

    def ct_divergence(self, phi):
        div = self.torch.zeros(self.nci, dtype=self.torch.float64, device=self.device)
        bhac_ct_divergence(self.h, phi, div)
        return div

    def init_ct(self, prim_interior, phi_host):
        """Device P (field rows from the face field, ghosts filled), U = prim2con(P),
        the face field on the device, and the initial wave-speed reduction."""
        P = self.pack(prim_interior)
        phi = self.torch.from_numpy(np.ascontiguousarray(phi_host, dtype=np.float64)).to(self.device)
        bhac_ct_center(self.h, phi, P)
        U = self.new_state("U")
        self.fill_ghosts(P)
        self.prim2con(P, U)
        self.compute_dt(P)
        return U, P, phi

    def rk2_step_ct(self, U, P, phi, U1, P1, phi1):
        """One SSP-RK2 step in place on (U, P, phi) with scratch (U1, P1, phi1)."""
        self.substep_ct(U, U, P, phi, phi, U1, P1, phi1, 0.0, 1.0)
        self.substep_ct(U, U1, P1, phi, phi1, U, P, phi, 0.5, 0.5)

    def init(self, prim_interior):
        """Device P (ghosts filled), U = prim2con(P) and the initial wave-speed reduction."""
        P = self.pack(prim_interior)
        U = self.new_state("U")
        self.fill_ghosts(P)
        self.prim2con(P, U)
        self.compute_dt(P)
        return U, P

    def rk2_step(self, U, P, U1, P1):
        """One SSP-RK2 step in place on (U, P) with scratch (U1, P1). The substeps
        read each block's halo from its neighbours, so no ghost fill is needed."""
        self.substep(U, U, P, U1, P1, 0.0, 1.0)
        self.substep(U, U1, P1, U, P, 0.5, 0.5)

    def capture_rk2_step(self, U, P, U1, P1):
        bhac_capture_rk2_step(self.h, U, P, U1, P1)

    def capture_rk2_step_ct(self, U, P, U1, P1, phi, phi1):
        bhac_capture_rk2_step_ct(self.h, U, P, U1, P1, phi, phi1)

    def launch_rk2_step(self):
        bhac_launch_rk2_step(self.h)

    def run(self, prim_interior, steps):
        U, P = self.init(prim_interior)
        U1, P1 = self.new_state("U"), self.new_state("P")
        for _ in range(steps):
            self.rk2_step(U, P, U1, P1)
        return U, P

    def timestep(self):
        return bhac_get_timestep(self.h)

    def stats(self):
        return bhac_get_stats(self.h)

    def schedule(self):
        return bhac_get_schedule(self.h)

    def reset_stats(self):
        bhac_reset_stats(self.h)
