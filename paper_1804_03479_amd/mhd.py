"""Thin Python binding of libmhd (ctypes).  Argument marshalling only: every
step of the update runs in the library's HIP kernels.  PyTorch provides the
device memory and the stream.

The library must have been built (``paper_1804_03479_amd.build``); loading
fails loudly otherwise, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhd.so")

VL, CTU = 0, 1
PLM, PPM = 0, 1
ROE, HLLE, HLLD, MLP = 0, 1, 2, 3
F64, F32, F32_MIXED = 0, 1, 2

SCHEMES = {"vl": VL, "ctu": CTU}
RECONS = {"plm": PLM, "ppm": PPM}
SOLVERS = {"roe": ROE, "hlle": HLLE, "hlld": HLLD, "mlp": MLP}
PRECS = {"f64": F64, "f32": F32, "f32_mixed": F32_MIXED}

ERRORS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "ghost too small", -4: "HIP error",
          -5: "non-physical state", -6: "no device", -7: "out of memory"}


class MHDError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(status, status)} ({status})")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("recon", ctypes.c_int), ("riemann", ctypes.c_int),
                ("prec", ctypes.c_int), ("gamma", ctypes.c_double), ("courant", ctypes.c_double),
                ("beta_fp64", ctypes.c_double), ("mlp_dp", ctypes.c_double), ("mlp_drho", ctypes.c_double)]


class LevelDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx", ctypes.c_double),
                ("n_groups", ctypes.c_int), ("group_edge", ctypes.c_int), ("groups", ctypes.c_void_p),
                ("U", ctypes.c_void_p), ("B", ctypes.c_void_p), ("E64", ctypes.c_void_p)]


_lib = None

EXPORTS = ["mhd_abi_version", "mhd_strerror", "mhd_required_ghost", "mhd_init", "mhd_finalize",
           "mhd_check_level", "mhd_prim_to_cons", "mhd_cfl_dt", "mhd_step", "mhd_step_devdt",
           "mhd_advance", "mhd_divB", "mhd_sums", "mhd_fallback_count", "mhd_sync",
           "mhd_profile_step", "mhd_num_stages", "mhd_stage_name"]


def load(path: str = LIB_PATH):
    """Load libmhd.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmhd not built: {path} is missing (run paper_1804_03479_amd.build())")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.mhd_strerror.restype = ctypes.c_char_p
    lib.mhd_strerror.argtypes = [I]
    lib.mhd_required_ghost.argtypes = [I, I]
    lib.mhd_init.argtypes = [ctypes.POINTER(Config), P, ctypes.POINTER(P)]
    lib.mhd_finalize.argtypes = [P]
    lib.mhd_check_level.argtypes = [P, ctypes.POINTER(LevelDesc)]
    lib.mhd_prim_to_cons.argtypes = [P, ctypes.POINTER(LevelDesc), P]
    lib.mhd_cfl_dt.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(D), P]
    lib.mhd_step.argtypes = [P, ctypes.POINTER(LevelDesc), D]
    lib.mhd_step_devdt.argtypes = [P, ctypes.POINTER(LevelDesc), P]
    lib.mhd_advance.argtypes = [P, ctypes.POINTER(LevelDesc), P, P]
    lib.mhd_divB.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.mhd_sums.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(D * 7)]
    lib.mhd_fallback_count.argtypes = [P, ctypes.POINTER(ctypes.c_longlong)]
    lib.mhd_sync.argtypes = [P]
    lib.mhd_profile_step.argtypes = [P, ctypes.POINTER(LevelDesc), I, P]
    lib.mhd_num_stages.argtypes = [P]
    lib.mhd_stage_name.restype = ctypes.c_char_p
    lib.mhd_stage_name.argtypes = [P, I]
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        raise MHDError(status, what)


def dtype_of(prec: int):
    return torch.float64 if prec == F64 else torch.float32


class Level:
    """A dense periodic level: conserved U (5, nz, ny, nx), face B (3, nz, ny, nx).

    ``groups`` is an optional int32 tensor (n, 3) of group origins in cells; only
    those patch groups are updated and the rest of the grid acts as ghosts.
    """

    def __init__(self, U: torch.Tensor, B: torch.Tensor, dx: float, groups: torch.Tensor | None = None,
                 group_edge: int = 16, E64: torch.Tensor | None = None):
        if U.dim() != 4 or U.shape[0] != 5 or B.shape != (3,) + tuple(U.shape[1:]):
            raise ValueError("U must be (5, nz, ny, nx) and B (3, nz, ny, nx)")
        if not (U.is_cuda and B.is_cuda and U.is_contiguous() and B.is_contiguous()):
            raise ValueError("U and B must be contiguous device tensors")
        if U.dtype != B.dtype:
            raise ValueError("U and B must share a dtype")
        self.U, self.B, self.dx = U, B, float(dx)
        self.E64 = E64
        self.group_edge = int(group_edge)
        self.set_groups(groups)

    def set_groups(self, groups):
        if groups is not None:
            if groups.dtype != torch.int32 or not groups.is_cuda or groups.dim() != 2 or groups.shape[1] != 3:
                raise ValueError("groups must be an int32 device tensor of shape (n, 3)")
            groups = groups.contiguous()
        self.groups = groups

    @property
    def shape(self):
        return tuple(self.U.shape[1:])

    def desc(self) -> LevelDesc:
        nz, ny, nx = self.shape
        g = self.groups
        return LevelDesc(nx, ny, nz, self.dx, 0 if g is None else int(g.shape[0]), self.group_edge,
                         None if g is None else g.data_ptr(), self.U.data_ptr(), self.B.data_ptr(),
                         None if self.E64 is None else self.E64.data_ptr())


class Solver:
    """One libmhd context on the current torch stream."""

    def __init__(self, scheme="vl", recon="plm", riemann="roe", prec="f64", gamma=5.0 / 3.0,
                 courant=0.5, beta_fp64=0.1, mlp_dp=0.3, mlp_drho=0.3, stream: torch.cuda.Stream | None = None):
        self.lib = load()
        self.cfg = Config(SCHEMES[scheme], RECONS[recon], SOLVERS[riemann], PRECS[prec], gamma, courant,
                          beta_fp64, mlp_dp, mlp_drho)
        self.prec = PRECS[prec]
        self.dtype = dtype_of(self.prec)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(self.lib.mhd_init(ctypes.byref(self.cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "mhd_init")
        self.h = h

    def close(self):
        if self.h:
            self.lib.mhd_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state set-up
    def level_from_primitives(self, W5: torch.Tensor, B: torch.Tensor, dx: float, groups=None,
                              group_edge: int = 16) -> Level:
        W5 = W5.to(device="cuda", dtype=self.dtype).contiguous()
        B = B.to(device="cuda", dtype=self.dtype).contiguous()
        U = torch.empty_like(W5)
        lv = Level(U, B, dx, groups, group_edge)
        self.prim_to_cons(lv, W5)
        return lv

    def prim_to_cons(self, lv: Level, W5: torch.Tensor):
        if W5.shape != lv.U.shape or W5.dtype != self.dtype or not W5.is_contiguous():
            raise ValueError("W5 must match U in shape and dtype")
        d = lv.desc()
        _check(self.lib.mhd_prim_to_cons(self.h, ctypes.byref(d), ctypes.c_void_p(W5.data_ptr())), "mhd_prim_to_cons")

    def _check_level(self, lv: Level):
        if lv.U.dtype != self.dtype:
            raise ValueError(f"level dtype {lv.U.dtype} does not match solver precision {self.dtype}")

    # -- the update
    def cfl_dt(self, lv: Level) -> float:
        self._check_level(lv)
        d = lv.desc()
        dt = ctypes.c_double()
        _check(self.lib.mhd_cfl_dt(self.h, ctypes.byref(d), ctypes.byref(dt), None), "mhd_cfl_dt")
        return dt.value

    def cfl_dt_device(self, lv: Level, out: torch.Tensor):
        d = lv.desc()
        _check(self.lib.mhd_cfl_dt(self.h, ctypes.byref(d), None, ctypes.c_void_p(out.data_ptr())), "mhd_cfl_dt")

    def step(self, lv: Level, dt: float):
        self._check_level(lv)
        d = lv.desc()
        _check(self.lib.mhd_step(self.h, ctypes.byref(d), float(dt)), "mhd_step")

    def step_devdt(self, lv: Level, dt_dev: torch.Tensor):
        d = lv.desc()
        _check(self.lib.mhd_step_devdt(self.h, ctypes.byref(d), ctypes.c_void_p(dt_dev.data_ptr())), "mhd_step_devdt")

    def advance(self, lv: Level, dt_dev: torch.Tensor | None = None, t_dev: torch.Tensor | None = None):
        self._check_level(lv)
        d = lv.desc()
        _check(self.lib.mhd_advance(self.h, ctypes.byref(d),
                                    None if dt_dev is None else ctypes.c_void_p(dt_dev.data_ptr()),
                                    None if t_dev is None else ctypes.c_void_p(t_dev.data_ptr())), "mhd_advance")

    # -- diagnostics
    def divb(self, lv: Level):
        d = lv.desc()
        mx, l1 = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.mhd_divB(self.h, ctypes.byref(d), ctypes.byref(mx), ctypes.byref(l1)), "mhd_divB")
        return mx.value, l1.value

    def sums(self, lv: Level):
        d = lv.desc()
        out = (ctypes.c_double * 7)()
        _check(self.lib.mhd_sums(self.h, ctypes.byref(d), ctypes.byref(out)), "mhd_sums")
        return list(out)

    def fallback_count(self) -> int:
        v = ctypes.c_longlong()
        _check(self.lib.mhd_fallback_count(self.h, ctypes.byref(v)), "mhd_fallback_count")
        return v.value

    def sync(self):
        _check(self.lib.mhd_sync(self.h), "mhd_sync")

    def profile_step(self, lv: Level, nrep: int = 5) -> dict:
        """Mean milliseconds per stage over nrep advancing steps."""
        n = self.lib.mhd_num_stages(self.h)
        out = (ctypes.c_double * n)()
        d = lv.desc()
        _check(self.lib.mhd_profile_step(self.h, ctypes.byref(d), int(nrep), ctypes.cast(out, ctypes.c_void_p)),
               "mhd_profile_step")
        return {self.lib.mhd_stage_name(self.h, s).decode(): out[s] for s in range(n)}
