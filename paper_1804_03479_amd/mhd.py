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

ERRORS = {0: "ok", -1: "invalid argument", -2: "unsupported", -4: "HIP error",
          -5: "non-physical state", -6: "no device", -7: "out of memory", -8: "static scratch too small"}
SCRATCH_LIMIT = -8


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
                ("U", ctypes.c_void_p), ("B", ctypes.c_void_p), ("E64", ctypes.c_void_p),
                ("n_groups_dev", ctypes.c_void_p)]


_lib = None

EXPORTS = ["mhd_abi_version", "mhd_strerror", "mhd_required_ghost", "mhd_init", "mhd_finalize",
           "mhd_check_level", "mhd_prim_to_cons", "mhd_cfl_dt", "mhd_step", "mhd_step_devdt",
           "mhd_advance", "mhd_divB", "mhd_sums", "mhd_fallback_count", "mhd_sync",
           "mhd_profile_step", "mhd_num_stages", "mhd_stage_name",
           "mhd_mlp_num_params", "mhd_mlp_set_weights", "mhd_mlp_forward", "mhd_mlp_backward",
           "mhd_mlp_train_step", "mhd_mlp_prepare", "mhd_mlp_face_flux", "mhd_set_capture", "mhd_correct",
           "mhd_advance_graph", "mhd_set_launch", "mhd_cfl_dt_min", "mhd_prolong", "mhd_restrict",
           "mhd_prolong_time", "mhd_accumulate_registers", "mhd_dt_subdivide", "mhd_regrid_flag",
           "mhd_prolong_new_groups", "mhd_workspace_bytes", "mhd_step_noalloc"]


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
    lib.mhd_step_noalloc.argtypes = [P, ctypes.POINTER(LevelDesc), P]
    lib.mhd_advance.argtypes = [P, ctypes.POINTER(LevelDesc), P, P]
    lib.mhd_divB.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.mhd_sums.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(D * 7)]
    lib.mhd_fallback_count.argtypes = [P, ctypes.POINTER(ctypes.c_longlong)]
    lib.mhd_sync.argtypes = [P]
    lib.mhd_profile_step.argtypes = [P, ctypes.POINTER(LevelDesc), I, P]
    lib.mhd_num_stages.argtypes = [P]
    lib.mhd_stage_name.restype = ctypes.c_char_p
    lib.mhd_stage_name.argtypes = [P, I]
    lib.mhd_mlp_num_params.argtypes = []
    lib.mhd_mlp_set_weights.argtypes = [P, P]
    lib.mhd_mlp_forward.argtypes = [P, P, P, I, P]
    lib.mhd_mlp_backward.argtypes = [P, P, P, P, I, P]
    lib.mhd_mlp_train_step.argtypes = [P, P, P, P, P, I, P, P, I, ctypes.c_float, P]
    lib.mhd_mlp_prepare.argtypes = [P, P, I, P, P, P]
    lib.mhd_mlp_face_flux.argtypes = [P, P, I, P, P]
    lib.mhd_set_capture.argtypes = [P, P, ctypes.c_longlong, P, I]
    lib.mhd_advance_graph.argtypes = [P, ctypes.POINTER(LevelDesc), P, P]
    lib.mhd_set_launch.argtypes = [P, I, I, I, I]
    lib.mhd_cfl_dt_min.argtypes = [P, ctypes.POINTER(LevelDesc), D, P]
    lib.mhd_dt_subdivide.argtypes = [P, P, I, P]
    lib.mhd_prolong_time.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(LevelDesc), D,
                                     ctypes.POINTER(LevelDesc), I]
    lib.mhd_accumulate_registers.argtypes = [P, ctypes.POINTER(LevelDesc), D, I]
    lib.mhd_workspace_bytes.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(ctypes.c_size_t)]
    lib.mhd_regrid_flag.argtypes = [P, ctypes.POINTER(LevelDesc), D, I, I, P, I, P, P]
    lib.mhd_prolong_new_groups.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(LevelDesc),
                                           ctypes.POINTER(LevelDesc)]
    lib.mhd_prolong.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(LevelDesc), I]
    lib.mhd_restrict.argtypes = [P, ctypes.POINTER(LevelDesc), ctypes.POINTER(LevelDesc)]
    lib.mhd_correct.argtypes = [P, ctypes.POINTER(LevelDesc), P, ctypes.POINTER(LevelDesc), P, I]
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        raise MHDError(status, what)


def dtype_of(prec: int):
    return torch.float64 if prec == F64 else torch.float32


def check_group_origins(origins, shape, edge: int):
    """Raise ValueError unless every (x, y, z) origin row is a multiple of edge
    inside the grid of shape (nz, ny, nx) and no origin is listed twice."""
    import numpy as np
    o = np.asarray(origins, dtype=np.int64).reshape(-1, 3)
    nz, ny, nx = shape
    if edge <= 0 or nx % edge or ny % edge or nz % edge:
        raise ValueError(f"group edge {edge} must divide the grid {shape}")
    if o.size == 0:
        return
    if (o < 0).any() or (o[:, 0] >= nx).any() or (o[:, 1] >= ny).any() or (o[:, 2] >= nz).any():
        raise ValueError("group origins must lie inside the grid")
    if (o % edge).any():
        raise ValueError(f"group origins must be multiples of the group edge {edge}")
    if len(np.unique(o, axis=0)) != len(o):
        raise ValueError("group origins must be unique")


def check_dt_tensor(t, what: str = "dt"):
    """A device time step or time: one contiguous float64 element on the GPU."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() >= 1):
        raise ValueError(f"{what} must be a contiguous float64 device tensor")


class Level:
    """A dense periodic level: conserved U (5, nz, ny, nx), face B (3, nz, ny, nx).

    ``groups`` is an optional int32 tensor (n, 3) of group origins in cells; only
    those patch groups are updated and the rest of the grid acts as ghosts.
    """

    def __init__(self, U: torch.Tensor, B: torch.Tensor, dx: float, groups: torch.Tensor | None = None,
                 group_edge: int = 16, E64: torch.Tensor | None = None, validate_groups: bool = True):
        if U.dim() != 4 or U.shape[0] != 5 or B.shape != (3,) + tuple(U.shape[1:]):
            raise ValueError("U must be (5, nz, ny, nx) and B (3, nz, ny, nx)")
        if not (U.is_cuda and B.is_cuda and U.is_contiguous() and B.is_contiguous()):
            raise ValueError("U and B must be contiguous device tensors")
        if U.dtype != B.dtype:
            raise ValueError("U and B must share a dtype")
        self.U, self.B, self.dx = U, B, float(dx)
        self.E64 = E64
        self.group_edge = int(group_edge)
        self.n_groups_dev = None
        self.set_groups(groups, validate=validate_groups)

    def set_groups(self, groups, validate: bool = True):
        """Group list of the level.  With validate (the default) the origins are
        checked on the host: multiples of group_edge inside the grid, no
        duplicates (a duplicate would update its cells twice in place).  Lists
        written on the device by the library's regridding are valid by
        construction and pass validate=False (their contents are not on the
        host)."""
        if groups is not None:
            if groups.dtype != torch.int32 or not groups.is_cuda or groups.dim() != 2 or groups.shape[1] != 3:
                raise ValueError("groups must be an int32 device tensor of shape (n, 3)")
            groups = groups.contiguous()
            if validate:
                check_group_origins(groups.cpu().numpy(), self.shape, self.group_edge)
        self.groups = groups

    @property
    def shape(self):
        return tuple(self.U.shape[1:])

    def desc(self) -> LevelDesc:
        nz, ny, nx = self.shape
        g = self.groups
        return LevelDesc(nx, ny, nz, self.dx, 0 if g is None else int(g.shape[0]), self.group_edge,
                         None if g is None else g.data_ptr(), self.U.data_ptr(), self.B.data_ptr(),
                         None if self.E64 is None else self.E64.data_ptr(),
                         None if self.n_groups_dev is None else self.n_groups_dev.data_ptr())


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
        E64 = None
        if self.prec == F32_MIXED:
            E64 = torch.empty(tuple(U.shape[1:]), dtype=torch.float64, device="cuda")
        lv = Level(U, B, dx, groups, group_edge, E64=E64)
        self.prim_to_cons(lv, W5)
        return lv

    def prim_to_cons(self, lv: Level, W5: torch.Tensor):
        self._check_level(lv)
        if W5.shape != lv.U.shape or W5.dtype != self.dtype or not W5.is_contiguous():
            raise ValueError("W5 must match U in shape and dtype")
        d = lv.desc()
        _check(self.lib.mhd_prim_to_cons(self.h, ctypes.byref(d), ctypes.c_void_p(W5.data_ptr())), "mhd_prim_to_cons")

    def _check_level(self, lv: Level):
        """dtype and shape checks the C side cannot make (it sees no element size)."""
        if not isinstance(lv, Level):
            raise ValueError("expected a Level")
        if lv.U.dtype != self.dtype or lv.B.dtype != self.dtype:
            raise ValueError(f"level dtype {lv.U.dtype} does not match solver precision {self.dtype}")
        if self.prec == F32_MIXED:
            e = lv.E64
            if e is None or e.dtype != torch.float64 or tuple(e.shape) != lv.shape or not e.is_contiguous():
                raise ValueError("the mixed form needs a contiguous float64 E64 of the grid's shape")

    # -- the update
    def cfl_dt(self, lv: Level) -> float:
        self._check_level(lv)
        d = lv.desc()
        dt = ctypes.c_double()
        _check(self.lib.mhd_cfl_dt(self.h, ctypes.byref(d), ctypes.byref(dt), None), "mhd_cfl_dt")
        return dt.value

    def cfl_dt_device(self, lv: Level, out: torch.Tensor):
        self._check_level(lv)
        check_dt_tensor(out, "out")
        d = lv.desc()
        _check(self.lib.mhd_cfl_dt(self.h, ctypes.byref(d), None, ctypes.c_void_p(out.data_ptr())), "mhd_cfl_dt")

    def step(self, lv: Level, dt: float):
        self._check_level(lv)
        d = lv.desc()
        _check(self.lib.mhd_step(self.h, ctypes.byref(d), float(dt)), "mhd_step")

    def step_devdt(self, lv: Level, dt_dev: torch.Tensor):
        self._check_level(lv)
        check_dt_tensor(dt_dev, "dt_dev")
        d = lv.desc()
        _check(self.lib.mhd_step_devdt(self.h, ctypes.byref(d), ctypes.c_void_p(dt_dev.data_ptr())), "mhd_step_devdt")

    def step_noalloc(self, lv: Level, dt_dev: torch.Tensor):
        """mhd_step_devdt with the library's static scratch (no device allocation)."""
        self._check_level(lv)
        check_dt_tensor(dt_dev, "dt_dev")
        d = lv.desc()
        _check(self.lib.mhd_step_noalloc(self.h, ctypes.byref(d), ctypes.c_void_p(dt_dev.data_ptr())),
               "mhd_step_noalloc")

    def advance(self, lv: Level, dt_dev: torch.Tensor | None = None, t_dev: torch.Tensor | None = None):
        self._check_level(lv)
        for t, nm in ((dt_dev, "dt_dev"), (t_dev, "t_dev")):
            if t is not None:
                check_dt_tensor(t, nm)
        d = lv.desc()
        _check(self.lib.mhd_advance(self.h, ctypes.byref(d),
                                    None if dt_dev is None else ctypes.c_void_p(dt_dev.data_ptr()),
                                    None if t_dev is None else ctypes.c_void_p(t_dev.data_ptr())), "mhd_advance")

    def advance_graph(self, lv: Level, dt_dev: torch.Tensor | None = None, t_dev: torch.Tensor | None = None):
        """mhd_advance replayed from a captured HIP graph (needs a non-default stream)."""
        self._check_level(lv)
        for t, nm in ((dt_dev, "dt_dev"), (t_dev, "t_dev")):
            if t is not None:
                check_dt_tensor(t, nm)
        d = lv.desc()
        _check(self.lib.mhd_advance_graph(self.h, ctypes.byref(d),
                                          None if dt_dev is None else ctypes.c_void_p(dt_dev.data_ptr()),
                                          None if t_dev is None else ctypes.c_void_p(t_dev.data_ptr())),
               "mhd_advance_graph")

    def set_launch(self, blocks_per_cu: int = 0, threads: int = 0, batch: int = 0, tiles: int = 0):
        """Launch shape of the stage kernels: blocks per CU of the persistent
        grid (0: one item per thread), threads per block (0: 256), the
        group-list batch of the middle stages (0: the whole list) and, for
        CTU with PPM, the reconstruction stage on LDS tiles (1) or per cell
        (0)."""
        _check(self.lib.mhd_set_launch(self.h, int(blocks_per_cu), int(threads), int(batch), int(tiles)),
               "mhd_set_launch")

    def cfl_dt_min(self, lv: Level, dt_dev: torch.Tensor, scale: float = 1.0):
        self._check_level(lv)
        check_dt_tensor(dt_dev, "dt_dev")
        d = lv.desc()
        _check(self.lib.mhd_cfl_dt_min(self.h, ctypes.byref(d), float(scale), ctypes.c_void_p(dt_dev.data_ptr())),
               "mhd_cfl_dt_min")

    def dt_subdivide(self, dt_coarse: torch.Tensor, parts: int, dt_fine: torch.Tensor):
        check_dt_tensor(dt_coarse, "dt_coarse")
        check_dt_tensor(dt_fine, "dt_fine")
        _check(self.lib.mhd_dt_subdivide(self.h, ctypes.c_void_p(dt_coarse.data_ptr()), int(parts),
                                         ctypes.c_void_p(dt_fine.data_ptr())), "mhd_dt_subdivide")

    def prolong(self, coarse: Level, fine: Level, halo: int = 4, coarse_old: Level | None = None,
                alpha: float = 1.0):
        """Fine level (or its ghost halos) from the coarse level; with coarse_old,
        from old + alpha (coarse - old)."""
        self._check_level(coarse)
        self._check_level(fine)
        if coarse_old is not None:
            self._check_level(coarse_old)
        dc, df = coarse.desc(), fine.desc()
        if coarse_old is None and alpha == 1.0:
            _check(self.lib.mhd_prolong(self.h, ctypes.byref(dc), ctypes.byref(df), int(halo)), "mhd_prolong")
            return
        do = None if coarse_old is None else ctypes.byref(coarse_old.desc())
        _check(self.lib.mhd_prolong_time(self.h, do, ctypes.byref(dc), float(alpha), ctypes.byref(df), int(halo)),
               "mhd_prolong_time")

    def workspace_bytes(self, lv: Level) -> int:
        """Device bytes of stage scratch this context needs to update lv."""
        self._check_level(lv)
        d = lv.desc()
        v = ctypes.c_size_t()
        _check(self.lib.mhd_workspace_bytes(self.h, ctypes.byref(d), ctypes.byref(v)), "mhd_workspace_bytes")
        return v.value

    def regrid_flag(self, coarse: Level, threshold: float, buffer: int, fine_edge: int, groups_out: torch.Tensor,
                    count: torch.Tensor, wanted: torch.Tensor):
        """Group list of the level above coarse from the refinement criterion
        into groups_out (int32 (capacity, 3)), count and wanted (int32 (1,))."""
        for t in (groups_out, count, wanted):
            if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("regrid outputs must be contiguous int32 device tensors")
        if groups_out.dim() != 2 or groups_out.shape[1] != 3:
            raise ValueError("groups_out must be (capacity, 3)")
        self._check_level(coarse)
        d = coarse.desc()
        _check(self.lib.mhd_regrid_flag(self.h, ctypes.byref(d), float(threshold), int(buffer), int(fine_edge),
                                        ctypes.c_void_p(groups_out.data_ptr()), int(groups_out.shape[0]),
                                        ctypes.c_void_p(count.data_ptr()), ctypes.c_void_p(wanted.data_ptr())),
               "mhd_regrid_flag")

    def prolong_new_groups(self, coarse: Level, fine_new: Level, fine_old: Level | None):
        for lv in (coarse, fine_new) + (() if fine_old is None else (fine_old,)):
            self._check_level(lv)
        dc, dn = coarse.desc(), fine_new.desc()
        do = None if fine_old is None else ctypes.byref(fine_old.desc())
        _check(self.lib.mhd_prolong_new_groups(self.h, ctypes.byref(dc), ctypes.byref(dn), do),
               "mhd_prolong_new_groups")

    def accumulate_registers(self, lv: Level, weight: float, reset: bool):
        self._check_level(lv)
        d = lv.desc()
        _check(self.lib.mhd_accumulate_registers(self.h, ctypes.byref(d), float(weight), int(bool(reset))),
               "mhd_accumulate_registers")

    def correct(self, coarse: Level, fine_solver: "Solver", fine: Level, dt_dev: torch.Tensor,
                fine_registers: bool = False):
        """Coarse-fine flux and EMF correction after both levels covered the coarse
        step dt_dev (fine_registers: the fine level sub-cycled and accumulated)."""
        self._check_level(coarse)
        fine_solver._check_level(fine)
        check_dt_tensor(dt_dev, "dt_dev")
        dc, df = coarse.desc(), fine.desc()
        _check(self.lib.mhd_correct(self.h, ctypes.byref(dc), fine_solver.h, ctypes.byref(df),
                                    ctypes.c_void_p(dt_dev.data_ptr()), int(bool(fine_registers))), "mhd_correct")

    def restrict(self, fine: Level, coarse: Level):
        self._check_level(fine)
        self._check_level(coarse)
        dc, df = coarse.desc(), fine.desc()
        _check(self.lib.mhd_restrict(self.h, ctypes.byref(df), ctypes.byref(dc)), "mhd_restrict")

    # -- diagnostics
    def divb(self, lv: Level):
        self._check_level(lv)
        d = lv.desc()
        mx, l1 = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.mhd_divB(self.h, ctypes.byref(d), ctypes.byref(mx), ctypes.byref(l1)), "mhd_divB")
        return mx.value, l1.value

    def sums(self, lv: Level):
        self._check_level(lv)
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
        self._check_level(lv)
        n = self.lib.mhd_num_stages(self.h)
        out = (ctypes.c_double * n)()
        d = lv.desc()
        _check(self.lib.mhd_profile_step(self.h, ctypes.byref(d), int(nrep), ctypes.cast(out, ctypes.c_void_p)),
               "mhd_profile_step")
        return {self.lib.mhd_stage_name(self.h, s).decode(): out[s] for s in range(n)}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, shape=None, what="tensor"):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {shape}, got {tuple(t.shape)}")
    return t


class MlpOps:
    """Learned-flux entry points of one Solver (its context and stream)."""

    def __init__(self, solver: Solver):
        self.s = solver
        self.lib = solver.lib
        self.nparam = self.lib.mhd_mlp_num_params()

    def set_weights(self, params):
        _dev_f32(params, (self.nparam,), "params")
        _check(self.lib.mhd_mlp_set_weights(self.s.h, _ptr(params)), "mhd_mlp_set_weights")

    def forward(self, params, X):
        n = X.shape[0]
        _dev_f32(params, (self.nparam,), "params")
        _dev_f32(X, (n, 15), "X")
        Y = torch.empty((n, 7), dtype=torch.float32, device="cuda")
        _check(self.lib.mhd_mlp_forward(self.s.h, _ptr(params), _ptr(X), n, _ptr(Y)), "mhd_mlp_forward")
        return Y

    def backward(self, params, X, dY):
        n = X.shape[0]
        _dev_f32(params, (self.nparam,), "params")
        _dev_f32(X, (n, 15), "X")
        _dev_f32(dY, (n, 7), "dY")
        G = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check(self.lib.mhd_mlp_backward(self.s.h, _ptr(params), _ptr(X), _ptr(dY), n, _ptr(G)), "mhd_mlp_backward")
        return G

    def train_step(self, params, m, v, grads, step: int, X, T, lr: float, loss=None):
        n = X.shape[0]
        for t, nm in ((params, "params"), (m, "adam_m"), (v, "adam_v"), (grads, "grads")):
            _dev_f32(t, (self.nparam,), nm)
        _dev_f32(X, (n, 15), "X")
        _dev_f32(T, (n, 7), "T")
        _check(self.lib.mhd_mlp_train_step(self.s.h, _ptr(params), _ptr(m), _ptr(v), _ptr(grads), int(step), _ptr(X),
                                           _ptr(T), n, float(lr), _ptr(loss)), "mhd_mlp_train_step")

    def prepare(self, samples):
        n = samples.shape[0]
        _dev_f32(samples, (n, 22), "samples")
        X = torch.empty((n, 15), dtype=torch.float32, device="cuda")
        T = torch.empty((n, 7), dtype=torch.float32, device="cuda")
        F = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(self.lib.mhd_mlp_prepare(self.s.h, _ptr(samples), n, _ptr(X), _ptr(T), _ptr(F)), "mhd_mlp_prepare")
        return X, T, F

    def face_flux(self, states):
        n = states.shape[0]
        _dev_f32(states, (n, 15), "states")
        Fl = torch.empty((n, 7), dtype=torch.float32, device="cuda")
        used = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(self.lib.mhd_mlp_face_flux(self.s.h, _ptr(states), n, _ptr(Fl), _ptr(used)), "mhd_mlp_face_flux")
        return Fl, used

    def set_capture(self, buf=None, count=None, stride: int = 1):
        if buf is None:
            _check(self.lib.mhd_set_capture(self.s.h, None, 0, None, 1), "mhd_set_capture")
            return
        _dev_f32(buf, (buf.shape[0], 22), "capture buffer")
        if not (count.is_cuda and count.dtype == torch.int64 and count.numel() == 1):
            raise ValueError("count must be a one-element int64 device tensor")
        _check(self.lib.mhd_set_capture(self.s.h, _ptr(buf), buf.shape[0], _ptr(count), int(stride)),
               "mhd_set_capture")
