"""FP64 CPU oracle of the unsplit ideal-MHD update (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never loads
it, shares no source with it, and has no CPU fallback through it.

The arithmetic lives in ``mhd_oracle.c`` / ``mhd_oracle_ctu.c`` (plain C99,
compiled with ``-O2 -ffp-contract=off``); this module only builds the shared
library and marshals numpy arrays.  Arrays are float64, C-ordered
``[z][y][x]``; conserved state ``U`` is (5, nz, ny, nx) = (rho, Mx, My, Mz, e),
face field ``B`` is (3, nz, ny, nx) = (bx, by, bz) on lower faces.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["mhd_oracle.c", "mhd_oracle_ctu.c"]

VL, CTU = 0, 1
PLM, PPM, FIRST_ORDER = 0, 1, 2
ROE, HLLE, HLLD = 0, 1, 2
GAMMA = 5.0 / 3.0

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so in place with gcc."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-o", _LIB_PATH + ".tmp"] + srcs + ["-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    D = ctypes.c_double
    I = ctypes.c_int
    P = ctypes.c_void_p
    lib.or_cfl_dt.restype = D
    lib.or_cfl_dt.argtypes = [I, I, I, D, D, D, P, P]
    lib.or_step.restype = I
    lib.or_step.argtypes = [I, I, I, D, D, I, I, I, P, P, D, P, P, ctypes.POINTER(I)]
    lib.or_step_ex.restype = I
    lib.or_step_ex.argtypes = [I, I, I, D, D, I, I, I, P, P, D, P, P, ctypes.POINTER(I), P, P]
    lib.or_prim_to_cons.argtypes = [I, I, I, D, P, P, P]
    lib.or_cons_to_prim.argtypes = [I, I, I, D, P, P, P]
    lib.or_divb.argtypes = [I, I, I, D, P, P]
    lib.or_sums.argtypes = [I, I, I, D, P, P, P]
    lib.or_phys_flux.argtypes = [D, P, D, P]
    lib.or_w_to_u.argtypes = [D, P, D, P]
    lib.or_u_to_w.argtypes = [D, P, D, P]
    lib.or_fast_speed.restype = D
    lib.or_fast_speed.argtypes = [D, P, D]
    lib.or_riemann.restype = I
    lib.or_riemann.argtypes = [I, D, P, P, D, P]
    lib.or_roe_eigen.argtypes = [D, P, P, D, P, P]
    lib.or_ppm_edges.argtypes = [P, P, P]
    lib.or_set_threads.argtypes = [I]
    lib.or_get_threads.restype = I
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def prim_to_cons(W5, B, gamma: float = GAMMA) -> np.ndarray:
    """(rho, vx, vy, vz, p) cells + face B -> conserved U (Eq. 5, cell B = face mean)."""
    W5, B = _f64(W5), _f64(B)
    nz, ny, nx = W5.shape[1:]
    U = np.empty((5, nz, ny, nx))
    _load().or_prim_to_cons(nx, ny, nz, gamma, _p(W5), _p(B), _p(U))
    return U


def cons_to_prim(U, B, gamma: float = GAMMA) -> np.ndarray:
    """Conserved U + face B -> (rho, vx, vy, vz, p, Bcx, Bcy, Bcz)."""
    U, B = _f64(U), _f64(B)
    nz, ny, nx = U.shape[1:]
    W = np.empty((8, nz, ny, nx))
    _load().or_cons_to_prim(nx, ny, nz, gamma, _p(U), _p(B), _p(W))
    return W


def cfl_dt(U, B, dx: float, gamma: float = GAMMA, courant: float = 0.5) -> float:
    U, B = _f64(U), _f64(B)
    nz, ny, nx = U.shape[1:]
    return float(_load().or_cfl_dt(nx, ny, nz, dx, gamma, courant, _p(U), _p(B)))


def divb(B, dx: float) -> np.ndarray:
    B = _f64(B)
    nz, ny, nx = B.shape[1:]
    out = np.empty((nz, ny, nx))
    _load().or_divb(nx, ny, nz, dx, _p(B), _p(out))
    return out


def sums(U, B, dx: float) -> np.ndarray:
    """(mass, Mx, My, Mz, E_T, U_B, U_V) volume totals."""
    U, B = _f64(U), _f64(B)
    nz, ny, nx = U.shape[1:]
    out = np.empty(7)
    _load().or_sums(nx, ny, nz, dx, _p(U), _p(B), _p(out))
    return out


def step(U, B, dt: float, dx: float, scheme: int = VL, recon: int = PLM, riemann: int = ROE,
         gamma: float = GAMMA, return_fallbacks: bool = False, return_fluxes: bool = False):
    """One full update of the periodic grid; returns (U_new, B_new), then
    the fallback count if asked for, then, if asked for, the full update's
    fluxes F [3, 5, nz, ny, nx] (through the lower d-face of each cell) and
    edge EMFs E [3, nz, ny, nx] (at each cell's lower corner edges)."""
    U, B = _f64(U), _f64(B)
    nz, ny, nx = U.shape[1:]
    Uo = np.empty_like(U)
    Bo = np.empty_like(B)
    F = np.empty((3, 5) + U.shape[1:]) if return_fluxes else None
    E = np.empty((3,) + U.shape[1:]) if return_fluxes else None
    nfb = ctypes.c_int(0)
    rc = _load().or_step_ex(nx, ny, nz, dx, gamma, scheme, recon, riemann, _p(U), _p(B), float(dt),
                            _p(Uo), _p(Bo), ctypes.byref(nfb), _p(F) if return_fluxes else None,
                            _p(E) if return_fluxes else None)
    if rc != 0:
        raise RuntimeError(f"oracle step failed with status {rc}")
    out = (Uo, Bo)
    if return_fallbacks:
        out += (int(nfb.value),)
    if return_fluxes:
        out += (F, E)
    return out


def run(U, B, nsteps: int, dx: float, courant: float = 0.5, **kw):
    """nsteps CFL-limited steps; returns (U, B, t, dts)."""
    t = 0.0
    dts = []
    for _ in range(nsteps):
        dt = cfl_dt(U, B, dx, kw.get("gamma", GAMMA), courant)
        if dt <= 0:
            raise RuntimeError("non-physical state")
        U, B = step(U, B, dt, dx, **kw)
        t += dt
        dts.append(dt)
    return U, B, t, dts


# ---- 1D helpers for unit tests; w = (rho, vn, vt1, vt2, p, bt1, bt2) ----
def phys_flux(w, bn, gamma: float = GAMMA) -> np.ndarray:
    w = _f64(w)
    f = np.empty(7)
    _load().or_phys_flux(gamma, _p(w), float(bn), _p(f))
    return f


def w_to_u(w, bn, gamma: float = GAMMA) -> np.ndarray:
    w = _f64(w)
    u = np.empty(7)
    _load().or_w_to_u(gamma, _p(w), float(bn), _p(u))
    return u


def u_to_w(u, bn, gamma: float = GAMMA) -> np.ndarray:
    u = _f64(u)
    w = np.empty(7)
    _load().or_u_to_w(gamma, _p(u), float(bn), _p(w))
    return w


def fast_speed(w, bn, gamma: float = GAMMA) -> float:
    w = _f64(w)
    return float(_load().or_fast_speed(gamma, _p(w), float(bn)))


def riemann(solver: int, wl, wr, bn, gamma: float = GAMMA):
    wl, wr = _f64(wl), _f64(wr)
    f = np.empty(7)
    fb = _load().or_riemann(solver, gamma, _p(wl), _p(wr), float(bn), _p(f))
    return f, fb


def roe_eigen(wl, wr, bn, gamma: float = GAMMA):
    wl, wr = _f64(wl), _f64(wr)
    lam = np.empty(7)
    R = np.empty((7, 7))
    _load().or_roe_eigen(gamma, _p(wl), _p(wr), float(bn), _p(lam), _p(R))
    return lam, R


def ppm_edges(q):
    """PPM (limited, CW84) values at the lower and upper edge of the centre
    cell of five consecutive cell averages q[0..4]."""
    q = _f64(q)
    assert q.shape == (5,)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _load().or_ppm_edges(_p(q), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def initial_state(prob, gamma: float = GAMMA):
    """Convert a problem dict from the input generator to (U, B)."""
    W5 = np.stack([prob["rho"], prob["vx"], prob["vy"], prob["vz"], prob["p"]])
    B = np.stack([prob["bx"], prob["by"], prob["bz"]])
    return prim_to_cons(W5, B, gamma), _f64(B)
