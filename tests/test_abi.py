"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhd.h")


@pytest.fixture(scope="module")
def mhd():
    import torch  # noqa: F401  (load torch's HIP runtime first)
    from paper_1804_03479_amd import mhd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1804_03479_amd import build
        build.build()
    m.load()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-zA-Z0-9_]+)\s*\(", text)))


def test_header_matches_exports(mhd):
    lib = mhd.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mhd.EXPORTS)


def test_abi_version_and_strings(mhd):
    lib = mhd.load()
    assert lib.mhd_abi_version() == 4
    for s in (0, -1, -2, -4, -5, -6, -7, -8):
        assert len(lib.mhd_strerror(s)) > 0 and lib.mhd_strerror(s) != b"unknown status"
    assert lib.mhd_strerror(-3) == b"unknown status"      # retired code
    assert lib.mhd_strerror(-999) == b"unknown status"


def test_required_ghost(mhd):
    lib = mhd.load()
    assert lib.mhd_required_ghost(mhd.VL, mhd.PLM) == 3
    assert lib.mhd_required_ghost(mhd.CTU, mhd.PPM) == 4
    assert lib.mhd_required_ghost(mhd.VL, mhd.PPM) == 4
    assert lib.mhd_required_ghost(7, mhd.PLM) == -1
    assert lib.mhd_required_ghost(mhd.VL, 9) == -1


def _cfg(mhd, **kw):
    c = dict(scheme=mhd.VL, recon=mhd.PLM, riemann=mhd.ROE, prec=mhd.F64, gamma=5 / 3, courant=0.5,
             beta_fp64=0.1, mlp_dp=0.3, mlp_drho=0.3)
    c.update(kw)
    return mhd.Config(**c)


@pytest.mark.parametrize("bad", [dict(scheme=5), dict(recon=-1), dict(riemann=9), dict(prec=3),
                                 dict(gamma=1.0), dict(gamma=float("nan")), dict(courant=0.0),
                                 dict(courant=1.5)])
def test_init_rejects_invalid_config(mhd, bad):
    lib = mhd.load()
    h = ctypes.c_void_p()
    cfg = _cfg(mhd, **bad)
    assert lib.mhd_init(ctypes.byref(cfg), None, ctypes.byref(h)) == -1
    assert not h.value


def test_init_null_arguments(mhd):
    lib = mhd.load()
    h = ctypes.c_void_p()
    assert lib.mhd_init(None, None, ctypes.byref(h)) == -1
    cfg = _cfg(mhd)
    assert lib.mhd_init(ctypes.byref(cfg), None, None) == -1


def test_init_without_device(mhd):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = mhd.load()
    h = ctypes.c_void_p()
    cfg = _cfg(mhd)
    assert lib.mhd_init(ctypes.byref(cfg), None, ctypes.byref(h)) == -6


def _level(mhd, **kw):
    d = dict(nx=16, ny=16, nz=16, dx=1 / 16, n_groups=0, group_edge=16, groups=None, U=0x1000, B=0x2000, E64=None)
    d.update(kw)
    return mhd.LevelDesc(**d)


@pytest.mark.parametrize("bad", [dict(nx=3), dict(nz=0), dict(dx=0.0), dict(dx=-1.0), dict(U=None), dict(B=None),
                                 dict(n_groups=2, groups=None), dict(n_groups=0, groups=0x3000),
                                 dict(nx=48, ny=48, nz=48, n_groups=1, groups=0x3000, group_edge=3),
                                 dict(nx=40, ny=48, nz=48, n_groups=1, groups=0x3000, group_edge=16),
                                 dict(nx=16, ny=16, nz=16, n_groups=1, groups=0x3000, group_edge=16)])
def test_check_level_rejects(mhd, bad):
    lib = mhd.load()
    lv = _level(mhd, **bad)
    assert lib.mhd_check_level(None, ctypes.byref(lv)) == -1


def test_check_level_accepts(mhd):
    lib = mhd.load()
    assert lib.mhd_check_level(None, ctypes.byref(_level(mhd))) == 0
    lv = _level(mhd, nx=48, ny=32, nz=32, n_groups=3, groups=0x3000)
    assert lib.mhd_check_level(None, ctypes.byref(lv)) == 0


def test_null_context_calls(mhd):
    lib = mhd.load()
    lv = _level(mhd)
    d = ctypes.c_double()
    assert lib.mhd_step(None, ctypes.byref(lv), 0.1) == -1
    assert lib.mhd_cfl_dt(None, ctypes.byref(lv), ctypes.byref(d), None) == -1
    assert lib.mhd_advance(None, ctypes.byref(lv), None, None) == -1
    assert lib.mhd_divB(None, ctypes.byref(lv), ctypes.byref(d), ctypes.byref(d)) == -1
    assert lib.mhd_sync(None) == -1
    assert lib.mhd_finalize(None) == -1
    sz = ctypes.c_size_t()
    i = ctypes.c_int()
    assert lib.mhd_workspace_bytes(None, ctypes.byref(lv), ctypes.byref(sz)) == -1
    assert lib.mhd_prolong(None, ctypes.byref(lv), ctypes.byref(lv), 4) == -1
    assert lib.mhd_prolong_time(None, None, ctypes.byref(lv), 0.5, ctypes.byref(lv), 4) == -1
    assert lib.mhd_restrict(None, ctypes.byref(lv), ctypes.byref(lv)) == -1
    assert lib.mhd_correct(None, ctypes.byref(lv), None, ctypes.byref(lv), None, 0) == -1
    assert lib.mhd_accumulate_registers(None, ctypes.byref(lv), 0.5, 1) == -1
    assert lib.mhd_dt_subdivide(None, None, 2, None) == -1
    assert lib.mhd_regrid_flag(None, ctypes.byref(lv), 1.0, 1, 16, None, 4, ctypes.byref(i), ctypes.byref(i)) == -1
    assert lib.mhd_prolong_new_groups(None, ctypes.byref(lv), ctypes.byref(lv), None) == -1


def test_binding_fails_loudly_without_library(tmp_path):
    import torch  # noqa: F401
    from paper_1804_03479_amd import mhd as m
    saved = m._lib
    try:
        m._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            m.load(str(tmp_path / "missing.so"))
    finally:
        m._lib = saved
