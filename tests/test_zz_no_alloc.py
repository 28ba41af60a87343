"""The allocation-free step (mhd_step_noalloc) against mhd_step_devdt on the
same input, through the C ABI: identical kernels on a different scratch, so
the results must be identical bit for bit.  Two calls in a row, the second
with a smaller input, then a group list (occupancy map in the static array)
and an FP64 VL level; a level whose scratch exceeds the static array is
refused with MHD_ERR_SCRATCH_LIMIT."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1804_03479_amd import inputs  # noqa: E402
from paper_1804_03479_amd.mhd import SCRATCH_LIMIT, Level, MHDError, Solver  # noqa: E402


def level(p, dtype, groups=None):
    U, B = oracle.initial_state(p)
    return Level(torch.from_numpy(U).to("cuda", dtype).contiguous(),
                 torch.from_numpy(B).to("cuda", dtype).contiguous(), p["dx"], groups=groups)


def pair(s, p, dtype, groups=None, steps=2):
    a, b = level(p, dtype, groups), level(p, dtype, groups)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        s.cfl_dt_device(a, dt)
        s.step_devdt(a, dt)
        s.step_noalloc(b, dt)
    torch.cuda.synchronize()
    return a, b


def same(a, b):
    return torch.equal(a.U, b.U) and torch.equal(a.B, b.B)


def test_noalloc_equals_devdt_two_calls_then_smaller():
    s = Solver("ctu", "ppm", "hlld", "f32")
    a, b = pair(s, inputs.abc_problem(40, 0.1, seed=3), torch.float32)
    assert same(a, b)
    # second call, smaller and ragged: the array still holds the first call's values
    a, b = pair(s, inputs.smooth_problem(24, 20, 16, seed=9), torch.float32)
    assert same(a, b)
    s.close()


def test_noalloc_group_list_and_fp64_vl():
    s = Solver("ctu", "ppm", "hlld", "f32")
    g = torch.tensor([(16, 0, 0), (0, 16, 16)], dtype=torch.int32, device="cuda")
    a, b = pair(s, inputs.abc_problem(32, 0.1, seed=4), torch.float32, groups=g)
    assert same(a, b)
    s.close()
    s = Solver("vl", "plm", "roe", "f64")
    a, b = pair(s, inputs.abc_problem(32, 0.01, seed=0), torch.float64, steps=3)
    assert same(a, b)
    s.close()


def test_noalloc_refuses_levels_beyond_the_array():
    s = Solver("ctu", "ppm", "hlld", "f32")
    lv = level(inputs.abc_problem(64, 0.1, seed=0), torch.float32)   # 64^3 x 98 words x 4 B > 64 MiB
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    U0 = lv.U.clone()
    with pytest.raises(MHDError) as e:
        s.step_noalloc(lv, dt)
    assert e.value.status == SCRATCH_LIMIT
    torch.cuda.synchronize()
    assert torch.equal(lv.U, U0)
    s.close()
