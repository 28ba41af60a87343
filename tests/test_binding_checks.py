"""Host-side argument checks of the Python binding (no GPU needed): what the
C side cannot check because it sees neither element sizes nor the contents
of device group lists."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1804_03479_amd.mhd import check_dt_tensor, check_group_origins  # noqa: E402


def test_valid_group_list_passes():
    check_group_origins(np.array([[0, 0, 0], [16, 0, 0], [16, 32, 48]]), (64, 64, 64), 16)
    check_group_origins(np.zeros((0, 3)), (32, 32, 32), 16)


@pytest.mark.parametrize("origins, why", [
    ([[8, 0, 0]], "multiples"),            # not on the group lattice
    ([[0, 0, 64]], "inside"),              # past the grid
    ([[-16, 0, 0]], "inside"),             # negative
    ([[0, 16, 0], [0, 16, 0]], "unique"),  # listed twice: in-place double update
])
def test_bad_group_lists_rejected(origins, why):
    with pytest.raises(ValueError, match=why):
        check_group_origins(np.array(origins), (64, 64, 64), 16)


def test_edge_must_divide_grid():
    with pytest.raises(ValueError, match="divide"):
        check_group_origins(np.array([[0, 0, 0]]), (40, 48, 48), 16)


@pytest.mark.parametrize("t", [
    torch.zeros(1, dtype=torch.float64),              # host memory
    torch.zeros(1, dtype=torch.float32),              # wrong dtype
    torch.zeros(2, 2, dtype=torch.float64).t(),       # not contiguous
    0.5,                                              # not a tensor
])
def test_bad_dt_tensors_rejected(t):
    with pytest.raises(ValueError, match="float64 device tensor"):
        check_dt_tensor(t, "dt")
