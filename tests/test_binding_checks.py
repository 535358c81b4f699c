"""Host-side checks of the binding's argument validation (no GPU needed):
every entry point that hands a device pointer to the kernels rejects an
output or input tensor that is not a contiguous int32 / uint8 device tensor
of the right shape before anything reaches the library."""
import types

import pytest
import torch

from paper_1708_08180_amd import binding

# stands in for a device image: _check_out only reads its shape and device
DEV_IMG = types.SimpleNamespace(shape=(4, 5), device=torch.device("cuda", 0))


@pytest.mark.parametrize("out,err", [
    (torch.zeros((4, 5), dtype=torch.int32), ValueError),                  # host tensor
    (torch.zeros((4, 6), dtype=torch.int32), ValueError),                  # wrong shape
    (torch.zeros((4, 5), dtype=torch.int64), ValueError),                  # wrong dtype
    (torch.zeros((5, 4), dtype=torch.int32).t(), ValueError),              # not contiguous
    (torch.zeros((4, 5), dtype=torch.int32, device="meta"), ValueError),   # not a device tensor
    (object(), TypeError),
])
def test_check_out_rejects(out, err):
    with pytest.raises(err):
        binding._check_out(out, DEV_IMG)


def test_entry_points_reject_host_images():
    img = torch.zeros((4, 5), dtype=torch.uint8)
    for fn in (binding.label, binding.label_plain, binding.label_equal, binding.label_timed):
        with pytest.raises(ValueError):
            fn(img, 8)


def test_component_stats_rejects_host_labels():
    with pytest.raises(ValueError):
        binding.component_stats(torch.zeros((4, 5), dtype=torch.int32))


def test_label3d_rejects_host_volume():
    with pytest.raises(ValueError):
        binding.label3d(torch.zeros((2, 3, 4), dtype=torch.uint8), 26)


def test_server_submit_validates_image():
    srv = object.__new__(binding.Server)   # no device server: submit must fail first
    srv._h = None
    with pytest.raises(ValueError):
        binding.Server.submit(srv, torch.zeros((4, 5), dtype=torch.uint8), 0)
    with pytest.raises(ValueError):
        binding.Server.submit(srv, torch.zeros((4, 5), dtype=torch.int32), 0)
