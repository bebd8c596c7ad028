"""The library's plain device copy, which bench.py times as the practical
bandwidth ceiling: it must copy exactly, on the stream it is given."""
import pytest
import torch

from paper_1810_09299_amd import abi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (64 << 20) + 16 * 257])
def test_device_copy_is_exact(nbytes):
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    src = torch.randint(-2**31, 2**31 - 1, (nbytes // 4 + 8,), dtype=torch.int32, generator=g).to("cuda")
    dst = torch.zeros_like(src)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    abi.lbm_axi_device_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    stream.synchronize()
    n = nbytes // 4
    assert torch.equal(dst[:n], src[:n])
    assert int(dst[n:].abs().sum()) == 0          # nothing beyond the requested bytes


def test_device_copy_rejects_misaligned_sizes():
    src = torch.zeros(64, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    with pytest.raises(abi.LbmAxiError):
        abi.lbm_axi_device_copy(src.data_ptr(), dst.data_ptr(), 20)
    with pytest.raises(abi.LbmAxiError):
        abi.lbm_axi_device_copy(src.data_ptr() + 4, dst.data_ptr(), 32)
