"""The allocation-free read-back (lbm_axi_moments_noalloc) against
lbm_axi_moments: the same fields and diagnostics, bit for bit, on two calls in
a row on one device, the second on a smaller grid (its shared reduction
scratch then holds the first call's partials beyond what the second writes)."""
import ctypes

import numpy as np
import pytest

from paper_1810_09299_amd import abi, inputs

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "rho", "uz", "ur", "p")


def _device_outputs(torch, nr, nz):
    out = {k: torch.full((nr, nz), float("nan"), dtype=torch.float64, device="cuda") for k in FIELDS}
    diag = torch.full((ctypes.sizeof(abi.lbm_axi_diag) // 8,), float("nan"), dtype=torch.float64, device="cuda")
    return out, diag


def _diag_from(torch_buf):
    raw = torch_buf.cpu().numpy().tobytes()
    return abi.lbm_axi_diag.from_buffer_copy(raw).as_dict()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_noalloc_equals_moments_on_two_calls(precision):
    import torch
    from paper_1810_09299_amd.case import AxiCase
    big = inputs.oscillating_droplet(nr=96, nz=160, R0=24.0, zc=80.0, W=4.0, sigma=1e-3, mobility=0.05)
    small = inputs.static_droplet(nr=20, nz=36, R=7.0, zc=18.0, W=4.0, sigma=1e-3, mobility=0.1, z_periodic=False)
    cases = [AxiCase(s, precision=precision) for s in (big, small)]
    for c, n in zip(cases, (37, 23)):
        c.step(n)
    outs = []
    for c in cases:                                   # the two calls, back to back
        o, d = _device_outputs(torch, c.nr, c.nz)
        abi.lbm_axi_moments_noalloc(c.handle, *(o[k].data_ptr() for k in FIELDS), d.data_ptr())
        outs.append((o, d))
    torch.cuda.synchronize()
    for c, (o, d) in zip(cases, outs):
        ref, ref_diag, rc = c.moments()
        assert rc == 0
        for k in FIELDS:
            assert np.array_equal(o[k].cpu().numpy(), ref[k]), k
        got = _diag_from(d)
        for k, v in ref_diag.items():
            assert got[k] == v, (k, got[k], v)


def test_noalloc_rejects_null_outputs_and_handles():
    import torch
    from paper_1810_09299_amd.case import AxiCase
    spec = inputs.static_droplet(nr=20, nz=36, R=7.0, zc=18.0, W=4.0, sigma=1e-3, mobility=0.1)
    c = AxiCase(spec, precision="fp32")
    o, d = _device_outputs(torch, c.nr, c.nz)
    ptrs = [o[k].data_ptr() for k in FIELDS]
    lib = abi.load()
    P = ctypes.c_void_p
    assert lib.lbm_axi_moments_noalloc(None, *(P(x) for x in ptrs), P(d.data_ptr())) == abi.LBM_AXI_ESTATE
    for q in range(6):
        args = [P(x) for x in ptrs] + [P(d.data_ptr())]
        args[q] = None
        assert lib.lbm_axi_moments_noalloc(P(c.handle), *args) == abi.LBM_AXI_EINVAL
