"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and validates parameters without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1810_09299_amd import abi, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm_axi.h")).read()
    return sorted(set(re.findall(r"\b(lbm_axi_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    for name in _declared():
        assert hasattr(lib, name), name


def _params(**kw):
    spec = inputs.static_droplet(nr=16, nz=32, R=5, zc=16, W=4)
    prec = kw.pop("precision", "fp64")
    p = abi.make_params(spec, prec if isinstance(prec, str) else "fp64")
    if not isinstance(prec, str):
        p.precision = prec
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_state_bytes_layout():
    p64 = _params()
    p32 = _params(precision="fp32")
    b64 = abi.lbm_axi_state_bytes(p64)
    b32 = abi.lbm_axi_state_bytes(p32)
    plane = 16 * 32
    # 36 population planes + 3 aux planes in the storage type, 5 double planes of scratch
    assert b64 >= (36 + 3) * plane * 8 + 5 * plane * 8
    assert b32 >= (36 + 3) * plane * 4 + 5 * plane * 8
    assert b32 < b64
    assert b64 % 256 == 0
    # FP16-deviation storage: per buffer an FP32 f_0 plane, 8 FP16 f planes and
    # 9 FP16 g planes; 4 FP32 aux planes (phase field of both sides, u_z, u_r)
    b16 = abi.lbm_axi_state_bytes(_params(precision="fp16"))
    assert b16 >= 2 * (4 + 8 * 2 + 9 * 2) * plane + 4 * 4 * plane + 5 * plane * 8
    assert b16 < b32
    assert b16 % 256 == 0


@pytest.mark.parametrize("field,value", [
    ("nr", 3), ("nz", 2), ("W", 0.0), ("mobility", 0.0), ("rho_g", -1.0), ("nu_l", 0.0),
    ("sigma", -0.1), ("precision", 7), ("z_periodic", 2), ("collision", 3), ("W", float("nan")),
    ("g_z", float("inf")),
])
def test_invalid_parameters_rejected(field, value):
    p = _params(**{field: value})
    assert abi.lbm_axi_state_bytes(p) == 0
    h = ctypes.c_void_p()
    rc = abi.load().lbm_axi_init(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30, None, None,
                                 ctypes.byref(h))
    assert rc == abi.LBM_AXI_EINVAL
    assert h.value is None


@pytest.mark.parametrize("which,idx,value", [("s_f", 0, 2.0), ("s_f", 7, -0.5), ("s_g", 2, 0.0),
                                              ("s_g", 4, 2.5), ("s_f", 8, float("nan"))])
def test_invalid_rates_rejected(which, idx, value):
    p = _params()
    getattr(p, which)[idx] = value
    assert abi.lbm_axi_state_bytes(p) == 0


def test_fp16_rounding_option():
    """Stochastic g rounding belongs to FP16-deviation storage: the binding
    sets it for that precision only, the library rejects it for the others and
    any value other than the two modes."""
    spec = inputs.static_droplet(nr=16, nz=32, R=5, zc=16, W=4)
    spec.fp16_stochastic = True
    p16 = abi.make_params(spec, "fp16")
    assert p16.fp16_rounding == abi.LBM_AXI_ROUND_STOCHASTIC and abi.lbm_axi_state_bytes(p16) > 0
    p32 = abi.make_params(spec, "fp32")
    assert p32.fp16_rounding == abi.LBM_AXI_ROUND_NEAREST and abi.lbm_axi_state_bytes(p32) > 0
    p32.fp16_rounding = abi.LBM_AXI_ROUND_STOCHASTIC
    assert abi.lbm_axi_state_bytes(p32) == 0
    for bad in (2, -1):
        p16.fp16_rounding = bad
        assert abi.lbm_axi_state_bytes(p16) == 0


@pytest.mark.parametrize("form", ["mrt", "srt", "nmrt"])
def test_every_collision_form_is_accepted(form):
    spec = inputs.static_droplet(nr=16, nz=32, R=5, zc=16, W=4)
    spec.collision = form
    p = abi.make_params(spec, "fp32")
    assert p.collision == abi.COLLISIONS[form]
    assert abi.lbm_axi_state_bytes(p) > 0


def test_derived_rates_are_not_validated():
    # s_f[3..6] and s_g[1,7,8] come from the mobility and the viscosity
    p = _params()
    p.s_f[3] = 5.0
    p.s_g[7] = -3.0
    assert abi.lbm_axi_state_bytes(p) > 0


def test_small_block_and_null_handle():
    p = _params()
    lib = abi.load()
    h = ctypes.c_void_p()
    phi0 = (ctypes.c_double * (16 * 32))()
    rc = lib.lbm_axi_init(ctypes.byref(p), ctypes.c_void_p(256), 1024, phi0, None, ctypes.byref(h))
    assert rc == abi.LBM_AXI_ENOMEM
    rc = lib.lbm_axi_init(ctypes.byref(p), ctypes.c_void_p(257), 1 << 30, phi0, None, ctypes.byref(h))
    assert rc == abi.LBM_AXI_EINVAL            # misaligned block
    assert lib.lbm_axi_step(None, 1) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_destroy(None) == abi.LBM_AXI_OK
    assert abi.strerror(abi.LBM_AXI_EUNSTABLE).startswith("non-finite")


def test_device_copy_rejects_bad_arguments_on_the_host():
    """Size and alignment are checked before anything reaches the device (the
    pointers here are never dereferenced)."""
    lib = abi.load()
    P = ctypes.c_void_p
    a, b = 1 << 20, 1 << 24
    assert lib.lbm_axi_device_copy(P(a), P(b), 0, None) == abi.LBM_AXI_OK          # nothing to do
    assert lib.lbm_axi_device_copy(P(a), P(b), 24, None) == abi.LBM_AXI_EINVAL     # not 16-byte units
    assert lib.lbm_axi_device_copy(P(a + 4), P(b), 32, None) == abi.LBM_AXI_EINVAL  # misaligned source
    assert lib.lbm_axi_device_copy(P(a), P(b + 8), 32, None) == abi.LBM_AXI_EINVAL  # misaligned target
    assert lib.lbm_axi_device_copy(None, P(b), 32, None) == abi.LBM_AXI_EINVAL
    assert lib.lbm_axi_device_copy(P(a), P(a + 16), 32, None) == abi.LBM_AXI_EINVAL  # overlapping ranges


def test_grid_size_limit():
    """The library keeps every population plane's byte offsets in 32 bits:
    nr * nz up to 2^25 is accepted, one node more is not."""
    p = _params()
    p.nr, p.nz = 4096, 8192
    assert abi.lbm_axi_state_bytes(p) > 0
    p.nz = 8193
    assert abi.lbm_axi_state_bytes(p) == 0


def test_null_batch_handles_are_rejected():
    lib = abi.load()
    n = ctypes.c_int32()
    assert lib.lbm_axi_batch_run(None, 1) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_batch_prepare(None, 1) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_batch_poll(None, None, 0, ctypes.byref(n)) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_batch_release(None, 0) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_batch_set_config(None, 8, 0, 1, 16) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_batch_sync(None) == abi.LBM_AXI_ESTATE
    assert lib.lbm_axi_batch_destroy(None) == abi.LBM_AXI_OK          # NULL is accepted
    assert lib.lbm_axi_set_tile(None, 8) == abi.LBM_AXI_ESTATE


def test_pool_sizing_covers_head_and_blocks():
    """A pool of Batch.pool_for(specs) holds the head (case table and work
    list) and one block per case: blocks are whole multiples of the 256-byte
    alignment the pool's first-fit allocator uses, so the sum is exact."""
    from paper_1810_09299_amd import inputs
    from paper_1810_09299_amd.batch import Batch
    specs = [inputs.static_droplet(nr=nr, nz=nz, R=3, zc=nz / 2, W=4) for nr, nz in ((5, 7), (16, 32), (33, 130))]
    for prec in ("fp64", "fp32", "fp16"):
        head = Batch.head_bytes(len(specs), prec)
        # the work list's reserved room alone is 16-byte items, a million of them
        assert head >= 16 * (1 << 20) and head % 256 == 0
        assert Batch.head_bytes(2 * len(specs), prec) > head
        for s in specs:
            assert Batch.footprint(s, prec) % 256 == 0
        assert Batch.pool_for(specs, prec) == head + sum(Batch.footprint(s, prec) for s in specs)
    assert abi.lbm_axi_batch_reserved_bytes(0, abi.PRECISIONS["fp32"]) == 0
    assert abi.lbm_axi_batch_reserved_bytes(4, 7) == 0
