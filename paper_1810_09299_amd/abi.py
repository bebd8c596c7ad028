"""ctypes binding of liblbm_axi.so: the C-ABI of include/lbm_axi.h, same names.

Argument marshalling only.  The library must have been built (build.py); if it
is missing, loading raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_axi.so")

LBM_AXI_OK = 0
LBM_AXI_EINVAL = -1
LBM_AXI_ENOMEM = -2
LBM_AXI_EDEVICE = -3
LBM_AXI_EUNSTABLE = -4
LBM_AXI_EBUSY = -5
LBM_AXI_ESTATE = -6

LBM_AXI_FP64 = 0
LBM_AXI_FP32 = 1
LBM_AXI_FP16D = 2
LBM_AXI_ROUND_NEAREST = 0
LBM_AXI_ROUND_STOCHASTIC = 1
LBM_AXI_MRT = 0
LBM_AXI_SRT = 1
LBM_AXI_NMRT = 2
COLLISIONS = {"mrt": LBM_AXI_MRT, "srt": LBM_AXI_SRT, "nmrt": LBM_AXI_NMRT}
PRECISIONS = {"fp64": LBM_AXI_FP64, "fp32": LBM_AXI_FP32, "fp16": LBM_AXI_FP16D}

# every symbol include/lbm_axi.h declares
EXPORTS = (
    "lbm_axi_state_bytes", "lbm_axi_init", "lbm_axi_step", "lbm_axi_moments", "lbm_axi_moments_noalloc",
    "lbm_axi_get_state", "lbm_axi_set_state", "lbm_axi_time", "lbm_axi_set_tile",
    "lbm_axi_destroy", "lbm_axi_strerror",
    "lbm_axi_batch_reserved_bytes", "lbm_axi_batch_create", "lbm_axi_batch_admit",
    "lbm_axi_batch_run", "lbm_axi_batch_prepare", "lbm_axi_batch_poll", "lbm_axi_batch_moments",
    "lbm_axi_batch_get_state", "lbm_axi_batch_release", "lbm_axi_batch_set_config",
    "lbm_axi_batch_info", "lbm_axi_batch_sync", "lbm_axi_batch_destroy",
    "lbm_axi_device_copy",
)


class lbm_axi_params(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("z_periodic", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dispersed_gas", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("free_s1", ctypes.c_int32), ("fp16_rounding", ctypes.c_int32),
                ("W", ctypes.c_double), ("mobility", ctypes.c_double), ("sigma", ctypes.c_double),
                ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
                ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double), ("g_z", ctypes.c_double),
                ("g_ramp", ctypes.c_double),
                ("s_f", ctypes.c_double * 9), ("s_g", ctypes.c_double * 9)]


class lbm_axi_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("phase_mass", ctypes.c_double),
                ("fluid_mass", ctypes.c_double), ("mom_z", ctypes.c_double),
                ("umax", ctypes.c_double), ("p_in", ctypes.c_double), ("p_out", ctypes.c_double),
                ("dp", ctypes.c_double), ("R_eq", ctypes.c_double), ("semi_z", ctypes.c_double),
                ("semi_r", ctypes.c_double), ("centroid_z", ctypes.c_double),
                ("rise_u", ctypes.c_double), ("min_axis_phi", ctypes.c_double),
                ("nonfinite", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class LbmAxiError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1810_09299_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.lbm_axi_state_bytes.restype = ctypes.c_size_t
    lib.lbm_axi_state_bytes.argtypes = [ctypes.POINTER(lbm_axi_params)]
    lib.lbm_axi_init.restype = ctypes.c_int
    lib.lbm_axi_init.argtypes = [ctypes.POINTER(lbm_axi_params), _P, ctypes.c_size_t, _D, _P,
                                 ctypes.POINTER(_P)]
    lib.lbm_axi_step.restype = ctypes.c_int
    lib.lbm_axi_step.argtypes = [_P, ctypes.c_int64]
    lib.lbm_axi_moments.restype = ctypes.c_int
    lib.lbm_axi_moments.argtypes = [_P, _D, _D, _D, _D, _D, ctypes.POINTER(lbm_axi_diag)]
    lib.lbm_axi_moments_noalloc.restype = ctypes.c_int
    lib.lbm_axi_moments_noalloc.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    lib.lbm_axi_get_state.restype = ctypes.c_int
    lib.lbm_axi_get_state.argtypes = [_P, _D, _D, _D, ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_axi_set_state.restype = ctypes.c_int
    lib.lbm_axi_set_state.argtypes = [_P, _D, _D, _D, ctypes.c_int64]
    lib.lbm_axi_time.restype = ctypes.c_int
    lib.lbm_axi_time.argtypes = [_P, ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_axi_set_tile.restype = ctypes.c_int
    lib.lbm_axi_set_tile.argtypes = [_P, ctypes.c_int32]
    lib.lbm_axi_destroy.restype = ctypes.c_int
    lib.lbm_axi_destroy.argtypes = [_P]
    lib.lbm_axi_strerror.restype = ctypes.c_char_p
    lib.lbm_axi_strerror.argtypes = [ctypes.c_int]
    I32P = ctypes.POINTER(ctypes.c_int32)
    lib.lbm_axi_batch_reserved_bytes.restype = ctypes.c_size_t
    lib.lbm_axi_batch_reserved_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.lbm_axi_batch_create.restype = ctypes.c_int
    lib.lbm_axi_batch_create.argtypes = [_P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _P,
                                         ctypes.POINTER(_P)]
    lib.lbm_axi_batch_admit.restype = ctypes.c_int
    lib.lbm_axi_batch_admit.argtypes = [_P, ctypes.POINTER(lbm_axi_params), _D, ctypes.c_int64, I32P]
    lib.lbm_axi_batch_run.restype = ctypes.c_int
    lib.lbm_axi_batch_run.argtypes = [_P, ctypes.c_int32]
    lib.lbm_axi_batch_prepare.restype = ctypes.c_int
    lib.lbm_axi_batch_prepare.argtypes = [_P, ctypes.c_int32]
    lib.lbm_axi_batch_poll.restype = ctypes.c_int
    lib.lbm_axi_batch_poll.argtypes = [_P, I32P, ctypes.c_int32, I32P]
    lib.lbm_axi_batch_moments.restype = ctypes.c_int
    lib.lbm_axi_batch_moments.argtypes = [_P, ctypes.c_int32, _D, _D, _D, _D, _D,
                                          ctypes.POINTER(lbm_axi_diag)]
    lib.lbm_axi_batch_get_state.restype = ctypes.c_int
    lib.lbm_axi_batch_get_state.argtypes = [_P, ctypes.c_int32, _D, _D, _D, ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_axi_batch_release.restype = ctypes.c_int
    lib.lbm_axi_batch_release.argtypes = [_P, ctypes.c_int32]
    lib.lbm_axi_batch_set_config.restype = ctypes.c_int
    lib.lbm_axi_batch_set_config.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.lbm_axi_batch_info.restype = ctypes.c_int
    lib.lbm_axi_batch_info.argtypes = [_P, I32P, I32P, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_axi_batch_sync.restype = ctypes.c_int
    lib.lbm_axi_batch_sync.argtypes = [_P]
    lib.lbm_axi_batch_destroy.restype = ctypes.c_int
    lib.lbm_axi_batch_destroy.argtypes = [_P]
    lib.lbm_axi_device_copy.restype = ctypes.c_int
    lib.lbm_axi_device_copy.argtypes = [_P, _P, ctypes.c_size_t, _P]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().lbm_axi_strerror(int(code)).decode()


def _check(rc: int, where: str, ok=(LBM_AXI_OK,)) -> int:
    if rc not in ok:
        raise LbmAxiError(rc, where)
    return rc


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


# ---------------------------------------------------------------- same names

def lbm_axi_state_bytes(params: lbm_axi_params) -> int:
    return int(load().lbm_axi_state_bytes(ctypes.byref(params)))


def lbm_axi_init(params: lbm_axi_params, dev_state: int, dev_bytes: int, phi0_host, hip_stream: int):
    """Returns the opaque handle (an int)."""
    h = _P()
    rc = load().lbm_axi_init(ctypes.byref(params), _P(dev_state), dev_bytes, _dptr(phi0_host),
                             _P(hip_stream), ctypes.byref(h))
    _check(rc, "lbm_axi_init")
    return h.value


def lbm_axi_step(handle: int, nsteps: int) -> None:
    _check(load().lbm_axi_step(_P(handle), int(nsteps)), "lbm_axi_step")


def lbm_axi_moments(handle: int, phi=None, rho=None, uz=None, ur=None, p=None, raise_unstable=False):
    """Fills the given float64 host arrays; returns (rc, diag dict)."""
    d = lbm_axi_diag()
    ok = (LBM_AXI_OK,) if raise_unstable else (LBM_AXI_OK, LBM_AXI_EUNSTABLE)
    rc = load().lbm_axi_moments(_P(handle), _dptr(phi), _dptr(rho), _dptr(uz), _dptr(ur), _dptr(p),
                                ctypes.byref(d))
    _check(rc, "lbm_axi_moments", ok)
    return rc, d.as_dict()


def lbm_axi_moments_noalloc(handle: int, phi: int, rho: int, uz: int, ur: int, p: int, diag: int) -> None:
    """Device pointers in, nothing copied back; asynchronous on the case's stream."""
    _check(load().lbm_axi_moments_noalloc(_P(handle), _P(phi), _P(rho), _P(uz), _P(ur), _P(p), _P(diag)),
           "lbm_axi_moments_noalloc")


def lbm_axi_get_state(handle: int, f=None, g=None, aux=None) -> int:
    t = ctypes.c_int64()
    _check(load().lbm_axi_get_state(_P(handle), _dptr(f), _dptr(g), _dptr(aux), ctypes.byref(t)),
           "lbm_axi_get_state")
    return t.value


def lbm_axi_set_state(handle: int, f, g, aux, t: int) -> None:
    _check(load().lbm_axi_set_state(_P(handle), _dptr(f), _dptr(g), _dptr(aux), int(t)),
           "lbm_axi_set_state")


def lbm_axi_time(handle: int) -> int:
    t = ctypes.c_int64()
    _check(load().lbm_axi_time(_P(handle), ctypes.byref(t)), "lbm_axi_time")
    return t.value


def lbm_axi_set_tile(handle: int, tile_r: int) -> None:
    _check(load().lbm_axi_set_tile(_P(handle), int(tile_r)), "lbm_axi_set_tile")


def lbm_axi_destroy(handle: int) -> None:
    _check(load().lbm_axi_destroy(_P(handle)), "lbm_axi_destroy")


def lbm_axi_strerror(code: int) -> str:
    return strerror(code)


def lbm_axi_batch_reserved_bytes(max_cases: int, precision: int) -> int:
    return int(load().lbm_axi_batch_reserved_bytes(int(max_cases), int(precision)))


def lbm_axi_batch_create(dev_pool: int, pool_bytes: int, max_cases: int, precision: int,
                         hip_stream: int):
    h = _P()
    _check(load().lbm_axi_batch_create(_P(dev_pool), pool_bytes, int(max_cases), int(precision),
                                       _P(hip_stream), ctypes.byref(h)), "lbm_axi_batch_create")
    return h.value


def lbm_axi_batch_admit(batch: int, params: lbm_axi_params, phi0_host, nsteps: int):
    """Returns the slot, or None when the batch is busy (no slot or memory
    right now); raises for a case that can never fit (LBM_AXI_ENOMEM)."""
    slot = ctypes.c_int32()
    rc = load().lbm_axi_batch_admit(_P(batch), ctypes.byref(params), _dptr(phi0_host), int(nsteps),
                                    ctypes.byref(slot))
    if rc == LBM_AXI_EBUSY:
        return None
    _check(rc, "lbm_axi_batch_admit")
    return slot.value


def lbm_axi_batch_run(batch: int, chunk_steps: int) -> None:
    _check(load().lbm_axi_batch_run(_P(batch), int(chunk_steps)), "lbm_axi_batch_run")


def lbm_axi_batch_prepare(batch: int, chunk_steps: int) -> None:
    _check(load().lbm_axi_batch_prepare(_P(batch), int(chunk_steps)), "lbm_axi_batch_prepare")


def lbm_axi_batch_poll(batch: int, cap: int = 4096):
    arr = (ctypes.c_int32 * max(cap, 1))()
    n = ctypes.c_int32()
    _check(load().lbm_axi_batch_poll(_P(batch), arr, int(cap), ctypes.byref(n)), "lbm_axi_batch_poll")
    return [arr[q] for q in range(min(n.value, cap))]


def lbm_axi_batch_moments(batch: int, slot: int, phi=None, rho=None, uz=None, ur=None, p=None):
    d = lbm_axi_diag()
    rc = load().lbm_axi_batch_moments(_P(batch), int(slot), _dptr(phi), _dptr(rho), _dptr(uz),
                                      _dptr(ur), _dptr(p), ctypes.byref(d))
    _check(rc, "lbm_axi_batch_moments", (LBM_AXI_OK, LBM_AXI_EUNSTABLE))
    return rc, d.as_dict()


def lbm_axi_batch_get_state(batch: int, slot: int, f=None, g=None, aux=None) -> int:
    t = ctypes.c_int64()
    _check(load().lbm_axi_batch_get_state(_P(batch), int(slot), _dptr(f), _dptr(g), _dptr(aux),
                                          ctypes.byref(t)), "lbm_axi_batch_get_state")
    return t.value


def lbm_axi_batch_release(batch: int, slot: int) -> None:
    _check(load().lbm_axi_batch_release(_P(batch), int(slot)), "lbm_axi_batch_release")


def lbm_axi_batch_set_config(batch: int, tile_r: int, persistent: int, schedule: int, bands: int = 0) -> None:
    _check(load().lbm_axi_batch_set_config(_P(batch), int(tile_r), int(persistent), int(schedule), int(bands)),
           "lbm_axi_batch_set_config")


def lbm_axi_batch_info(batch: int) -> dict:
    u, r = ctypes.c_int32(), ctypes.c_int32()
    fb, la = ctypes.c_size_t(), ctypes.c_int64()
    _check(load().lbm_axi_batch_info(_P(batch), ctypes.byref(u), ctypes.byref(r), ctypes.byref(fb),
                                     ctypes.byref(la)), "lbm_axi_batch_info")
    return {"used": u.value, "running": r.value, "free_bytes": fb.value, "launches": la.value}


def lbm_axi_batch_sync(batch: int) -> None:
    _check(load().lbm_axi_batch_sync(_P(batch)), "lbm_axi_batch_sync")


def lbm_axi_batch_destroy(batch: int) -> None:
    _check(load().lbm_axi_batch_destroy(_P(batch)), "lbm_axi_batch_destroy")


def lbm_axi_device_copy(src: int, dst: int, nbytes: int, stream: int = 0) -> None:
    """Plain device-to-device copy (device pointers), asynchronous on stream."""
    _check(load().lbm_axi_device_copy(_P(src), _P(dst), int(nbytes), _P(stream)), "lbm_axi_device_copy")


def make_params(spec, precision: str = "fp64") -> lbm_axi_params:
    """Copy a case description (nr, nz, z_periodic, W, mobility, sigma, rho_l,
    rho_g, nu_l, nu_g, g_z, dispersed_gas, collision, s_f, s_g) into the C struct."""
    p = lbm_axi_params()
    p.nr, p.nz = int(spec.nr), int(spec.nz)
    p.z_periodic = int(bool(spec.z_periodic))
    p.precision = PRECISIONS[precision]
    p.dispersed_gas = int(bool(getattr(spec, "dispersed_gas", False)))
    p.collision = COLLISIONS[getattr(spec, "collision", "mrt")]
    p.W, p.mobility, p.sigma = float(spec.W), float(spec.mobility), float(spec.sigma)
    p.rho_l, p.rho_g = float(spec.rho_l), float(spec.rho_g)
    p.nu_l, p.nu_g = float(spec.nu_l), float(spec.nu_g)
    p.g_z = float(getattr(spec, "g_z", 0.0))
    p.free_s1 = int(bool(getattr(spec, "free_s1", False)))
    # the g rounding of FP16-deviation storage (not a parameter of the other precisions)
    stochastic = precision == "fp16" and bool(getattr(spec, "fp16_stochastic", False))
    p.fp16_rounding = LBM_AXI_ROUND_STOCHASTIC if stochastic else LBM_AXI_ROUND_NEAREST
    p.g_ramp = float(getattr(spec, "g_ramp", 0.0))
    for a in range(9):
        p.s_f[a] = float(spec.s_f[a])
        p.s_g[a] = float(spec.s_g[a])
    return p
