"""ctypes wrapper of the plain FP64 CPU oracle (axi_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It never imports
the HIP library's package, and the HIP library never imports it.

Case objects are duck-typed: anything with the attributes nr, nz, z_periodic,
dispersed_gas, W, mobility, sigma, rho_l, rho_g, nu_l, nu_g, g_z, s_f, s_g and
phi0 (float64 (nr, nz)) will do.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "axi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_axi.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("z_periodic", ctypes.c_int32), ("dispersed_gas", ctypes.c_int32),
                ("collision", ctypes.c_int32), ("alt", ctypes.c_int32),
                ("free_s1", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("W", ctypes.c_double), ("mobility", ctypes.c_double), ("sigma", ctypes.c_double),
                ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
                ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double), ("g_z", ctypes.c_double),
                ("g_ramp", ctypes.c_double),
                ("s_f", ctypes.c_double * 9), ("s_g", ctypes.c_double * 9)]


class Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("phase_mass", ctypes.c_double),
                ("fluid_mass", ctypes.c_double), ("mom_z", ctypes.c_double),
                ("umax", ctypes.c_double), ("p_in", ctypes.c_double), ("p_out", ctypes.c_double),
                ("dp", ctypes.c_double), ("R_eq", ctypes.c_double), ("semi_z", ctypes.c_double),
                ("semi_r", ctypes.c_double), ("centroid_z", ctypes.c_double),
                ("rise_u", ctypes.c_double), ("min_axis_phi", ctypes.c_double),
                ("nonfinite", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_D = ctypes.POINTER(ctypes.c_double)

# alternative readings (axi_oracle.h ORA_ALT_*), set through a case's `alt`
ALT_JOINT_PU = 1
ALT_ODD_AXIS = 2
ALT_FREE_S1 = 4


def _load():
    global _lib
    if _lib is None:
        # (re)build when missing or older than its sources
        srcs = (_SRC, os.path.join(os.path.dirname(_SRC), "axi_oracle.h"))
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(x) for x in srcs):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.ora_create.restype = ctypes.c_void_p
        lib.ora_create.argtypes = [ctypes.POINTER(_Params), _D]
        lib.ora_destroy.argtypes = [ctypes.c_void_p]
        lib.ora_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.ora_step_debug.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
        lib.ora_time.restype = ctypes.c_int64
        lib.ora_time.argtypes = [ctypes.c_void_p]
        lib.ora_moments.argtypes = [ctypes.c_void_p, _D, _D, _D, _D, _D]
        lib.ora_diagnostics.argtypes = [ctypes.c_void_p, ctypes.POINTER(Diag)]
        lib.ora_get_state.argtypes = [ctypes.c_void_p, _D, _D, _D]
        lib.ora_set_state.argtypes = [ctypes.c_void_p, _D, _D, _D, ctypes.c_int64]
        lib.ora_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                    _D, _D, _D]
        lib.ora_stencil.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _D]
        lib.ora_stream.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _D, _D]
        lib.ora_rates.argtypes = [ctypes.c_void_p, _D, _D]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _params(spec) -> _Params:
    p = _Params()
    p.nr, p.nz = int(spec.nr), int(spec.nz)
    p.z_periodic = int(bool(spec.z_periodic))
    p.dispersed_gas = int(bool(getattr(spec, "dispersed_gas", False)))
    p.collision = {"mrt": 0, "srt": 1, "nmrt": 2}[getattr(spec, "collision", "mrt")]
    p.W, p.mobility, p.sigma = float(spec.W), float(spec.mobility), float(spec.sigma)
    p.rho_l, p.rho_g = float(spec.rho_l), float(spec.rho_g)
    p.nu_l, p.nu_g = float(spec.nu_l), float(spec.nu_g)
    p.g_z = float(getattr(spec, "g_z", 0.0))
    for a in range(9):
        p.s_f[a] = float(spec.s_f[a])
        p.s_g[a] = float(spec.s_g[a])
    p.alt = int(getattr(spec, "alt", 0))
    p.free_s1 = int(bool(getattr(spec, "free_s1", False)))
    p.g_ramp = float(getattr(spec, "g_ramp", 0.0))
    return p


class OracleCase:
    """One case advanced by the FP64 oracle."""

    def __init__(self, spec, phi0=None):
        lib = _load()
        self.nr, self.nz = int(spec.nr), int(spec.nz)
        phi0 = spec.phi0 if phi0 is None else phi0
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(self.nr, self.nz)
        self._p = _params(spec)
        self._h = lib.ora_create(ctypes.byref(self._p), _ptr(phi0))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ora_destroy(self._h)
            self._h = None

    @property
    def t(self) -> int:
        return int(_lib.ora_time(self._h))

    def step(self, n: int = 1):
        _lib.ora_step(self._h, int(n))

    def step_debug(self):
        nr, nz = self.nr, self.nz
        fp = np.empty((9, nr, nz))
        gp = np.empty((9, nr, nz))
        Fz = np.empty((nr, nz))
        Fr = np.empty((nr, nz))
        _lib.ora_step_debug(self._h, _ptr(fp), _ptr(gp), _ptr(Fz), _ptr(Fr))
        return fp, gp, Fz, Fr

    def moments(self):
        nr, nz = self.nr, self.nz
        out = {k: np.empty((nr, nz)) for k in ("phi", "rho", "uz", "ur", "p")}
        _lib.ora_moments(self._h, *(_ptr(out[k]) for k in ("phi", "rho", "uz", "ur", "p")))
        return out

    def diagnostics(self) -> dict:
        d = Diag()
        _lib.ora_diagnostics(self._h, ctypes.byref(d))
        return d.as_dict()

    def get_state(self):
        nr, nz = self.nr, self.nz
        f = np.empty((9, nr, nz))
        g = np.empty((9, nr, nz))
        aux = np.empty((3, nr, nz))
        _lib.ora_get_state(self._h, _ptr(f), _ptr(g), _ptr(aux))
        return f, g, aux

    def set_state(self, f, g, aux, t=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        aux = np.ascontiguousarray(aux, dtype=np.float64)
        _lib.ora_set_state(self._h, _ptr(f), _ptr(g), _ptr(aux), int(t))

    def rates(self):
        sf = np.empty(9)
        sg = np.empty(9)
        _lib.ora_rates(self._h, _ptr(sf), _ptr(sg))
        return sf, sg


def lattice():
    lib = _load()
    cz = (ctypes.c_int32 * 9)()
    cr = (ctypes.c_int32 * 9)()
    w = np.empty(9)
    M = np.empty((9, 9))
    Minv = np.empty((9, 9))
    lib.ora_lattice(cz, cr, _ptr(w), _ptr(M), _ptr(Minv))
    return np.array(list(cz)), np.array(list(cr)), w, M, Minv


def stencil(chi, z_periodic: bool):
    lib = _load()
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    nr, nz = chi.shape
    dz, dr, lap = np.empty_like(chi), np.empty_like(chi), np.empty_like(chi)
    lib.ora_stencil(nr, nz, int(bool(z_periodic)), _ptr(chi), _ptr(dz), _ptr(dr), _ptr(lap))
    return dz, dr, lap


def stream(post, z_periodic: bool):
    lib = _load()
    post = np.ascontiguousarray(post, dtype=np.float64)
    _, nr, nz = post.shape
    out = np.empty_like(post)
    lib.ora_stream(nr, nz, int(bool(z_periodic)), _ptr(post), _ptr(out))
    return out
