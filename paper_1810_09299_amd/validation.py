"""Physics checks of the GPU path against the paper's test problems (Sec. 3).

- Miller-Scriven / Lamb frequency of the n-th shape mode of a drop (Eqs. 43-45).
- Droplet oscillation (Sec. 3.2, Table 1): the radial half-axis R_r(t) of an
  ellipsoidal drop, and its angular frequency from a damped-cosine fit.
- Thread breakup (Sec. 3.3): time until the phase field on the axis first
  drops below 1/2, in units of the capillary time sqrt(R^3 rho_l / sigma).
- Young-Laplace pressure jump of a drop at rest, 2 sigma / R.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs


def lamb_frequency(n: int, Re: float, rho_l: float, rho_g: float, sigma: float,
                   nu_l: float, nu_g: float) -> float:
    """omega_n of Eq. 43: Lamb's frequency (Eq. 44) with the viscous correction alpha (Eq. 45)."""
    w_star = math.sqrt(n * (n - 1) * (n + 1) * (n + 2) * sigma / (Re ** 3 * (n * rho_g + (n + 1) * rho_l)))
    alpha = ((2 * n + 1) ** 2 * rho_l * rho_g * math.sqrt(nu_l * nu_g)) / (
        math.sqrt(2) * Re * (n * rho_g + (n + 1) * rho_l) * (rho_l * math.sqrt(nu_l) + rho_g * math.sqrt(nu_g)))
    return w_star - 0.5 * alpha * math.sqrt(w_star) + 0.25 * alpha ** 2


def first_extremum(t: np.ndarray, y: np.ndarray, window: int = 20) -> int:
    """Index of the first local extremum of y that is extreme within +-window samples."""
    for q in range(window, len(y) - window):
        seg = y[q - window:q + window + 1]
        if y[q] == seg.max() or y[q] == seg.min():
            if abs(y[q] - y[0]) > 1e-6 * max(1.0, abs(y[0])):
                return q
    return 0


def lamb_damping(n: int, Re: float, rho_l: float, rho_g: float, nu_l: float, nu_g: float) -> float:
    """Amplitude decay rate of the n-th shape mode from the viscous dissipation
    of the potential flows inside and outside the drop (Lamb's dissipation
    method; for a drop alone it is (n-1)(2n+1) nu / R^2, for a bubble alone
    (n+2)(2n+1) nu / R^2):  gamma = (2n+1) [(n^2-1) mu_l + n(n+2) mu_g] /
    (R^2 [(n+1) rho_l + n rho_g])."""
    mu_l, mu_g = rho_l * nu_l, rho_g * nu_g
    return (2 * n + 1) * ((n * n - 1) * mu_l + n * (n + 2) * mu_g) / (Re ** 2 * ((n + 1) * rho_l + n * rho_g))


def damped_frequency(t: np.ndarray, y: np.ndarray, with_decay: bool = False):
    """Angular frequency of y(t) from a least-squares fit of
    A exp(-g t) cos(w t + p) + c to the record after its first extremum (the
    first half-period of a large deformation is not yet the free oscillation);
    with `with_decay`, (w, g)."""
    from scipy.optimize import curve_fit
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    q0 = first_extremum(t, y)
    tt, yy = t[q0:], y[q0:]
    c0 = yy[-max(1, len(yy) // 4):].mean()
    d = yy - c0
    sgn = np.sign(d)
    cr = np.where(sgn[:-1] * sgn[1:] < 0)[0]
    w0 = math.pi / np.median(np.diff(tt[cr][:4])) if len(cr) > 2 else 2 * math.pi / (tt[-1] - tt[0])
    A0 = d[0]

    def model(x, A, g, w, p, c):
        return A * np.exp(-g * (x - tt[0])) * np.cos(w * (x - tt[0]) + p) + c

    p, _ = curve_fit(model, tt, yy, p0=[A0, 1e-4, w0, 0.0, c0], maxfev=20000)
    if with_decay:
        return abs(float(p[2])), float(p[1])
    return abs(float(p[2]))


def run_oscillation(Rr: float, Rz: float = 90.0, ratio: float = 100.0, steps: int = 40000,
                    every: int = 50, precision: str = "fp64", nr: int = 150, nz: int = 300,
                    sigma: float = 0.3, mobility: float = 0.01, W: float = 4.0, nu=(0.1, 0.1),
                    fp16_stochastic: bool = False):
    """Sec. 3.2 setup (rho_g = 1, rho_l = ratio): returns (t, R_r(t), R_e, spec)."""
    from .case import AxiCase
    spec = inputs.ellipsoidal_droplet(nr=nr, nz=nz, Rz=Rz, Rr=Rr, W=W, ratio=ratio, sigma=sigma,
                                      mobility=mobility, nu=nu, rho_g=1.0, z_periodic=True)
    spec.fp16_stochastic = fp16_stochastic
    case = AxiCase(spec, precision=precision)
    ts, rr = [], []
    for _ in range(steps // every):
        case.step(every)
        d = case.diagnostics()
        ts.append(d["t"])
        rr.append(d["semi_r"])
    return np.array(ts, float), np.array(rr), spec.meta["Re"], spec


def oscillation_frequency(Rr: float, **kw):
    """The fitted (damped) frequency omega_lb and decay rate gamma of R_r(t),
    Eq. 43's omega_ana, Lamb's decay rate gamma_lamb, and omega_undamped =
    sqrt(omega_lb^2 + gamma^2): a damped oscillator s^2 + 2 gamma s + omega_0^2
    = 0 rings at sqrt(omega_0^2 - gamma^2), which at nu = 0.1 and these radii
    (gamma / omega_0 of 0.37-0.5) sits 7-13 % below omega_0."""
    t, rr, Re, spec = run_oscillation(Rr, **kw)
    w, g = damped_frequency(t, rr, with_decay=True)
    wa = lamb_frequency(2, Re, spec.rho_l, spec.rho_g, spec.sigma, spec.nu_l, spec.nu_g)
    gl = lamb_damping(2, Re, spec.rho_l, spec.rho_g, spec.nu_l, spec.nu_g)
    return {"Rr": Rr, "Re": Re, "omega_lb": w, "omega_ana": wa, "gamma": g, "gamma_lamb": gl,
            "omega_undamped": math.sqrt(w * w + g * g), "t": t, "semi_r": rr}


def thread_breakup_time(wavelength: int, ratio: float = 100.0, R: float = 60.0, nr: int = 200,
                        sigma: float = 0.3, mobility: float = 0.01, W: float = 4.0, nu=(0.1, 0.1),
                        max_tc: float = 40.0, every: int = 100, precision: str = "fp64"):
    """Sec. 3.3 setup (N_z x N_r = wavelength x 200, R = 60, d = 0.1 R cos(2 pi z / wavelength),
    rho_g = 1): first time, in capillary times, at which phi on the axis drops below 1/2."""
    from .case import AxiCase
    spec = inputs.liquid_thread(nr=nr, nz=wavelength, R0=R, amp=0.1, waves=1, noise=0.0, W=W,
                                ratio=ratio, sigma=sigma, mobility=mobility, rho_l=ratio)
    spec.nu_l, spec.nu_g = nu
    tc = math.sqrt(R ** 3 * spec.rho_l / sigma)
    case = AxiCase(spec, precision=precision)
    while case.t < max_tc * tc:
        case.step(every)
        d = case.diagnostics()
        if d["nonfinite"]:
            return float("nan"), tc
        if d["min_axis_phi"] < 0.5:
            return d["t"] / tc, tc
    return float("inf"), tc


def laplace_run(nr=48, nz=96, R=16.0, W=4.0, ratio=100.0, sigma=1e-4, mobility=0.1, steps=20000,
                every=2000, rho_l=1.0, precision="fp64"):
    """Drop at rest: (t, dp / (2 sigma / R_eq)) over time."""
    from .case import AxiCase
    spec = inputs.static_droplet(nr=nr, nz=nz, R=R, zc=nz / 2, W=W, ratio=ratio, sigma=sigma,
                                 mobility=mobility, z_periodic=True, rho_l=rho_l)
    case = AxiCase(spec, precision=precision)
    out = []
    for _ in range(steps // every):
        case.step(every)
        d = case.diagnostics()
        out.append((d["t"], d["dp"] / (2 * sigma / d["R_eq"]) if d["R_eq"] > 0 else float("nan"), d["umax"]))
    return out
