"""Seeded synthetic inputs: case parameters and initial phase fields.

This module feeds both the HIP library and the FP64 oracle with identical
inputs.  It holds none of the method's arithmetic: only geometry (interface
profiles of the paper's test cases), parameter bookkeeping (density and
viscosity ratios, Eotvos/Morton numbers), and a counter-based random number
generator for jitter and random states.

Every field is a float64 array of shape (nr, nz): row j sits at r = j + 1/2
(the first lattice line is at half a lattice unit from the axis, Sec. 2.3 of
the paper), column k at z = k.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, index) -> np.ndarray:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based generator.

    Output number c = seed * 2^32 + index of the sequence started from state 0:
    the state (c + 1) * 0x9E3779B97F4A7C15 passed through the published
    finaliser.  Returns uint64.
    """
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        c = np.uint64((seed << 32) & _MASK64) + idx + np.uint64(1)
        z = c * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, index) -> np.ndarray:
    """Uniform deviates in [-1, 1) from the top 53 bits of SplitMix64."""
    u = (splitmix64(seed, index) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


@dataclasses.dataclass
class CaseSpec:
    """Physical parameters of one axisymmetric case plus its initial phase field."""

    name: str
    nr: int
    nz: int
    z_periodic: bool
    W: float
    mobility: float
    sigma: float
    rho_l: float
    rho_g: float
    nu_l: float
    nu_g: float
    g_z: float = 0.0
    dispersed_gas: bool = False
    s_f: tuple = (1.0,) * 9
    s_g: tuple = (1.0,) * 9
    collision: str = "mrt"      # "mrt"; "srt": every rate 1/tau (Sec. 2.2); "nmrt": raw-moment MRT (Sec. 4)
    free_s1: bool = False       # extension: the energy moment relaxes at s_g[1], not 1/tau_g
    g_ramp: float = 0.0         # steps over which g_z is reached linearly (0: at once)
    fp16_stochastic: bool = False   # FP16-deviation storage: g rounded stochastically (unbiased)
    phi0: np.ndarray | None = None
    steps: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.nr * self.nz


def node_coords(nr: int, nz: int):
    """(z, r) of every node: z_k = k, r_j = j + 1/2."""
    z = np.arange(nz, dtype=np.float64)[None, :].repeat(nr, axis=0)
    r = (np.arange(nr, dtype=np.float64) + 0.5)[:, None].repeat(nz, axis=1)
    return z, r


PAPER_NU = 0.1   # nu_l = nu_g = 0.1 in every test of Sec. 3
# viscosities the paper's tied rate s1 = s7 = s8 = 1/tau_g (Eq. 34) runs
# stably (tau_g in about (0.65, 1.15); tests/test_oracle_stability.py)
TIED_RATE_NU = (0.05, 0.2)


def viscosities(ratio: float, mu_ratio: float | None, nu_min: float = PAPER_NU):
    """Kinematic viscosities (nu_l, nu_g) of a workload.

    mu_ratio None: both phases get the paper's nu = 0.1.  Otherwise the
    dynamic viscosity ratio mu_l/mu_g is honoured: nu_l/nu_g =
    (mu_l/mu_g)(rho_g/rho_l), the smaller of the two being nu_min."""
    if mu_ratio is None:
        return nu_min, nu_min
    q = mu_ratio / ratio
    if q <= 1.0:
        return nu_min, nu_min / q
    return nu_min * q, nu_min


def energy_rate(nu_l: float, nu_g: float):
    """(free_s1, s_g) for a pair of viscosities: the paper's tied rate when
    both lie where it is stable, else the extension that relaxes the energy
    moment at its own rate s_g[1] = 1."""
    lo, hi = TIED_RATE_NU
    free = not (lo <= min(nu_l, nu_g) and max(nu_l, nu_g) <= hi)
    return free, (1.0,) * 9


def _with_viscosities(spec: "CaseSpec", ratio: float, mu_ratio: float | None) -> "CaseSpec":
    spec.nu_l, spec.nu_g = viscosities(ratio, mu_ratio)
    spec.free_s1, spec.s_g = energy_rate(spec.nu_l, spec.nu_g)
    spec.meta["mu_ratio"] = mu_ratio if mu_ratio is not None else ratio * spec.nu_l / spec.nu_g
    return spec


def tanh_profile(dist_inside: np.ndarray, W: float) -> np.ndarray:
    """0.5 + 0.5 tanh(2 s / W): the interface profile of Eqs. 41, 46 and 47."""
    return 0.5 + 0.5 * np.tanh(2.0 * dist_inside / W)


# --------------------------------------------------------------------------
# the paper's own test cases (Sec. 3)
# --------------------------------------------------------------------------

def static_droplet(nr=64, nz=128, R=20.0, zc=None, W=5.0, ratio=1000.0, mu_ratio=None,
                   sigma=0.01, mobility=0.1, z_periodic=False, rho_l=1.0, nu=None,
                   name="static_droplet") -> CaseSpec:
    """Spherical drop centred on the axis (Eq. 41).  nu = (nu_l, nu_g) sets the
    viscosities directly (mu_ratio must then be None)."""
    if nu is not None and mu_ratio is not None:
        raise ValueError("give nu or mu_ratio, not both")
    zc = nz / 2 if zc is None else zc
    z, r = node_coords(nr, nz)
    d = np.sqrt((z - zc) ** 2 + r ** 2)
    s = CaseSpec(name=name, nr=nr, nz=nz, z_periodic=z_periodic, W=W, mobility=mobility,
                 sigma=sigma, rho_l=rho_l, rho_g=rho_l / ratio, nu_l=PAPER_NU, nu_g=PAPER_NU,
                 phi0=tanh_profile(R - d, W), meta=dict(R=R, zc=zc))
    if nu is not None:
        s.nu_l, s.nu_g = nu
        return s
    return _with_viscosities(s, ratio, mu_ratio)


def ellipsoidal_droplet(nr=150, nz=300, Rz=90.0, Rr=30.0, zc=None, W=4.0, ratio=100.0,
                        sigma=0.3, mobility=0.01, nu=(0.1, 0.1), rho_g=1.0, z_periodic=True,
                        name="ellipsoidal_droplet") -> CaseSpec:
    """Ellipsoidal drop of Eq. 46 with R_e = (R_r^2 R_z)^(1/3)."""
    zc = nz / 2 if zc is None else zc
    z, r = node_coords(nr, nz)
    Re = (Rr * Rr * Rz) ** (1.0 / 3.0)
    s = Re * (1.0 - np.sqrt((z - zc) ** 2 / Rz ** 2 + r ** 2 / Rr ** 2))
    return CaseSpec(name=name, nr=nr, nz=nz, z_periodic=z_periodic, W=W, mobility=mobility,
                    sigma=sigma, rho_l=rho_g * ratio, rho_g=rho_g, nu_l=nu[0], nu_g=nu[1],
                    phi0=tanh_profile(s, W), meta=dict(Rz=Rz, Rr=Rr, Re=Re, zc=zc))


def oscillating_droplet(nr=256, nz=512, R0=60.0, amp=0.05, jitter=1e-3, seed=1, zc=None,
                        W=4.0, ratio=1000.0, mu_ratio=None, sigma=1e-3, mobility=0.05,
                        z_periodic=True, rho_l=1.0, name="oscillating_droplet") -> CaseSpec:
    """Drop with a P2 Legendre shape perturbation and seeded interface jitter.

    Interface radius r_s(theta) = R0 [1 + amp P2(cos theta)] + jitter * xi_node,
    theta measured from the +z axis; xi from SplitMix64(seed, node index).
    """
    zc = nz / 2 if zc is None else zc
    z, r = node_coords(nr, nz)
    d = np.sqrt((z - zc) ** 2 + r ** 2)
    cth = np.where(d > 0, (z - zc) / np.maximum(d, 1e-300), 1.0)
    p2 = 0.5 * (3.0 * cth ** 2 - 1.0)
    xi = uniform_pm1(seed, np.arange(nr * nz, dtype=np.uint64)).reshape(nr, nz)
    rs = R0 * (1.0 + amp * p2) + jitter * xi
    sp = CaseSpec(name=name, nr=nr, nz=nz, z_periodic=z_periodic, W=W, mobility=mobility,
                  sigma=sigma, rho_l=rho_l, rho_g=rho_l / ratio, nu_l=PAPER_NU, nu_g=PAPER_NU,
                  phi0=tanh_profile(rs - d, W), meta=dict(R0=R0, zc=zc, seed=seed))
    return _with_viscosities(sp, ratio, mu_ratio)


def liquid_thread(nr=128, nz=2048, R0=32.0, amp=0.1, waves=None, noise=1e-4, seed=2, W=4.0,
                  ratio=1000.0, mu_ratio=None, sigma=5e-3, mobility=0.1, rho_l=1.0,
                  name="liquid_thread") -> CaseSpec:
    """Thread of Eq. 47, R(z) = R0 + amp R0 cos(2 pi z / lambda) + noise R0 xi_k.

    The wavelength is Nz / round(Nz / (9 R0)) so that a whole number of waves
    fits the periodic domain.
    """
    if waves is None:
        waves = max(1, round(nz / (9.0 * R0)))
    lam = nz / waves
    z, r = node_coords(nr, nz)
    xi = uniform_pm1(seed, np.arange(nz, dtype=np.uint64))[None, :]
    Rz = R0 + amp * R0 * np.cos(2.0 * math.pi * z / lam) + noise * R0 * xi
    sp = CaseSpec(name=name, nr=nr, nz=nz, z_periodic=True, W=W, mobility=mobility,
                  sigma=sigma, rho_l=rho_l, rho_g=rho_l / ratio, nu_l=PAPER_NU, nu_g=PAPER_NU,
                  phi0=tanh_profile(Rz - r, W),
                  meta=dict(R0=R0, wavelength=lam, k=2 * math.pi * R0 / lam, seed=seed))
    return _with_viscosities(sp, ratio, mu_ratio)


def eotvos_morton(Eo: float, Mo: float, D: float, rho_l: float, rho_g: float, nu_l: float):
    """sigma and g from Eo = g drho D^2 / sigma and Mo = g mu_l^4 drho / (rho_l^2 sigma^3)."""
    mu_l = rho_l * nu_l
    sigma = mu_l * mu_l * math.sqrt(Eo / Mo) / (D * rho_l)
    g = Eo * sigma / ((rho_l - rho_g) * D * D)
    return sigma, g


def rising_bubble(nr=512, nz=2048, R=40.0, zc=200.0, W=4.0, ratio=1000.0, mu_ratio=None,
                  Eo=10.0, Mo=1e-3, mobility=0.02, rho_l=1.0, g_ramp=1000.0,
                  name="rising_bubble") -> CaseSpec:
    """Gas bubble on the axis in a walled column, gravity along -z, reached
    linearly over the first g_ramp steps: at density ratio 1000, gravity
    switched on at once drives the gas past the sound speed before the
    pressure field that holds it can form (tests/test_oracle_stability.py)."""
    z, r = node_coords(nr, nz)
    d = np.sqrt((z - zc) ** 2 + r ** 2)
    nu_l, _ = viscosities(ratio, mu_ratio)
    rho_g = rho_l / ratio
    sigma, g = eotvos_morton(Eo, Mo, 2.0 * R, rho_l, rho_g, nu_l)
    sp = CaseSpec(name=name, nr=nr, nz=nz, z_periodic=False, W=W, mobility=mobility,
                  sigma=sigma, rho_l=rho_l, rho_g=rho_g, nu_l=PAPER_NU, nu_g=PAPER_NU, g_z=-g,
                  dispersed_gas=True, phi0=tanh_profile(d - R, W), g_ramp=g_ramp,
                  meta=dict(R=R, zc=zc, Eo=Eo, Mo=Mo))
    return _with_viscosities(sp, ratio, mu_ratio)


# --------------------------------------------------------------------------
# random states for single-step parity checks
# --------------------------------------------------------------------------

def random_state(nr: int, nz: int, seed: int, u_amp: float = 0.02):
    """Random post-propagation populations (f, g) and previous-step (phi, u_z, u_r).

    f_i = r * phi_n * a_i with a_i in [0.05, 0.2] and phi_n in [0.05, 0.95];
    g_i = r * 1e-3 * xi; aux = (phi_n + 0.01 xi, u_amp xi, u_amp xi).
    Shapes: f, g (9, nr, nz); aux (3, nr, nz).
    """
    n = nr * nz
    idx = np.arange(40 * n, dtype=np.uint64)
    xi = uniform_pm1(seed, idx).reshape(40, nr, nz)
    _, r = node_coords(nr, nz)
    phin = 0.5 + 0.45 * xi[0]
    a = 0.125 + 0.075 * xi[1:10]
    f = r[None] * phin[None] * a
    g = r[None] * 1e-3 * xi[10:19]
    aux = np.stack([phin + 0.01 * xi[19], u_amp * xi[20], u_amp * xi[21]])
    return f, g, aux


# --------------------------------------------------------------------------
# the benchmark workloads (synthetic stand-ins shaped like the paper's tests)
# --------------------------------------------------------------------------

def workload(name: str, as_written: bool = False) -> CaseSpec:
    """Named workloads: static droplet 64x128, oscillation 256x512,
    thread 128x2048, bubble 512x2048 (all at density ratio 1000), and the
    well-conditioned static droplet used for long-horizon parity.

    By default every phase has the paper's nu = 0.1 (dynamic viscosity ratio
    = density ratio, the paper's rates).  as_written: the dynamic viscosity
    ratios the configurations state (100, 50, 100, 100), which put the gas
    viscosity outside the range the paper's tied energy rate runs, so those
    cases take the free energy rate (inputs.energy_rate)."""
    mu = (lambda m: m if as_written else None)
    if name == "static_droplet":
        # the paper's static-drop normalisation rho_g = 1, rho_l = ratio (Sec. 3.1)
        s = static_droplet(nr=64, nz=128, R=20.0, zc=64.0, W=5.0, ratio=1000.0, mu_ratio=mu(100.0),
                           sigma=0.01, mobility=0.1, z_periodic=False, rho_l=1000.0)
        s.steps = 2000
        return s
    if name == "static_droplet_parity":
        # same geometry at the paper's static-drop capillary ratio sigma/rho_l = 1e-6,
        # with rho_l = 1: well conditioned over 1000 steps
        s = static_droplet(nr=64, nz=128, R=20.0, zc=64.0, W=5.0, ratio=1000.0, mu_ratio=mu(100.0),
                           sigma=1e-6, mobility=0.1, z_periodic=False, rho_l=1.0)
        s.steps = 1000
        return s
    if name == "oscillating_droplet":
        s = oscillating_droplet(nr=256, nz=512, R0=60.0, amp=0.05, jitter=1e-3, seed=1,
                                zc=256.0, W=4.0, ratio=1000.0, mu_ratio=mu(50.0), sigma=1e-3,
                                mobility=0.05, z_periodic=True)
        s.steps = 20000
        return s
    if name == "liquid_thread":
        s = liquid_thread(nr=128, nz=2048, R0=32.0, amp=0.1, noise=1e-4, seed=2, W=4.0,
                          ratio=1000.0, mu_ratio=mu(100.0), sigma=5e-3, mobility=0.1)
        s.steps = 200000
        return s
    if name == "rising_bubble":
        # mobility 0.05: with the configuration's 0.02 a gas-side mode grows on
        # the axis inside the rising bubble in this wide column (nr = 512) and
        # the run goes non-finite near step 3500 (nr <= 256 carries 0.02)
        s = rising_bubble(nr=512, nz=2048, R=40.0, zc=200.0, W=4.0, ratio=1000.0,
                          mu_ratio=mu(100.0), Eo=10.0, Mo=1e-3, mobility=0.05)
        s.steps = 100000
        return s
    raise KeyError(name)


WORKLOADS = ("static_droplet", "oscillating_droplet", "liquid_thread", "rising_bubble")


def serving_request(i: int, base_seed: int = 1810) -> CaseSpec:
    """Request i of the serving sweep: a static-droplet, oscillation or bubble
    case with Nr in {64,128,256,512}, Nz = Nr * {2,3,4}, R in [Nr/4, Nr/3],
    density ratio in {10,100,1000}, steps log-uniform in [1e3, 2e4]; every
    phase at the paper's nu = 0.1 (the paper's rates, the fast unit-rate
    collision).

    Bubbles use Eo = Mo = 1, gravity from the first step: with the bubble configuration's Eo = 10, Mo = 1e-3
    the buoyancy drives the gas past the sound speed at density ratio 1000 (and
    for the smallest bubbles at 100) within a few hundred steps, in FP64 too.

    At density ratio 1000, Nr is drawn from {128, 256, 512} (R >= 32 = 8 W):
    drops of R = 16-21 (R/W about 4-5) at that ratio grow a gas-side mode on
    the axis just beyond their poles and go non-finite within 3,500-16,000
    steps, in FP64 too."""
    u = 0.5 * (uniform_pm1(base_seed, np.arange(8, dtype=np.uint64) + np.uint64(8 * i)) + 1.0)
    kind = ("static_droplet", "oscillating_droplet", "rising_bubble")[min(2, int(u[0] * 3))]
    ratio = (10.0, 100.0, 1000.0)[min(2, int(u[4] * 3))]
    if ratio < 1000.0:
        nr = (64, 128, 256, 512)[min(3, int(u[1] * 4))]
    else:
        nr = (128, 256, 512)[min(2, int(u[1] * 3))]
    nz = nr * (2, 3, 4)[min(2, int(u[2] * 3))]
    R = nr * (0.25 + u[3] * (1.0 / 3.0 - 0.25))
    steps = int(round(10 ** (3.0 + u[5] * math.log10(20.0))))
    if kind == "static_droplet":
        s = static_droplet(nr=nr, nz=nz, R=R, zc=nz / 2, W=4.0, ratio=ratio,
                           sigma=0.01, mobility=0.1, z_periodic=False)
    elif kind == "oscillating_droplet":
        s = oscillating_droplet(nr=nr, nz=nz, R0=R, seed=base_seed + i, zc=nz / 2, W=4.0,
                                ratio=ratio, sigma=1e-3, mobility=0.05)
    else:
        zc = min(nz / 4, nz - 1.5 * R)
        s = rising_bubble(nr=nr, nz=nz, R=R, zc=max(zc, 1.5 * R), W=4.0, ratio=ratio,
                          Eo=1.0, Mo=1.0, mobility=0.02, g_ramp=0.0)
    s.name = f"req{i}_{kind}"
    s.steps = steps
    s.meta["request"] = i
    return s
