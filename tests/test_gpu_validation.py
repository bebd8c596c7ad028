"""The GPU path on the paper's own test problems (Sec. 3), against the numbers
the paper prints.  These are physics checks, not parity: the paper's numbers
come from its own implementation, whose initial populations and measurement
details it does not give, so the comparisons with them use the paper's own
level of agreement with theory (Table 1: up to 8.9 %); the oscillation
frequencies are also checked, more tightly, against the damped-mode
prediction of Eq. 43 and Lamb's decay rate."""
import os

import numpy as np
import pytest

from paper_1810_09299_amd import inputs, validation
from paper_1810_09299_amd.case import AxiCase

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _breakup_rows():
    return np.loadtxt(os.path.join(GOLD, "thread_breakup_times.txt"))


@pytest.mark.parametrize("ratio,wavelength", [(100, 600), (100, 1200), (100, 1800), (10, 600), (10, 1200),
                                              (10, 1800)])
def test_thread_breakup_time_matches_paper(ratio, wavelength):
    rows = _breakup_rows()
    ref = [r[3] for r in rows if r[0] == ratio and r[1] == wavelength][0]
    tb, _ = validation.thread_breakup_time(wavelength, ratio=float(ratio))
    assert abs(tb - ref) <= 0.03 * ref, (tb, ref)


def _damped_prediction(r):
    """sqrt(omega_43^2 - gamma_Lamb^2): where a shape mode of Eq. 43's
    frequency rings when its amplitude decays at Lamb's rate."""
    return (r["omega_ana"] ** 2 - r["gamma_lamb"] ** 2) ** 0.5


def _report(tag, r, paper):
    pred = _damped_prediction(r)
    print(f"\n{tag}: omega_lb {r['omega_lb'] * 1e4:.4f}e-4 (paper {paper:.4f}e-4, {r['omega_lb'] * 1e4 / paper - 1:+.2%}); "
          f"damped prediction {pred * 1e4:.4f}e-4 ({r['omega_lb'] / pred - 1:+.2%}); gamma {r['gamma'] * 1e4:.4f}e-4 "
          f"vs Lamb {r['gamma_lamb'] * 1e4:.4f}e-4 ({r['gamma'] / r['gamma_lamb'] - 1:+.2%}); undamped "
          f"{r['omega_undamped'] * 1e4:.4f}e-4 vs Eq. 43 {r['omega_ana'] * 1e4:.4f}e-4")


@pytest.mark.parametrize("ratio,omega_lb", [(10, 15.2504), (20, 11.0000), (50, 7.0439)])
def test_oscillation_frequency_matches_paper_table2(ratio, omega_lb):
    """Table 2 (R_r = 30, R_z = 90, density ratios 10, 20, 50; ratio 100 is
    Table 1's first column): omega_LB within 8.9 % of the paper's LB column
    (measured -2.8, -2.5, -3.2 %), and within 6 % of the damped prediction
    (measured -5.2, -4.8, -2.6 %: the denser the outer fluid, the more the
    walls and the periodic images 300 cells apart slow it), and the fitted
    decay rate 0.6-1.1 of Lamb's (measured 0.80, 0.75, 0.73).  The table's
    analytic column is not what Eqs. 43-45 give for these ratios, so only its
    LB column is compared."""
    r = validation.oscillation_frequency(30, ratio=float(ratio), steps=60000, every=20)
    _report(f"Table 2, ratio {ratio}", r, omega_lb)
    assert abs(r["omega_lb"] * 1e4 - omega_lb) <= 0.089 * omega_lb, r["omega_lb"]
    assert abs(r["omega_lb"] / _damped_prediction(r) - 1.0) <= 0.06
    assert 0.6 <= r["gamma"] / r["gamma_lamb"] <= 1.1


@pytest.mark.parametrize("Rr,omega_lb", [(30, 4.8934), (45, 3.4074), (60, 2.5964), (75, 2.1313)])
def test_oscillation_frequency_matches_paper_table1(Rr, omega_lb):
    """Every column of Table 1 (R_z = 90, density ratio 100, R_e = (R_r^2 R_z)^(1/3)
    = 43.3, 56.7, 68.7, 79.7).

    At nu = 0.1 these drops are strongly damped: Lamb's decay rate is 0.37-0.51
    of Eq. 43's frequency, so the mode rings at sqrt(omega^2 - gamma^2), 7-14 %
    below Eq. 43.  The fitted frequency is checked against that damped
    prediction within 3 % (measured +2.2, -0.2, -0.9, -1.2 %); this detects a
    shift of the frequency that the paper's own 8.9 % spread would not.  The
    fitted decay rate is 0.6-1.1 of Lamb's (measured 0.73-0.76, and 0.73-0.80
    in Table 2): Lamb's rate is the small-viscosity limit, and these drops,
    with omega R^2 / nu of only 9-20, decay more slowly.  With the fitted
    rate, sqrt(omega^2 + gamma^2) lies 4.1-4.7 % below Eq. 43 in every column.  Against the
    paper's LB column: within that 8.9 % (measured -3.2, -5.8, -6.0, -7.4 %;
    the paper's values lie between the damped and the undamped frequency, and
    it does not say how it measured them).  For R_r = 30 the first oblate
    extreme at t ~ 8600 (Sec. 3.2)."""
    r = validation.oscillation_frequency(Rr, steps=60000, every=20)
    _report(f"Table 1, R_r {Rr}", r, omega_lb)
    assert abs(r["omega_lb"] / _damped_prediction(r) - 1.0) <= 0.03
    assert 0.6 <= r["gamma"] / r["gamma_lamb"] <= 1.1
    assert abs(r["omega_lb"] * 1e4 - omega_lb) <= 0.089 * omega_lb, r["omega_lb"]
    if Rr == 30:
        t, rr = r["t"], r["semi_r"]
        q = validation.first_extremum(t, rr)
        assert abs(t[q] - 8600) <= 0.05 * 8600, t[q]


def test_oscillation_frequency_in_every_precision():
    """Table 1's first column (R_r = 30) in FP32 and in FP16-deviation storage
    (g rounded to nearest and stochastically): the fitted frequency and decay
    rate of R_r(t) against the FP64 path's over the same 60k steps."""
    ref = validation.oscillation_frequency(30, steps=60000, every=20)
    for prec, sr, bound in (("fp32", False, 2e-3), ("fp16", False, 1e-2), ("fp16", True, 1e-2)):
        r = validation.oscillation_frequency(30, steps=60000, every=20, precision=prec, fp16_stochastic=sr)
        dw = r["omega_lb"] / ref["omega_lb"] - 1.0
        dg = r["gamma"] / ref["gamma"] - 1.0
        print(f"\n{prec}{' stochastic' if sr else ''}: omega_lb {dw:+.2e}, gamma {dg:+.2e} relative to FP64")
        assert abs(dw) <= bound and abs(dg) <= 3 * bound, (prec, sr, dw, dg)


def test_laplace_pressure_converges():
    out = validation.laplace_run(nr=48, nz=96, R=16.0, W=4.0, ratio=100.0, sigma=1e-4, steps=12000,
                                 every=2000)
    assert abs(out[-1][1] - 1.0) <= 0.01, out


def _gold(name):
    return dict(l.split() for l in open(os.path.join(GOLD, name))
                if l.strip() and not l.startswith("#"))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_paper_static_droplet_at_equilibrium(precision):
    """The Sec. 3.1 static drop (Nz x Nr = 200 x 100, R = 50 at (100, 0),
    rho_l / rho_g = 1000 / 1, W = 4, sigma = 1e-3, M = 0.01, nu = 0.1,
    periodic z, no-slip top wall), run to equilibrium and then sampled every
    500 steps over another 20000:

    - |u|max is of the order 1e-6 the paper reports (Fig. 1a);
    - the density across the interface at the equator follows Eq. 42 within
      1 % of rho_l - rho_g (Fig. 1b; measured 0.6 %);
    - the drop keeps its radius: R_eq within 0.1 cell of R, semi_r within
      0.05 cell (measured 0.055 and 0.006);
    - the pressure jump, averaged over the samples, is 2 sigma / R_eq within
      5 % (an acoustic oscillation of a few per cent is still ringing;
      measured mean 0.975)."""
    spec = inputs.static_droplet(nr=100, nz=200, R=50, zc=100, W=4, ratio=1000, sigma=1e-3,
                                 mobility=0.01, z_periodic=True, rho_l=1000.0, nu=(0.1, 0.1))
    case = AxiCase(spec, precision=precision)
    case.step(20000)
    lap, umax = [], []
    for _ in range(40):
        case.step(500)
        _, d, rc = case.moments(fields=False)
        assert rc == 0
        lap.append(d["dp"] / (2 * spec.sigma / d["R_eq"]))
        umax.append(d["umax"])
    m, d, _ = case.moments()
    ref = float(_gold("static_droplet_spurious.txt")["umax_order"])
    assert ref / 10 < max(umax) < ref * 10, max(umax)
    rho_an = spec.rho_g + (spec.rho_l - spec.rho_g) * spec.phi0
    equator = np.abs(m["rho"][:, 100] - rho_an[:, 100]) / (spec.rho_l - spec.rho_g)
    assert equator.max() <= 0.01, equator.max()
    assert abs(d["R_eq"] - 50) <= 0.1 and abs(d["semi_r"] - 50) <= 0.05, (d["R_eq"], d["semi_r"])
    assert abs(np.mean(lap) - 1.0) <= 0.05, lap


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_static_droplet_workload_laplace_and_conservation(precision):
    """The static-droplet workload (64 x 128, z walls, R = 20, W = 5, density
    ratio 1000 at rho_l = 1000, sigma = 0.01, M = 0.1).  Its closed box rings
    acoustically for about 30k steps (dp / (2 sigma / R_eq) is 2.05 at step
    2000); averaged over steps 30k-40k the jump is 2 sigma / R_eq within 2 %
    (measured 1.005 in every precision), |u|max stays of order 1e-5, and the
    phase mass drifts by at most FP64 roundoff, FP32 rounding (measured
    2.8e-4 over 40k steps) or not at all (FP16-deviation storage)."""
    spec = inputs.workload("static_droplet")
    case = AxiCase(spec, precision=precision)
    _, d0, _ = case.moments(fields=False)
    case.step(30000)
    lap, umax = [], []
    for _ in range(20):
        case.step(500)
        _, d, rc = case.moments(fields=False)
        assert rc == 0
        lap.append(d["dp"] / (2 * spec.sigma / d["R_eq"]))
        umax.append(d["umax"])
    assert abs(np.mean(lap) - 1.0) <= 0.02, np.mean(lap)
    assert max(umax) < 1e-4, max(umax)
    drift = abs(d["phase_mass"] / d0["phase_mass"] - 1)
    assert drift <= {"fp64": 1e-12, "fp32": 1e-3, "fp16": 0.0}[precision], drift


@pytest.mark.parametrize("precision,nr,tol,stochastic", [("fp64", 64, 2e-3, False), ("fp32", 64, 2e-3, False),
                                                         ("fp16", 16, 1e-2, False), ("fp16", 64, 1e-2, True)])
def test_pipe_flow_bessel_mode(precision, nr, tol, stochastic):
    """Axial flow in the pipe bounded by the r-wall (R_w = nr): u_z =
    U J_0(alpha r / R_w) keeps its shape and decays at nu (alpha / R_w)^2, the
    slowest mode of d_t u_z = nu (d_r^2 + d_r / r) u_z (the axisymmetric
    viscous terms of Eqs. 6 and 30, nu of Eq. 34).  FP16-deviation storage
    rounds every stored g / r to 11 bits each step, so a change of less than
    half an FP16 ulp (2^-12 of the value) per step is lost: at nr = 64 the
    mode decays by 1.4e-4 of itself per step and FP16 keeps only 0.6 of the
    rate; at nr = 16 (2.3e-3 per step) it is within 1 %.  Stochastic g
    rounding stores every g unbiased, and the rate at nr = 64 is within 1 %."""
    from scipy.special import j0
    nz, nu, U = 8, 0.1, 1e-3
    alpha = 2.404825557695773
    spec = inputs.static_droplet(nr=nr, nz=nz, R=2, W=4, sigma=0.0, mobility=0.05, z_periodic=True,
                                 nu=(nu, nu))
    spec.phi0 = np.ones((nr, nz))
    spec.fp16_stochastic = stochastic
    case = AxiCase(spec, precision=precision)
    f, _, aux, _ = case.get_state()
    z, r = inputs.node_coords(nr, nz)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cz = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    uz = U * j0(alpha * r / nr)
    cu = cz[:, None, None] * uz[None]
    g = r[None] * spec.rho_l * w[:, None, None] * (3 * cu + 4.5 * cu ** 2 - 1.5 * (uz ** 2)[None])
    aux[1] = uz
    case.set_state(f, g, aux, 0)
    lam = nu * (alpha / nr) ** 2
    case.step(int(0.1 / lam))
    u0 = case.moments()[0]["uz"][:, 0].copy()
    steps = int(0.85 / lam)
    case.step(steps)
    u1 = case.moments()[0]["uz"][:, 0].copy()
    rate = -np.log(u1[0] / u0[0]) / steps
    assert abs(rate / (nu * (alpha / nr) ** 2) - 1) <= tol, rate / (nu * (alpha / nr) ** 2)
    assert np.abs(u1 / u1[0] - j0(alpha * r[:, 0] / nr)).max() <= 5 * tol


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_radial_phase_field_diffusion_bessel_mode(precision):
    """phi = 1/2 + eps J_0(a r / R_w), a the first zero of J_1 (no flux at the
    r-wall), with u = 0 and the counter term negligible (W = 1e6): the slowest
    radial mode of d_t phi = M (d_r^2 + d_r / r) phi (Eq. 5), decaying at
    M (a / R_w)^2.  At nr = 64 it changes by 3.6e-4 of itself per step; the
    FP16-deviation storage keeps it (f is stored as a deviation from the
    reader's phi, which is FP32), unlike the slow g of the pipe-flow mode."""
    from scipy.special import j0
    a1 = 3.8317059702075125
    nr, nz, M = 64, 8, 0.1
    spec = inputs.static_droplet(nr=nr, nz=nz, R=2, W=1e6, sigma=0.0, mobility=M, z_periodic=True)
    _, r = inputs.node_coords(nr, nz)
    spec.phi0 = 0.5 + 0.1 * j0(a1 * r / nr)
    case = AxiCase(spec, precision=precision)
    lam = M * (a1 / nr) ** 2
    case.step(int(0.1 / lam))
    p0 = case.moments()[0]["phi"][:, 0] - 0.5
    n = int(1.0 / lam)
    case.step(n)
    p1 = case.moments()[0]["phi"][:, 0] - 0.5
    assert abs(-np.log(p1[0] / p0[0]) / n / lam - 1) <= 5e-3
    assert np.abs(p1 / p1[0] - j0(a1 * r[:, 0] / nr)).max() <= 5e-3
