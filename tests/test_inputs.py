"""Host-side workload definitions (no GPU): the viscosities each workload
gets, the energy-rate extension they switch to, and the gravity ramp of the
bubble."""
import math

import pytest

from paper_1810_09299_amd import inputs


def _mu_ratio(spec):
    return (spec.rho_l * spec.nu_l) / (spec.rho_g * spec.nu_g)


def test_viscosities_honour_the_dynamic_viscosity_ratio():
    assert inputs.viscosities(1000.0, None) == (0.1, 0.1)
    for ratio, mu in ((1000.0, 100.0), (1000.0, 50.0), (10.0, 100.0), (100.0, 100.0)):
        nl, ng = inputs.viscosities(ratio, mu)
        assert min(nl, ng) == 0.1
        assert math.isclose(ratio * nl / ng, mu, rel_tol=1e-12)


def test_energy_rate_switches_outside_the_tied_rates_window():
    lo, hi = inputs.TIED_RATE_NU
    assert inputs.energy_rate(0.1, 0.1)[0] is False
    assert inputs.energy_rate(lo, hi)[0] is False
    for nl, ng in ((0.1, 1.0), (0.1, 2.0), (0.03, 0.1), (0.3, 0.1)):
        free, sg = inputs.energy_rate(nl, ng)
        assert free is True and sg[1] == 1.0


@pytest.mark.parametrize("name,mu", [("static_droplet", 100.0), ("oscillating_droplet", 50.0),
                                     ("liquid_thread", 100.0), ("rising_bubble", 100.0)])
def test_workloads_as_written_have_the_stated_viscosity_ratio(name, mu):
    paper = inputs.workload(name)
    assert paper.nu_l == paper.nu_g == 0.1 and not paper.free_s1
    assert math.isclose(_mu_ratio(paper), paper.rho_l / paper.rho_g, rel_tol=1e-12)
    written = inputs.workload(name, as_written=True)
    assert math.isclose(_mu_ratio(written), mu, rel_tol=1e-12)
    assert written.free_s1 and written.meta["mu_ratio"] == mu
    # the same geometry and interface in both forms
    assert (written.nr, written.nz, written.W, written.sigma) == (paper.nr, paper.nz, paper.W, paper.sigma)


def test_a_viscosity_pair_and_a_ratio_are_not_both_accepted():
    with pytest.raises(ValueError):
        inputs.static_droplet(nr=16, nz=32, R=5, zc=16, W=4, ratio=1000.0, mu_ratio=100.0, nu=(0.1, 0.1))


def test_bubble_gravity_is_ramped_and_sized_by_eo_and_mo():
    s = inputs.workload("rising_bubble")
    assert s.g_ramp == 1000.0 and s.g_z < 0.0 and s.mobility == 0.05
    R, D = s.meta["R"], 2 * s.meta["R"]
    # Eo = g drho D^2 / sigma (R20)
    assert math.isclose(abs(s.g_z) * (s.rho_l - s.rho_g) * D * D / s.sigma, 10.0, rel_tol=1e-9)
    assert R == 40.0
