"""FP32 storage and arithmetic against the FP64 oracle.

Bound (from the method's specification): after 1000 steps
||phi32 - phi64||_inf <= 1e-4 and ||u32 - u64||_inf / ||u64||_inf <= 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_1810_09299_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("zper,collision", [(False, "mrt"), (True, "mrt"), (True, "srt"), (True, "nmrt")])
def test_fp32_static_droplet_1000_steps(zper, collision):
    from paper_1810_09299_amd.case import AxiCase
    spec = inputs.workload("static_droplet_parity")
    spec.z_periodic = zper
    spec.collision = collision
    ora = oracle.OracleCase(spec)
    gpu = AxiCase(spec, precision="fp32")
    ora.step(1000)
    gpu.step(1000)
    mo = ora.moments()
    mg, dg, rc = gpu.moments()
    assert rc == 0
    assert np.abs(mg["phi"] - mo["phi"]).max() <= 1e-4
    un = max(np.abs(mo["uz"]).max(), np.abs(mo["ur"]).max())
    for k in ("uz", "ur"):
        assert np.abs(mg[k] - mo[k]).max() <= 1e-4 * un, k
    # the conserved phase mass stays within FP32 rounding of the FP64 value
    assert abs(dg["phase_mass"] - ora.diagnostics()["phase_mass"]) <= 1e-5 * dg["phase_mass"]


def test_fp32_one_step_random_state():
    """One step from the same random state: FP32 within FP32 rounding of FP64."""
    from paper_1810_09299_amd.case import AxiCase
    spec = inputs.static_droplet(nr=33, nz=130, R=10, zc=65, W=4, sigma=1e-3, mobility=0.1)
    f, g, aux = inputs.random_state(33, 130, seed=5)
    ora = oracle.OracleCase(spec)
    ora.set_state(f, g, aux, 0)
    gpu = AxiCase(spec, precision="fp32")
    gpu.set_state(f, g, aux, 0)
    ora.step(1)
    gpu.step(1)
    fo, go, ao = ora.get_state()
    fg, gg, ag, _ = gpu.get_state()
    for a, b in ((fg, fo), (gg, go)):
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()


def test_fp32_one_step_free_energy_rate_and_ramp():
    """The same with the energy moment at its own rate and gravity mid-ramp."""
    from paper_1810_09299_amd.case import AxiCase
    spec = inputs.static_droplet(nr=33, nz=130, R=10, zc=65, W=4, sigma=1e-3, mobility=0.1)
    spec.free_s1, spec.g_ramp, spec.g_z = True, 50.0, -1e-4
    spec.s_g = (1.0, 1.3, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0)
    f, g, aux = inputs.random_state(33, 130, seed=6)
    ora = oracle.OracleCase(spec)
    ora.set_state(f, g, aux, 20)
    gpu = AxiCase(spec, precision="fp32")
    gpu.set_state(f, g, aux, 20)
    ora.step(1)
    gpu.step(1)
    fo, go, ao = ora.get_state()
    fg, gg, ag, _ = gpu.get_state()
    for a, b in ((fg, fo), (gg, go)):
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
