"""The oscillation and thread configurations in every storage precision,
against the FP64 GPU path (which matches the oracle, tests/test_gpu_parity.py).

Bounds.  FP32 agrees with FP64 to ~1e-5 in phi after 1000 steps and FP16
deviation storage to ~1e-4 (tests/test_gpu_fp32.py, tests/test_gpu_fp16.py).
The semi-axes come from linear interpolation of the psi = 1/2 crossings,
where |d phi / dz| is about 1/W = 0.25 per cell, so a phi error e moves them by
about 4e; over 20k steps of the oscillation the bounds 0.01 cell (FP32) and
0.02 cell (FP16) leave a margin of 10 or more on e.  Pinch-off is sampled
every 100 steps: the times agree within 1% plus one sample.
"""
import numpy as np
import pytest

from paper_1810_09299_amd import inputs

pytestmark = pytest.mark.gpu


def _semi_axes(precision, steps=20000, every=500):
    from paper_1810_09299_amd.case import AxiCase
    c = AxiCase(inputs.workload("oscillating_droplet"), precision=precision)
    out = []
    for _ in range(steps // every):
        c.step(every)
        d = c.diagnostics()
        assert not d["nonfinite"]
        out.append((d["semi_z"], d["semi_r"]))
    return np.array(out)


def test_oscillation_semi_axes_in_every_precision():
    """256 x 512 oscillating droplet (ratio 1000, P2 amplitude 0.05 R0), 20k steps."""
    ref = _semi_axes("fp64")
    assert ref[:, 0].max() - ref[:, 0].min() > 1.0          # the drop does oscillate
    for prec, bound in (("fp32", 0.01), ("fp16", 0.02)):
        got = _semi_axes(prec)
        assert np.abs(got - ref).max() <= bound, prec


def _pinch_off(precision, every=100, limit=200000):
    from paper_1810_09299_amd.case import AxiCase
    c = AxiCase(inputs.workload("liquid_thread"), precision=precision)
    while c.t < limit:
        c.step(every)
        d = c.diagnostics()
        assert not d["nonfinite"]
        if d["min_axis_phi"] < 0.5:
            return d["t"]
    return None


def test_thread_pinch_off_time_in_every_precision():
    """128 x 2048 periodic thread (ratio 1000, 7 waves, seeded noise)."""
    t64 = _pinch_off("fp64")
    assert t64 is not None
    for prec in ("fp32", "fp16"):
        t = _pinch_off(prec)
        assert t is not None and abs(t - t64) <= 0.01 * t64 + 100, (prec, t, t64)
