"""Host checks of bench.py: the timed region holds exactly the
requested number of steps for any --steps >= 1, and runs on more than one
GPU are refused with a message."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("steps", [1, 5, 20, 99, 100, 101, 250, 1000, 2000, 12345])
def test_step_plan_sums_to_steps(steps):
    plan = bench.step_plan(steps)
    assert sum(plan) == steps
    assert all(m >= 1 for m in plan)
    # every run but the last has the replayed length min(chunk, steps)
    c = min(bench.CHUNK, steps)
    assert all(m == c for m in plan[:-1])
    assert 1 <= plan[-1] <= c


def test_step_plan_examples():
    assert bench.step_plan(20) == [20]          # a short run: one replay of 20
    assert bench.step_plan(5) == [5]
    assert bench.step_plan(250) == [100, 100, 50]
    assert bench.step_plan(300) == [100, 100, 100]
    assert bench.step_plan(0) == []
    assert bench.step_plan(7, chunk=3) == [3, 3, 1]


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_refuses_zero_steps():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "0"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
