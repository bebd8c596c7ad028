"""Continuous batching: requests admitted while others run, results equal to
running each request alone."""
import numpy as np
import pytest

from paper_1810_09299_amd import inputs

pytestmark = pytest.mark.gpu


def _small_requests(n=12):
    from paper_1810_09299_amd import serving
    reqs = []
    i = 0
    while len(reqs) < n:
        s = inputs.serving_request(i)
        i += 1
        if s.nr > 128:
            continue
        steps = min(s.steps, 1500)
        reqs.append(serving.Request(rid=i, arrival=0.0, spec=s, steps=steps))
    return reqs


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_serving_results_equal_alone_runs(precision):
    """Poisson arrivals, admission by footprint under a pool that cannot hold
    every request at once: every request completes with exactly its steps,
    and 8 sampled requests' fields are bit-identical to running them alone."""
    from paper_1810_09299_amd import serving
    from paper_1810_09299_amd.batch import Batch
    from paper_1810_09299_amd.case import AxiCase
    reqs = _small_requests()
    serving.poisson_arrivals(reqs, rate_per_s=200.0)
    need = sorted(Batch.footprint(r.spec, precision) for r in reqs)
    pool = sum(need[-4:]) + Batch.head_bytes(16, precision)   # room for about four at a time
    reqs, summ = serving.serve(reqs, pool_bytes=pool, max_cases=16, precision=precision, chunk=100,
                               keep_fields=True)
    assert summ["requests"] == len(reqs)
    assert 1 < summ["max_running"] < len(reqs)       # admission bound by memory, work overlapped
    for r in reqs:
        assert r.diag["t"] == r.steps
        assert r.finished >= r.admitted >= r.arrival
    for r in reqs[:8]:
        alone = AxiCase(r.spec, precision=precision)
        alone.step(r.steps)
        fields, diag, _ = alone.moments()
        for k in ("phi", "rho", "uz", "ur", "p"):
            assert np.array_equal(fields[k], r.fields[k], equal_nan=True), (r.rid, k)
        assert diag["t"] == r.steps


def test_latency_percentiles_reported():
    from paper_1810_09299_amd import serving
    reqs = _small_requests(8)
    serving.poisson_arrivals(reqs, rate_per_s=100.0)
    _, summ = serving.serve(reqs, pool_bytes=512 << 20, max_cases=8, precision="fp32", chunk=100)
    assert 0 < summ["p50_latency_s"] <= summ["p99_latency_s"]
    assert summ["aggregate_mlups"] > 0
