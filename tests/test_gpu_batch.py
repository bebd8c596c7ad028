"""Batches: many uneven cases in one launch per step (C-ABI lbm_axi_batch_*)."""
import numpy as np
import pytest

from paper_1810_09299_amd import inputs

pytestmark = pytest.mark.gpu


def _mix():
    a = inputs.static_droplet(nr=40, nz=96, R=12, zc=48, W=4, sigma=1e-4, mobility=0.1, z_periodic=False)
    b = inputs.oscillating_droplet(nr=64, nz=128, R0=20, zc=64, W=4, sigma=1e-4, mobility=0.05)
    c = inputs.liquid_thread(nr=33, nz=200, R0=10, W=4, sigma=1e-4, mobility=0.1)
    d = inputs.rising_bubble(nr=48, nz=160, R=10, zc=40, W=4, Eo=1.0, Mo=1.0, g_ramp=40.0)
    e = inputs.static_droplet(nr=36, nz=80, R=10, zc=40, W=4, sigma=1e-4, mobility=0.1, z_periodic=True)
    e.collision = "srt"
    f = inputs.oscillating_droplet(nr=40, nz=90, R0=12, zc=45, W=4, sigma=1e-4, mobility=0.05)
    f.s_g = (1.0, 1.15, 1.2, 1.1, 1.1, 0.9, 0.9, 1.0, 1.0)
    f.free_s1 = True                                  # the energy moment at its own rate
    h = inputs.liquid_thread(nr=20, nz=130, R0=7, W=4, sigma=1e-4, mobility=0.1)
    h.collision = "nmrt"
    h.s_g = (1.0, 1.0, 1.2, 1.1, 1.1, 0.9, 0.9, 1.0, 1.0)
    # collision forms: unit-rate MRT (a-d), SRT (e), MRT with other rates and
    # the free energy rate (f), non-orthogonal MRT (h); d's gravity ramps up
    # over its first 40 of 81 steps (direct launches until then)
    return [(a, 37), (b, 64), (c, 50), (d, 81), (e, 45), (f, 29), (h, 33)]


def _alone(spec, steps, precision):
    from paper_1810_09299_amd.case import AxiCase
    c = AxiCase(spec, precision=precision)
    c.step(steps)
    return c.get_state()


def _run_batch(mix, precision, chunk=16, tile=8, persistent=0, schedule=1, bands=16):
    from paper_1810_09299_amd.batch import Batch
    b = Batch(pool_bytes=256 << 20, max_cases=8, precision=precision)
    b.set_config(tile, persistent, schedule, bands)
    slots = [b.admit(s, n) for s, n in mix]
    assert None not in slots
    for _ in range(200):
        if len(b.poll()) == len(mix):
            break
        b.run(chunk)
    states = [b.get_state(s) for s in slots]
    info = b.info()
    b.close()
    return states, info


@pytest.mark.parametrize("precision,chunk", [("fp32", 16), ("fp64", 16), ("fp16", 16), ("fp32", 7), ("fp16", 7)])
def test_alone_equals_mix_bitwise(precision, chunk):
    """Each case's populations after its own step count are bit-identical
    alone and in the mixed batch (graph replays of full chunks, direct
    launches for the tails where cases finish).  Odd chunks replay the graphs
    of both buffer phases in turn."""
    mix = _mix()
    states, info = _run_batch(mix, precision, chunk=chunk)
    assert info["running"] == 0
    for (spec, n), st in zip(mix, states):
        f, g, aux, t = st
        fa, ga, xa, ta = _alone(spec, n, precision)
        assert t == ta == n
        assert np.isfinite(f).all() and np.isfinite(g).all()
        assert np.array_equal(f, fa) and np.array_equal(g, ga) and np.array_equal(aux, xa)


def test_stochastic_fp16_rounding_alone_equals_mix_bitwise():
    """FP16-deviation cases with stochastic g rounding beside cases rounded to
    nearest (two kernels per collision form): every case's populations after
    its own step count are bit-identical alone and in the batch, through graph
    replays and direct launches, since the random words depend only on the
    node and the case's own time, which the batch keeps on the device."""
    mix = _mix()
    for i, (spec, _) in enumerate(mix):
        spec.fp16_stochastic = i % 2 == 0
    states, info = _run_batch(mix, "fp16", chunk=16)
    assert info["running"] == 0
    for (spec, n), st in zip(mix, states):
        f, g, aux, t = st
        fa, ga, xa, ta = _alone(spec, n, "fp16")
        assert t == ta == n
        assert np.isfinite(f).all() and np.isfinite(g).all()
        assert np.array_equal(f, fa) and np.array_equal(g, ga) and np.array_equal(aux, xa)
    # the option reaches the kernel: the same case rounded to nearest differs
    spec, n = mix[1]
    spec.fp16_stochastic = True
    g_sr = _alone(spec, n, "fp16")[1]
    spec.fp16_stochastic = False
    assert not np.array_equal(g_sr, _alone(spec, n, "fp16")[1])


@pytest.mark.parametrize("tile,persistent,schedule,bands,precision",
                         [(2, 0, 0, 8, "fp32"), (4, 1, 1, 32, "fp32"), (16, 1, 0, 16, "fp32"),
                          (8, 1, 1, 8, "fp32"), (8, 0, 3, 32, "fp32"), (4, 1, 2, 16, "fp32"),
                          (4, 1, 0, 32, "fp16"), (16, 0, 1, 8, "fp16"), (8, 0, 3, 16, "fp16"),
                          (8, 1, 1, 32, "fp16sr"), (2, 0, 3, 8, "fp16sr"),
                          (4, 0, 0, 32, "fp64"), (4, 0, 3, 32, "fp64")])
def test_launch_configuration_does_not_change_results(tile, persistent, schedule, bands, precision):
    """fp16sr: FP16-deviation storage with stochastic g rounding for every
    other case (its random words follow each case's own time, kept on the
    device, whichever workgroup or launch advances it)."""
    mix = _mix()
    if precision == "fp16sr":
        precision = "fp16"
        for i, (spec, _) in enumerate(mix):
            spec.fp16_stochastic = i % 2 == 0
    ref, _ = _run_batch(mix, precision)
    got, _ = _run_batch(mix, precision, chunk=10, tile=tile, persistent=persistent, schedule=schedule,
                        bands=bands)
    for a, b in zip(ref, got):
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y)


def test_admission_by_footprint_and_release():
    from paper_1810_09299_amd import abi
    from paper_1810_09299_amd.batch import Batch
    spec = inputs.static_droplet(nr=64, nz=128, R=20, zc=64, W=5)
    need = Batch.footprint(spec, "fp32")
    head = abi.lbm_axi_batch_reserved_bytes(16, abi.LBM_AXI_FP32)
    b = Batch(pool_bytes=head + 3 * need + 100, max_cases=16, precision="fp32")
    slots = [b.admit(spec, 10) for _ in range(3)]
    assert None not in slots
    assert b.admit(spec, 10) is None            # the pool is full
    b.release(slots[1])
    s = b.admit(spec, 10)
    assert s is not None
    assert b.info()["used"] == 3
    b.run(10)
    assert sorted(b.poll()) == sorted([slots[0], slots[2], s])
    _, diag, rc = b.moments(s, fields=False)
    assert rc == 0 and diag["t"] == 10
    b.close()


def test_finished_cases_stop_exactly():
    from paper_1810_09299_amd.batch import Batch
    spec = inputs.static_droplet(nr=20, nz=40, R=6, zc=20, W=4)
    b = Batch(pool_bytes=64 << 20, max_cases=4, precision="fp64")
    s1 = b.admit(spec, 5)
    s2 = b.admit(spec, 23)
    b.run(8)
    assert b.poll() == [s1]
    b.run(100)
    assert sorted(b.poll()) == sorted([s1, s2])
    assert b.get_state(s1)[3] == 5 and b.get_state(s2)[3] == 23
    b.run(50)                                   # nothing left to run
    assert b.get_state(s2)[3] == 23
    b.close()


@pytest.mark.parametrize("precision,rel", [("fp64", (1e-12,) * 3), ("fp32", (1e-5,) * 3),
                                           ("fp16", (3e-4, 3e-3, 1e-5))])
def test_full_size_batch_step_matches_oracle(precision, rel):
    """The benchmark's path: 256 x 512 oscillating droplets in one batch (tile
    64 x 8, one workgroup per tile, per-XCD bands).  After 100 batched steps,
    one more batched step of the second case equals one oracle step from the
    batch's exported state, at every node.  FP64: the parity bound of
    test_gpu_parity; FP32: one step from FP32-representable values rounds each
    operation once more than FP64, well inside 1e-5 of the largest value.
    FP16-deviation storage: the step's arithmetic is FP32 as above, then f and
    g are stored in FP16 again -- f deviations of at most ~0.03 r at the
    interface keep 11 bits (~2e-5 of max|f|, bound 3e-4), g keeps 11 bits of
    its own value (bound 3e-3 of max|g|); phi and u stay FP32 (1e-5)."""
    import bench
    import oracle
    from paper_1810_09299_amd.batch import Batch
    specs = bench.batch_specs(2)
    pool = Batch.pool_for(specs, precision)
    b = Batch(pool_bytes=pool, max_cases=2, precision=precision)
    b.set_config(8, 0, 1)
    slots = [b.admit(s, 10 ** 6) for s in specs]
    b.run(100)
    f, g, aux, t = b.get_state(slots[1])
    assert t == 100
    ora = oracle.OracleCase(specs[1])
    ora.set_state(f, g, aux, t)
    ora.step(1)
    b.run(1)
    fg, gg, ag, t1 = b.get_state(slots[1])
    b.close()
    assert t1 == 101
    for x, y, bound, name in zip((fg, gg, ag), ora.get_state(), rel, "fga"):
        err = np.abs(x - y).max()
        assert err <= bound * np.abs(y).max(), (name, err)


def test_case_placed_beyond_4_gib_of_the_pool():
    """Case state addresses are 64-bit in the batch's case table (only offsets
    within one case are 32-bit): a case that the first-fit pool places after a
    filler of more than 4 GiB steps bit-identically to the same case alone."""
    from paper_1810_09299_amd.batch import Batch
    filler = inputs.static_droplet(nr=2048, nz=8192, R=600, zc=4096, W=4, sigma=1e-4, mobility=0.1)
    need = Batch.footprint(filler, "fp64")
    assert need > (4 << 30)
    spec, n = _mix()[1]
    b = Batch(pool_bytes=need + (256 << 20), max_cases=4, precision="fp64")
    b.set_config(8, 0, 1)
    s_fill = b.admit(filler, 2)
    s_case = b.admit(spec, n)
    assert s_fill is not None and s_case is not None
    for _ in range(50):
        if len(b.poll()) == 2:
            break
        b.run(16)
    f, g, aux, t = b.get_state(s_case)
    b.close()
    fa, ga, xa, ta = _alone(spec, n, "fp64")
    assert t == ta == n
    assert np.array_equal(f, fa) and np.array_equal(g, ga) and np.array_equal(aux, xa)


def test_autotuner_picks_a_candidate_and_answers_do_not_change():
    """tune_batch times every candidate launch configuration and returns the
    fastest; the batch gives bit-identical populations under every candidate
    of the tuner's default search space (tile height x persistence x case
    order x band count)."""
    import itertools
    from paper_1810_09299_amd import autotune
    from paper_1810_09299_amd.batch import Batch
    mix = [(s, 400) for s, _ in _mix()[:4]]

    def make():
        b = Batch(pool_bytes=256 << 20, max_cases=8, precision="fp32")
        for s, n in mix:
            assert b.admit(s, n) is not None
        return b

    best, timings = autotune.tune_batch(make, tiles=(8, 4), persistent=(0, 1), schedules=(1, 0),
                                        bands=(16, 8), chunk=20, steps=40)
    assert set(timings) == set(itertools.product((8, 4), (0, 1), (1, 0), (16, 8)))
    assert all(t > 0 for t in timings.values()) and best == min(timings, key=timings.get)
    short = [(s, 37) for s, _ in _mix()]
    ref, _ = _run_batch(short, "fp32", tile=best[0], persistent=best[1], schedule=best[2], bands=best[3])
    defaults = autotune.tune_batch.__defaults__
    space = itertools.product(defaults[0], defaults[1], defaults[2], defaults[3])
    for cfg in space:
        st, _ = _run_batch(short, "fp32", chunk=11, tile=cfg[0], persistent=cfg[1], schedule=cfg[2],
                           bands=cfg[3])
        for a, b in zip(ref, st):
            for x, y in zip(a[:3], b[:3]):
                assert np.array_equal(x, y), cfg


def test_prepare_captures_without_stepping():
    """prepare() leaves every case at its time; the runs after it give the
    same populations as runs without it."""
    from paper_1810_09299_amd.batch import Batch
    mix = [(s, 40) for s, _ in _mix()[:3]]
    ref, _ = _run_batch(mix, "fp32", chunk=20)
    b = Batch(pool_bytes=256 << 20, max_cases=8, precision="fp32")
    slots = [b.admit(s, n) for s, n in mix]
    b.run(3)                                         # odd: the next run starts at the other phase
    for m in (20, 17):
        b.prepare(m)
    assert all(b.get_state(s)[3] == 3 for s in slots)
    b.run(20)
    b.run(17)
    got = [b.get_state(s) for s in slots]
    b.close()
    for a, g in zip(ref, got):
        assert g[3] == 40
        for x, y in zip(a[:3], g[:3]):
            assert np.array_equal(x, y)


def test_block_reused_while_steps_are_queued():
    """A case released while its steps are still queued: the next case placed
    in its pool block waits for them (the steps would otherwise overwrite the
    new case's state), and its result equals the case run alone."""
    from paper_1810_09299_amd.batch import Batch
    (a, _), (c, nc) = _mix()[1], _mix()[5]
    b_spec = inputs.oscillating_droplet(nr=40, nz=90, R0=12, zc=45, W=4, sigma=1e-4, mobility=0.05, seed=9)
    need = [Batch.footprint(x, "fp32") for x in (a, b_spec)]
    from paper_1810_09299_amd import abi
    head = abi.lbm_axi_batch_reserved_bytes(4, abi.LBM_AXI_FP32)
    bt = Batch(pool_bytes=head + sum(need) + 512, max_cases=4, precision="fp32")
    sa = bt.admit(a, 10 ** 6)
    sb = bt.admit(b_spec, 10 ** 6)
    for _ in range(5):
        bt.run(50)                                   # queued, not waited for
    bt.release(sb)                                   # still running on the GPU
    sc = bt.admit(c, nc)                             # only b's block fits
    assert sc is not None
    for _ in range(20):
        if sc in bt.poll():
            break
        bt.run(16)
    f, g, aux, t = bt.get_state(sc)
    assert t == nc
    bt.release(sa)
    bt.close()
    fa, ga, xa, ta = _alone(c, nc, "fp32")
    assert np.array_equal(f, fa) and np.array_equal(g, ga) and np.array_equal(aux, xa)


def test_bench_short_run_times_exactly_the_requested_steps():
    """The benchmark's timed region holds exactly --steps steps after exactly
    --warmup steps, for short and odd counts (20 after 5, for one)."""
    import bench
    specs = bench.batch_specs(2)
    for steps, warmup in ((20, 5), (1, 0), (7, 3), (130, 1)):
        res = bench.run_batch(specs, "fp32", steps, warmup, config=(8, 0, 1, 16))
        assert res["steps"] == steps
        assert res["t_final"] == steps + warmup
        assert res["finite"] and res["kernel_ms"] > 0


def test_degenerate_step_counts():
    """Zero steps leave a state untouched; a negative count is rejected; a
    batch with nothing running accepts run() as a no-op; a case admitted with
    zero steps is done at once and holds its initial state."""
    from paper_1810_09299_amd import abi
    from paper_1810_09299_amd.batch import Batch
    from paper_1810_09299_amd.case import AxiCase
    spec, _ = _mix()[0]
    c = AxiCase(spec, precision="fp64")
    f0, g0, a0, t0 = c.get_state()
    c.step(0)
    f1, g1, a1, t1 = c.get_state()
    assert t1 == t0 == 0 and np.array_equal(f0, f1) and np.array_equal(g0, g1) and np.array_equal(a0, a1)
    with pytest.raises(abi.LbmAxiError):
        c.step(-1)
    c.close()
    b = Batch(pool_bytes=64 << 20, max_cases=4, precision="fp64")
    b.run(16)                                        # nothing admitted: a no-op
    assert b.info()["launches"] == 0
    s0 = b.admit(spec, 0)
    s1 = b.admit(spec, 5)
    b.run(16)
    assert sorted(b.poll()) == sorted([s0, s1])
    fz, gz, az, tz = b.get_state(s0)
    assert tz == 0 and np.array_equal(fz, f0) and np.array_equal(gz, g0) and np.array_equal(az, a0)
    assert b.get_state(s1)[3] == 5
    with pytest.raises(abi.LbmAxiError):
        b.run(-1)
    b.close()


def test_invalid_configurations_and_slots_are_rejected():
    from paper_1810_09299_amd import abi
    from paper_1810_09299_amd.batch import Batch
    from paper_1810_09299_amd.case import AxiCase
    spec, _ = _mix()[0]
    c = AxiCase(spec, precision="fp32")
    for tr in (3, 32, -1):
        with pytest.raises(abi.LbmAxiError):
            c.set_tile(tr)
    c.close()
    b = Batch(pool_bytes=64 << 20, max_cases=2, precision="fp32")
    for cfg in ((5, 0, 1, 16), (8, 2, 1, 16), (8, 0, 4, 16), (8, 0, -1, 16), (8, 0, 1, 12), (8, 0, 1, 64)):
        with pytest.raises(abi.LbmAxiError):
            b.set_config(*cfg)
    s = b.admit(spec, 3)
    with pytest.raises(abi.LbmAxiError):
        abi.lbm_axi_batch_release(b.handle, 1)        # slot 1 is not in use
    with pytest.raises(abi.LbmAxiError):
        abi.lbm_axi_batch_release(b.handle, 7)        # beyond max_cases
    b.run(3)
    assert b.poll() == [s]
    b.close()
