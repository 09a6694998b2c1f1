"""GPU tests of the batch API (mwax_batch_*): many uneven instances as one
persistent, graph-replayed unit of device work per call.

Parity bar: a batch instance must give exactly what the same plan gives when
driven alone with mwax_channelise + mwax_correlate (bit for bit, INT8 and
FP16), and its INT8 sums must equal the oracle's integer X-engine on the
channelised codes the batch produced.  Every input is seeded and synthetic.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_11557_amd import mwax  # noqa: E402
from paper_2303_11557_amd.mwax import Batch, Plan, make_config  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    mwax.lib()
    yield


def log(msg):
    print(msg, flush=True)


# (tiles, L, T): uneven tile counts (ragged 128-input tiles), FFT lengths and
# integration lengths; T chosen so integrations end inside calls.
SHAPES = [(3, 32, 200), (70, 128, 50), (16, 1024, 10), (64, 32, 600), (5, 128, 30), (130, 64, 100)]
CHUNK = 16384          # samples per instance per call: a multiple of every L
CALLS = 3


def make_volts(i, n_in, S):
    v = synth.gaussian_volts(n_in, S, seed=synth.MWAX_SEED + 3 + i, sources=[synth.Source(3.0, 5 + i)], L=32)
    d = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    return d


@pytest.fixture(scope="module")
def volts():
    return [make_volts(i, 2 * t, CHUNK * CALLS) for i, (t, L, T) in enumerate(SHAPES)]


def cfgs(prec, shapes=SHAPES, chunk=CHUNK):
    return [make_config(t, L=L, T=T, xprec=prec, max_samples=chunk) for (t, L, T) in shapes]


def drain(p, prec, max_ints=64):
    if prec == "int8":
        raw, sc = p.integrate_raw(max_ints)
        return raw.cpu().numpy(), sc.cpu().numpy()
    return p.integrate(max_ints).cpu().numpy(), None


def run_single(prec, volts, shapes=SHAPES, chunk=CHUNK, calls=CALLS):
    outs = []
    for i, c in enumerate(cfgs(prec, shapes, chunk)):
        got = []
        with Plan(c) as p:
            for k in range(calls):
                p.channelise(volts[i][:, k * chunk:(k + 1) * chunk])
                p.correlate()
                got.append(drain(p, prec))
            torch.cuda.synchronize()
        outs.append(got)
    return outs


def run_batch(prec, volts, graph=True, tuning=None, autotune=False, between=None, shapes=SHAPES,
              chunk=CHUNK, calls=CALLS, tiles=None):
    outs = [[] for _ in shapes]
    volts = volts[:len(shapes)]
    with Batch(cfgs(prec, shapes, chunk)) as b:
        b.set_graph(graph)
        if tuning is not None:
            b.set_tuning(*tuning)
        if tiles is not None:
            b.set_tiles(tiles)
            assert b.tiles() == list(tiles)
        if autotune:
            kc, grid = b.autotune([v[:, :chunk] for v in volts], trials=2)
            log(f"autotuned kchunk={kc} grid={grid}")
        for k in range(calls):
            b.run([v[:, k * chunk:(k + 1) * chunk] for v in volts])
            if between is not None:
                between(k)
            for i, p in enumerate(b.plans):
                outs[i].append(drain(p, prec))
        b.sync()
    return outs


def assert_same(a, b, what):
    for i, (ga, gb) in enumerate(zip(a, b)):
        for k, (x, y) in enumerate(zip(ga, gb)):
            assert x[0].shape == y[0].shape, f"{what}: instance {i} call {k} emitted {x[0].shape} vs {y[0].shape}"
            assert np.array_equal(x[0], y[0]), f"{what}: instance {i} call {k} differs"
            if x[1] is not None:
                assert np.array_equal(x[1], y[1]), f"{what}: instance {i} call {k} scales differ"


@pytest.fixture(scope="module")
def single_int8(volts):
    log("single plans int8")
    return run_single("int8", volts)


def test_batch_int8_graph_equals_single_plans(volts, single_int8):
    log("batch int8 graph")
    got = run_batch("int8", volts, graph=True)
    emitted = sum(x[0].shape[0] for g in got for x in g)
    assert emitted > 10
    assert_same(got, single_int8, "batch(graph) vs single")


def test_batch_int8_eager_equals_graph_with_work_between(volts, single_int8):
    # graph replays with unrelated eager device work and synchronisations between them
    junk = torch.zeros(1 << 20, device="cuda")

    def between(k):
        junk.add_(1.0)
        torch.cuda.synchronize()

    log("batch int8 eager")
    got = run_batch("int8", volts, graph=False, between=between)
    assert_same(got, single_int8, "batch(eager) vs single")
    log("batch int8 graph, work between replays")
    got = run_batch("int8", volts, graph=True, between=between)
    assert_same(got, single_int8, "batch(graph, eager work between) vs single")


@pytest.mark.parametrize("kc", [128, 1000])
def test_batch_int8_chunked_items_are_exact(volts, single_int8, kc):
    # chunked work items flush with int64 atomics: still bit-exact
    log(f"batch int8 kchunk={kc}")
    got = run_batch("int8", volts, tuning=([kc] * len(SHAPES), 200))
    assert_same(got, single_int8, f"batch kchunk={kc} vs single")


def test_batch_autotune_then_exact(volts, single_int8):
    log("batch int8 autotune")
    got = run_batch("int8", volts, autotune=True)
    assert_same(got, single_int8, "autotuned batch vs single")


@pytest.mark.parametrize("kc", [0, 128])
def test_batch_int8_small_tiles_equal_single_plans(volts, single_int8, kc):
    # 64 x 64 MFMA tiles (one 32 x 32 block per wave), whole-segment and chunked
    # items: the same integer sums as the single plans' 128 x 128 tiles
    log(f"batch int8 tile 64 kchunk={kc}")
    got = run_batch("int8", volts, tuning=([kc] * len(SHAPES), 0), tiles=[64] * len(SHAPES))
    assert_same(got, single_int8, f"batch tile 64 kchunk={kc} vs single")


def test_batch_fp16_small_tiles_equal_single_plans(volts):
    # every 32 x 32 output block runs the same MFMA chain over the same row
    # groups whatever the tile edge, so the FP16 sums are bit-identical too
    shapes = SHAPES[:3]
    ref = run_single("fp16", volts, shapes)
    log("batch fp16 tile 64")
    got = run_batch("fp16", volts, shapes=shapes, tiles=[64] * len(shapes))
    assert_same(got, ref, "fp16 batch tile 64 vs single")


def test_batch_small_tiles_match_oracle_integer_xengine():
    # 128, 200 (ragged against 64) and 6 inputs on 64-edge tiles, chunked
    # items: the oracle's int64 X-engine on the codes the batch wrote
    shapes = [(64, 32, 256), (100, 128, 64), (3, 1024, 8)]
    S = 8192
    vs = [make_volts(20 + i, 2 * t, S) for i, (t, L, T) in enumerate(shapes)]
    with Batch(cfgs("int8", shapes, S)) as b:
        b.set_tuning([3] * len(shapes), 0)
        b.set_tiles([64] * len(shapes))
        b.run(vs)
        for i, p in enumerate(b.plans):
            q = p.read_channelised().cpu().numpy()
            raw, _ = p.integrate_raw(2)
            raw = raw.cpu().numpy()
            L, T = shapes[i][1], shapes[i][2]
            log(f"oracle int check, tile 64, instance {i} n={2 * shapes[i][0]} L={L} T={T}")
            ref = oracle.correlate_i64(q, T)
            assert raw.shape == ref.shape
            assert np.array_equal(raw, ref)


def test_batch_tuning_cache(volts, tmp_path):
    shapes = [SHAPES[3], SHAPES[4]]                # 128 and 10 inputs
    vs = [volts[3], volts[4]]
    cache = tmp_path / "mwax_tuning.txt"
    with Batch(cfgs("int8", shapes)) as b:
        with pytest.raises(mwax.MwaxError) as e:
            b.set_tiles([32, 128])
        assert e.value.status == mwax.MWAX_E_INVAL
        kc, grid = b.autotune([v[:, :CHUNK] for v in vs], trials=1, cache=str(cache))
        tiles = b.tiles()
    lines = cache.read_text().split("\n")
    shape_lines = sorted(l.split() for l in lines if l.startswith("shape "))
    grid_lines = [l.split() for l in lines if l.startswith("grid ")]
    log(f"tuning cache: {shape_lines} {grid_lines}")
    assert len(shape_lines) == 2 and len(grid_lines) == 1
    want = sorted([["shape", shape_lines[0][1], str(2 * t), str(L), str(mwax.X_INT8), str(te), str(k)]
                   for (t, L, T), te, k in zip(shapes, tiles, kc)])
    assert shape_lines == want
    assert int(grid_lines[0][4]) == grid
    # a second batch takes the cached choices without timing anything: plant a
    # choice the tuner would not make and check that it is the one in force
    arch = shape_lines[0][1]
    planted = [f"shape {arch} {2 * t} {L} {mwax.X_INT8} 64 256" for (t, L, T) in shapes]
    cache.write_text("garbage line\n" + "\n".join(planted) + f"\n{' '.join(grid_lines[0][:4])} 100\n")
    outs = [[] for _ in shapes]
    with Batch(cfgs("int8", shapes)) as b:
        kc2, grid2 = b.autotune([v[:, :CHUNK] for v in vs], trials=1, cache=str(cache))
        assert (kc2, grid2, b.tiles()) == ([256, 256], 100, [64, 64])
        for k in range(CALLS):
            b.run([v[:, k * CHUNK:(k + 1) * CHUNK] for v in vs])
            for i, p in enumerate(b.plans):
                outs[i].append(drain(p, "int8"))
        b.sync()
    assert_same(outs, run_single("int8", vs, shapes), "batch on cached tuning vs single")


def test_batch_fp16_equals_single_plans(volts):
    shapes = SHAPES[:3]
    log("single fp16")
    ref = run_single("fp16", volts, shapes)
    log("batch fp16")
    got = run_batch("fp16", volts, shapes=shapes)
    assert_same(got, ref, "fp16 batch vs single")


def test_batch_int8_matches_oracle_integer_xengine():
    # one integration per call: the oracle's int64 X-engine on the codes the batch wrote
    shapes = [(6, 32, 256), (65, 128, 64), (2, 1024, 8)]
    S = 8192
    vs = [make_volts(10 + i, 2 * t, S) for i, (t, L, T) in enumerate(shapes)]
    with Batch(cfgs("int8", shapes, S)) as b:
        b.set_tuning([3] * len(shapes), 0)          # several chunks per segment
        b.run(vs)
        for i, p in enumerate(b.plans):
            q = p.read_channelised().cpu().numpy()
            raw, sc = p.integrate_raw(2)
            raw = raw.cpu().numpy()
            L, T = shapes[i][1], shapes[i][2]
            log(f"oracle int check instance {i} n={2 * shapes[i][0]} L={L} T={T}")
            ref = oracle.correlate_i64(q, T)
            assert raw.shape == ref.shape
            assert np.array_equal(raw, ref)
            assert np.all(sc.cpu().numpy() > 0)


def test_batch_skip_and_errors(volts):
    shapes = SHAPES[:2]
    with Batch(cfgs("int8", shapes)) as b:
        # instance 1 skipped: it stays at stream position 0 and emits nothing
        n0 = n1 = 0
        for k in range(2):
            b.run([volts[0][:, k * CHUNK:(k + 1) * CHUNK], None])
            n0 += b.plans[0].integrate_raw(64)[0].shape[0]
            n1 += b.plans[1].integrate_raw(64)[0].shape[0]
        assert n0 == 2 * CHUNK // (32 * 200) and n1 == 0
        # bad length on one instance: nothing changes anywhere
        with pytest.raises(mwax.MwaxError) as e:
            b.run([volts[0][:, :CHUNK], volts[1][:, :100]])
        assert e.value.status == mwax.MWAX_E_INVAL and "instance 1" in str(e.value)
        # the batch's plans are owned by it
        assert mwax.lib().mwax_plan_destroy(b.plans[0].h) == mwax.MWAX_E_INVAL
        # the autotuner needs fresh instances
        with pytest.raises(mwax.MwaxError) as e:
            b.autotune([v[:, :CHUNK] for v in volts[:2]])
        assert e.value.status == mwax.MWAX_E_STATE
        b.sync()
    with pytest.raises(mwax.MwaxError) as e:
        Batch(cfgs("fp32", shapes))
    assert e.value.status == mwax.MWAX_E_UNSUPPORTED
    with pytest.raises(mwax.MwaxError) as e:
        Batch([make_config(3, L=32, T=200, xprec="int8", max_samples=CHUNK),
               make_config(3, L=32, T=200, xprec="fp16", max_samples=CHUNK)])
    assert e.value.status == mwax.MWAX_E_UNSUPPORTED


def test_batch_slot_exhaustion_is_atomic(volts):
    # T = one call: without mwax_integrate the slots fill; the failing call must
    # leave every instance as it was
    shapes = [(3, 32, 512), (4, 32, 512)]
    with Batch(cfgs("int8", shapes)) as b:
        nslots = b.plans[0].dims.n_slots
        k = 0
        with pytest.raises(mwax.MwaxError) as e:
            for k in range(nslots + 1):
                b.run([volts[0][:, :CHUNK], volts[3][:8, :CHUNK]])
        assert e.value.status == mwax.MWAX_E_STATE
        r0, _ = b.plans[0].integrate_raw(64)
        r1, _ = b.plans[1].integrate_raw(64)
        assert r0.shape[0] == r1.shape[0] == k


def test_batch_int8_whole_segment_partial_at_the_int32_bound():
    """70,000 spectra of +-127 on every input in one whole-segment work item of the
    persistent X-engine: the int32 partial reaches 2 * 127^2 * 65536 = 2.114e9
    (just below 2^31) before its flush, and the int64 sums pass 2^31.  With L = 1
    the transform is the identity and with scale 1 the codes are the samples, so
    the oracle's integer X-engine on the same values is the reference."""
    n_tiles, L, M = 2, 1, 70000
    q = np.full((M, L, 4, 2), 127, np.int8)
    q[:, :, 1, 1] = -127
    q[::3, :, 2, 0] = -127
    volts = torch.from_numpy(np.ascontiguousarray(q[:, 0].transpose(1, 0, 2))).cuda()   # [n][M][2]
    with Batch([make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=L * M)]) as b:
        b.set_tuning([0], 0)                       # whole segments: one item of 4375 row groups
        p = b.plans[0]
        p.set_scales(np.ones(L, np.float32))
        b.run([volts])
        assert np.array_equal(p.read_channelised().cpu().numpy(), q)
        raw, _ = p.integrate_raw(1)
        raw = raw.cpu().numpy()
    ref = oracle.correlate_i64(q, M)
    assert np.abs(ref).max() > 2 ** 31
    assert np.array_equal(raw, ref)


def test_batch_slots_emitted_without_clearing_are_cleared_before_atomic_use():
    """Whole-segment items overwrite a slot with their first flush, so emitting
    does not clear it.  Work that adds atomically into such a slot must find it
    cleared: (a) after switching the batch to chunked items, (b) when a batch
    instance is driven through the single-plan path, whose 128-group segments
    are split into chunks.  Both must equal the plan driven alone."""
    call = 65536                                    # one integration per call, 128 row groups
    shape = [(3, 32, call // 32)]
    with Plan(cfgs("int8", shape, call)[0]) as q:
        nslots = q.dims.n_slots
    ncalls = 2 * nslots + 2
    v = make_volts(20, 6, call * ncalls)
    ref = run_single("int8", [v], shape, call, ncalls)[0]
    for mode in ("retune", "single"):
        got = []
        with Batch(cfgs("int8", shape, call)) as b:
            p = b.plans[0]
            for k in range(ncalls):
                chunk = v[:, k * call:(k + 1) * call]
                if k == nslots and mode == "retune":
                    b.set_tuning([64], 0)           # chunked items from here on
                if k >= nslots and mode == "single":
                    p.channelise(chunk)
                    p.correlate()
                else:
                    b.run([chunk])
                got.append(drain(p, "int8"))
            b.sync()
        log(f"{mode}: {ncalls} integrations, {nslots} slots")
        assert_same([got], [ref], f"batch ({mode}) vs single")


def test_int32_integrators_at_their_bound():
    """Integrations of 65,536 spectra use int32 integrators; with every sample
    at +-127 the autos reach 2 * 127^2 * 65536 = 2.114e9 (just below 2^31).
    The single-plan path (which splits the segment into atomically added
    chunks) and the batch path (whole segments, first flush stores) must both
    equal the oracle's int64 sums bit for bit."""
    n_tiles, L, M = 2, 1, 65536
    q = np.full((M, L, 4, 2), 127, np.int8)
    q[:, :, 1, 1] = -127
    q[1::2, :, 3, 0] = -127
    volts = torch.from_numpy(np.ascontiguousarray(q[:, 0].transpose(1, 0, 2))).cuda()   # [n][M][2]
    cfg = make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=L * M)
    ref = oracle.correlate_i64(q, M)
    assert np.abs(ref).max() == 2 * 127 ** 2 * M
    with Plan(cfg) as p:
        p.set_scales(np.ones(L, np.float32))
        p.channelise(volts)
        p.correlate()
        raw, _ = p.integrate_raw(1)
        assert np.array_equal(raw.cpu().numpy(), ref)
    with Batch([cfg]) as b:
        b.plans[0].set_scales(np.ones(L, np.float32))
        b.run([volts])
        raw, _ = b.plans[0].integrate_raw(1)
        assert np.array_equal(raw.cpu().numpy(), ref)
