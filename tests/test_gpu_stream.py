"""GPU tests of the streaming runtime (mwax_stream_*): HBM-budget admission,
ingest from pinned host memory or a device producer, one plan per coarse
channel with integrators kept on the device across blocks, output rings and
block timing.

Parity bar: every integration a stream emits equals, bit for bit, what the same
plan gives when driven alone over the same voltages (same kernels, same
summation order).  Every input is seeded and synthetic.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_11557_amd import mwax  # noqa: E402
from paper_2303_11557_amd.mwax import Plan, Stream, device_view, make_config  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    mwax.lib()
    yield


def log(msg):
    print(msg, flush=True)


N_TILES, L, T = 8, 128, 100          # integration = 12,800 samples
CALL = 6400                          # samples per plan call
BLOCK = 4 * CALL                     # 2 integrations per block
N_CH, N_BLOCKS = 3, 4


def cfg(prec="int8"):
    return make_config(N_TILES, L=L, T=T, xprec=prec, max_samples=CALL)


def host_volts(ch):
    v = synth.gaussian_volts(2 * N_TILES, BLOCK * N_BLOCKS, seed=synth.MWAX_SEED + 4 + ch,
                             sources=[synth.Source(2.0, 9 + ch)], L=L)
    t = torch.from_numpy(np.ascontiguousarray(v)).pin_memory()
    return t


def reference(volts_dev, prec="int8"):
    """The same plan driven alone over the whole stream of one channel."""
    with Plan(cfg(prec)) as p:
        outs = []
        for off in range(0, volts_dev.shape[1], CALL):
            p.channelise(volts_dev[:, off:off + CALL])
            p.correlate()
            outs.append(p.integrate(8).clone())
        torch.cuda.synchronize()
    return torch.cat(outs).cpu().numpy()


def ring_ints(s, ch, n):
    dims = s.plans[ch].dims
    got = []
    for j in range(n):
        ptr = s.vis_ptr(ch, j)
        got.append(device_view(ptr, (dims.fft_len, dims.n_pairs), torch.complex64).clone())
    torch.cuda.synchronize()
    return torch.stack(got).cpu().numpy()


def test_stream_from_pinned_host_equals_single_plans():
    hv = [host_volts(ch) for ch in range(N_CH)]
    budget = 2 * (2 * N_TILES) * BLOCK * 2
    with Stream(cfg(), N_CH, BLOCK, budget, out_depth=N_BLOCKS * 2 + 1) as s:
        assert s.info.pool_slots == 2
        done = []
        for b in range(N_BLOCKS):
            for ch in range(N_CH):
                slot, _ = s.acquire(wait_ms=-1)
                s.copy_in(slot, hv[ch][:, b * BLOCK:(b + 1) * BLOCK])
                s.submit(slot, ch, t_arrival=s.now())
                done += s.poll(0)
        while len(done) < N_BLOCKS * N_CH:
            done += s.poll(-1)
        log(f"{len(done)} blocks; latency p50 {np.median([d['t_ready_s'] - d['t_arrival_s'] for d in done]):.4f} s")
        assert [d["block"] for d in done if d["channel"] == 0] == list(range(N_BLOCKS))
        for d in done:
            assert d["n_ints"] == 2
            assert d["t_ready_s"] >= d["t_submit_s"] - 1e-3 >= d["t_arrival_s"] - 2e-3
        for ch in range(N_CH):
            got = ring_ints(s, ch, 2 * N_BLOCKS)
            ref = reference(hv[ch].cuda())
            assert got.shape == ref.shape
            assert np.array_equal(got, ref), f"channel {ch} differs from the plan driven alone"


def test_stream_admission_by_budget():
    budget = 2 * (2 * N_TILES) * BLOCK * 2 + 12345       # two buffers, not three
    hv = host_volts(0)
    with Stream(cfg(), 1, BLOCK, budget, out_depth=4) as s:
        a, _ = s.acquire(0)
        b, _ = s.acquire(0)
        assert a != b
        with pytest.raises(mwax.MwaxError) as e:
            s.acquire(0)
        assert e.value.status == mwax.MWAX_E_STATE and "budget" in str(e.value)
        s.copy_in(a, hv[:, :BLOCK])
        s.submit(a, 0, s.now())
        with pytest.raises(mwax.MwaxError):
            s.submit(a, 0, s.now())                         # no longer acquired
        c, _ = s.acquire(-1)                                # waits for block 0 to finish
        assert c == a
        recs = s.poll(0)
        assert len(recs) == 1 and recs[0]["slot"] == a and recs[0]["n_ints"] == 2
        with pytest.raises(mwax.MwaxError) as e:
            s.vis_ptr(0, 2)
        assert e.value.status == mwax.MWAX_E_STATE
    with pytest.raises(mwax.MwaxError) as e:
        Stream(cfg(), 1, BLOCK, 1000)
    assert e.value.status == mwax.MWAX_E_INVAL
    with pytest.raises(mwax.MwaxError) as e:
        Stream(cfg(), 1, BLOCK + 100, 1 << 30)
    assert e.value.status == mwax.MWAX_E_INVAL


def test_stream_device_producer_and_fp16():
    # a producer kernel writes the admitted buffer on the ingest stream
    n_in = 2 * N_TILES
    for prec in ("int8", "fp16"):
        with Stream(cfg(prec), 1, BLOCK, 3 * n_in * BLOCK * 2, out_depth=2 * N_BLOCKS) as s:
            for b in range(N_BLOCKS):
                slot, ptr = s.acquire(-1)
                view = device_view(ptr, (n_in, BLOCK, 2), torch.int8)
                synth.device_volts(view, seed=synth.MWAX_SEED + 40, L=L, s0=b * BLOCK,
                                   sources=[synth.Source(3.0, -20)], stream=s.info.ingest_stream)
                s.submit(slot, 0, s.now())
            recs = []
            while len(recs) < N_BLOCKS:
                recs += s.poll(-1)
            got = ring_ints(s, 0, 2 * N_BLOCKS)
        whole = torch.empty((n_in, BLOCK * N_BLOCKS, 2), dtype=torch.int8, device="cuda")
        synth.device_volts(whole, seed=synth.MWAX_SEED + 40, L=L, sources=[synth.Source(3.0, -20)])
        ref = reference(whole, prec)
        log(f"device producer {prec}: {len(recs)} blocks")
        assert np.array_equal(got, ref)


def test_stream_output_ring_back_pressure():
    # A ring of two blocks' integrations: block b overwrites the entries of block
    # b - 2, so its submit is refused until poll has returned block b - 2; block
    # b - 1's visibilities are read after poll returns it, while block b runs on
    # the lane.  Everything read equals the plan driven alone.
    hv = host_volts(0)
    budget = 3 * (2 * N_TILES) * BLOCK * 2
    P = 2 * N_TILES * (2 * N_TILES + 1) // 2
    got = {}
    with Stream(cfg(), 1, BLOCK, budget, out_depth=4) as s:
        seen = []

        def wait_block(k):
            while not any(r["block"] == k for r in seen):
                seen.extend(s.poll(-1))

        def read(j):
            got[j] = device_view(s.vis_ptr(0, j), (L, P), torch.complex64).clone()

        for b in range(N_BLOCKS):
            slot, _ = s.acquire(wait_ms=-1)
            s.copy_in(slot, hv[:, b * BLOCK:(b + 1) * BLOCK])
            if b == 2:
                # block 2 takes the entries of block 0, which poll has not returned
                with pytest.raises(mwax.MwaxError) as e:
                    s.submit(slot, 0, s.now())
                assert e.value.status == mwax.MWAX_E_STATE and "poll" in str(e.value)
                wait_block(0)
                read(0)
                read(1)
                torch.cuda.synchronize()                   # read before block 2 reuses them
            s.submit(slot, 0, s.now())
            if b >= 2:
                wait_block(b - 1)                          # block b may still be running
                read(2 * b - 2)
                read(2 * b - 1)
                torch.cuda.synchronize()
        wait_block(N_BLOCKS - 1)
        read(2 * N_BLOCKS - 2)
        read(2 * N_BLOCKS - 1)
        torch.cuda.synchronize()
        with pytest.raises(mwax.MwaxError) as e:
            s.vis_ptr(0, 2 * N_BLOCKS - 5)                 # overwritten by the last block
        assert e.value.status == mwax.MWAX_E_STATE
    ref = reference(hv.cuda())
    assert sorted(got) == list(range(2 * N_BLOCKS))
    assert np.array_equal(torch.stack([got[j] for j in range(2 * N_BLOCKS)]).cpu().numpy(), ref)
