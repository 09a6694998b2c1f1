"""GPU parity of the 6,400-point F-engine (Sec. 2.5.1: 5 ms frames of 6,400
samples -> 200 Hz ultra-fine channels) and of the averaging of its visibilities
(Sec. 2.6), against the FP64 oracle (whose mixed-radix FFT is pinned against
the O(L^2) DFT).  Bounds as in test_gpu_parity: FP32 spectra within
2e-6 log2(L) of the rms, int8 codes and binary16 values equal to the oracle's
rounding of its FP64 spectra except next to a rounding boundary, FP32
visibilities within 1e-5 (relative Frobenius per channel), INT8 sums bit-exact
against the integer oracle on the GPU's codes.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_11557_amd import mwax  # noqa: E402
from paper_2303_11557_amd.mwax import Plan, make_config  # noqa: E402

L = 6400


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    mwax.lib()
    yield


def log(msg):
    print(msg, flush=True)


def rel_frob(got, ref):
    return np.linalg.norm(got - ref, axis=-1) / np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)


def test_fft6400_fp32_spectra():
    n_tiles, M = 3, 21                   # 21 frames: ragged against the 4-frame rows
    v = synth.gaussian_volts(2 * n_tiles, L * M, seed=640, sources=[synth.Source(3.0, 77)], L=L)
    with Plan(make_config(n_tiles, L=L, T=M, xprec="fp32", max_samples=L * M)) as p:
        p.channelise(torch.from_numpy(v).cuda())
        got = p.read_channelised().cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    ref = oracle.channelise(v, L)
    assert got.shape == ref.shape == (M, L, 2 * n_tiles)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.max(np.abs(got - ref)) / rms
    log(f"fft6400 fp32: max error {err:.3g} of rms")
    assert err < 2e-6 * math.log2(L)


def test_fft6400_tone_lands_in_closed_form_channel():
    # the quarter-turn tone i^q: exact samples, all power in bin 1600 = channel 4800
    M = 5
    v = synth.tone_volts(4, L * M, L, L // 4, 20, [0, 1, 2, 3])
    with Plan(make_config(2, L=L, T=M, xprec="fp32", max_samples=L * M)) as p:
        p.channelise(torch.from_numpy(v).cuda())
        got = p.read_channelised().cpu().numpy()
    mag = np.abs(got[..., 0] + 1j * got[..., 1])
    assert np.allclose(mag[:, 4800, :], 20 * L, rtol=1e-6)
    assert np.delete(mag, 4800, axis=1).max() < 1e-4 * 20 * L


def test_fft6400_int8_fixed_scales():
    n_tiles, M = 2, 18
    v = synth.gaussian_volts(2 * n_tiles, L * M, seed=641, sources=[synth.Source(3.0, -1234)], L=L)
    ref = oracle.channelise(v, L)
    s = (5.0 * np.sqrt(L * 64.0) / 127.0 * (1.0 + 0.01 * np.arange(L) / L)).astype(np.float32)
    inv = (np.float32(1.0) / s).astype(np.float32)
    with Plan(make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=L * M)) as p:
        p.set_scales(s)
        p.channelise(torch.from_numpy(v).cuda())
        q = p.read_channelised().cpu().numpy().astype(np.int64)
    qo = oracle.requantise(ref, inv).astype(np.int64)
    diff = q != qo
    xs = np.stack([ref.real, ref.imag], -1) * inv[None, :, None, None].astype(np.float64)
    frac = np.abs(np.abs(xs - np.floor(xs)) - 0.5)
    log(f"fft6400 int8: {np.count_nonzero(diff)} of {diff.size} codes differ from the FP64 requantisation")
    assert np.all(np.abs(q - qo)[diff] == 1)
    assert np.all(frac[diff] < 1e-3 * math.log2(L) / 7.0)
    assert diff.mean() <= 1e-4
    assert q.min() >= -127 and q.max() <= 127


def test_fft6400_fp16_rounding():
    n_tiles, M = 2, 10
    v = synth.gaussian_volts(2 * n_tiles, L * M, seed=642)
    ref = oracle.channelise(v, L)
    e = (int(math.ceil(math.log2(L))) + 1) // 2
    with Plan(make_config(n_tiles, L=L, T=M, xprec="fp16", max_samples=L * M)) as p:
        p.channelise(torch.from_numpy(v).cuda())
        h = p.read_channelised().cpu().numpy().astype(np.float64)
    x = np.stack([ref.real, ref.imag], -1) * 2.0 ** -e
    fft_err = 2e-6 * math.log2(L) * np.sqrt(np.mean(np.abs(ref) ** 2)) * 2.0 ** -e
    half_ulp = np.maximum(2.0 ** (np.floor(np.log2(np.maximum(np.abs(h), 2.0 ** -14))) - 11), 2.0 ** -25)
    assert np.all(np.abs(h - x) <= half_ulp * 1.0001 + fft_err)
    want = np.stack([oracle.round_fp16(ref.real, 2.0 ** -e), oracle.round_fp16(ref.imag, 2.0 ** -e)], -1)
    assert (h != want).mean() < 1e-2


def run_plan(v, n_tiles, T, prec, chunks, max_ints=8):
    outs = []
    d = torch.from_numpy(v).cuda()
    with Plan(make_config(n_tiles, L=L, T=T, xprec=prec, max_samples=max(chunks))) as p:
        s0 = 0
        for n in chunks:
            p.channelise(d[:, s0:s0 + n])
            p.correlate()
            s0 += n
            outs.append(p.integrate(max_ints).clone())
        torch.cuda.synchronize()
    return torch.cat(outs).cpu().numpy().astype(np.complex128)


def test_fft6400_fp32_end_to_end_and_fscrunch():
    # 3 tiles, integrations of 12 frames (60 ms), calls crossing them; then the
    # averaging of the paper's three output widths (fscrunch 200, 50, 5)
    n_tiles, T = 3, 12
    S = 2 * T * L
    v = synth.gaussian_volts(2 * n_tiles, S, seed=643, sources=[synth.Source(4.0, 900)], L=L)
    ref = oracle.fx_correlate(v, L, T, threads=8)
    got = run_plan(v, n_tiles, T, "fp32", [5 * L, 14 * L, 5 * L])
    assert got.shape == ref.shape == (2, L, 21)
    err = rel_frob(got, ref)
    log(f"fft6400 fp32 end to end: max per-channel rel-Frobenius {err.max():.3g}")
    assert err.max() <= 1e-5
    d_vis = torch.from_numpy(got.astype(np.complex64)).cuda()
    for F in (200, 50, 5):
        avg = mwax.fscrunch(d_vis, F).cpu().numpy().astype(np.complex128)
        want = oracle.fscrunch(ref, F)
        e = rel_frob(avg, want)
        log(f"fscrunch {F}: {avg.shape[1]} channels, max rel-Frobenius {e.max():.3g}")
        assert avg.shape == (2, L // F, 21) and e.max() <= 1e-5


def test_fft6400_int8_end_to_end():
    # automatic scales from the first 21 frames of each integration; int64 sums
    # bit-exact against the integer oracle on the GPU's codes
    n_tiles, T = 4, 30
    S = T * L
    v = synth.gaussian_volts(2 * n_tiles, S, seed=644, sources=[synth.Source(3.0, -2000)], L=L)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=S)) as p:
        ncal = p.dims.cal_spectra
        assert ncal == 21
        p.channelise(torch.from_numpy(v).cuda())
        q = p.read_channelised().cpu().numpy()
        p.correlate()
        raw, sc = p.integrate_raw(1)
        raw, sc = raw.cpu().numpy(), sc.cpu().numpy()
    assert raw.shape == (1, L, 36, 2)
    assert np.array_equal(raw, oracle.correlate_i64(q, T))
    spec = oracle.channelise(v, L)
    _, s_o, inv_o = oracle.calibrate(spec[:ncal])
    assert np.max(np.abs(sc[0] / s_o - 1)) < 1e-5
    qo = oracle.requantise(spec, inv_o)
    d = q.astype(np.int32) - qo.astype(np.int32)
    assert np.abs(d).max() <= 1 and np.count_nonzero(d) <= 1e-4 * d.size
    # against FP64: the error of the encoding itself (30 spectra leave the
    # requantisation noise of the cross pairs barely averaged), measured on the
    # oracle's own INT8 chain
    ref = oracle.correlate(spec, T)
    got = (raw[..., 0] + 1j * raw[..., 1]) * (sc.astype(np.float64) ** 2)[:, :, None]
    vi = oracle.correlate_i64(qo, T).astype(np.float64)
    v8 = (vi[..., 0] + 1j * vi[..., 1]) * (s_o.astype(np.float64) ** 2)[None, :, None]
    err, e_chain = rel_frob(got, ref), rel_frob(v8, ref)
    log(f"fft6400 int8 end to end: max per-channel rel-Frobenius vs FP64 {err.max():.3g} "
        f"(oracle int8 chain {e_chain.max():.3g})")
    assert err.max() < 1.25 * e_chain.max() + 1e-4
    # against the oracle's INT8 chain: channels whose codes all agree differ only
    # by the scales (<= 1e-5 relative, squared in V); a code one step off at a
    # rounding boundary moves its channel by more, and is allowed above
    same = ~np.any(d != 0, axis=(0, 2, 3))
    assert np.count_nonzero(same) > 0.99 * L
    assert rel_frob(got, v8)[:, same].max() < 3e-5


def test_fft6400_rejected_by_batches():
    with pytest.raises(mwax.MwaxError) as e:
        mwax.Batch([make_config(2, L=L, T=10, xprec="int8", max_samples=10 * L)])
    assert e.value.status == mwax.MWAX_E_UNSUPPORTED


@pytest.mark.parametrize("prec,Lc,F", [("fp32", L, 200), ("fp32", L, 5), ("int8", L, 50), ("int8", 1024, 8),
                                       ("fp16", 256, 4)])
def test_integrate_averaged_equals_averaging_of_the_visibilities(prec, Lc, F):
    # emission with the averaging of Sec. 2.6 in the same pass over the
    # integrators: equal (to one FP32 rounding of an FP64 mean) to the oracle's
    # averaging of the plan's own exact visibilities, with and without weights
    n_tiles = 3
    n = 2 * n_tiles
    T = 12 if Lc == L else 40
    S = 2 * T * Lc
    v = synth.gaussian_volts(n, S, seed=650 + Lc + F, sources=[synth.Source(4.0, Lc // 5)], L=Lc)
    d = torch.from_numpy(v).cuda()
    w = np.full((2, n * (n + 1) // 2), 0.75, np.float32)
    w[:, 3] = 0.0
    cfg = make_config(n_tiles, L=Lc, T=T, xprec=prec, max_samples=S)
    with Plan(cfg) as p:
        p.channelise(d)
        p.correlate()
        if prec == "int8":
            raw, sc = p.integrate_raw(2)
            exact = (raw.cpu().numpy()[..., 0] + 1j * raw.cpu().numpy()[..., 1]) * \
                (sc.cpu().numpy().astype(np.float64) ** 2)[:, :, None]
        else:
            exact = p.integrate(2).cpu().numpy().astype(np.complex128)
    outs = {}
    for weighted in (False, True):
        with Plan(cfg) as p:
            p.channelise(d)
            p.correlate()
            wt = torch.from_numpy(w).cuda() if weighted else None
            outs[weighted] = p.integrate_averaged(F, 2, weights=wt).cpu().numpy().astype(np.complex128)
    want = oracle.fscrunch(exact, F)
    assert outs[False].shape == want.shape == (2, Lc // F, n * (n + 1) // 2)
    if prec == "int8":
        # the exact sums, averaged in FP64 and rounded once to FP32
        assert np.all(np.abs(outs[False] - want) <= 2.0 ** -23 * np.abs(want) + 1e-30)
    else:
        # the plan's FP32 visibilities were rounded once more before the oracle averaged them
        assert np.max(rel_frob(outs[False], want)) < 1e-6
    ww = oracle.apply_weights(want, w.astype(np.float64))
    assert np.max(rel_frob(outs[True], ww)) < 1e-6
    assert np.array_equal(outs[True][:, :, 3], outs[False][:, :, 3])


@pytest.mark.parametrize("prec,Lc,F,n_tiles", [("int8", L, 200, 3), ("int8", L, 50, 40), ("int8", L, 5, 3),
                                               ("fp16", L, 50, 3), ("int8", 1024, 8, 40), ("fp16", 128, 4, 40),
                                               ("int8", 128, 1, 3),
                                               # more than 256 fine channels per output channel: the
                                               # kernel's table of channel weights is reloaded
                                               ("int8", 1024, 512, 3), ("fp16", L, 1280, 3)])
def test_x_engine_averaging_equals_averaging_of_the_visibilities(prec, Lc, F, n_tiles):
    # a plan that averages inside its X-engine (mwax_set_averaging) emits what
    # the oracle's averaging of the same plan's exact visibilities gives, to
    # FP32 accumulation; the block comes in two calls that split an
    # integration, so segments accumulate into the FP64 integrators
    n = 2 * n_tiles
    T = 12 if Lc == L else 40
    S = 3 * T * Lc
    call = S // 2                                 # 1.5 integrations per call
    v = synth.gaussian_volts(n, S, seed=700 + Lc + F + n, sources=[synth.Source(4.0, Lc // 5)], L=Lc)
    d = torch.from_numpy(v).cuda()
    cfg = make_config(n_tiles, L=Lc, T=T, xprec=prec, max_samples=call)
    with Plan(cfg) as p:
        for k in range(2):
            p.channelise(d[:, k * call:(k + 1) * call])
            p.correlate()
        if prec == "int8":
            raw, sc = p.integrate_raw(3)
            exact = (raw.cpu().numpy()[..., 0] + 1j * raw.cpu().numpy()[..., 1]) * \
                (sc.cpu().numpy().astype(np.float64) ** 2)[:, :, None]
        else:
            exact = p.integrate(3).cpu().numpy().astype(np.complex128)
    with Plan(cfg) as p:
        p.set_averaging(F)
        for k in range(2):
            p.channelise(d[:, k * call:(k + 1) * call])
            p.correlate()
        got = p.integrate(3).cpu().numpy().astype(np.complex128)
    want = oracle.fscrunch(exact, F)
    assert got.shape == want.shape == (3, Lc // F, n * (n + 1) // 2)
    err = np.max(rel_frob(got, want))
    log(f"X-engine averaging {prec} L={Lc} F={F} n={n}: max rel. Frobenius {err:.3g}")
    # FP32 sums of up to F + 1 weighted terms, one rounding each
    assert err < max(2e-6, (F + 1) * 2.0 ** -24)
    autos = [a * (a + 1) // 2 + a for a in range(n)]
    assert np.all(np.abs(got[:, :, autos].imag) <= 1e-6 * np.abs(got[:, :, autos].real) + 1e-30)


def test_x_engine_averaging_tile_order_and_errors():
    n_tiles, Lc, T, F = 4, 256, 20, 4
    n = 2 * n_tiles
    S = T * Lc
    v = synth.gaussian_volts(n, S, seed=730, sources=[synth.Source(4.0, 9)], L=Lc)
    d = torch.from_numpy(v).cuda()
    cfg = make_config(n_tiles, L=Lc, T=T, xprec="int8", max_samples=S)
    with Plan(cfg) as p:
        p.set_averaging(F)
        p.channelise(d)
        p.correlate()
        tri = p.integrate(1, order="tri")
    with Plan(cfg) as p:
        p.set_averaging(F)
        p.channelise(d)
        p.correlate()
        tb = p.integrate(1, order="tile_bl").cpu().numpy()
        for call in (lambda: p.integrate_raw(1), lambda: p.integrate_averaged(2, 1)):
            with pytest.raises(mwax.MwaxError) as e:
                call()
            assert e.value.status == mwax.MWAX_E_STATE
        with pytest.raises(mwax.MwaxError) as e:
            p.set_averaging(2)                           # not before the first block
        assert e.value.status == mwax.MWAX_E_STATE
        p.reset()
        with pytest.raises(mwax.MwaxError) as e:
            p.set_averaging(3)                           # 3 does not divide 256
        assert e.value.status == mwax.MWAX_E_INVAL
        p.set_averaging(2)
        assert p.favg == 2
    # the tile-baseline order over L / F channels holds the same numbers
    tri = tri.cpu().numpy()[0]
    for a in range(n_tiles):
        for b in range(a + 1):
            bl = a * (a + 1) // 2 + b
            for p1 in range(2):
                for p2 in range(2):
                    n1, n2 = 2 * a + p1, 2 * b + p2
                    want = tri[:, n1 * (n1 + 1) // 2 + n2] if n1 >= n2 else np.conj(tri[:, n2 * (n2 + 1) // 2 + n1])
                    assert np.array_equal(tb[0, bl, :, 2 * p1 + p2], want)
    with Plan(make_config(2, L=Lc, T=T, xprec="fp32", max_samples=S)) as p:
        with pytest.raises(mwax.MwaxError) as e:
            p.set_averaging(F)
        assert e.value.status == mwax.MWAX_E_UNSUPPORTED
