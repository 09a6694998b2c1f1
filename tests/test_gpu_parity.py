"""GPU parity of the HIP hot path against the FP64 oracle, through the C ABI.

Every input is seeded and synthetic; the oracle only ever sees voltages or
channelised data that the seeded generators (or numpy) produced, never values
computed by the HIP path.  Tolerances:
  * integer work (int8 X-engine on given int8 data, exact-integer L <= 4): bit-exact;
  * FP32 path: <= 1e-5 relative Frobenius error per fine channel vs FP64;
  * quantisation decisions (int8 codes, binary16 rounding): equal except where
    the FP64 value lies within the FP32 transform's error of a rounding
    boundary, where either neighbour is valid;
  * FP16 / INT8 end to end: the error envelope derived in the test (stated).
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


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    mwax.lib()
    yield


def log(msg):
    print(msg, flush=True)


def to_np_vis(t):
    return t.cpu().numpy().astype(np.complex128)


def rel_frob(got, ref):
    """per-channel relative Frobenius error, arrays [..., L, P]."""
    num = np.linalg.norm(got - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return num / np.maximum(den, 1e-300)


def dev_volts(volts_np):
    """Copy voltages to the device with rows padded to a multiple of 8 samples
    (the C ABI wants 16-byte aligned rows); returns the [n][S][2] view."""
    n, S = volts_np.shape[:2]
    ld = -(-S // 8) * 8
    d = torch.zeros((n, ld, 2), dtype=torch.int8, device="cuda")
    d[:, :S] = torch.from_numpy(np.ascontiguousarray(volts_np)).cuda()
    return d[:, :S]


def run_fx(volts_np, n_tiles, L, T, prec, chunks=None, scales=None, max_ints=8, order="tri"):
    """Channelise + correlate in the given chunk sizes (samples), emit all integrations."""
    S = volts_np.shape[1]
    chunks = chunks or [S]
    assert sum(chunks) == S
    d = dev_volts(volts_np)
    outs = []
    with Plan(make_config(n_tiles, L=L, T=T, xprec=prec, max_samples=max(chunks))) as p:
        if scales is not None:
            p.set_scales(scales)
        s0 = 0
        for n in chunks:
            p.channelise(d[:, s0:s0 + n])
            p.correlate()
            s0 += n
            outs.append(p.integrate(max_ints, order=order).clone())
        torch.cuda.synchronize()
    return torch.cat(outs)


# ---------------------------------------------------------------------------
# F-engine: spectra, channel order and the transpose
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
def test_fengine_fp32_spectra(L):
    n_tiles = 3
    M = 37                                   # ragged against every row group
    v = synth.gaussian_volts(2 * n_tiles, L * M, seed=100 + L)
    log(f"fengine fp32 L={L}")
    with Plan(make_config(n_tiles, L=L, T=M, xprec="fp32", max_samples=L * M)) as p:
        p.channelise(dev_volts(v))
        got = p.read_channelised().cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    ref = oracle.channelise(v, L)
    assert got.shape == ref.shape
    if L <= 4:
        assert np.array_equal(got, ref), "exact-integer transform must be bit-exact"
    else:
        rms = np.sqrt(np.mean(np.abs(ref) ** 2))
        err = np.max(np.abs(got - ref)) / rms
        assert err < 2e-6 * math.log2(L), f"max error {err:.3g} of rms"


def test_fengine_tone_lands_in_closed_form_channel():
    L, T = 128, 32
    for q in range(4):
        k0 = q * L // 4
        v = synth.tone_volts(4, L * T, L, k0, 50, [0, 1, 2, 3])
        with Plan(make_config(2, L=L, T=T, xprec="fp32", max_samples=L * T)) as p:
            p.channelise(dev_volts(v))
            got = p.read_channelised().cpu().numpy()
        mag = np.abs(got[..., 0] + 1j * got[..., 1])
        c0 = (k0 + L // 2) % L
        assert np.allclose(mag[:, c0, :], 50 * L, rtol=1e-6)
        others = np.delete(mag, c0, axis=1)
        assert others.max() < 1e-3 * 50 * L


@pytest.mark.parametrize("L", [4, 16, 32, 128, 512, 1024])
def test_fengine_int8_requantisation_fixed_scales(L):
    # one case per F-engine decomposition: whole FFT per lane (L <= 16, one or two
    # frames per group) and the two-pass split with 4 .. 32 lanes per FFT
    M, n_tiles = 48, 4
    log(f"fengine int8 requantisation L={L}")
    v = synth.gaussian_volts(2 * n_tiles, L * M, seed=7, sources=[synth.Source(3.0, -37)], L=L)
    ref = oracle.channelise(v, L)
    # oracle-chosen scales: 5 sigma of each channel maps to 127 (slightly varied per channel)
    s = (5.0 * np.sqrt(L * 64.0) / 127.0 * (1.0 + 0.01 * np.arange(L) / L)).astype(np.float32)
    inv = (np.float32(1.0) / s).astype(np.float32)
    with Plan(make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=L * M)) as p:
        p.set_scales(s)
        p.channelise(dev_volts(v))
        q = p.read_channelised().cpu().numpy().astype(np.int64)
    qo = oracle.requantise(ref, inv).astype(np.int64)
    diff = q != qo
    # where they differ: by one step, and the FP64 value sits next to a half-integer
    xs = np.stack([ref.real, ref.imag], -1) * inv[None, :, None, None].astype(np.float64)
    frac = np.abs(np.abs(xs - np.floor(xs)) - 0.5)
    assert np.all(np.abs(q - qo)[diff] == 1)
    # the FP32 transform's error grows like log2(L) (see test_fengine_fp32_spectra)
    tol = 1e-3 * max(1.0, math.log2(L) / 7.0)
    assert np.all(frac[diff] < tol), "a differing code is not at a rounding boundary"
    log(f"fengine int8 L={L}: {np.count_nonzero(diff)} of {diff.size} codes differ from the FP64 requantisation")
    assert diff.mean() <= 1e-4
    assert q.min() >= -127 and q.max() <= 127


@pytest.mark.parametrize("L", [8, 128, 512, 1024])
def test_fengine_fp16_rounding(L):
    M, n_tiles = 40, 4
    log(f"fengine fp16 rounding L={L}")
    v = synth.gaussian_volts(2 * n_tiles, L * M, seed=8)
    ref = oracle.channelise(v, L)
    e = (int(math.log2(L)) + 1) // 2
    with Plan(make_config(n_tiles, L=L, T=M, xprec="fp16", max_samples=L * M)) as p:
        p.channelise(dev_volts(v))
        h = p.read_channelised().cpu().numpy().astype(np.float64)
    want = np.stack([oracle.round_fp16(ref.real, 2.0 ** -e), oracle.round_fp16(ref.imag, 2.0 ** -e)], -1)
    x = np.stack([ref.real, ref.imag], -1) * 2.0 ** -e
    diff = h != want
    # h must be a binary16 neighbour of the FP32 spectrum, which lies within the
    # transform's absolute error of the FP64 value x (the same bound as the FP32 test)
    fft_err = 2e-6 * math.log2(L) * np.sqrt(np.mean(np.abs(ref) ** 2)) * 2.0 ** -e
    half_ulp = np.maximum(2.0 ** (np.floor(np.log2(np.maximum(np.abs(h), 2.0 ** -14))) - 11), 2.0 ** -25)
    assert np.all(np.abs(h - x) <= half_ulp * 1.0001 + fft_err)
    assert diff.mean() < 1e-2


# ---------------------------------------------------------------------------
# X-engine on given channelised data (the X-engine input order of Sec. 2.5.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_tiles,L,M,T", [(1, 4, 40, 40), (3, 8, 53, 21), (17, 2, 70, 35),
                                           (65, 1, 33, 33), (129, 2, 20, 20), (64, 4, 100, 37)])
def test_xengine_int8_bit_exact(n_tiles, L, M, T):
    n = 2 * n_tiles
    rng = np.random.default_rng(n + L + M)
    q = rng.integers(-127, 128, size=(M, L, n, 2)).astype(np.int8)
    q[:, :, 0, :] = 127                       # extremes on one input
    q[:, :, -1, :] = -127
    log(f"xengine int8 n={n} L={L} M={M} T={T}")
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=L * M)) as p:
        p.load_channelised(torch.from_numpy(q).cuda())
        p.correlate()
        raw, sc = p.integrate_raw(M // T + 1)
        raw = raw.cpu().numpy()
    ref = oracle.correlate_i64(q, T)
    assert raw.shape == ref.shape
    assert np.array_equal(raw, ref)
    assert np.all(sc.cpu().numpy() == 1.0)


def test_xengine_int8_steady_state_512_inputs():
    # 256 tiles x 2 pols, 2 channels, 8192 spectra = 512 row groups per tile: the
    # launch splits every tile into K-chunks of 64 groups (well past the loop's
    # steady state), flushed with int32 atomic adds; every tile, wave and
    # fragment position is compared, element by element
    n_tiles, L, M = 256, 2, 8192
    n = 2 * n_tiles
    rng = np.random.default_rng(2024)
    q = rng.integers(-127, 128, size=(M, L, n, 2)).astype(np.int8)
    q[:, :, 5, :] = 127
    q[:, :, 300, :] = -127
    log(f"xengine int8 steady state n={n} L={L} M={M}")
    with Plan(make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=L * M)) as p:
        p.load_channelised(torch.from_numpy(q).cuda())
        p.correlate()
        raw, _ = p.integrate_raw(1)
        raw = raw.cpu().numpy()
    ref = oracle.correlate_i64(q, M)
    assert raw.shape == ref.shape
    bad = np.argwhere(raw != ref)
    assert bad.size == 0, f"{len(bad)} entries differ, first at {bad[:4].tolist()}"


def test_xengine_int8_many_spectra_exceed_int32():
    # 70,000 spectra of +-127 on every input: sums pass 2^31 (int32 -> int64 flushes)
    n_tiles, L, M = 2, 1, 70000
    q = np.full((M, L, 4, 2), 127, np.int8)
    q[:, :, 1, 1] = -127
    q[::3, :, 2, 0] = -127
    with Plan(make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=L * M)) as p:
        p.load_channelised(torch.from_numpy(q).cuda())
        p.correlate()
        raw, _ = p.integrate_raw(1)
    ref = oracle.correlate_i64(q, M)
    assert np.abs(ref).max() > 2 ** 31
    assert np.array_equal(raw.cpu().numpy(), ref)


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
@pytest.mark.parametrize("n_tiles,L,M,T", [(3, 8, 45, 15), (70, 2, 24, 24), (130, 1, 17, 17)])
def test_xengine_float_vs_fp64(prec, n_tiles, L, M, T):
    n = 2 * n_tiles
    rng = np.random.default_rng(n * 3 + L)
    x = rng.normal(size=(M, L, n, 2)) * 100.0
    x = x.astype(np.float16).astype(np.float64)        # exactly representable in both
    dt = torch.float16 if prec == "fp16" else torch.float32
    with Plan(make_config(n_tiles, L=L, T=T, xprec=prec, max_samples=L * M)) as p:
        # loaded binary16 data are taken as spectra * 2^-e; output is scaled back by 2^2e
        p.load_channelised(torch.from_numpy(x).to(dt).cuda())
        p.correlate()
        vis = to_np_vis(p.integrate(M // T))
    spec = x[..., 0] + 1j * x[..., 1]
    ref = oracle.correlate(spec, T)
    if prec == "fp16":
        e = (int(math.log2(L)) + 1) // 2 if L > 1 else 0
        ref = ref * 2.0 ** (2 * e)
    err = rel_frob(vis, ref)
    assert err.max() < 2e-6, err.max()


# ---------------------------------------------------------------------------
# Whole path
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 4])
def test_exact_integer_lengths_fp32_and_int8(L):
    # twiddles are +-1, +-i: FP32 results are exact integers (< 2^24 per partial)
    n_tiles, T = 5, 24
    rng = np.random.default_rng(L)
    v = rng.integers(-20, 21, size=(2 * n_tiles, L * T * 2, 2)).astype(np.int8)
    ref = oracle.fx_correlate(v, L, T)
    got = to_np_vis(run_fx(v, n_tiles, L, T, "fp32"))
    assert np.array_equal(got, ref)
    # int8 with s_c = 1: codes equal the exact spectra, sums are exact
    d = dev_volts(v)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=L * T * 2)) as p:
        p.set_scales(np.ones(L, np.float32))
        p.channelise(d)
        p.correlate()
        raw, _ = p.integrate_raw(2)
    q = np.stack([oracle.channelise(v, L).real, oracle.channelise(v, L).imag], -1)
    assert np.abs(q).max() <= 127
    assert np.array_equal(raw.cpu().numpy(), oracle.correlate_i64(q.astype(np.int8), T))


def test_16_tiles_plain_fp32_full():
    """16 tiles x 2 pols, 128,000 samples, L = 128, one integration."""
    n_tiles, L, T = 16, 128, 1000
    v = synth.gaussian_volts(32, L * T, sigma=8.0, seed=synth.MWAX_SEED)
    ref = oracle.fx_correlate(v, L, T, threads=8)
    got = to_np_vis(run_fx(v, n_tiles, L, T, "fp32"))
    err = rel_frob(got, ref)
    log(f"16 tiles fp32 max per-channel rel-Frobenius {err.max():.3g}")
    assert got.shape == (1, L, 32 * 33 // 2)
    assert err.max() <= 1e-5
    # autos real (imaginary part at FP32 rounding level) and positive
    autos = got[0][:, [n * (n + 1) // 2 + n for n in range(32)]]
    assert np.all(autos.real > 0)
    assert np.max(np.abs(autos.imag) / autos.real) < 1e-6


def test_tile_baseline_order():
    n_tiles, L, T = 6, 32, 40
    v = synth.gaussian_volts(12, L * T, seed=3)
    ref = oracle.pack_tilebl(oracle.fx_correlate(v, L, T)[0], n_tiles)
    got = to_np_vis(run_fx(v, n_tiles, L, T, "fp32", order="tile_bl"))[0]
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_tile_baseline_order_int8():
    """INT8 integrators hold Im V minus a row term that the pack step removes
    with the autos (see pack.hip); the tile-baseline view reads entries of both
    triangles' orientations, so it must equal the oracle's tile-baseline packing
    of the oracle's integer X-engine on the GPU's codes, to FP32 output rounding."""
    n_tiles, L, T = 6, 32, 40
    v = synth.gaussian_volts(12, L * T, seed=5, sources=[synth.Source(3.0, 7)], L=L)
    s = np.full(L, 0.25, np.float32)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=L * T)) as p:
        p.set_scales(s)
        p.channelise(dev_volts(v))
        q = p.read_channelised().cpu().numpy()
        p.correlate()
        got = to_np_vis(p.integrate(1, order="tile_bl"))[0]
    vi = oracle.correlate_i64(q, T)[0].astype(np.float64)
    ref = oracle.pack_tilebl((vi[..., 0] + 1j * vi[..., 1]) * 0.0625, n_tiles)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))
    assert np.any(ref.imag != 0)


def test_chunking_and_integration_boundaries():
    # integrations of T = 37 spectra, calls of uneven sizes crossing boundaries
    n_tiles, L, T = 5, 16, 37
    S = L * T * 4
    v = synth.gaussian_volts(10, S, seed=11)
    ref = oracle.fx_correlate(v, L, T)
    chunks = [L * 5, L * 50, L * 3, L * 70, S - L * 128]
    for prec, tol in (("fp32", 1e-5),):
        got = to_np_vis(run_fx(v, n_tiles, L, T, prec, chunks=chunks))
        assert got.shape == ref.shape
        assert rel_frob(got, ref).max() <= tol
    # int8 with fixed scales: chunking cannot change a single bit
    s = np.full(L, 5.0 * math.sqrt(L * 64.0) / 127.0, np.float32)
    a = run_fx(v, n_tiles, L, T, "int8", scales=s).cpu().numpy()
    b = run_fx(v, n_tiles, L, T, "int8", chunks=chunks, scales=s).cpu().numpy()
    assert np.array_equal(a, b)


def test_int8_auto_scales_and_error_envelope():
    n_tiles, L, T = 8, 128, 800
    v = synth.gaussian_volts(16, L * T, seed=21, sources=[synth.Source(4.0, 41)], L=L)
    spec = oracle.channelise(v, L)
    ref = oracle.correlate(spec, T)
    d = dev_volts(v)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=L * T)) as p:
        ncal = p.dims.cal_spectra
        p.channelise(d)
        p.correlate()
        raw, sc = p.integrate_raw(1)
        p.reset()
        p.channelise(d)
        p.correlate()
        vis = to_np_vis(p.integrate(1))
    _, s_orc, inv_orc = oracle.calibrate(spec[:ncal])
    sc = sc.cpu().numpy()[0]
    assert np.max(np.abs(sc / s_orc - 1)) < 1e-5
    # output = V_int * s^2 exactly as documented
    raw = raw.cpu().numpy()[0]
    want = ((raw[..., 0].astype(np.float64) * sc.astype(np.float64)[:, None] * sc.astype(np.float64)[:, None])
            .astype(np.float32))
    assert np.array_equal(vis[0].real.astype(np.float32), want)
    # error envelope vs FP64: quantisation noise of step s = 5 sigma / 127 is s^2/12
    # per component against sigma^2, a relative 1.3e-4 bias on the autos
    err = rel_frob(vis, ref)
    log(f"int8 e2e max per-channel rel-Frobenius vs FP64 {err.max():.3g}")
    assert err.max() < 3e-3
    # the oracle's own int chain (its own scales) agrees closely
    q_orc = oracle.requantise(spec, inv_orc)
    v_orc = oracle.correlate_i64(q_orc, T)[0].astype(np.float64)
    v_orc = (v_orc[..., 0] + 1j * v_orc[..., 1]) * (s_orc.astype(np.float64) ** 2)[:, None]
    assert rel_frob(vis[0], v_orc).max() < 1e-4


def test_get_scales():
    # the scales of the most recently begun integration, read without emitting it
    n_tiles, L, T = 3, 32, 40
    v = synth.gaussian_volts(2 * n_tiles, L * T * 2, seed=31)
    d = dev_volts(v)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=L * T)) as p:
        with pytest.raises(mwax.MwaxError) as e:
            p.get_scales()
        assert e.value.status == mwax.MWAX_E_STATE
        p.channelise(d[:, :L * T])
        s0 = p.get_scales().clone()
        p.correlate()
        p.channelise(d[:, L * T:])
        s1 = p.get_scales().clone()
        p.correlate()
        _, sc = p.integrate_raw(2)
        torch.cuda.synchronize()
        assert torch.equal(sc[0], s0) and torch.equal(sc[1], s1)
        assert not torch.equal(s0, s1)
        p.set_scales(np.full(L, 0.5, np.float32))
        p.channelise(d[:, :L * T])
        assert bool(torch.all(p.get_scales() == 0.5))
        p.correlate()
        p.reset()
        with pytest.raises(mwax.MwaxError) as e:
            p.get_scales()
        assert e.value.status == mwax.MWAX_E_STATE
    spec = oracle.channelise(v, L)
    for j, s in enumerate((s0, s1)):
        _, s_o, _ = oracle.calibrate(spec[j * T:j * T + min(T, -(-131072 // L))])
        assert np.max(np.abs(s.cpu().numpy() / s_o - 1)) < 1e-5
    with Plan(make_config(n_tiles, L=L, T=T, xprec="fp16", max_samples=L * T)) as p:
        with pytest.raises(mwax.MwaxError) as e:
            p.get_scales()
        assert e.value.status == mwax.MWAX_E_UNSUPPORTED


def test_point_source_phase_on_gpu():
    n_tiles, L, T, A, k0 = 8, 128, 2000, 2.0, 17
    seed = synth.MWAX_SEED + 1
    v = synth.gaussian_volts(16, L * T, seed=seed, sources=[synth.Source(A, k0)], L=L)
    got = to_np_vis(run_fx(v, n_tiles, L, T, "int8"))
    taus = synth.source_delays(16, seed)
    nu = synth.NU_C + k0 * synth.F_S / L
    c0 = (k0 + L // 2) % L
    vv = L * 2 * (64 + 1 / 12)
    sig = T * L * L * A * A
    rms = math.sqrt(T * (vv * vv + 2 * vv * L * L * A * A))
    for a in range(16):
        for b in range(a):
            want = sig * np.exp(-2j * np.pi * nu * (taus[a] - taus[b]))
            assert abs(got[0, c0, a * (a + 1) // 2 + b] - want) < 6 * rms


def test_determinism():
    n_tiles, L, T = 20, 64, 64
    v = synth.gaussian_volts(40, L * T, seed=5)
    for prec in ("fp32", "fp16", "int8"):
        a = run_fx(v, n_tiles, L, T, prec).cpu().numpy()
        b = run_fx(v, n_tiles, L, T, prec).cpu().numpy()
        assert a.tobytes() == b.tobytes(), prec


def test_state_machine_errors():
    with Plan(make_config(2, L=16, T=10, xprec="int8", max_samples=16 * 10)) as p:
        d = torch.zeros((4, 16 * 10, 2), dtype=torch.int8, device="cuda")
        with pytest.raises(mwax.MwaxError) as e:
            p.correlate()
        assert e.value.status == mwax.MWAX_E_STATE
        with pytest.raises(mwax.MwaxError) as e:
            p.channelise(d, n_samples=15)
        assert e.value.status == mwax.MWAX_E_INVAL
        p.channelise(d)
        with pytest.raises(mwax.MwaxError) as e:
            p.channelise(d)
        assert e.value.status == mwax.MWAX_E_STATE
        with pytest.raises(mwax.MwaxError) as e:
            p.set_scales(np.ones(16, np.float32))
        assert e.value.status == mwax.MWAX_E_STATE
        p.correlate()
        # fill every slot with completed integrations, then one more must be refused
        slots = p.dims.n_slots
        for _ in range(slots - 1):
            p.channelise(d)
            p.correlate()
        with pytest.raises(mwax.MwaxError) as e:
            p.channelise(d)
        assert e.value.status == mwax.MWAX_E_STATE
        out = p.integrate(100)
        assert out.shape[0] == slots
        assert torch.count_nonzero(out) == 0
    with Plan(make_config(2, L=16, T=10, xprec="fp32", max_samples=160)) as p:
        with pytest.raises(mwax.MwaxError) as e:
            p.integrate_raw(1)
        assert e.value.status == mwax.MWAX_E_UNSUPPORTED


# ---------------------------------------------------------------------------
# Full-size configurations: sampled outputs and invariants
# ---------------------------------------------------------------------------
def sampled_check(vis, volts_dev, inputs, L, T, j, tol_fn):
    v = volts_dev[inputs].cpu().numpy()
    spec = oracle.channelise(v, L, m0=j * T, nm=T)
    ref = oracle.correlate(spec, T, threads=8)[0]        # [L][p(sel)]
    n = len(inputs)
    worst = 0.0
    for a in range(n):
        for b in range(a + 1):
            n1, n2 = inputs[a], inputs[b]
            if n1 < n2:
                n1, n2 = n2, n1
                r = np.conj(ref[:, a * (a + 1) // 2 + b])
            else:
                r = ref[:, a * (a + 1) // 2 + b]
            g = vis[:, n1 * (n1 + 1) // 2 + n2]
            scale = np.sqrt(np.abs(ref[:, a * (a + 1) // 2 + a].real) * np.abs(ref[:, b * (b + 1) // 2 + b].real))
            worst = max(worst, float(np.max(np.abs(g - r) / scale)))
    assert worst < tol_fn, worst
    return worst


def test_128_tiles_plain_fp32_sampled():
    """128 tiles, 1.28 M samples (1 s), one point source, 0.5 s integrations."""
    n_tiles, L, T, S = 128, 128, 5000, 1_280_000
    n = 2 * n_tiles
    d = torch.empty((n, S, 2), dtype=torch.int8, device="cuda")
    seed = synth.MWAX_SEED + 1
    synth.device_volts(d, seed=seed, sources=[synth.Source(2.0, 17)], L=L)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="fp32", max_samples=S)) as p:
        p.channelise(d)
        p.correlate()
        vis = p.integrate(2)
        torch.cuda.synchronize()
    assert vis.shape == (2, L, n * (n + 1) // 2)
    inputs = [0, 1, 2, 77, 128, 200, 254, 255]
    for j in range(2):
        w = sampled_check(to_np_vis(vis[j]), d, inputs, L, T, j, 1e-5)
        log(f"128 tiles fp32 integration {j}: worst sampled error {w:.3g} (of sqrt(auto1 auto2))")
    # closed-form phase of the source in channel c0 on the sampled pairs
    taus = synth.source_delays(n, seed)
    nu = synth.NU_C + 17 * synth.F_S / L
    c0 = (17 + L // 2) % L
    g = to_np_vis(vis[0][c0])
    ph_err = []
    for a in inputs:
        for b in inputs:
            if a > b:
                ph = np.angle(g[a * (a + 1) // 2 + b] * np.exp(2j * np.pi * nu * (taus[a] - taus[b])))
                ph_err.append(abs(ph))
    assert max(ph_err) < 0.1        # expected phase noise ~0.011 rad


# Sampled inputs of the 256-tile tests: both inputs of the first and last
# tiles, and inputs in the upper column half (64..127) of every 128-row tile,
# so that sampled pairs of off-diagonal tiles reach both column halves.
FULL_INPUTS = [0, 1, 2, 3, 100, 130, 200, 257, 330, 400, 460, 510, 511]


@pytest.mark.parametrize("prec,tol", [("int8", 2e-3), ("fp16", 5e-4), ("fp32", 1e-5)])
def test_channel_precision_full_size_sampled(prec, tol):
    """256 tiles, 8 s (10.24 M samples), three sources, one 8 s integration.
    INT8 (80,000 spectra: int64 integrators, two K-chunks per tile flushed with
    int64 atomic adds, a flush at 65,536 spectra): the int64 sums at the sampled
    pairs equal the oracle's integer X-engine on the GPU's own codes, bit for
    bit; every precision is within its bound of FP64."""
    n_tiles, L, S = 256, 128, 10_240_000
    T = S // L
    n = 2 * n_tiles
    log(f"256 tiles {prec}: generating 10.5 GB of voltages")
    d = torch.empty((n, S, 2), dtype=torch.int8, device="cuda")
    srcs = [synth.Source(2.0, -37), synth.Source(3.0, 5), synth.Source(4.0, 41)]
    synth.device_volts(d, seed=synth.MWAX_SEED + 2, sources=srcs, L=L)
    inputs = FULL_INPUTS
    cols = [max(a, b) * (max(a, b) + 1) // 2 + min(a, b) for ai, a in enumerate(inputs) for b in inputs[:ai + 1]]
    autos_idx = torch.tensor([k * (k + 1) // 2 + k for k in range(n)], device="cuda")
    with Plan(make_config(n_tiles, L=L, T=T, xprec=prec, max_samples=S)) as p:
        p.channelise(d)
        if prec == "int8":
            sel = torch.tensor(inputs, device="cuda")
            codes = p.read_channelised().index_select(2, sel).cpu().numpy()     # [T][L][k][2]
            p.correlate()
            raw, sc = p.integrate_raw(1)
            torch.cuda.synchronize()
            assert raw.shape == (1, L, n * (n + 1) // 2, 2)
            auto_raw = raw[0][:, autos_idx]
            assert bool(torch.all(auto_raw[..., 0] > 0)) and bool(torch.all(auto_raw[..., 1] == 0))
            raw_s = raw[0].index_select(1, torch.tensor(cols, device="cuda")).cpu().numpy()
            s2 = sc[0].cpu().numpy().astype(np.float64) ** 2
            del raw
        else:
            p.correlate()
            vis = p.integrate(1)
            torch.cuda.synchronize()
    log(f"256 tiles {prec}: correlated")
    if prec == "int8":
        want = oracle.correlate_i64(codes, T)[0]
        bad = np.argwhere(raw_s != want)
        assert bad.size == 0, f"{len(bad)} sampled int64 sums differ, first at {bad[:4].tolist()}"
        log(f"256 tiles int8: {raw_s.shape[1]} sampled pairs x {L} channels bit-exact against the integer oracle")
        # the sampled visibilities V = V_int s^2 against FP64
        got = np.zeros((L, n * (n + 1) // 2), np.complex128)
        got[:, cols] = (raw_s[..., 0] + 1j * raw_s[..., 1]) * s2[:, None]
    else:
        assert vis.shape == (1, L, n * (n + 1) // 2)
        v0 = vis[0]
        autos = v0[:, autos_idx]
        assert bool(torch.all(autos.real > 0))
        got = to_np_vis(v0)
        del vis
    w = sampled_check(got, d, inputs, L, T, 0, tol)
    log(f"256 tiles {prec}: worst sampled error {w:.3g} (bound {tol})")
    del d
    torch.cuda.empty_cache()
