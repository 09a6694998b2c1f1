"""GPU parity of the fractional delay and phase correction (Sec. 2.5.1 delay
paragraph, Sec. 4.3) fused into the F-engines, against the FP64 oracle's
correction of its own spectra (pinned by the delay theorem, signed-frequency
tones, the sky-frequency offset and a phased-up point source).

Bounds: FP32 spectra within 3e-6 log2(L) of the rms (the transform's bound of
the uncorrected F-engine plus the FP32 gain evaluation); int8 codes equal to
the oracle's requantisation of its corrected FP64 spectra except next to a
rounding boundary (<= 1e-4 of them, by one step); visibilities of a point
source delayed by tau_n and corrected by -tau_n real to 0.05 rad.
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

NU = synth.NU_C / synth.F_S


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    mwax.lib()
    yield


def log(msg):
    print(msg, flush=True)


def delay_table(n_in, n_steps, seed, scale=0.5):
    """Seeded fractional delays in (-scale, scale) samples, float32 [n_in][n_steps]."""
    u = synth.uniform(np.arange(n_in * n_steps, dtype=np.uint64), seed)
    return ((2.0 * u - 1.0) * scale).astype(np.float32).reshape(n_in, n_steps)


@pytest.mark.parametrize("L,step", [(16, 64), (128, 6400), (512, 1024), (1024, 1024), (6400, 6400)])
def test_delay_fp32_spectra(L, step):
    n_tiles = 2
    M = 12 if L == 6400 else 40
    S = L * M
    n_steps = -(-S // step)
    v = synth.gaussian_volts(2 * n_tiles, S, seed=700 + L, sources=[synth.Source(3.0, L // 8)], L=L)
    dl = delay_table(2 * n_tiles, n_steps, seed=701 + L)
    with Plan(make_config(n_tiles, L=L, T=M, xprec="fp32", max_samples=S)) as p:
        p.set_delays(torch.from_numpy(dl).cuda(), step, synth.NU_C)
        p.channelise(torch.from_numpy(v).cuda())
        got = p.read_channelised().cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    ref = oracle.delay_correct(oracle.channelise(v, L), dl.astype(np.float64), step, NU)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.max(np.abs(got - ref)) / rms
    log(f"delay fp32 L={L} step={step}: max error {err:.3g} of rms")
    assert err < 3e-6 * math.log2(L)
    assert np.max(np.abs(got - oracle.channelise(v, L))) > 1e-2 * rms       # the correction did something


@pytest.mark.parametrize("L", [128, 6400])
def test_delay_int8_codes(L):
    n_tiles = 2
    M = 16 if L == 6400 else 64
    S = L * M
    step = 6400
    v = synth.gaussian_volts(2 * n_tiles, S, seed=710 + L)
    dl = delay_table(2 * n_tiles, -(-S // step), seed=711 + L)
    s = np.full(L, 5.0 * math.sqrt(L * 64.0) / 127.0, np.float32)
    with Plan(make_config(n_tiles, L=L, T=M, xprec="int8", max_samples=S)) as p:
        p.set_scales(s)
        p.set_delays(torch.from_numpy(dl).cuda(), step, synth.NU_C)
        p.channelise(torch.from_numpy(v).cuda())
        q = p.read_channelised().cpu().numpy().astype(np.int64)
    ref = oracle.delay_correct(oracle.channelise(v, L), dl.astype(np.float64), step, NU)
    qo = oracle.requantise(ref, (1.0 / s).astype(np.float32)).astype(np.int64)
    diff = q != qo
    log(f"delay int8 L={L}: {np.count_nonzero(diff)} of {diff.size} codes differ")
    assert np.all(np.abs(q - qo)[diff] == 1)
    assert diff.mean() <= 1e-4


@pytest.mark.parametrize("L,prec", [(128, "int8"), (6400, "fp32"), (6400, "int8")])
def test_delay_point_source_phased_up(L, prec):
    # a point source reaches input n tau_n late (phase -2 pi nu tau_n); applying
    # d_n = -tau_n f_s every 5 ms leaves its visibilities real in the source
    # channel: flat phase after the correction (Sec. 4.3)
    n_tiles, k0, A = 4, (17 if L == 128 else 1234), 3.0
    n_in = 2 * n_tiles
    T = 2000 if L == 128 else 40
    S = L * T
    seed = synth.MWAX_SEED + 9
    v = synth.gaussian_volts(n_in, S, seed=seed, sources=[synth.Source(A, k0)], L=L)
    taus = synth.source_delays(n_in, seed)
    n_steps = -(-S // 6400)
    dl = np.repeat((-taus * synth.F_S).astype(np.float32)[:, None], n_steps, axis=1)
    with Plan(make_config(n_tiles, L=L, T=T, xprec=prec, max_samples=S)) as p:
        p.set_delays(torch.from_numpy(np.ascontiguousarray(dl)).cuda(), 6400, synth.NU_C)
        p.channelise(torch.from_numpy(v).cuda())
        p.correlate()
        vis = p.integrate(1)[0].cpu().numpy().astype(np.complex128)
    c0 = (k0 + L // 2) % L
    sig = T * L * L * A * A
    worst = 0.0
    for a in range(n_in):
        for b in range(a):
            g = vis[c0, a * (a + 1) // 2 + b]
            worst = max(worst, abs(np.angle(g)))
            assert abs(abs(g) / sig - 1) < 0.2
    log(f"delay point source L={L} {prec}: worst phase {worst:.3g} rad after correction")
    assert worst < 0.05


def test_delay_table_follows_the_stream():
    # one table set before two calls: the second call continues at the step its
    # stream position falls in; a call past the table's end is refused
    n_tiles, L, step = 2, 64, 256
    M1, M2 = 20, 28
    S = L * (M1 + M2)
    v = synth.gaussian_volts(2 * n_tiles, S, seed=720)
    dl = delay_table(2 * n_tiles, S // step, seed=721, scale=3.0)
    d = torch.from_numpy(v).cuda()
    tab = torch.from_numpy(dl).cuda()
    got = []
    with Plan(make_config(n_tiles, L=L, T=M1 + M2, xprec="fp32", max_samples=L * M2)) as p:
        p.set_delays(tab, step, 0.0)
        p.channelise(d[:, :L * M1])
        got.append(p.read_channelised().cpu().numpy())
        p.correlate()
        p.channelise(d[:, L * M1:])
        got.append(p.read_channelised().cpu().numpy())
        p.correlate()
        with pytest.raises(mwax.MwaxError) as e:
            p.channelise(d[:, :L])                       # step S // step: past the table
        assert e.value.status == mwax.MWAX_E_INVAL
        with pytest.raises(mwax.MwaxError) as e:
            p.set_delays(tab, 100, 0.0)                  # not a whole number of frames
        assert e.value.status == mwax.MWAX_E_INVAL
    g = np.concatenate(got).astype(np.float64)
    g = g[..., 0] + 1j * g[..., 1]
    ref = oracle.delay_correct(oracle.channelise(v, L), dl.astype(np.float64), step, 0.0)
    assert np.max(np.abs(g - ref)) < 3e-6 * math.log2(L) * np.sqrt(np.mean(np.abs(ref) ** 2))


def test_delay_refused_for_batch_instances():
    with mwax.Batch([make_config(2, L=32, T=10, xprec="int8", max_samples=320)]) as b:
        with pytest.raises(mwax.MwaxError) as e:
            b.plans[0].set_delays(torch.zeros((4, 1), dtype=torch.float32, device="cuda"), 320, 0.0)
        assert e.value.status == mwax.MWAX_E_UNSUPPORTED
