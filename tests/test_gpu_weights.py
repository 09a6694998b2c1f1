"""GPU parity of the visibility weights (Sec. 4.1) against the FP64 oracle.

The weights kernel counts, per pair and integration, the 50 ms sub-blocks
populated in both inputs and divides by the sub-blocks of the integration in
FP32; the normalisation divides the FP32 visibilities by the FP32 weights.
Both divisions are correctly rounded, so every result lies within half an
FP32 ulp (relative 2^-24) of the oracle's FP64 quotient of the same inputs;
zero weights are exactly 0 and leave the visibilities bit-for-bit unchanged.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_11557_amd import mwax  # noqa: E402
from paper_2303_11557_amd.mwax import Plan, make_config  # noqa: E402

HALF_ULP = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    mwax.lib()
    yield


def log(msg):
    print(msg, flush=True)


def flags_for(n_in, subs, n_ints, p, seed):
    f = synth.zero_flags(n_in, subs * n_ints, p, seed=seed)
    f[0, :subs] = 1                   # input 0 lost its whole first integration
    if n_in > 1:
        f[-1, :] = 0                  # the last input never lost a packet
    return f


@pytest.mark.parametrize("n_in,subs,n_ints,p", [
    (1, 1, 1, 0.5),
    (2, 160, 3, 0.1),
    (130, 40, 2, 0.2),          # ragged 64-input blocks
    (200, 1100, 1, 0.05),       # two LDS passes, ragged last mask word
    (512, 160, 1, 0.01),        # 256 tiles, 8 s integration
    (2048, 160, 1, 0.002),      # largest array
])
def test_vis_weights_parity(n_in, subs, n_ints, p):
    log(f"weights n_in={n_in} subs={subs} n_ints={n_ints}")
    f = flags_for(n_in, subs, n_ints, p, seed=n_in * 7 + subs)
    want = oracle.vis_weights(f, subs)
    got = mwax.vis_weights(torch.from_numpy(f).cuda(), subs)
    torch.cuda.synchronize()
    g = got.cpu().numpy().astype(np.float64)
    assert g.shape == want.shape
    assert np.all(np.abs(g - want) <= HALF_ULP * want)
    assert np.array_equal(g == 0, want == 0)
    assert np.count_nonzero(want == 0) > 0
    if n_in > 1:
        assert np.count_nonzero(want == 1) > 0


def test_vis_weights_zero_integrations():
    out = torch.full((1, 3), 7.0, device="cuda")
    f = torch.zeros((2, 0), dtype=torch.uint8, device="cuda")
    mwax.vis_weights(f, 4, out=out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)


@pytest.mark.parametrize("n_in,L,n_ints", [(1, 1, 1), (3, 5, 3), (130, 7, 2), (512, 128, 1)])
def test_apply_weights_parity(n_in, L, n_ints):
    log(f"apply n_in={n_in} L={L} n_ints={n_ints}")
    P = n_in * (n_in + 1) // 2
    rng = np.random.default_rng(n_in + 31 * L)
    vis = (rng.standard_normal((n_ints, L, P)) * 1e6 + 1j * rng.standard_normal((n_ints, L, P)) * 1e6)
    vis = vis.astype(np.complex64)
    w = oracle.vis_weights(flags_for(n_in, 40, n_ints, 0.3, seed=n_in), 40).astype(np.float32)
    d_vis = torch.from_numpy(vis).cuda()
    mwax.apply_weights(d_vis, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    g = d_vis.cpu().numpy()
    want = oracle.apply_weights(vis.astype(np.complex128), w.astype(np.float64))
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(g).astype(np.float64) - part(want)) <= HALF_ULP * np.abs(part(want)))
    zero = np.broadcast_to((w == 0)[:, None, :], vis.shape)
    assert np.count_nonzero(zero) > 0
    bits = lambda a: a.view(np.uint32).reshape(a.shape + (2,))  # noqa: E731
    assert np.array_equal(bits(g)[zero], bits(vis)[zero])


def test_weights_end_to_end_fp32():
    # voltages with zeroed sub-blocks through the FP32 correlator, then the
    # weights and the normalisation, against the oracle's whole chain
    n_tiles, L, sub_len, subs, J = 8, 16, 64, 10, 3
    n_in = 2 * n_tiles
    T = subs * sub_len // L
    S = J * subs * sub_len
    flags = synth.zero_flags(n_in, J * subs, 0.2, seed=11)
    flags[3, subs:2 * subs] = 1
    v = synth.zero_subblocks(synth.gaussian_volts(n_in, S, seed=synth.MWAX_SEED + 5,
                                                  sources=[synth.Source(3.0, 5)], L=L), flags, sub_len)
    d = torch.from_numpy(v).cuda()
    with Plan(make_config(n_tiles, L=L, T=T, xprec="fp32", max_samples=S)) as p:
        p.channelise(d)
        p.correlate()
        vis = p.integrate(J).clone()
        w = mwax.vis_weights(torch.from_numpy(flags).cuda(), subs)
        mwax.apply_weights(vis, w)
        torch.cuda.synchronize()
    assert vis.shape == (J, L, n_in * (n_in + 1) // 2)
    w_orc = oracle.vis_weights(flags, subs)
    want = oracle.apply_weights(oracle.fx_correlate(v, L, T), w_orc)
    got = vis.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(got - want, axis=-1) / np.linalg.norm(want, axis=-1)
    assert err.max() <= 1e-5
    for j in range(J):
        assert np.all(got[j][:, w_orc[j] == 0] == 0)
    assert np.count_nonzero(w_orc == 0) > 0
    assert np.count_nonzero((w_orc > 0) & (w_orc < 1)) > 0


def test_weights_end_to_end_int8_zeroed_calibration():
    """INT8 with zeroed sub-blocks inside the calibration windows.  Zeroed frames
    are left out of the scale calibration, and a window with none populated
    keeps the previous integration's scales, as the oracle defines; the int64
    sums equal the oracle's integer X-engine on the GPU's codes, the codes agree
    with the oracle's requantisation of its FP64 spectra, few codes clip, and the
    normalised result matches the oracle's chain."""
    n_tiles, L, sub_len, subs, J = 8, 16, 256, 10, 3
    n_in = 2 * n_tiles
    T = subs * sub_len // L                   # 160 spectra: the whole integration calibrates
    S = J * subs * sub_len
    flags = synth.zero_flags(n_in, J * subs, 0.2, seed=12)
    flags[:, subs:2 * subs] = 1               # integration 1: every input zeroed throughout
    flags[:, 2 * subs + 1:3 * subs] = 1       # integration 2: only its first sub-block is live
    v = synth.zero_subblocks(synth.gaussian_volts(n_in, S, seed=synth.MWAX_SEED + 6,
                                                  sources=[synth.Source(3.0, 5)], L=L), flags, sub_len)
    d = torch.from_numpy(v).cuda()
    with Plan(make_config(n_tiles, L=L, T=T, xprec="int8", max_samples=S)) as p:
        ncal = p.dims.cal_spectra
        assert ncal == T
        p.channelise(d)
        q = p.read_channelised().cpu().numpy()
        p.correlate()
        raw, sc = p.integrate_raw(J)
        p.reset()
        p.channelise(d)
        p.correlate()
        vis = p.integrate(J).clone()
        w = mwax.vis_weights(torch.from_numpy(flags).cuda(), subs)
        mwax.apply_weights(vis, w)
        torch.cuda.synchronize()
    raw, sc = raw.cpu().numpy(), sc.cpu().numpy()
    assert raw.shape[0] == J
    assert np.array_equal(raw, oracle.correlate_i64(q, T)), "int64 sums differ from the integer oracle"
    spec = oracle.channelise(v, L)
    prev, s_o, inv_o = None, [], []
    for j in range(J):
        _, s_j, inv_j, pop = oracle.calibrate(spec[j * T:j * T + ncal], prev=prev, return_populated=True)
        assert (pop == 0) == (j == 1)
        prev = (s_j, inv_j)
        s_o.append(s_j)
        inv_o.append(inv_j)
    assert np.array_equal(sc[1], sc[0]), "an empty window must keep the previous scales"
    for j in (0, 2):
        assert np.max(np.abs(sc[j] / s_o[j] - 1)) < 1e-5
    qo = np.concatenate([oracle.requantise(spec[j * T:(j + 1) * T], inv_o[j]) for j in range(J)])
    dq = q.astype(np.int32) - qo.astype(np.int32)
    assert np.abs(dq).max() <= 1 and np.count_nonzero(dq) <= 1e-4 * dq.size
    # integration 2: one live sub-block in ten; with zeroed frames in the mean its
    # sigma would be ~3x low and ~1/3 of the live codes would clip at +-127
    live = np.any(q[2 * T:3 * T] != 0, axis=(1, 3))           # [T][n_in] populated frames
    clipped = np.count_nonzero(np.abs(q[2 * T:3 * T].astype(np.int32)) == 127)
    frac = clipped / max(1, np.count_nonzero(live) * L * 2)
    log(f"int8 zeroed calibration: clip fraction {frac:.3g} over {np.count_nonzero(live)} live frames")
    assert frac < 1e-3
    w_orc = oracle.vis_weights(flags, subs)
    vi = oracle.correlate_i64(qo, T).astype(np.float64)
    v8 = (vi[..., 0] + 1j * vi[..., 1]) * np.stack([s.astype(np.float64) ** 2 for s in s_o])[:, :, None]
    want = oracle.apply_weights(v8, w_orc)
    got = vis.cpu().numpy().astype(np.complex128)
    scale = np.linalg.norm(want, axis=-1, keepdims=True)
    ok = scale[..., 0] > 0
    err = np.linalg.norm(got - want, axis=-1)[ok] / scale[ok][:, 0]
    assert err.max() < 1e-4
    assert np.all(got[1] == 0)


def test_weights_with_frames_straddling_sub_blocks():
    # L = 1024 frames over 1280-sample sub-blocks: frames mix zeroed and live
    # samples.  The weight still counts sub-blocks (it does not depend on L); a
    # pair with w = 0 can then hold nonzero visibilities, which the normalisation
    # leaves as they are.  Input 0 loses the even sub-blocks, input 1 the odd ones.
    n_tiles, L, sub_len, subs = 2, 1024, 1280, 8
    n_in = 2 * n_tiles
    T = subs * sub_len // L
    S = subs * sub_len
    flags = np.zeros((n_in, subs), np.uint8)
    flags[0, 0::2] = 1
    flags[1, 1::2] = 1
    v = synth.zero_subblocks(synth.gaussian_volts(n_in, S, seed=synth.MWAX_SEED + 7), flags, sub_len)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="fp32", max_samples=S)) as p:
        p.channelise(torch.from_numpy(v).cuda())
        p.correlate()
        vis = p.integrate(1).clone()
        before = vis.clone()
        w = mwax.vis_weights(torch.from_numpy(flags).cuda(), subs)
        mwax.apply_weights(vis, w)
        torch.cuda.synchronize()
    w_orc = oracle.vis_weights(flags, subs)
    p01 = 1 * 2 // 2 + 0
    assert w_orc[0, p01] == 0 and w.cpu().numpy()[0, p01] == 0
    ref = oracle.fx_correlate(v, L, T)
    assert np.any(ref[0, :, p01] != 0), "straddling frames correlate although w = 0"
    assert torch.equal(vis[0, :, p01], before[0, :, p01])
    want = oracle.apply_weights(ref, w_orc)
    got = vis.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(got - want, axis=-1) / np.linalg.norm(want, axis=-1)
    assert err.max() <= 1e-5
