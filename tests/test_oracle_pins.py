"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here touches the GPU or the HIP library.  Each pin is chosen so that a
plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a missing fftshift) fails at least one of them; the
``test_pins_catch_*`` tests plant such slips in copies of the oracle's output
and check that the pins notice.

Paper: Morrison et al. 2023, "MWAX: A New Correlator for the MWA".
"""
import cmath
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rng(seed=1):
    return np.random.default_rng(seed)


def rand_volts(n, S, seed=1, amp=127):
    v = rng(seed).integers(-amp, amp + 1, size=(n, S, 2))
    return v.astype(np.int8)


# ---------------------------------------------------------------------------
# Pin checks, written as functions so the mutation tests can reuse them.
# ---------------------------------------------------------------------------
def brute_force_vis(volts, L, T):
    """Definition written out in pure Python (Sec. 2.5.1 F step, Sec. 2.5.2 X step).

    Returns full matrices V[j][c][n1][n2] as nested lists of Python complex.
    """
    n_in, S = volts.shape[0], volts.shape[1]
    M = S // L
    X = [[[0j] * L for _ in range(M)] for _ in range(n_in)]
    for n in range(n_in):
        for m in range(M):
            for k in range(L):
                acc = 0j
                for q in range(L):
                    x = complex(int(volts[n, m * L + q, 0]), int(volts[n, m * L + q, 1]))
                    acc += x * cmath.exp(-2j * math.pi * k * q / L)
                X[n][m][(k + L // 2) % L] = acc
    n_int = M // T
    V = [[[[0j] * n_in for _ in range(n_in)] for _ in range(L)] for _ in range(n_int)]
    for j in range(n_int):
        for c in range(L):
            for a in range(n_in):
                for b in range(n_in):
                    V[j][c][a][b] = sum(X[a][m][c] * X[b][m][c].conjugate()
                                        for m in range(j * T, (j + 1) * T))
    return V


def check_brute_force(vis_packed, V, tol):
    n_int, L, P = vis_packed.shape
    n_in = len(V[0][0])
    for j in range(n_int):
        for c in range(L):
            for a in range(n_in):
                for b in range(a + 1):
                    got = vis_packed[j, c, a * (a + 1) // 2 + b]
                    want = V[j][c][a][b]
                    if abs(got - want) > tol * max(1.0, abs(want)):
                        return False
    return True


def tone_channel_ok(vis, L, k0, T, amp, phases):
    """P4: all power in c0 = (k0 + L/2) mod L with V = T L^2 A^2 i^(p1 - p2)."""
    c0 = (k0 + L // 2) % L
    n_in = len(phases)
    peak = T * L * L * amp * amp
    for c in range(L):
        for a in range(n_in):
            for b in range(a + 1):
                got = vis[0, c, a * (a + 1) // 2 + b]
                want = peak * (1j ** ((phases[a] - phases[b]) % 4)) if c == c0 else 0
                if abs(got - want) > 1e-9 * peak:
                    return False
    return True


def point_source_ok(vis, c0, taus, nu, T, L, amp, sigma2_c):
    """P5: E V[c0][n1,n2] = T L^2 A^2 exp(-2 pi i nu (tau1 - tau2)) within 6 sigma."""
    n_in = len(taus)
    v = L * sigma2_c
    s = T * L * L * amp * amp
    rms = math.sqrt(T * (v * v + 2 * v * L * L * amp * amp))
    for a in range(n_in):
        for b in range(a):
            want = s * cmath.exp(-2j * math.pi * nu * (taus[a] - taus[b]))
            got = vis[0, c0, a * (a + 1) // 2 + b]
            if abs(got - want) > 6 * rms:
                return False
    return True


# ---------------------------------------------------------------------------
# DFT / FFT pins
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 4, 8, 16, 64])
def test_dft_closed_forms(orc, L):
    # delta at q0 -> X[k] = exp(-2 pi i k q0 / L)
    for q0 in range(L):
        x = np.zeros(L, complex)
        x[q0] = 1
        X = orc.dft(x)
        want = np.array([cmath.exp(-2j * math.pi * k * q0 / L) for k in range(L)])
        assert np.max(np.abs(X - want)) < 1e-12
    # constant -> L at DC only
    X = orc.dft(np.full(L, 3 - 2j))
    want = np.zeros(L, complex)
    want[0] = L * (3 - 2j)
    assert np.max(np.abs(X - want)) < 1e-12 * L
    # positive-frequency tone exp(+2 pi i k0 q / L) -> L at bin k0 (forward sign)
    k0 = L // 4 if L >= 4 else 0
    x = np.array([cmath.exp(2j * math.pi * k0 * q / L) for q in range(L)])
    X = orc.dft(x)
    want = np.zeros(L, complex)
    want[k0] = L
    assert np.max(np.abs(X - want)) < 1e-11 * L


@pytest.mark.parametrize("L", [1, 2, 4, 8, 16, 32, 64])
def test_fft_matches_dft(orc, L):
    x = rng(L).normal(size=L) + 1j * rng(L + 100).normal(size=L)
    assert np.max(np.abs(orc.fft(x) - orc.dft(x))) < 1e-12 * L


@pytest.mark.parametrize("L", [2, 32, 128, 1024, 4096])
def test_fft_matches_numpy(orc, L):
    # numpy.fft.fft uses the same forward sign and no normalisation.
    x = rng(L).normal(size=L) * 50 + 1j * rng(L + 1).normal(size=L) * 50
    X = orc.fft(x)
    ref = np.fft.fft(x)
    assert np.max(np.abs(X - ref)) < 1e-12 * np.max(np.abs(ref)) * math.log2(L)


@pytest.mark.parametrize("L", [3, 5, 6, 10, 20, 25, 50, 100, 400, 1000])
def test_fft_mixed_radix_matches_dft(orc, L):
    # lengths with prime factors 2, 3 and 5 take the mixed-radix path
    x = rng(L).normal(size=L) * 30 + 1j * rng(L + 7).normal(size=L) * 30
    ref = orc.dft(x)
    assert np.max(np.abs(orc.fft(x) - ref)) < 1e-12 * np.max(np.abs(ref)) * math.log2(L) * 4


def test_fft_6400_matches_numpy_and_parseval(orc):
    # the F-engine length of Sec. 2.5.1: 6,400 points (2^8 5^2), 200 Hz channels
    L = 6400
    x = rng(64).normal(size=L) * 50 + 1j * rng(65).normal(size=L) * 50
    X = orc.fft(x)
    ref = np.fft.fft(x)
    assert np.max(np.abs(X - ref)) < 1e-12 * np.max(np.abs(ref)) * math.log2(L)
    assert np.sum(np.abs(X) ** 2) == pytest.approx(L * np.sum(np.abs(x) ** 2), rel=1e-12)


@pytest.mark.parametrize("k0", [1600, 1, 3199, 4813])
def test_fft_6400_tone(orc, k0):
    # exp(+2 pi i k0 q / L) puts L at bin k0 and nothing elsewhere; k0 = L/4 is
    # the quarter-turn tone i^q, whose samples are exact
    L = 6400
    q = np.arange(L)
    x = np.exp(2j * np.pi * ((k0 * q) % L) / L) if k0 != L // 4 else 1j ** (q % 4)
    X = orc.fft(x)
    want = np.zeros(L, complex)
    want[k0] = L
    assert np.max(np.abs(X - want)) < 1e-9 * L


def test_channelise_6400_against_dft(orc):
    # two frames of two inputs by the O(L^2) definition; the tone bin k0 = 1600
    # lands in channel (1600 + 3200) mod 6400 = 4800
    L = 6400
    v = rand_volts(2, 2 * L, seed=64)
    a = orc.channelise(v, L)
    b = orc.channelise(v, L, use_dft=True)
    assert np.max(np.abs(a - b)) < 1e-9 * np.max(np.abs(b))
    t = synth.tone_volts(1, L, L, L // 4, 20, [0])
    mag = np.abs(orc.channelise(t, L)[0, :, 0])
    assert int(np.argmax(mag)) == 4800 and mag.max() == pytest.approx(20 * L)
    assert np.sort(mag)[-2] < 1e-6


# ---------------------------------------------------------------------------
# Channel order: centre-symmetric channels with DC at c = L/2 (Sec. 2.6)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [4, 8, 128])
def test_channel_order(orc, L):
    # a DC (constant) input lands in the centre channel
    v = np.zeros((1, 2 * L, 2), np.int8)
    v[0, :, 0] = 5
    spec = orc.channelise(v, L)
    assert np.count_nonzero(np.abs(spec) > 1e-9) == 2
    assert np.allclose(spec[:, L // 2, 0], 5 * L)
    # an exact tone at bin k0 = L/4 lands in channel (k0 + L/2) mod L = 3L/4
    v = synth.tone_volts(1, 2 * L, L, L // 4, 10, [0])
    spec = orc.channelise(v, L)
    mag = np.abs(spec[0, :, 0])
    assert int(np.argmax(mag)) == (L // 4 + L // 2) % L
    assert mag.max() == pytest.approx(10 * L)


def test_channelise_dft_and_fft_agree(orc):
    v = rand_volts(3, 16 * 5, seed=7)
    a = orc.channelise(v, 16)
    b = orc.channelise(v, 16, use_dft=True)
    assert np.max(np.abs(a - b)) < 1e-10


def test_channelise_subsets(orc):
    v = rand_volts(5, 64 * 6, seed=3)
    full = orc.channelise(v, 64)
    part = orc.channelise(v, 64, inputs=[4, 1], m0=2, nm=3)
    assert np.array_equal(part[:, :, 0], full[2:5, :, 4])
    assert np.array_equal(part[:, :, 1], full[2:5, :, 1])


# ---------------------------------------------------------------------------
# P1 brute force on 2-4 inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_in,L,M,T", [(2, 4, 3, 3), (3, 8, 4, 2), (4, 2, 6, 3), (2, 1, 5, 5)])
def test_brute_force_small(orc, n_in, L, M, T):
    v = rand_volts(n_in, L * M, seed=n_in * 10 + L)
    vis = orc.fx_correlate(v, L, T)
    V = brute_force_vis(v, L, T)
    assert vis.shape == (M // T, L, n_in * (n_in + 1) // 2)
    assert check_brute_force(vis, V, 1e-9)


# ---------------------------------------------------------------------------
# P2 exact-integer special cases L in {1, 2, 4}
# ---------------------------------------------------------------------------
def _exact_vis(volts, L, T):
    """Gaussian-integer arithmetic: exp(-2 pi i k q / L) = (-i)^(4kq/L) for L | 4."""
    powers = [(1, 0), (0, -1), (-1, 0), (0, 1)]          # (-i)^0..3
    n_in, S = volts.shape[0], volts.shape[1]
    M = S // L
    X = np.zeros((n_in, M, L, 2), dtype=object)
    for n in range(n_in):
        for m in range(M):
            for k in range(L):
                re = im = 0
                for q in range(L):
                    a, b = int(volts[n, m * L + q, 0]), int(volts[n, m * L + q, 1])
                    wr, wi = powers[(4 * k * q // L) % 4]
                    re += a * wr - b * wi
                    im += a * wi + b * wr
                X[n, m, (k + L // 2) % L] = (re, im)
    out = np.zeros((M // T, L, n_in * (n_in + 1) // 2, 2), dtype=object)
    for j in range(M // T):
        for c in range(L):
            for a in range(n_in):
                for b in range(a + 1):
                    sr = si = 0
                    for m in range(j * T, (j + 1) * T):
                        r1, i1 = X[a, m, c]
                        r2, i2 = X[b, m, c]
                        sr += r1 * r2 + i1 * i2
                        si += i1 * r2 - r1 * i2
                    out[j, c, a * (a + 1) // 2 + b] = (sr, si)
    return out


@pytest.mark.parametrize("L", [1, 2, 4])
def test_exact_integer_cases(orc, L):
    v = rand_volts(4, L * 12, seed=L)
    vis = orc.fx_correlate(v, L, 6)
    ex = _exact_vis(v, L, 6)
    assert np.array_equal(vis.real, ex[..., 0].astype(np.float64))
    assert np.array_equal(vis.imag, ex[..., 1].astype(np.float64))


def test_L1_is_textbook_outer_product(orc):
    # L = 1: no transform, V = sum_m x x^H (a ZHERK), checked with numpy matmul.
    v = rand_volts(6, 40, seed=11)
    vis = orc.fx_correlate(v, 1, 40)
    x = v[..., 0].astype(np.float64) + 1j * v[..., 1]
    full = x @ x.conj().T
    tri = np.array([full[a, b] for a in range(6) for b in range(a + 1)])
    assert np.array_equal(vis[0, 0], tri)


# ---------------------------------------------------------------------------
# P3 Parseval, P6 Hermitian/auto invariants, numpy matmul cross-check
# ---------------------------------------------------------------------------
def test_parseval(orc):
    L, T = 128, 20
    v = rand_volts(6, L * T * 2, seed=5)
    vis = orc.fx_correlate(v, L, T)
    for j in range(2):
        for n in range(6):
            lhs = vis[j, :, n * (n + 1) // 2 + n].real.sum()
            seg = v[n, j * T * L:(j + 1) * T * L].astype(np.int64)
            rhs = L * int((seg ** 2).sum())
            assert abs(lhs - rhs) <= 1e-12 * rhs


def test_hermitian_and_autos(orc):
    L, T = 16, 8
    v = rand_volts(5, L * T, seed=9)
    spec = orc.channelise(v, L)
    full = orc.correlate_full(spec, T)
    packed = orc.correlate(spec, T)
    n = 5
    for a in range(n):
        # bitwise conjugate symmetry (same summation order)
        for b in range(n):
            assert full[0, :, b, a].real.tobytes() == full[0, :, a, b].real.tobytes()
            assert np.array_equal(full[0, :, b, a].imag, -full[0, :, a, b].imag)
        assert np.all(full[0, :, a, a].imag == 0)
        assert np.all(full[0, :, a, a].real >= 0)
        for b in range(a + 1):
            assert np.array_equal(packed[0, :, a * (a + 1) // 2 + b], full[0, :, a, b])


def test_correlate_matches_numpy_matmul(orc):
    L, T, n = 32, 10, 7
    v = rand_volts(n, L * T, seed=12)
    spec = orc.channelise(v, L)
    vis = orc.correlate(spec, T, threads=3)
    for c in range(L):
        X = spec[:, c, :].T                  # [n][T]
        full = X @ X.conj().T
        tri = np.array([full[a, b] for a in range(n) for b in range(a + 1)])
        assert np.max(np.abs(vis[0, c] - tri)) <= 1e-10 * np.max(np.abs(tri))


def test_threads_do_not_change_results(orc):
    L, T, n = 64, 6, 6
    v = rand_volts(n, L * T * 2, seed=13)
    spec = orc.channelise(v, L)
    assert np.array_equal(orc.correlate(spec, T, 1), orc.correlate(spec, T, 5))


# ---------------------------------------------------------------------------
# P4 closed-form tones (the method of Sec. 3.1: phase-rotated tones)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [4, 32, 128])
@pytest.mark.parametrize("quarter", [0, 1, 2, 3])
def test_tone_closed_form(orc, L, quarter):
    k0 = quarter * L // 4
    phases = [0, 1, 2, 3, 1, 0]
    T = 7
    v = synth.tone_volts(6, L * T, L, k0, 11, phases)
    vis = orc.fx_correlate(v, L, T)
    assert tone_channel_ok(vis, L, k0, T, 11, phases)


# ---------------------------------------------------------------------------
# P5 point source with seeded delays: closed-form visibility phase
# ---------------------------------------------------------------------------
def test_point_source_phase(orc):
    L, T, n, A, k0 = 128, 2000, 8, 2.0, 17
    seed = synth.MWAX_SEED + 1
    v = synth.gaussian_volts(n, L * T, sigma=8.0, seed=seed, sources=[synth.Source(A, k0)], L=L)
    vis = orc.fx_correlate(v, L, T, threads=4)
    taus = synth.source_delays(n, seed)
    nu = synth.NU_C + k0 * synth.F_S / L
    c0 = (k0 + L // 2) % L
    assert point_source_ok(vis, c0, taus, nu, T, L, A, 2 * (64 + 1 / 12))


# ---------------------------------------------------------------------------
# P7 noise statistics of rounded Gaussian voltages (sigma = 8)
# ---------------------------------------------------------------------------
def test_noise_statistics(orc):
    L, T, n = 128, 400, 6
    v = synth.gaussian_volts(n, L * T, sigma=8.0, seed=synth.MWAX_SEED)
    vis = orc.fx_correlate(v, L, T, threads=4)
    var_c = 2 * (64 + 1 / 12)             # per complex sample, incl. rounding noise
    vX = L * var_c
    autos = np.array([vis[0, :, a * (a + 1) // 2 + a].real for a in range(n)])
    ratio = autos.mean() / (vX * T)
    assert abs(ratio - 1) < 5 / math.sqrt(T * L * n)
    cross = np.concatenate([vis[0, :, a * (a + 1) // 2 + b] for a in range(n) for b in range(a)])
    z = np.concatenate([cross.real, cross.imag]) / (vX * math.sqrt(T / 2))
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs((z ** 2).mean() - 1) < 5 * math.sqrt(2 / z.size)


# ---------------------------------------------------------------------------
# int64 X step, requantiser, calibration, fp16 rounding, tile-baseline view
# ---------------------------------------------------------------------------
def test_correlate_i64_brute(orc):
    q = rng(3).integers(-127, 128, size=(9, 4, 3, 2)).astype(np.int8)
    vis = orc.correlate_i64(q, 3)
    for j in range(3):
        for c in range(4):
            for a in range(3):
                for b in range(a + 1):
                    sr = si = 0
                    for m in range(3 * j, 3 * j + 3):
                        r1, i1 = int(q[m, c, a, 0]), int(q[m, c, a, 1])
                        r2, i2 = int(q[m, c, b, 0]), int(q[m, c, b, 1])
                        sr += r1 * r2 + i1 * i2
                        si += i1 * r2 - r1 * i2
                    assert tuple(vis[j, c, a * (a + 1) // 2 + b]) == (sr, si)


def test_correlate_i64_exceeds_int32(orc):
    M = 100_000
    q = np.empty((M, 1, 2, 2), np.int8)
    q[:, 0, 0] = (127, -127)
    q[:, 0, 1] = (-127, 127)
    vis = orc.correlate_i64(q, M)
    assert tuple(vis[0, 0, 0]) == (2 * 127 * 127 * M, 0)
    # x0 conj(x1) with x0 = 127(1 - i), x1 = -127(1 - i): re = -2*127^2, im = 0
    assert tuple(vis[0, 0, 1]) == (-2 * 127 * 127 * M, 0)
    assert tuple(vis[0, 0, 2]) == (2 * 127 * 127 * M, 0)
    assert vis.max() > 2 ** 31


def test_requantise_rule(orc):
    vals = np.array([2.5, 3.5, -2.5, -3.5, 0.5, -0.5, 1.49999, 126.6, 127.5, 300.0, -300.0,
                     -127.5, -128.0, 0.0], np.float64)
    spec = (vals + 1j * vals[::-1]).reshape(1, 1, -1)
    q = orc.requantise(spec, np.array([1.0], np.float32))
    expect_re = np.clip(np.rint(vals), -127, 127)           # numpy rint: ties to even
    expect_im = np.clip(np.rint(vals[::-1]), -127, 127)
    assert np.array_equal(q[0, 0, :, 0], expect_re.astype(np.int8))
    assert np.array_equal(q[0, 0, :, 1], expect_im.astype(np.int8))
    assert q.min() == -127
    # per-channel scale applies per channel
    spec = np.array([[[10 + 10j], [10 + 10j]]])
    q = orc.requantise(spec, np.array([0.5, 0.25], np.float32))
    assert q[0, 0, 0].tolist() == [5, 5] and q[0, 1, 0].tolist() == [2, 2]   # 2.5 -> 2


def test_calibrate_rule(orc):
    spec = np.zeros((3, 2, 4), complex)
    spec[:, 0, :] = 3 + 4j          # |x|^2 / 2 = 12.5 everywhere
    sig2, s, inv = orc.calibrate(spec)
    assert sig2[0] == 12.5 and sig2[1] == 0.0
    assert s[0] == np.float32(5 * math.sqrt(12.5) / 127)
    assert inv[0] == np.float32(127 / (5 * math.sqrt(12.5)))
    assert s[1] == 1.0 and inv[1] == 1.0


def test_calibrate_white_noise(orc):
    L = 64
    v = synth.gaussian_volts(8, L * 200, sigma=8.0, seed=42)
    sig2, _, _ = orc.calibrate(orc.channelise(v, L))
    # E|X|^2 = L * 2 * 64.083, so sigma^2 per component = L * 64.083
    assert abs(sig2.mean() / (L * (64 + 1 / 12)) - 1) < 0.02


def test_calibrate_leaves_out_zeroed_frames(orc):
    # Frames of zeroed samples (Sec. 2.4: lost packets are zeroed) have all-zero
    # spectra; interleaving such frames with the populated ones must leave the
    # scales bit-for-bit as they were (the sums keep their order, the count its
    # value).  Dividing by every frame instead would halve sigma^2 here.
    L, n = 16, 6
    v = synth.gaussian_volts(n, L * 40, sigma=8.0, seed=77)
    a = orc.channelise(v, L)
    b = np.zeros((2 * a.shape[0],) + a.shape[1:], complex)
    b[0::2] = a
    sa, s_a, i_a, pa = orc.calibrate(a, return_populated=True)
    sb, s_b, i_b, pb = orc.calibrate(b, return_populated=True)
    assert pa == pb == 40 * n
    assert np.array_equal(sa, sb) and np.array_equal(s_a, s_b) and np.array_equal(i_a, i_b)
    # zero some whole frames of single inputs: only those drop out of the count
    z = synth.zero_subblocks(v, np.eye(n, 4, dtype=np.uint8) * 1, 10 * L)  # input k loses frames 10k..10k+9
    _, _, _, pz = orc.calibrate(orc.channelise(z, L), return_populated=True)
    assert pz == 40 * n - 4 * 10
    # a frame with a single nonzero sample counts as populated
    w = np.zeros((1, 2 * L, 2), np.int8)
    w[0, 3] = (1, 0)
    _, _, _, pw = orc.calibrate(orc.channelise(w, L), return_populated=True)
    assert pw == 1


def test_calibrate_empty_window_keeps_previous_scales(orc):
    spec = np.zeros((5, 8, 3), complex)
    prev = (np.arange(1, 9, dtype=np.float32), 1 / np.arange(1, 9, dtype=np.float32))
    sig2, s, inv, pop = orc.calibrate(spec, prev=prev, return_populated=True)
    assert pop == 0 and np.all(sig2 == 0)
    assert np.array_equal(s, prev[0]) and np.array_equal(inv, prev[1])
    _, s1, i1 = orc.calibrate(spec)            # no previous integration: unit scales
    assert np.all(s1 == 1) and np.all(i1 == 1)


def test_round_fp16_matches_numpy(orc):
    r = rng(21)
    x = np.concatenate([
        r.normal(size=2000) * 1000, r.normal(size=500) * 1e-5, r.normal(size=200) * 6e4,
        np.array([0.0, -0.0, 65504.0, 65519.9, 65520.0, -70000.0, 2.0 ** -24, 2.0 ** -25,
                  3 * 2.0 ** -26, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 2049.0, 2051.0]),
    ])
    y = orc.round_fp16(x)
    ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(y, ref)
    assert np.array_equal(orc.round_fp16(x, 0.25), (x * 0.25).astype(np.float16).astype(np.float64))


def test_pack_tilebl(orc):
    n_tiles, L = 3, 2
    n = 2 * n_tiles
    P = n * (n + 1) // 2
    vis = (np.arange(L * P) + 1j * (1000 + np.arange(L * P))).reshape(L, P)
    out = orc.pack_tilebl(vis, n_tiles)
    assert out.shape == (6, L, 4)

    def V(c, r, s):
        return vis[c, r * (r + 1) // 2 + s] if r >= s else np.conj(vis[c, s * (s + 1) // 2 + r])

    for a in range(n_tiles):
        for b in range(a + 1):
            bl = a * (a + 1) // 2 + b
            for c in range(L):
                assert out[bl, c, 0] == V(c, 2 * a, 2 * b)          # XX
                assert out[bl, c, 1] == V(c, 2 * a, 2 * b + 1)      # XY
                assert out[bl, c, 2] == V(c, 2 * a + 1, 2 * b)      # YX
                assert out[bl, c, 3] == V(c, 2 * a + 1, 2 * b + 1)  # YY
    # auto-tile XY is the conjugate of YX
    assert out[0, 0, 1] == np.conj(out[0, 0, 2])


# ---------------------------------------------------------------------------
# The pins notice planted mistakes
# ---------------------------------------------------------------------------
def test_pins_catch_conjugation_error(orc):
    L, T, n, A, k0 = 128, 2000, 6, 2.0, 17
    seed = synth.MWAX_SEED + 1
    v = synth.gaussian_volts(n, L * T, seed=seed, sources=[synth.Source(A, k0)], L=L)
    vis = orc.fx_correlate(v, L, T, threads=4)
    taus = synth.source_delays(n, seed)
    nu = synth.NU_C + k0 * synth.F_S / L
    c0 = (k0 + L // 2) % L
    args = (c0, taus, nu, T, L, A, 2 * (64 + 1 / 12))
    assert point_source_ok(vis, *args)
    assert not point_source_ok(np.conj(vis), *args)          # x1* x2 instead of x1 x2*


def test_pins_catch_missing_fftshift_and_wrong_sign(orc):
    L, T = 32, 5
    phases = [0, 1, 3]
    v = synth.tone_volts(3, L * T, L, L // 4, 9, phases)
    vis = orc.fx_correlate(v, L, T)
    assert tone_channel_ok(vis, L, L // 4, T, 9, phases)
    assert not tone_channel_ok(np.roll(vis, L // 2, axis=1), L, L // 4, T, 9, phases)
    # inverse-sign transform puts the tone at -k0: channel mirrored about DC
    mirrored = np.concatenate([vis[:, :1], vis[:, :0:-1]], axis=1)
    assert not tone_channel_ok(mirrored, L, L // 4, T, 9, phases)


def test_pins_catch_dropped_term(orc):
    n_in, L, M, T = 3, 4, 4, 2
    v = rand_volts(n_in, L * M, seed=77)
    vis = orc.fx_correlate(v, L, T)
    V = brute_force_vis(v, L, T)
    assert check_brute_force(vis, V, 1e-9)
    # drop the i1*i2 term of the real part (equivalent: keep only r1 r2)
    spec = orc.channelise(v, L)
    bad = np.zeros_like(vis)
    for j in range(M // T):
        for a in range(n_in):
            for b in range(a + 1):
                s = spec[j * T:(j + 1) * T]
                bad[j, :, a * (a + 1) // 2 + b] = (
                    (s[:, :, a].real * s[:, :, b].real).sum(0)
                    + 1j * (s[:, :, a].imag * s[:, :, b].real - s[:, :, a].real * s[:, :, b].imag).sum(0))
    assert not check_brute_force(bad, V, 1e-9)
    # transposed operand (x2 x1*) breaks the brute-force comparison as well
    assert not check_brute_force(np.conj(vis), V, 1e-9)


# ---------------------------------------------------------------------------
# Visibility weights (Sec. 4.1; zeroing flags of Sec. 2.4): per pair and
# integration, the fraction of 50 ms sub-blocks populated in both inputs
# ---------------------------------------------------------------------------
def nested_losses(z, S, J):
    """Input n loses the first z[n] sub-blocks of each of J integrations."""
    flags = np.zeros((len(z), J * S), np.uint8)
    for n, zn in enumerate(z):
        for j in range(J):
            flags[n, j * S: j * S + zn] = 1
    return flags


def nested_weights_ok(w, z, S):
    """A pair keeps the sub-blocks after the later of its two losses."""
    for j in range(w.shape[0]):
        for a in range(len(z)):
            for b in range(a + 1):
                if w[j, a * (a + 1) // 2 + b] != (S - max(z[a], z[b])) / S:
                    return False
    return True


def test_weights_nested_losses_closed_form(orc):
    z, S = [0, 1, 5, 5, 7, 12, 19, 20, 3], 20
    w = orc.vis_weights(nested_losses(z, S, 3), S)
    assert w.shape == (3, 45)
    assert nested_weights_ok(w, z, S)


def test_weights_single_losses(orc):
    # input n loses only sub-block n: cross pairs keep S - 2, autos S - 1
    n, S = 7, 11
    flags = np.zeros((n, S), np.uint8)
    flags[np.arange(n), np.arange(n)] = 1
    w = orc.vis_weights(flags, S)[0]
    for a in range(n):
        for b in range(a + 1):
            assert w[a * (a + 1) // 2 + b] == ((S - 1) / S if a == b else (S - 2) / S)


def test_weights_are_the_gram_matrix_of_the_populated_masks(orc):
    # counting sub-blocks populated in both inputs is the product A A^T of the
    # 0/1 populated matrix with itself (numpy matmul, exact on small integers)
    n, S, J = 13, 37, 4
    flags = synth.zero_flags(n, J * S, 0.2, seed=5)
    w = orc.vis_weights(flags, S)
    r, c = np.tril_indices(n)
    order = np.argsort(r * (r + 1) // 2 + c)
    for j in range(J):
        A = (flags[:, j * S:(j + 1) * S] == 0).astype(np.float64)
        G = A @ A.T
        assert np.array_equal(w[j], G[r[order], c[order]] / S)


def test_weights_from_the_samples_themselves(orc):
    # the weight is the fraction of the integration's samples present in both
    # signal paths: counted sample by sample on a zeroed tone (whose samples are
    # never 0 unless zeroed)
    n, L, sub_len, S_int, J = 4, 8, 16, 5, 2
    flags = synth.zero_flags(n, J * S_int, 0.35, seed=9)
    v = synth.zero_subblocks(synth.tone_volts(n, J * S_int * sub_len, L, L // 4, 7, [0, 1, 2, 3]),
                             flags, sub_len)
    w = orc.vis_weights(flags, S_int)
    present = np.any(v != 0, axis=2)
    span = S_int * sub_len
    for j in range(J):
        for a in range(n):
            for b in range(a + 1):
                both = sum(1 for s in range(j * span, (j + 1) * span) if present[a, s] and present[b, s])
                assert w[j, a * (a + 1) // 2 + b] == both / span


def test_normalised_tone_recovers_the_unflagged_closed_form(orc):
    # P4 tone with zeroed sub-blocks (whole spectra each): before normalisation
    # V[c0] = w T L^2 A^2 i^(p1 - p2); after it, the closed form of the
    # unflagged tone; pairs without a common sub-block stay 0
    n, L, sub_len, S_int, J, amp = 5, 8, 16, 5, 2, 11
    phases = [0, 3, 1, 2, 1]
    T = S_int * sub_len // L
    flags = synth.zero_flags(n, J * S_int, 0.3, seed=4)
    flags[2, :S_int] = 1                           # input 2 lost the whole first integration
    v = synth.zero_subblocks(synth.tone_volts(n, J * S_int * sub_len, L, L // 4, amp, phases),
                             flags, sub_len)
    vis = orc.fx_correlate(v, L, T)
    w = orc.vis_weights(flags, S_int)
    normed = orc.apply_weights(vis, w)
    c0 = (L // 4 + L // 2) % L
    peak = T * L * L * amp * amp
    assert np.count_nonzero(w == 0) > 0 and np.count_nonzero((w > 0) & (w < 1)) > 0
    for j in range(J):
        for a in range(n):
            for b in range(a + 1):
                p = a * (a + 1) // 2 + b
                want = peak * (1j ** ((phases[a] - phases[b]) % 4))
                assert abs(vis[j, c0, p] - w[j, p] * want) <= 1e-9 * peak
                if w[j, p] > 0:
                    assert abs(normed[j, c0, p] - want) <= 1e-9 * peak
                else:
                    assert normed[j, c0, p] == 0
                others = np.delete(normed[j, :, p], c0)
                assert np.all(np.abs(others) <= 1e-9 * peak)


def test_weight_pins_catch_planted_slips(orc):
    # slips planted in copies of the oracle's weights: counting sub-blocks
    # lost in both inputs, populated in either, or in the first input only;
    # dividing by the sub-blocks of the whole flag row
    z, S, J = [0, 1, 5, 5, 7, 12, 19, 20, 3], 20, 2
    flags = nested_losses(z, S, J)
    good = orc.vis_weights(flags, S)
    assert nested_weights_ok(good, z, S)
    n = len(z)
    lost_both = np.zeros_like(good)
    either = np.zeros_like(good)
    first = np.zeros_like(good)
    for j in range(J):
        f = flags[:, j * S:(j + 1) * S].astype(bool)
        for a in range(n):
            for b in range(a + 1):
                p = a * (a + 1) // 2 + b
                lost_both[j, p] = np.sum(f[a] & f[b]) / S
                either[j, p] = np.sum(~f[a] | ~f[b]) / S
                first[j, p] = np.sum(~f[a]) / S
    for bad in (lost_both, either, first, good * S / (J * S)):
        assert not nested_weights_ok(bad, z, S)


def test_apply_weights_divides_only_where_weighted(orc):
    vis = np.array([[[2 + 4j, -3 + 1j, 0j]]])
    w = np.array([[0.5, 0.0, 0.25]])
    out = orc.apply_weights(vis, w)
    assert out[0, 0, 0] == 4 + 8j and out[0, 0, 1] == -3 + 1j and out[0, 0, 2] == 0


# ---------------------------------------------------------------------------
# Channel averaging (Sec. 2.6): centre-symmetric output channels of F fine
# channels, half-weight shared boundaries for even F, DC left out of the centre
# ---------------------------------------------------------------------------
AVG_CASES = [(16, 1), (16, 2), (16, 4), (16, 16), (20, 5), (30, 3), (32, 8), (12, 6)]


def band_weights(L, F):
    """weights[o][c] from the band edges in frequency: output channel o spans
    offsets (o - N/2) F +- F/2 from DC (in fine channels, modulo the coarse
    bandwidth L); a fine channel strictly inside counts 1, one centred on an
    edge 1/2 (both halves when the band spans the whole coarse channel, F = L,
    and its two edges meet at +-f_s/2), the DC channel 0 in the centre output
    channel."""
    N, oc = L // F, (L // F) // 2
    w = np.zeros((N, L))
    for o in range(N):
        for c in range(L):
            delta = ((c - L // 2 - (o - oc) * F + L // 2) % L) - L // 2
            for x in (delta - L, delta, delta + L):
                if F == 1:
                    w[o, c] += 1.0 if x == 0 else 0.0
                elif 2 * abs(x) < F:
                    w[o, c] += 1.0
                elif 2 * abs(x) == F:
                    w[o, c] += 0.5
            if F > 1 and o == oc and c == L // 2:
                w[o, c] = 0.0
    return w


def averaging_ok(out, vis, L, F):
    w = band_weights(L, F)
    want = np.einsum("oc,jcp->jop", w, vis) / w.sum(axis=1)[None, :, None]
    return np.allclose(out, want, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("L,F", AVG_CASES)
def test_averaging_matches_the_band_edges(orc, L, F):
    r = rng(L * 31 + F)
    vis = r.standard_normal((2, L, 6)) + 1j * r.standard_normal((2, L, 6))
    assert averaging_ok(orc.fscrunch(vis, F), vis, L, F)


@pytest.mark.parametrize("L,F", AVG_CASES)
def test_averaging_keeps_a_flat_spectrum(orc, L, F):
    vis = np.full((1, L, 3), 5.0 - 2.0j)
    assert np.allclose(orc.fscrunch(vis, F), 5.0 - 2.0j, rtol=1e-15, atol=0)


@pytest.mark.parametrize("L,F", [(c[0], c[1]) for c in AVG_CASES if c[1] > 1])
def test_averaging_counts_every_frequency_once_except_dc(orc, L, F):
    # Sec. 2.6: every frequency contributes equally to the total power; the
    # per-channel weights (F, or F - 1 at the centre) undo the means
    r = rng(L + F)
    vis = r.standard_normal((1, L, 10)) + 1j * r.standard_normal((1, L, 10))
    out = orc.fscrunch(vis, F)
    N = L // F
    W = np.full(N, float(F))
    W[N // 2] = F - 1
    total = np.einsum("o,jop->jp", W, out)
    assert np.allclose(total, vis.sum(axis=1) - vis[:, L // 2], rtol=1e-13, atol=1e-12)


def test_averaging_boundary_response_is_3db_down(orc):
    # even F: a signal in the fine channel on a boundary between two output
    # channels lands at half weight in each (Sec. 2.6: 3 dB at the boundaries)
    L, F = 32, 8
    N = L // F
    for c in range(L):
        vis = np.zeros((1, L, 1), complex)
        vis[0, c, 0] = 1.0
        resp = orc.fscrunch(vis, F)[0, :, 0].real * np.where(np.arange(N) == N // 2, F - 1, F)
        delta = (c - L // 2) % F
        if c == L // 2:
            assert np.all(resp == 0)
        elif delta == F // 2:
            assert sorted(resp[resp != 0]) == [0.5, 0.5]
            assert 10 * math.log10(0.5) == pytest.approx(-3.0103, abs=1e-4)
        else:
            assert sorted(resp[resp != 0]) == [1.0]


def test_averaging_pins_catch_planted_slips(orc):
    L, F = 32, 8
    r = rng(3)
    vis = r.standard_normal((1, L, 6)) + 1j * r.standard_normal((1, L, 6))
    good = orc.fscrunch(vis, F)
    assert averaging_ok(good, vis, L, F)
    N, oc = L // F, (L // F) // 2

    def slip(keep_dc=False, full_ends=False, centre=oc):
        out = np.zeros_like(good)
        for o in range(N):
            acc, ws = 0, 0
            for d in range(-F // 2, F // 2 + 1):
                if o == centre and d == 0 and not keep_dc:
                    continue
                w = 1.0 if full_ends or abs(d) < F // 2 else 0.5
                acc = acc + w * vis[:, (L // 2 + (o - centre) * F + d) % L]
                ws += w
            out[:, o] = acc / ws
        return out

    assert averaging_ok(slip(), vis, L, F)              # the slip helper itself is right
    for bad in (slip(keep_dc=True), slip(full_ends=True), slip(centre=oc - 1)):
        assert not averaging_ok(bad, vis, L, F)


# ---------------------------------------------------------------------------
# Fractional delay and phase correction (Sec. 2.5.1 delay paragraph, Sec. 4.3)
# ---------------------------------------------------------------------------
def shifted_spectra(frames):
    """fftshifted FFT of complex frames [M][L] -> [M][L][1] (numpy, FP64)."""
    X = np.fft.fftshift(np.fft.fft(frames, axis=1), axes=1)
    return X[:, :, None]


def test_delay_whole_samples_is_a_circular_shift(orc):
    # the delay theorem: delaying a frame by D whole samples (circularly) multiplies
    # bin k by exp(-2 pi i k D / L); with nu_c = 0 the correction must equal the
    # spectrum of the shifted frame, for either sign of D
    L, M = 64, 3
    x = rng(70).normal(size=(M, L)) + 1j * rng(71).normal(size=(M, L))
    for D in (1, 5, -3, 17):
        got = orc.delay_correct(shifted_spectra(x), np.full((1, 1), float(D)), L * M, 0.0)
        want = shifted_spectra(np.roll(x, D, axis=1))
        assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))


@pytest.mark.parametrize("k0", [-31, -1, 5, 31])
def test_delay_fractional_tone_uses_signed_frequency(orc, k0):
    # a tone at signed bin k0 sampled d samples late, exp(2 pi i k0 (q - d) / L),
    # has bin k0 = L exp(-2 pi i k0 d / L): the gradient runs over the signed
    # channel offset c - L/2, not the unsigned FFT bin
    L, d = 64, 0.3125
    q = np.arange(L)
    clean = np.exp(2j * np.pi * k0 * q / L)[None, :]
    late = np.exp(2j * np.pi * k0 * (q - d) / L)[None, :]
    got = orc.delay_correct(shifted_spectra(clean), np.full((1, 1), d), L, 0.0)
    c0 = (k0 + L // 2) % L
    assert abs(got[0, c0, 0] - L * np.exp(-2j * np.pi * k0 * d / L)) < 1e-9 * L
    assert abs(got[0, c0, 0] - shifted_spectra(late)[0, c0, 0]) < 1e-9 * L


def test_delay_sky_frequency_offset(orc):
    # L = 1: the only channel is the coarse-channel centre, so the gain is the
    # offset exp(-2 pi i (nu_c / f_s) d) alone; the offset is the same in every
    # channel of a longer transform, the gradient then varies across them
    nu = synth.NU_C / synth.F_S
    d = np.array([[0.37, -0.21]])
    x = np.array([[[3.0 + 4.0j]], [[-1.0 + 2.0j]]])        # [M=2][L=1][n=1]
    got = orc.delay_correct(x, d, 1, nu)
    for m in range(2):
        assert abs(got[m, 0, 0] - x[m, 0, 0] * np.exp(-2j * np.pi * nu * d[0, m])) < 1e-9
    L = 16
    ones = np.ones((1, L, 1), complex)
    g = orc.delay_correct(ones, np.full((1, 1), 0.25), L, nu)[0, :, 0]
    g0 = orc.delay_correct(ones, np.full((1, 1), 0.25), L, 0.0)[0, :, 0]
    ratio = g / g0
    assert np.allclose(ratio, np.exp(-2j * np.pi * nu * 0.25), atol=1e-12)
    assert np.allclose(np.abs(g), 1.0, atol=1e-14)          # power (and calibration) unchanged
    assert not np.allclose(g0, g0[0])                        # a gradient, not a constant


def test_delay_steps_follow_the_stream(orc):
    # a different whole-sample delay per step (step = 2 frames): every frame is
    # the circular shift by its own step's delay, with the stream offset m0
    L, M, step = 32, 6, 64
    x = rng(72).normal(size=(M, L)) + 1j * rng(73).normal(size=(M, L))
    m0 = 3                                  # frames 3..8 of the stream: steps 1..4
    D = np.array([[0.0, 2.0, -5.0, 7.0, 11.0]])
    got = orc.delay_correct(shifted_spectra(x), D, step, 0.0, m0=m0)
    for m in range(M):
        s = (m0 + m) * L // step
        want = shifted_spectra(np.roll(x[m:m + 1], int(D[0, s]), axis=1))
        assert np.max(np.abs(got[m:m + 1] - want)) < 1e-10 * np.max(np.abs(want))
    with pytest.raises(ValueError):
        orc.delay_correct(shifted_spectra(x), D[:, :3], step, 0.0, m0=m0)      # table too short


def test_delay_point_source_phased_up(orc):
    # the closed form of Sec. 4.3: a point source reaching input n tau_n late has
    # visibility phase -2 pi nu (tau_1 - tau_2); applying the delays d_n = -tau_n f_s
    # (advancing every path) leaves it real and positive in the source channel,
    # at the same amplitude, for two sources at different frequencies
    n_in, L, T, A = 6, 64, 400, 3.0
    seed = 0x51
    srcs = [synth.Source(A, 9), synth.Source(A, -20)]
    v = synth.gaussian_volts(n_in, L * T, sigma=2.0, seed=seed, sources=srcs, L=L)
    taus = synth.source_delays(n_in, seed)
    spec = orc.channelise(v, L)
    d = (-taus * synth.F_S)[:, None]
    cor = orc.delay_correct(spec, d, L * T, synth.NU_C / synth.F_S)
    V0 = orc.correlate(spec, T)[0]
    V = orc.correlate(cor, T)[0]
    for k0 in (9, -20):
        c0 = (k0 + L // 2) % L
        nu = synth.NU_C + k0 * synth.F_S / L
        for a in range(n_in):
            for b in range(a):
                p = a * (a + 1) // 2 + b
                want_before = np.angle(np.exp(-2j * np.pi * nu * (taus[a] - taus[b])))
                assert abs(np.angle(V0[c0, p] * np.exp(-1j * want_before))) < 0.05
                assert abs(np.angle(V[c0, p])) < 0.05
                assert abs(abs(V[c0, p]) / (T * L * L * A * A) - 1) < 0.1


def test_delay_pins_catch_planted_slips(orc):
    # numpy copies of the correction with one slip each; the pins above reject them
    L = 64

    def slipped(spec, d, nu, slip):
        c = np.arange(L) - L // 2
        if slip == "unsigned":
            c = (np.arange(L) + L // 2) % L            # the FFT bin instead of the signed offset
        ph = c / L * d + (0.0 if slip == "no_offset" else nu * d)
        g = np.exp((2j if slip == "sign" else -2j) * np.pi * ph)
        return spec * g[None, :, None]

    q = np.arange(L)
    x = rng(74).normal(size=(1, L)) + 1j * rng(75).normal(size=(1, L))
    want = shifted_spectra(np.roll(x, 3, axis=1))
    assert np.max(np.abs(slipped(shifted_spectra(x), 3.0, 0.0, "sign") - want)) > 1e-3
    tone = shifted_spectra(np.exp(2j * np.pi * -5 * q / L)[None, :])
    c0 = -5 + L // 2
    good = L * np.exp(-2j * np.pi * -5 * 0.3125 / L)
    assert abs(slipped(tone, 0.3125, 0.0, "unsigned")[0, c0, 0] - good) > 1e-3 * L
    assert abs(orc.delay_correct(tone, np.full((1, 1), 0.3125), L, 0.0)[0, c0, 0] - good) < 1e-9 * L
    one = np.ones((1, L, 1), complex)
    nu = synth.NU_C / synth.F_S
    ref = orc.delay_correct(one, np.full((1, 1), 0.37), L, nu)
    assert np.max(np.abs(slipped(one, 0.37, nu, "no_offset") - ref)) > 1e-3
    assert np.max(np.abs(slipped(one, 0.37, nu, "none") - ref)) < 1e-9


# ---------------------------------------------------------------------------
# Tied-array beamforming (Sec. 4.4)
# ---------------------------------------------------------------------------
def test_beamform_phased_source_closed_form(orc):
    # an exact tone reaching input n with phase i^p_n: weights conj(i^p_n) phase the
    # inputs up, so the coherent beam holds N A L in the tone channel (power
    # N^2 A^2 L^2, N times the incoherent sum N A^2 L^2); other channels are 0;
    # a beam pointed elsewhere (weights i^p_n) sums to a closed form too
    n, L, M, A, k0 = 8, 16, 3, 20, 4
    ph = np.array([0, 1, 2, 3, 1, 1, 0, 2])
    v = synth.tone_volts(n, L * M, L, k0, A, ph)
    spec = orc.channelise(v, L)
    c0 = (k0 + L // 2) % L
    w = np.zeros((L, 2, n), complex)
    w[:, 0, :] = (1j ** ph).conj()
    w[:, 1, :] = 1j ** ph
    B = orc.beamform(spec, w)
    assert B.shape == (M, L, 2)
    assert np.array_equal(B[:, c0, 0], np.full(M, n * A * L, complex))
    other = np.sum((1j ** ph) ** 2) * A * L
    assert np.allclose(B[:, c0, 1], other * (1j ** (np.arange(M) * 0)), atol=1e-9)
    assert np.max(np.abs(np.delete(B, c0, axis=1))) < 1e-9
    inc = orc.incoherent(spec, M, L)          # everything in one bin per polarisation
    assert inc.shape == (1, 1, 2)
    assert inc[0, 0].sum() == pytest.approx(M * n * A * A * L * L, rel=1e-12)
    assert np.abs(B[0, c0, 0]) ** 2 == pytest.approx(n * inc[0, 0].sum() / M, rel=1e-12)


def test_beamform_brute_force(orc):
    # tiny case written out in pure Python
    n, L, M, nb = 3, 4, 2, 2
    spec = rng(80).normal(size=(M, L, n)) + 1j * rng(81).normal(size=(M, L, n))
    w = rng(82).normal(size=(L, nb, n)) + 1j * rng(83).normal(size=(L, nb, n))
    B = orc.beamform(spec, w)
    for m in range(M):
        for c in range(L):
            for b in range(nb):
                want = sum(complex(w[c, b, k]) * complex(spec[m, c, k]) for k in range(n))
                assert abs(B[m, c, b] - want) < 1e-12


def test_incoherent_parseval_and_grouping(orc):
    # per spectrum and polarisation, the power over all channels is L times the
    # time-domain power of the frame (Parseval, exact integers); grouping sums
    # consecutive spectra and channels
    n, L, M = 6, 32, 8
    v = rand_volts(n, L * M, seed=84, amp=50)
    spec = orc.channelise(v, L)
    full = orc.incoherent(spec, 1, L)                     # [M][1][2]
    x = v.astype(np.int64)
    for m in range(M):
        fr = x[:, m * L:(m + 1) * L]
        for p in range(2):
            assert full[m, 0, p] == pytest.approx(L * np.sum(fr[p::2] ** 2), rel=1e-12)
    g = orc.incoherent(spec, 4, 8)                        # [2][4][2]
    fine = orc.incoherent(spec, 1, 1)                     # [M][L][2]
    assert np.allclose(g, fine.reshape(2, 4, 4, 8, 2).sum(axis=(1, 3)), rtol=1e-12)
    with pytest.raises(ValueError):
        orc.incoherent(spec, 3, 8)                        # 3 does not divide 8 spectra


def test_beamform_pins_catch_planted_slips(orc):
    n, L, M, A, k0 = 8, 16, 2, 20, 4
    ph = np.array([0, 1, 2, 3, 3, 2, 1, 0])
    spec = orc.channelise(synth.tone_volts(n, L * M, L, k0, A, ph), L)
    c0 = (k0 + L // 2) % L
    w = np.broadcast_to((1j ** ph).conj(), (L, 1, n))
    good = np.einsum("cbn,mcn->mcb", w, spec)                        # the definition, in numpy
    assert np.allclose(orc.beamform(spec, w), good, atol=1e-9)
    slip_conj = np.einsum("cbn,mcn->mcb", w.conj(), spec)            # weights conjugated
    assert abs(abs(slip_conj[0, c0, 0]) - n * A * L) > 1.0
    v = rand_volts(n, L * M, seed=85, amp=20)
    v[1::2] *= 3                                                      # Y paths 3x louder
    sp = orc.channelise(v, L)
    inc = orc.incoherent(sp, M, L)[0, 0]
    assert inc[1] > 5 * inc[0]                                        # so a swap is visible
    slip_pol = orc.incoherent(sp[:, :, ::-1], M, L)[0, 0]             # polarisations swapped
    assert abs(slip_pol[0] - inc[0]) > 0.5 * inc[0]
