"""GPU parity of the channel averaging (Sec. 2.6) against the FP64 oracle.

The kernel sums in FP64 in the oracle's order with weights 1 and 1/2 (exact
products) and divides in FP64, so its FP32 output equals the oracle's FP64
mean of the same FP32 visibilities rounded to FP32, bit for bit.
"""
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


def expected(vis_c64, F):
    want = oracle.fscrunch(vis_c64.astype(np.complex128), F)
    return want.real.astype(np.float32), want.imag.astype(np.float32)


@pytest.mark.parametrize("n_in,L,F,n_ints", [
    (1, 1, 1, 1),
    (3, 16, 1, 2),          # identity
    (3, 16, 2, 1),          # centre channel of weight 1
    (3, 16, 16, 1),         # one output channel over the whole band
    (4, 20, 5, 2),          # odd F
    (130, 32, 8, 1),        # ragged pair chunks
    (3, 40, 2, 1),          # 20 output channels: five runs of 4
    (3, 44, 4, 1),          # 11 output channels: a ragged last run
    (16, 1024, 8, 2),       # 1024 fine channels to 128
    (512, 128, 4, 1),       # 256 tiles
])
def test_fscrunch_parity_bit_exact(n_in, L, F, n_ints):
    log(f"fscrunch n_in={n_in} L={L} F={F} n_ints={n_ints}")
    P = n_in * (n_in + 1) // 2
    r = np.random.default_rng(n_in * 7 + L + F)
    vis = (r.standard_normal((n_ints, L, P)) * 1e5 + 1j * r.standard_normal((n_ints, L, P)) * 1e5)
    vis = vis.astype(np.complex64)
    got = mwax.fscrunch(torch.from_numpy(vis).cuda(), F)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert g.shape == (n_ints, L // F, P)
    re, im = expected(vis, F)
    assert np.array_equal(g.real, re) and np.array_equal(g.imag, im)


@pytest.mark.parametrize("n_in,L,F,n_ints", [(130, 32, 8, 2), (7, 20, 5, 1), (512, 128, 4, 1)])
def test_fscrunch_with_weights_bit_exact(n_in, L, F, n_ints):
    # weighting during the averaging equals the oracle's average followed by
    # its normalisation, both in FP64, rounded once
    log(f"weighted fscrunch n_in={n_in} L={L} F={F} n_ints={n_ints}")
    P = n_in * (n_in + 1) // 2
    r = np.random.default_rng(n_in + 5 * L)
    vis = (r.standard_normal((n_ints, L, P)) + 1j * r.standard_normal((n_ints, L, P))).astype(np.complex64)
    flags = synth.zero_flags(n_in, 40 * n_ints, 0.3, seed=n_in + 1)
    flags[0, :40] = 1
    w = oracle.vis_weights(flags, 40).astype(np.float32)
    assert np.count_nonzero(w == 0) > 0 and np.count_nonzero((w > 0) & (w < 1)) > 0
    got = mwax.fscrunch(torch.from_numpy(vis).cuda(), F, weights=torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    want = oracle.apply_weights(oracle.fscrunch(vis.astype(np.complex128), F), w.astype(np.float64))
    assert np.array_equal(g.real, want.real.astype(np.float32))
    assert np.array_equal(g.imag, want.imag.astype(np.float32))


def test_fscrunch_of_correlator_output():
    # FP32 correlator output averaged on the GPU: bit-exact against the oracle
    # averaging the same output, and within the FP32 path's 1e-5 of the oracle
    # averaging its own FP64 visibilities
    n_tiles, L, T, F = 4, 64, 24, 8
    n_in = 2 * n_tiles
    v = synth.gaussian_volts(n_in, L * T, seed=synth.MWAX_SEED + 9, sources=[synth.Source(3.0, 9)], L=L)
    with Plan(make_config(n_tiles, L=L, T=T, xprec="fp32", max_samples=L * T)) as p:
        p.channelise(torch.from_numpy(v).cuda())
        p.correlate()
        vis = p.integrate(1).clone()
        avg = mwax.fscrunch(vis, F)
        torch.cuda.synchronize()
    vis_h = vis.cpu().numpy()
    g = avg.cpu().numpy()
    re, im = expected(vis_h, F)
    assert np.array_equal(g.real, re) and np.array_equal(g.imag, im)
    ref = oracle.fscrunch(oracle.fx_correlate(v, L, T), F)
    err = np.linalg.norm(g - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
    assert err.max() <= 1e-5


def test_fscrunch_zero_integrations():
    vis = torch.zeros((0, 16, 3), dtype=torch.complex64, device="cuda")
    out = mwax.fscrunch(vis, 4)
    torch.cuda.synchronize()
    assert out.shape == (0, 4, 3)
