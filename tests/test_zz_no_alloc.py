"""The plan entry point that allocates nothing (mwax_plan_create_noalloc),
called through the C ABI: its results equal those of a plan created with
mwax_plan_create (the same kernels over the same inputs, so bit for bit), on
two plans in a row in the shared static workspace, the second smaller; sizes
beyond the workspace and a second live plan are refused."""
import ctypes

import numpy as np
import pytest

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


def drive(plan, d, chunk, prec, n_ints):
    outs, scs = [], []
    for off in range(0, d.shape[1], chunk):
        plan.channelise(d[:, off:off + chunk])
        plan.correlate()
        if prec == "int8":
            raw, sc = plan.integrate_raw(n_ints)
            outs.append(raw.clone())
            scs.append(sc.clone())
        else:
            outs.append(plan.integrate(n_ints).clone())
    torch.cuda.synchronize()
    return torch.cat(outs).cpu().numpy(), (torch.cat(scs).cpu().numpy() if scs else None)


@pytest.mark.parametrize("prec", ["int8", "fp32"])
def test_noalloc_plan_equals_plan(prec):
    # (tiles, L, T, chunk, calls): the second is smaller than the first
    for n_tiles, L, T, chunk, calls in ((24, 128, 60, 128 * 40, 6), (5, 32, 25, 32 * 30, 4)):
        v = synth.gaussian_volts(2 * n_tiles, chunk * calls, seed=n_tiles * 31 + L,
                                 sources=[synth.Source(3.0, 5)], L=L)
        d = torch.from_numpy(v).cuda()
        cfg = make_config(n_tiles, L=L, T=T, xprec=prec, max_samples=chunk)
        with Plan(cfg) as p:
            want, want_s = drive(p, d, chunk, prec, 8)
        with Plan(cfg, noalloc=True) as p:
            got, got_s = drive(p, d, chunk, prec, 8)
        assert got.shape == want.shape and got.shape[0] >= 2
        assert np.array_equal(got, want), f"{prec} {n_tiles} tiles: no-alloc plan differs"
        if prec == "int8":
            assert np.array_equal(got_s, want_s)


def test_noalloc_limits():
    lib = mwax.lib()
    h = ctypes.c_void_p()
    big = make_config(256, L=128, T=100, xprec="int8", max_samples=128 * 100)
    assert mwax.derive(big).workspace_bytes > 64 << 20
    assert lib.mwax_plan_create_noalloc(ctypes.byref(big), None, ctypes.byref(h)) == mwax.MWAX_E_INVAL
    assert "static workspace" in lib.mwax_last_error().decode()
    small = make_config(2, L=16, T=10, xprec="fp32", max_samples=160)
    with Plan(small, noalloc=True):
        assert lib.mwax_plan_create_noalloc(ctypes.byref(small), None, ctypes.byref(h)) == mwax.MWAX_E_STATE
    with Plan(small, noalloc=True):          # released by the first plan's destroy
        pass
