"""Host-side checks of libmwax that need no GPU: exports, plan derivation, errors.

Plan derivation is checked against arithmetic the paper prints
(tests/golden/printed_arithmetic.json, each item with its citation).
"""
import ctypes
import json
import os
import re

import pytest

from paper_2303_11557_amd import mwax

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "printed_arithmetic.json")))
PRINTED = {it["key"]: it["value"] for it in GOLDEN["items"]}


@pytest.fixture(scope="module")
def lib():
    return mwax.lib()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "mwax.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mwax_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mwax.h but not exported"
    assert set(names) == set(mwax.EXPORTS)


def test_synth_library_exports():
    lib = ctypes.CDLL(os.path.join(ROOT, "synth", "libsynth.so"))
    assert hasattr(lib, "synth_gaussian_volts")


def test_header_struct_layouts_match_binding():
    # the ctypes mirrors must have the C sizes (checked against the header's field list)
    assert ctypes.sizeof(mwax.Config) == 4 + 4 + 8 + 8 + 8 + 4 + 4 + 8 + 8
    assert ctypes.sizeof(mwax.Dims) == 4 + 4 + 8 * 4 + 4 + 4 + 8 * 3 + 8 * 3


def cfg(**kw):
    base = dict(n_tiles=128, L=128, T=100, xprec="fp32", max_samples=128 * 1000)
    base.update(kw)
    return mwax.make_config(**base)


def test_printed_arithmetic():
    fs = PRINTED["coarse_sample_rate_hz"]
    # sample time (Table 1)
    d = mwax.derive(cfg())
    assert d.sample_time_s * 1e9 == pytest.approx(PRINTED["sample_time_ns"], abs=1e-9)
    # 128 tiles -> 8,256 baselines (Sec. 1.4)
    assert d.n_baselines == PRINTED["baselines_128_tiles"]
    assert d.n_inputs == 256
    # 256 tiles -> 512 signal paths (Sec. 2.5)
    d256 = mwax.derive(cfg(n_tiles=256))
    assert d256.n_inputs == PRINTED["max_signal_paths"]
    # a 50 ms block holds 64,000 samples; 160 of them make 8 s (Sec. 2.5)
    assert round(0.05 * fs) == PRINTED["block_samples_50ms"]
    assert round(8.0 / 0.05) == PRINTED["blocks_per_subfile"]
    # 6,400-pt FFT <-> 200 Hz channels, 10 frames per 50 ms block, 5 ms each (Sec. 2.5.1)
    L6400 = fs / PRINTED["ultrafine_chan_hz"]
    assert L6400 == PRINTED["fengine_fft_len"]
    assert PRINTED["block_samples_50ms"] // PRINTED["fengine_fft_len"] == PRINTED["subblocks_per_block"]
    assert PRINTED["fengine_fft_len"] / fs == pytest.approx(PRINTED["subblock_s"])
    # the library derives L from the channel width: 200 Hz is the 6,400-point
    # transform; a 250 ms gulp holds 50 of its 5 ms frames, a 50 ms block 10
    d200 = mwax.derive(mwax.make_config(128, fine_chan_hz=PRINTED["ultrafine_chan_hz"],
                                        int_time_s=PRINTED["min_integration_s"],
                                        max_samples=PRINTED["block_samples_50ms"]))
    assert d200.fft_len == PRINTED["fengine_fft_len"]
    assert d200.spectra_per_int == 50 and d200.max_spectra == PRINTED["subblocks_per_block"]
    # other whole lengths that are not powers of two stay unsupported
    with pytest.raises(mwax.MwaxError) as e:
        mwax.derive(mwax.make_config(128, fine_chan_hz=fs / 3200, int_time_s=0.25, max_samples=64000))
    assert e.value.status == mwax.MWAX_E_UNSUPPORTED
    # 10 kHz channels (fscrunch 50, Sec. 2.6) are a 128-point FFT
    d10k = mwax.derive(mwax.make_config(128, fine_chan_hz=PRINTED["fscrunch50_chan_hz"],
                                        int_time_s=PRINTED["min_integration_s"],
                                        max_samples=PRINTED["block_samples_50ms"] * 5))
    assert d10k.fft_len == 128
    assert d10k.fine_chan_hz == PRINTED["fscrunch50_chan_hz"]
    # the minimum integration, one 250 ms gulp, is a whole number of 10 kHz spectra
    assert d10k.spectra_per_int == 2500
    assert d10k.int_time_s == pytest.approx(PRINTED["min_integration_s"])
    # an 8 s subfile of 256 tiles is ~10 GB of complex 8-bit samples (Sec. 2.4)
    gb = d256.n_inputs * 8 * fs * 2 / 1e9
    assert gb == pytest.approx(PRINTED["subfile_gb_256_tiles"], rel=0.06)


@pytest.mark.parametrize("L,T,prec,G", [(1, 5, "fp32", 4), (128, 1000, "int8", 16),
                                         (1024, 625, "fp16", 8), (32, 20000, "int8", 16),
                                         (16, 80000, "int8", 16)])
def test_derived_dimensions(L, T, prec, G):
    d = mwax.derive(cfg(n_tiles=7, L=L, T=T, xprec=prec, max_samples=L * T * 3))
    assert d.fft_len == L and d.spectra_per_int == T and d.group == G
    assert d.n_pairs == 14 * 15 // 2 and d.n_baselines == 7 * 8 // 2
    assert d.max_spectra == 3 * T
    assert d.vis_per_int == L * d.n_pairs
    assert d.n_slots >= 3 + 2
    assert d.cal_spectra == min(T, -(-131072 // L))
    assert d.fine_chan_hz == pytest.approx(1.28e6 / L)
    # INT8 integrators are int32 pairs up to 65,536 spectra per integration
    elem = 8 if prec == "int8" and T <= 65536 else 16
    assert d.workspace_bytes > d.n_slots * L * d.n_pairs * elem
    assert d.workspace_bytes < d.n_slots * L * d.n_pairs * elem + 3 * T * L * 14 * 32 + (1 << 24)


@pytest.mark.parametrize("bad", [
    dict(n_tiles=0), dict(n_tiles=1025), dict(max_samples=128 * 10 + 1), dict(max_samples=0),
    dict(xprec=7),
])
def test_invalid_configs(bad):
    with pytest.raises(mwax.MwaxError) as e:
        mwax.derive(cfg(**bad))
    assert e.value.status == mwax.MWAX_E_INVAL


def test_invalid_config_fields():
    c = cfg()
    c.n_pols = 1
    with pytest.raises(mwax.MwaxError):
        mwax.derive(c)
    c = cfg()
    c.flags = 1
    with pytest.raises(mwax.MwaxError):
        mwax.derive(c)
    c = cfg()
    c.int_time_s = 0.5 * 128 / 1.28e6 * 1.5   # 1.5 spectra
    with pytest.raises(mwax.MwaxError) as e:
        mwax.derive(c)
    assert "whole number" in str(e.value)
    c = cfg()
    c.fine_chan_hz = 1.28e6 / 100.5
    with pytest.raises(mwax.MwaxError) as e:
        mwax.derive(c)
    assert e.value.status == mwax.MWAX_E_INVAL


def test_null_arguments_are_rejected_without_a_device(lib):
    # every entry point checks its plan handle before touching the GPU
    assert lib.mwax_correlate(None) == mwax.MWAX_E_INVAL
    assert lib.mwax_channelise(None, None, 128, 128) == mwax.MWAX_E_INVAL
    n = ctypes.c_int32(5)
    assert lib.mwax_integrate(None, None, 1, ctypes.byref(n), 0) == mwax.MWAX_E_INVAL
    assert lib.mwax_sync(None) == mwax.MWAX_E_INVAL
    assert lib.mwax_plan_destroy(None) == mwax.MWAX_OK
    assert lib.mwax_plan_derive(None, None) == mwax.MWAX_E_INVAL
    assert b"null" in lib.mwax_last_error()
    out = ctypes.c_void_p()
    assert lib.mwax_plan_create(None, None, ctypes.byref(out)) == mwax.MWAX_E_INVAL
    assert out.value is None


def test_batch_and_stream_arguments_are_checked_without_a_device(lib):
    # every check below fails before the library touches the GPU
    out = ctypes.c_void_p()
    assert lib.mwax_batch_create(None, 0, None, ctypes.byref(out)) == mwax.MWAX_E_INVAL
    fp32 = (mwax.Config * 2)(cfg(xprec="fp32"), cfg(xprec="fp32"))
    assert lib.mwax_batch_create(fp32, 2, None, ctypes.byref(out)) == mwax.MWAX_E_UNSUPPORTED
    mixed = (mwax.Config * 2)(cfg(xprec="int8"), cfg(xprec="fp16"))
    assert lib.mwax_batch_create(mixed, 2, None, ctypes.byref(out)) == mwax.MWAX_E_UNSUPPORTED
    bad = (mwax.Config * 2)(cfg(xprec="int8"), cfg(xprec="int8", n_tiles=0))
    assert lib.mwax_batch_create(bad, 2, None, ctypes.byref(out)) == mwax.MWAX_E_INVAL
    assert b"instance 1" in lib.mwax_last_error()
    assert out.value is None
    assert lib.mwax_batch_run(None, None, None, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_batch_destroy(None) == mwax.MWAX_OK

    def stream_cfg(**kw):
        base = dict(n_channels=2, out_depth=4, cfg=cfg(xprec="int8", max_samples=128 * 100),
                    block_samples=128 * 400, hbm_budget_bytes=1 << 34)
        base.update(kw)
        return mwax.StreamConfig(base["n_channels"], base["out_depth"], base["cfg"],
                                 base["block_samples"], base["hbm_budget_bytes"])

    for kw in (dict(n_channels=0), dict(out_depth=0), dict(block_samples=128 * 450),
               dict(hbm_budget_bytes=1000), dict(cfg=cfg(n_tiles=0))):
        sc = stream_cfg(**kw)
        assert lib.mwax_stream_create(ctypes.byref(sc), ctypes.byref(out)) == mwax.MWAX_E_INVAL, kw
        assert out.value is None
    assert lib.mwax_stream_create(None, ctypes.byref(out)) == mwax.MWAX_E_INVAL
    n = ctypes.c_int32()
    assert lib.mwax_stream_poll(None, 0, None, 0, ctypes.byref(n)) == mwax.MWAX_E_INVAL
    assert lib.mwax_stream_destroy(None) == mwax.MWAX_OK


def test_stream_struct_layouts():
    assert ctypes.sizeof(mwax.StreamConfig) == 4 + 4 + ctypes.sizeof(mwax.Config) + 8 + 8
    assert ctypes.sizeof(mwax.BlockDone) == 4 + 4 + 8 + 8 + 4 + 4 + 8 * 3
    assert ctypes.sizeof(mwax.StreamInfo) == 4 + 4 + 8 + 8 + 8 + 8 + 8


def test_weight_arguments_are_checked_without_a_device(lib):
    vp = ctypes.c_void_p
    fake = vp(4096)          # never dereferenced: every call below fails its checks first
    assert lib.mwax_vis_weights(fake, 0, 4, 1, fake, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_vis_weights(fake, 2049, 4, 1, fake, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_vis_weights(fake, 8, 0, 1, fake, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_vis_weights(fake, 8, 4, -1, fake, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_vis_weights(None, 8, 4, 1, fake, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_vis_weights(fake, 8, 4, 1, vp(4098), None) == mwax.MWAX_E_INVAL
    assert lib.mwax_vis_weights(None, 8, 4, 0, None, None) == mwax.MWAX_OK      # nothing to do
    assert lib.mwax_apply_weights(fake, fake, 0, 16, 1, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_apply_weights(fake, fake, 8, 0, 1, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_apply_weights(fake, fake, 8, 16, -2, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_apply_weights(None, fake, 8, 16, 1, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_apply_weights(vp(4100), fake, 8, 16, 1, None) == mwax.MWAX_E_INVAL
    assert b"aligned" in lib.mwax_last_error()
    assert lib.mwax_apply_weights(None, None, 8, 16, 0, None) == mwax.MWAX_OK


def test_fscrunch_arguments_are_checked_without_a_device(lib):
    vp = ctypes.c_void_p
    a, b = vp(1 << 20), vp(1 << 30)   # never dereferenced: every call below fails its checks first
    assert lib.mwax_fscrunch(a, None, 0, 16, 1, 4, b, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(a, None, 8, 0, 1, 1, b, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(a, None, 8, 16, 1, 0, b, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(a, None, 8, 16, 1, 3, b, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(a, None, 8, 16, -1, 4, b, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(None, None, 8, 16, 1, 4, b, None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(a, None, 8, 16, 1, 4, vp((1 << 30) + 4), None) == mwax.MWAX_E_INVAL
    assert lib.mwax_fscrunch(a, None, 8, 16, 1, 4, vp((1 << 20) + 64), None) == mwax.MWAX_E_INVAL
    assert b"overlaps" in lib.mwax_last_error()
    assert lib.mwax_fscrunch(a, vp((1 << 28) + 2), 8, 16, 1, 4, b, None) == mwax.MWAX_E_INVAL
    assert b"weights" in lib.mwax_last_error()
    assert lib.mwax_fscrunch(None, None, 8, 16, 0, 4, None, None) == mwax.MWAX_OK


def test_bench_runs_on_one_gpu_only():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr
    h = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert h.returncode == 0
    for w in ("channel", "batch", "stream", "weights", "fscrunch"):
        assert w in h.stdout
