"""ctypes binding of libmwax (C ABI in include/mwax.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of ``libmwax.so``; PyTorch provides device memory and the stream.  There is no
CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmwax.so")

MWAX_OK, MWAX_E_INVAL, MWAX_E_NOMEM, MWAX_E_DEVICE, MWAX_E_STATE, MWAX_E_UNSUPPORTED = range(6)
X_FP32, X_FP16, X_INT8 = 0, 1, 2
ORDER_CHAN_TRI, ORDER_TILE_BL = 0, 1
FAMILY_F, FAMILY_X, FAMILY_PACK, FAMILY_CALIB, FAMILY_STEP = 0, 1, 2, 3, 4
F_S = 1.28e6

_PREC = {"fp32": X_FP32, "fp16": X_FP16, "int8": X_INT8}
_ORDER = {"tri": ORDER_CHAN_TRI, "tile_bl": ORDER_TILE_BL}

EXPORTS = (
    "mwax_plan_derive", "mwax_plan_create", "mwax_plan_create_noalloc", "mwax_plan_destroy", "mwax_plan_get_dims",
    "mwax_channelise", "mwax_load_channelised", "mwax_read_channelised", "mwax_correlate",
    "mwax_integrate", "mwax_integrate_raw_i64", "mwax_set_scales", "mwax_auto_scales", "mwax_get_scales",
    "mwax_set_delays", "mwax_beamform", "mwax_beamform_incoherent", "mwax_integrate_averaged",
    "mwax_set_averaging",
    "mwax_reset", "mwax_sync", "mwax_set_timing", "mwax_kernel_time", "mwax_last_error",
    "mwax_batch_create", "mwax_batch_destroy", "mwax_batch_plan", "mwax_batch_run",
    "mwax_batch_autotune", "mwax_batch_get_tuning", "mwax_batch_set_tuning", "mwax_batch_get_tiles",
    "mwax_batch_set_tiles", "mwax_batch_set_tuning_cache", "mwax_batch_set_graph",
    "mwax_batch_set_timing", "mwax_batch_kernel_time", "mwax_batch_sync",
    "mwax_stream_create", "mwax_stream_destroy", "mwax_stream_get_info", "mwax_stream_plan",
    "mwax_stream_now", "mwax_stream_acquire", "mwax_stream_copy_in", "mwax_stream_submit",
    "mwax_stream_poll", "mwax_stream_vis", "mwax_vis_weights", "mwax_apply_weights", "mwax_fscrunch",
)


class Config(ctypes.Structure):
    _fields_ = [
        ("n_tiles", ctypes.c_int32), ("n_pols", ctypes.c_int32),
        ("coarse_bw_hz", ctypes.c_double), ("fine_chan_hz", ctypes.c_double),
        ("int_time_s", ctypes.c_double), ("xprec", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("max_samples", ctypes.c_int64), ("flags", ctypes.c_uint64),
    ]


class Dims(ctypes.Structure):
    _fields_ = [
        ("n_inputs", ctypes.c_int32), ("fft_len", ctypes.c_int32),
        ("spectra_per_int", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
        ("n_baselines", ctypes.c_int64), ("max_spectra", ctypes.c_int64),
        ("n_slots", ctypes.c_int32), ("group", ctypes.c_int32),
        ("vis_per_int", ctypes.c_int64), ("cal_spectra", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_uint64), ("sample_time_s", ctypes.c_double),
        ("fine_chan_hz", ctypes.c_double), ("int_time_s", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StreamConfig(ctypes.Structure):
    _fields_ = [
        ("n_channels", ctypes.c_int32), ("out_depth", ctypes.c_int32), ("cfg", Config),
        ("block_samples", ctypes.c_int64), ("hbm_budget_bytes", ctypes.c_uint64),
    ]


class StreamInfo(ctypes.Structure):
    _fields_ = [
        ("pool_slots", ctypes.c_int32), ("n_inputs", ctypes.c_int32), ("block_bytes", ctypes.c_uint64),
        ("block_ld", ctypes.c_int64), ("ingest_stream", ctypes.c_void_p), ("compute_stream", ctypes.c_void_p),
        ("device_bytes", ctypes.c_uint64),
    ]


class BlockDone(ctypes.Structure):
    _fields_ = [
        ("channel", ctypes.c_int32), ("slot", ctypes.c_int32), ("block", ctypes.c_int64),
        ("first_int", ctypes.c_int64), ("n_ints", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("t_arrival_s", ctypes.c_double), ("t_submit_s", ctypes.c_double), ("t_ready_s", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class MwaxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"mwax error {status}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libmwax.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmwax is not built ({LIB_PATH} missing): run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER
        sig = {
            "mwax_plan_derive": [P(Config), P(Dims)],
            "mwax_plan_create": [P(Config), vp, P(vp)],
            "mwax_plan_create_noalloc": [P(Config), vp, P(vp)],
            "mwax_plan_destroy": [vp],
            "mwax_plan_get_dims": [vp, P(Dims)],
            "mwax_channelise": [vp, vp, i64, i64],
            "mwax_load_channelised": [vp, vp, i64],
            "mwax_read_channelised": [vp, vp, i64, P(i64)],
            "mwax_correlate": [vp],
            "mwax_integrate": [vp, vp, i32, P(i32), i32],
            "mwax_integrate_raw_i64": [vp, vp, vp, i32, P(i32)],
            "mwax_set_scales": [vp, P(ctypes.c_float)],
            "mwax_auto_scales": [vp],
            "mwax_get_scales": [vp, vp],
            "mwax_set_delays": [vp, vp, i64, i64, ctypes.c_double],
            "mwax_beamform": [vp, vp, i32, vp, i64, P(i64)],
            "mwax_integrate_averaged": [vp, i32, vp, vp, i32, P(i32)],
            "mwax_set_averaging": [vp, i32],
            "mwax_beamform_incoherent": [vp, i32, i32, vp, i64, P(i64)],
            "mwax_reset": [vp],
            "mwax_sync": [vp],
            "mwax_set_timing": [vp, i32],
            "mwax_kernel_time": [vp, i32, P(ctypes.c_double), P(i64)],
            "mwax_batch_create": [P(Config), i32, vp, P(vp)],
            "mwax_batch_destroy": [vp],
            "mwax_batch_plan": [vp, i32, P(vp)],
            "mwax_batch_run": [vp, P(vp), P(i64), P(i64)],
            "mwax_batch_autotune": [vp, P(vp), P(i64), P(i64), i32],
            "mwax_batch_get_tuning": [vp, P(i32), P(i32)],
            "mwax_batch_set_tuning": [vp, P(i32), i32],
            "mwax_batch_get_tiles": [vp, P(i32)],
            "mwax_batch_set_tiles": [vp, P(i32)],
            "mwax_batch_set_tuning_cache": [vp, ctypes.c_char_p],
            "mwax_batch_set_graph": [vp, i32],
            "mwax_batch_set_timing": [vp, i32],
            "mwax_batch_kernel_time": [vp, i32, P(ctypes.c_double), P(i64)],
            "mwax_batch_sync": [vp],
            "mwax_stream_create": [P(StreamConfig), P(vp)],
            "mwax_stream_destroy": [vp],
            "mwax_stream_get_info": [vp, P(StreamInfo)],
            "mwax_stream_plan": [vp, i32, P(vp)],
            "mwax_stream_now": [vp, P(ctypes.c_double)],
            "mwax_stream_acquire": [vp, i32, P(i32), P(vp)],
            "mwax_stream_copy_in": [vp, i32, vp, i64],
            "mwax_stream_submit": [vp, i32, i32, ctypes.c_double],
            "mwax_stream_poll": [vp, i32, P(BlockDone), i32, P(i32)],
            "mwax_stream_vis": [vp, i32, i64, P(vp)],
            "mwax_vis_weights": [vp, i32, i32, i32, vp, vp],
            "mwax_apply_weights": [vp, vp, i32, i32, i32, vp],
            "mwax_fscrunch": [vp, vp, i32, i32, i32, i32, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.mwax_last_error.argtypes = []
        L.mwax_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != MWAX_OK:
        raise MwaxError(status, lib().mwax_last_error().decode())


def make_config(n_tiles, L=None, fine_chan_hz=None, T=None, int_time_s=None, xprec="fp32",
                max_samples=None, coarse_bw_hz=F_S) -> Config:
    if fine_chan_hz is None:
        fine_chan_hz = coarse_bw_hz / L
    if L is None:
        L = int(round(coarse_bw_hz / fine_chan_hz))
    if int_time_s is None:
        int_time_s = T * L / coarse_bw_hz
    if max_samples is None:
        max_samples = int(round(int_time_s * coarse_bw_hz))
    prec = _PREC[xprec] if isinstance(xprec, str) else int(xprec)
    return Config(int(n_tiles), 2, float(coarse_bw_hz), float(fine_chan_hz), float(int_time_s),
                  prec, 0, int(max_samples), 0)


def derive(cfg: Config) -> Dims:
    d = Dims()
    _check(lib().mwax_plan_derive(ctypes.byref(cfg), ctypes.byref(d)))
    return d


class Plan:
    """One correlator plan on the current device and torch's current stream.

    A plan that belongs to a batch (``Batch.plans``) wraps the batch's handle and
    is released with the batch.  noalloc=True creates the plan in the library's
    static device workspace (mwax_plan_create_noalloc)."""

    def __init__(self, cfg: Config, stream=None, _handle=None, noalloc=False):
        import torch
        self.torch = torch
        self.cfg = cfg
        self._owned = _handle is None
        if _handle is None:
            if stream is None:
                stream = torch.cuda.current_stream()
            self.stream = stream
            h = ctypes.c_void_p()
            create = lib().mwax_plan_create_noalloc if noalloc else lib().mwax_plan_create
            _check(create(ctypes.byref(cfg), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        else:
            self.stream = None
            h = _handle
        self.h = h
        d = Dims()
        _check(lib().mwax_plan_get_dims(self.h, ctypes.byref(d)))
        self.dims = d
        self.L = d.fft_len
        self.n_in = d.n_inputs
        self.P = d.n_pairs
        self.T = d.spectra_per_int
        self.xprec = cfg.xprec
        self.favg = 1                 # set_averaging: fine channels per emitted channel

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            if self._owned:
                lib().mwax_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- hot path -------------------------------------------------------------
    def channelise(self, volts, n_samples=None):
        """volts: int8 cuda tensor [n_inputs][>= n_samples][2], rows may be strided."""
        t = self.torch
        assert volts.dtype == t.int8 and volts.is_cuda and volts.dim() == 3
        assert volts.shape[0] == self.n_in and volts.shape[2] == 2
        assert volts.stride(2) == 1 and volts.stride(1) == 2
        n = volts.shape[1] if n_samples is None else int(n_samples)
        ld = volts.stride(0) // 2
        _check(lib().mwax_channelise(self.h, ctypes.c_void_p(volts.data_ptr()), n, ld))

    def load_channelised(self, chan):
        """chan: [n_spectra][L][n_inputs][2] of int8 / int16 (binary16 bits) / float32."""
        assert chan.is_cuda and chan.is_contiguous() and chan.dim() == 4
        assert chan.shape[1] == self.L and chan.shape[2] == self.n_in and chan.shape[3] == 2
        _check(lib().mwax_load_channelised(self.h, ctypes.c_void_p(chan.data_ptr()), chan.shape[0]))

    def element_dtype(self):
        t = self.torch
        return {X_INT8: t.int8, X_FP16: t.float16, X_FP32: t.float32}[self.xprec]

    def read_channelised(self):
        t = self.torch
        out = t.empty((self.dims.max_spectra, self.L, self.n_in, 2), dtype=self.element_dtype(),
                      device="cuda")
        n = ctypes.c_int64()
        _check(lib().mwax_read_channelised(self.h, ctypes.c_void_p(out.data_ptr()),
                                           self.dims.max_spectra, ctypes.byref(n)))
        return out[: n.value]

    def beamform(self, weights, out=None):
        """Coherent beams of the last channelised block: weights complex64 [L][n_beams][n_inputs]
        -> beams complex64 [n_spectra][L][n_beams]."""
        t = self.torch
        assert weights.is_cuda and weights.dtype == t.complex64 and weights.is_contiguous()
        assert weights.dim() == 3 and weights.shape[0] == self.L and weights.shape[2] == self.n_in
        nb = weights.shape[1]
        if out is None:
            out = t.empty((self.dims.max_spectra, self.L, nb), dtype=t.complex64, device="cuda")
        assert out.is_cuda and out.dtype == t.complex64 and out.is_contiguous() and out.shape[1:] == (self.L, nb)
        n = ctypes.c_int64()
        _check(lib().mwax_beamform(self.h, ctypes.c_void_p(weights.data_ptr()), nb, ctypes.c_void_p(out.data_ptr()),
                                   out.shape[0], ctypes.byref(n)))
        return out[: n.value]

    def beamform_incoherent(self, t_avg=1, f_avg=1, out=None):
        """Incoherent beam of the last channelised block -> float32 [n_spectra/t_avg][L/f_avg][2]."""
        t = self.torch
        n_o = self.L // int(f_avg)
        if out is None:
            out = t.empty((self.dims.max_spectra // int(t_avg), n_o, 2), dtype=t.float32, device="cuda")
        assert out.is_cuda and out.dtype == t.float32 and out.is_contiguous() and out.shape[1:] == (n_o, 2)
        n = ctypes.c_int64()
        _check(lib().mwax_beamform_incoherent(self.h, int(t_avg), int(f_avg), ctypes.c_void_p(out.data_ptr()),
                                              out.shape[0] * n_o, ctypes.byref(n)))
        return out[: n.value]

    def correlate(self):
        _check(lib().mwax_correlate(self.h))

    def integrate(self, max_ints=1, order="tri", out=None):
        """Emit up to max_ints completed integrations -> complex64 tensor [n][...]
        (over L / fscrunch channels after set_averaging(fscrunch))."""
        t = self.torch
        o = _ORDER[order] if isinstance(order, str) else int(order)
        nc = self.L // self.favg
        shape = (max_ints, nc, self.P) if o == ORDER_CHAN_TRI else (max_ints, self.dims.n_baselines, nc, 4)
        if out is None:
            out = t.empty(shape, dtype=t.complex64, device="cuda")
        assert out.is_cuda and out.dtype == t.complex64 and out.is_contiguous()
        assert tuple(out.shape[1:]) == shape[1:] and out.shape[0] >= max_ints
        n = ctypes.c_int32()
        _check(lib().mwax_integrate(self.h, ctypes.c_void_p(out.data_ptr()), max_ints,
                                    ctypes.byref(n), o))
        return out[: n.value]

    def set_averaging(self, fscrunch):
        """Average by fscrunch inside the X-engine from the next block on (Sec. 2.6;
        INT8 and FP16 plans, before the first block or after reset)."""
        _check(lib().mwax_set_averaging(self.h, int(fscrunch)))
        self.favg = int(fscrunch)

    def integrate_averaged(self, fscrunch, max_ints=1, weights=None, out=None):
        """Emit completed integrations averaged by fscrunch (Sec. 2.6) in the same
        pass -> complex64 [n][L / fscrunch][P]; weights: [max_ints][P] float32 or None."""
        t = self.torch
        F = int(fscrunch)
        if out is None:
            out = t.empty((max_ints, self.L // F, self.P), dtype=t.complex64, device="cuda")
        assert out.is_cuda and out.dtype == t.complex64 and out.is_contiguous()
        assert out.shape[1:] == (self.L // F, self.P) and out.shape[0] >= max_ints
        wp = ctypes.c_void_p()
        if weights is not None:
            assert weights.is_cuda and weights.dtype == t.float32 and weights.is_contiguous()
            assert weights.shape[1] == self.P and weights.shape[0] >= max_ints
            wp = ctypes.c_void_p(weights.data_ptr())
        n = ctypes.c_int32()
        _check(lib().mwax_integrate_averaged(self.h, F, wp, ctypes.c_void_p(out.data_ptr()), max_ints,
                                             ctypes.byref(n)))
        return out[: n.value]

    def integrate_raw(self, max_ints=1):
        """INT8 plans: exact int64 sums [n][L][P][2] and the scales s_c [n][L]."""
        t = self.torch
        out = t.empty((max_ints, self.L, self.P, 2), dtype=t.int64, device="cuda")
        sc = t.empty((max_ints, self.L), dtype=t.float32, device="cuda")
        n = ctypes.c_int32()
        _check(lib().mwax_integrate_raw_i64(self.h, ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(sc.data_ptr()), max_ints,
                                            ctypes.byref(n)))
        return out[: n.value], sc[: n.value]

    def set_scales(self, scales):
        import numpy as np
        a = np.ascontiguousarray(scales, dtype=np.float32)
        assert a.shape == (self.L,)
        _check(lib().mwax_set_scales(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def auto_scales(self):
        _check(lib().mwax_auto_scales(self.h))

    def get_scales(self, out=None):
        """INT8 plans: the scales s_c [L] float32 of the most recently begun integration."""
        t = self.torch
        if out is None:
            out = t.empty((self.L,), dtype=t.float32, device="cuda")
        assert out.is_cuda and out.dtype == t.float32 and out.is_contiguous() and out.numel() >= self.L
        _check(lib().mwax_get_scales(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_delays(self, delays, step_samples=6400, sky_freq_hz=0.0):
        """Fractional delay and phase correction for the following channelise calls:
        delays = float32 cuda tensor [n_inputs][n_steps] (samples), kept alive by the
        caller; None turns it off."""
        if delays is None:
            _check(lib().mwax_set_delays(self.h, None, 0, 0, 0.0))
            self._delays = None
            return
        t = self.torch
        assert delays.is_cuda and delays.dtype == t.float32 and delays.is_contiguous() and delays.dim() == 2
        assert delays.shape[0] == self.n_in
        _check(lib().mwax_set_delays(self.h, ctypes.c_void_p(delays.data_ptr()), delays.shape[1],
                                     int(step_samples), float(sky_freq_hz)))
        self._delays = delays        # keep the table alive while the plan may read it

    def reset(self):
        _check(lib().mwax_reset(self.h))

    def sync(self):
        _check(lib().mwax_sync(self.h))

    def set_timing(self, on=True):
        _check(lib().mwax_set_timing(self.h, int(bool(on))))

    def kernel_time(self, family):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().mwax_kernel_time(self.h, family, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Batch:
    """Many plans run as one unit of device work per call (see mwax.h, Batches).

    stream=None lets the library create the batch's stream, which synchronises
    with the legacy default stream torch uses unless told otherwise."""

    def __init__(self, cfgs, stream=None):
        import torch
        self.torch = torch
        self.cfgs = list(cfgs)
        self.n = len(self.cfgs)
        arr = (Config * self.n)(*self.cfgs)
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p()
        _check(lib().mwax_batch_create(arr, self.n, sp, ctypes.byref(h)))
        self.h = h
        self.plans = []
        for i, c in enumerate(self.cfgs):
            ph = ctypes.c_void_p()
            _check(lib().mwax_batch_plan(self.h, i, ctypes.byref(ph)))
            self.plans.append(Plan(c, _handle=ph))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            for p in self.plans:
                p.close()
            lib().mwax_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _arrays(self, volts, n_samples):
        ptrs = (ctypes.c_void_p * self.n)()
        ns = (ctypes.c_int64 * self.n)()
        ld = (ctypes.c_int64 * self.n)()
        t = self.torch
        for i, v in enumerate(volts):
            if v is None:
                continue
            p = self.plans[i]
            assert v.dtype == t.int8 and v.is_cuda and v.dim() == 3
            assert v.shape[0] == p.n_in and v.shape[2] == 2 and v.stride(2) == 1 and v.stride(1) == 2
            ptrs[i] = v.data_ptr()
            ns[i] = v.shape[1] if n_samples is None or n_samples[i] is None else int(n_samples[i])
            ld[i] = v.stride(0) // 2
        return ptrs, ns, ld

    def run(self, volts, n_samples=None):
        """volts: one int8 [n_inputs][>= n][2] tensor (or None: skip) per instance."""
        assert len(volts) == self.n
        ptrs, ns, ld = self._arrays(volts, n_samples)
        _check(lib().mwax_batch_run(self.h, ptrs, ns, ld))

    def autotune(self, volts, trials=3, cache=None):
        """Tune on the given blocks; cache: path of the on-disk tuning cache to
        consult and update (None: keep the batch's setting)."""
        assert len(volts) == self.n
        if cache is not None:
            self.set_tuning_cache(cache)
        ptrs, ns, ld = self._arrays(volts, None)
        _check(lib().mwax_batch_autotune(self.h, ptrs, ns, ld, int(trials)))
        return self.tuning()

    def tiles(self):
        t = (ctypes.c_int32 * self.n)()
        _check(lib().mwax_batch_get_tiles(self.h, t))
        return list(t)

    def set_tiles(self, tiles):
        assert len(tiles) == self.n
        _check(lib().mwax_batch_set_tiles(self.h, (ctypes.c_int32 * self.n)(*[int(t) for t in tiles])))

    def set_tuning_cache(self, path):
        _check(lib().mwax_batch_set_tuning_cache(self.h, None if not path else os.fsencode(path)))

    def tuning(self):
        kc = (ctypes.c_int32 * self.n)()
        g = ctypes.c_int32()
        _check(lib().mwax_batch_get_tuning(self.h, kc, ctypes.byref(g)))
        return list(kc), g.value

    def set_tuning(self, kchunk=None, grid=0):
        kc = None if kchunk is None else (ctypes.c_int32 * self.n)(*[int(k) for k in kchunk])
        _check(lib().mwax_batch_set_tuning(self.h, kc, int(grid)))

    def set_graph(self, on=True):
        _check(lib().mwax_batch_set_graph(self.h, int(bool(on))))

    def set_timing(self, on=True):
        _check(lib().mwax_batch_set_timing(self.h, int(bool(on))))

    def kernel_time(self, family):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().mwax_batch_kernel_time(self.h, family, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def sync(self):
        _check(lib().mwax_batch_sync(self.h))


class Stream:
    """Real-time streaming of voltage blocks through one plan per coarse channel
    (see mwax.h, Real-time streaming).  The stream runs on its own HIP streams:
    call :meth:`ingest_stream` work before :meth:`submit`, and read output-ring
    visibilities only after :meth:`poll` has reported their block."""

    def __init__(self, cfg: Config, n_channels, block_samples, hbm_budget_bytes, out_depth=8):
        import torch
        self.torch = torch
        self.cfg = cfg
        sc = StreamConfig(int(n_channels), int(out_depth), cfg, int(block_samples), int(hbm_budget_bytes))
        h = ctypes.c_void_p()
        _check(lib().mwax_stream_create(ctypes.byref(sc), ctypes.byref(h)))
        self.h = h
        info = StreamInfo()
        _check(lib().mwax_stream_get_info(self.h, ctypes.byref(info)))
        self.info = info
        self.n_channels = int(n_channels)
        self.block_samples = int(block_samples)
        self.plans = []
        for k in range(self.n_channels):
            ph = ctypes.c_void_p()
            _check(lib().mwax_stream_plan(self.h, k, ctypes.byref(ph)))
            self.plans.append(Plan(cfg, _handle=ph))
        self.ingest = torch.cuda.ExternalStream(info.ingest_stream)
        self.compute = torch.cuda.ExternalStream(info.compute_stream)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            for p in self.plans:
                p.close()
            lib().mwax_stream_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def now(self):
        t = ctypes.c_double()
        _check(lib().mwax_stream_now(self.h, ctypes.byref(t)))
        return t.value

    def acquire(self, wait_ms=-1):
        """Admission -> (slot, device pointer of the free buffer [n_inputs][block_samples][2] int8);
        :func:`device_view` gives a tensor over it."""
        slot = ctypes.c_int32()
        ptr = ctypes.c_void_p()
        _check(lib().mwax_stream_acquire(self.h, int(wait_ms), ctypes.byref(slot), ctypes.byref(ptr)))
        return slot.value, ptr.value

    def copy_in(self, slot, host_block):
        """host_block: pinned int8 CPU tensor [n_inputs][>= block_samples][2]."""
        assert host_block.dtype == self.torch.int8 and host_block.dim() == 3
        assert host_block.stride(2) == 1 and host_block.stride(1) == 2
        _check(lib().mwax_stream_copy_in(self.h, int(slot), ctypes.c_void_p(host_block.data_ptr()),
                                         host_block.stride(0) // 2))

    def submit(self, slot, channel, t_arrival):
        _check(lib().mwax_stream_submit(self.h, int(slot), int(channel), float(t_arrival)))

    def poll(self, wait_ms=0, max_records=1024):
        recs = (BlockDone * max_records)()
        n = ctypes.c_int32()
        _check(lib().mwax_stream_poll(self.h, int(wait_ms), recs, max_records, ctypes.byref(n)))
        return [recs[i].as_dict() for i in range(n.value)]

    def vis_ptr(self, channel, j):
        ptr = ctypes.c_void_p()
        _check(lib().mwax_stream_vis(self.h, int(channel), int(j), ctypes.byref(ptr)))
        return ptr.value


def vis_weights(flags, subs_per_int, out=None, stream=None):
    """Occupancy weights [n_ints][P] float32 from zeroing flags
    [n_inputs][n_ints * subs_per_int] uint8 (nonzero = sub-block zeroed), both
    on the device (Sec. 4.1)."""
    import torch
    assert flags.is_cuda and flags.dtype == torch.uint8 and flags.is_contiguous() and flags.dim() == 2
    n_in, n_sub = flags.shape
    subs = int(subs_per_int)
    assert subs >= 1 and n_sub % subs == 0, "flags must hold a whole number of integrations"
    n_ints = n_sub // subs
    if out is None:
        out = torch.empty((n_ints, n_in * (n_in + 1) // 2), dtype=torch.float32, device=flags.device)
    assert out.is_contiguous() and out.dtype == torch.float32 and out.numel() >= n_ints * (n_in * (n_in + 1) // 2)
    assert out.is_cuda and out.device == flags.device, "out must be on the flags' device"
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().mwax_vis_weights(ctypes.c_void_p(flags.data_ptr()), n_in, subs, n_ints,
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    return out


def apply_weights(vis, weights, stream=None):
    """Normalise CHAN_TRI visibilities [n_ints][L][P] complex64 in place by the
    weights [n_ints][P] (V / w where w > 0); returns vis."""
    import torch
    assert vis.is_cuda and vis.dtype == torch.complex64 and vis.is_contiguous() and vis.dim() == 3
    n_ints, L, P = vis.shape
    n_in = int(round(((8 * P + 1) ** 0.5 - 1) / 2))
    assert n_in * (n_in + 1) // 2 == P, "P is not a triangular number"
    assert weights.is_contiguous() and weights.dtype == torch.float32 and tuple(weights.shape) == (n_ints, P)
    assert weights.is_cuda and weights.device == vis.device, "weights must be on the visibilities' device"
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().mwax_apply_weights(ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(weights.data_ptr()),
                                    n_in, L, n_ints, ctypes.c_void_p(st.cuda_stream)))
    return vis


def fscrunch(vis, F, out=None, stream=None, weights=None):
    """Centre-symmetric channel averaging (Sec. 2.6) of CHAN_TRI visibilities
    [n_ints][L][P] complex64 by F -> [n_ints][L/F][P], optionally divided by the
    occupancy weights [n_ints][P] (where positive) in the same pass."""
    import torch
    assert vis.is_cuda and vis.dtype == torch.complex64 and vis.is_contiguous() and vis.dim() == 3
    n_ints, L, P = vis.shape
    n_in = int(round(((8 * P + 1) ** 0.5 - 1) / 2))
    assert n_in * (n_in + 1) // 2 == P, "P is not a triangular number"
    F = int(F)
    assert F >= 1 and L % F == 0, "F must divide the channel count"
    if out is None:
        out = torch.empty((n_ints, L // F, P), dtype=torch.complex64, device=vis.device)
    assert out.is_contiguous() and out.dtype == torch.complex64 and tuple(out.shape) == (n_ints, L // F, P)
    assert out.is_cuda and out.device == vis.device, "out must be on the visibilities' device"
    wp = ctypes.c_void_p()
    if weights is not None:
        assert weights.is_contiguous() and weights.dtype == torch.float32 and tuple(weights.shape) == (n_ints, P)
        assert weights.is_cuda and weights.device == vis.device, "weights must be on the visibilities' device"
        wp = ctypes.c_void_p(weights.data_ptr())
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().mwax_fscrunch(ctypes.c_void_p(vis.data_ptr()), wp, n_in, L, n_ints, F,
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    return out


def device_view(ptr, shape, dtype):
    """A torch tensor over device memory owned by the library (no copy, no ownership)."""
    import torch
    n = 1
    for d in shape:
        n *= d
    esize = torch.empty((), dtype=dtype).element_size()

    class _Mem:
        pass

    typestr = {torch.int8: "|i1", torch.complex64: "<c8", torch.float32: "<f4", torch.int64: "<i8"}[dtype]
    holder = _Mem()
    holder.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                       "version": 3, "strides": None}
    assert n * esize > 0 and ptr
    return torch.as_tensor(holder, device="cuda")


def pair_index(n1, n2):
    return n1 * (n1 + 1) // 2 + n2
