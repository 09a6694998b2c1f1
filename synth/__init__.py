"""Seeded synthetic MWA-shaped voltages -- the one input generator both sides use.

This module holds none of the correlator's arithmetic: it only makes int8
complex voltage streams, laid out ``[n_inputs][n_samples][2]`` (re, im), with
input index n = 2*tile + pol.  The host version below (numpy) and the device
version (``synth.hip``, exposed through :func:`device_volts`) implement the
same counter-based definition:

* uniform draws: SplitMix64 output function (Steele, Lea and Flood 2014) on the
  counter ``seed + (idx + 1) * 0x9E3779B97F4A7C15``, top 53 bits, offset by half
  a step so a draw is never 0 or 1;
* Gaussian: Box-Muller on the pair (u1, u2) = draws 2*ctr and 2*ctr+1 with
  ctr = n * 2**36 + s;
* point sources: A exp(2 pi i (k0 s / L - nu tau_n)) with the tone centred on
  fine channel bin k0 (f0 = k0 f_s / L), sky frequency nu = nu_c + f0 and a
  seeded per-input delay tau_n in [0, max_delay);
* x = clip(rint(sigma * gauss + sources), -127, 127).

Host and device evaluate log/cos/sin with different maths libraries, so a
sample can on rare occasions round differently.  Parity tests therefore always
hand the oracle the exact int8 array the GPU consumed.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

F_S = 1.28e6            # complex samples per second per coarse channel
NU_C = 121 * 1.28e6     # sky centre frequency of coarse channel 121 (154.88 MHz)
MWAX_SEED = 0x4D574158  # "MWAX"

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_DELAY_STREAM = 0xD1B54A32D192ED03


@dataclass(frozen=True)
class Source:
    """A point source: complex amplitude ``amp`` centred on FFT bin ``k0``."""
    amp: float
    k0: int


def splitmix64(idx, seed: int) -> np.ndarray:
    """SplitMix64 output for counter values ``idx`` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (np.asarray(idx, np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(idx, seed: int) -> np.ndarray:
    """Uniform doubles in (0, 1) from the top 53 bits of SplitMix64."""
    z = splitmix64(idx, seed)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def source_delays(n_inputs: int, seed: int, max_delay: float = 50e-9) -> np.ndarray:
    """Seeded per-input delays tau_n, uniform in [0, max_delay) seconds."""
    return max_delay * uniform(np.arange(n_inputs, dtype=np.uint64), seed ^ _DELAY_STREAM)


def gaussian_volts(n_inputs: int, n_samples: int, sigma: float = 8.0, seed: int = MWAX_SEED,
                   sources=(), L: int = 128, nu_c: float = NU_C, max_delay: float = 50e-9,
                   s0: int = 0) -> np.ndarray:
    """Host generator: int8 [n_inputs][n_samples][2] (samples s0 .. s0+n_samples-1)."""
    out = np.empty((n_inputs, n_samples, 2), np.int8)
    s = np.arange(s0, s0 + n_samples, dtype=np.uint64)
    taus = source_delays(n_inputs, seed, max_delay) if sources else None
    for n in range(n_inputs):
        ctr = np.uint64(n) * np.uint64(1 << 36) + s
        u1 = uniform(ctr * np.uint64(2), seed)
        u2 = uniform(ctr * np.uint64(2) + np.uint64(1), seed)
        r = np.sqrt(-2.0 * np.log(u1))
        th = 2.0 * np.pi * u2
        re = sigma * r * np.cos(th)
        im = sigma * r * np.sin(th)
        for src in sources:
            f0 = src.k0 * F_S / L
            nu = nu_c + f0
            ks = (np.int64(src.k0) * s.astype(np.int64)) % L     # exact phase in turns * L
            turns = ks.astype(np.float64) / L - nu * taus[n]
            re = re + src.amp * np.cos(2.0 * np.pi * turns)
            im = im + src.amp * np.sin(2.0 * np.pi * turns)
        out[n, :, 0] = np.clip(np.rint(re), -127, 127).astype(np.int8)
        out[n, :, 1] = np.clip(np.rint(im), -127, 127).astype(np.int8)
    return out


def tone_volts(n_inputs: int, n_samples: int, L: int, k0: int, amp: int, phases) -> np.ndarray:
    """Exact integer tone: x_n[s] = amp * i^(s * 4 k0 / L + p_n), k0 a multiple of L/4.

    All power lands in FFT bin k0; every sample is an exact int8 value.
    """
    if (4 * k0) % L != 0:
        raise ValueError("k0 must be a multiple of L/4 for an exact integer tone")
    step = (4 * k0) // L
    unit = np.array([[1, 0], [0, 1], [-1, 0], [0, -1]], np.int64)   # i^0 .. i^3
    s = np.arange(n_samples, dtype=np.int64)
    out = np.empty((n_inputs, n_samples, 2), np.int8)
    for n in range(n_inputs):
        e = (s * step + int(phases[n])) % 4
        out[n] = (amp * unit[e]).astype(np.int8)
    return out


_FLAG_STREAM = 0x6A09E667F3BCC909


def zero_flags(n_inputs: int, n_sub: int, p: float, seed: int = MWAX_SEED) -> np.ndarray:
    """Seeded zeroing flags [n_inputs][n_sub] uint8: 1 marks a 50 ms sub-block
    whose packets were lost (probability p each)."""
    idx = np.arange(n_inputs * n_sub, dtype=np.uint64)
    return (uniform(idx, seed ^ _FLAG_STREAM) < p).astype(np.uint8).reshape(n_inputs, n_sub)


def zero_subblocks(volts: np.ndarray, flags: np.ndarray, sub_len: int) -> np.ndarray:
    """What the capture stage hands on: voltages [n][S][2] with every flagged
    sub-block of sub_len samples set to zero (S = n_sub * sub_len)."""
    n, S = volts.shape[:2]
    if flags.shape != (n, S // sub_len) or S % sub_len:
        raise ValueError("flags must cover the voltages in whole sub-blocks")
    keep = np.repeat(flags == 0, sub_len, axis=1)
    return (volts * keep[:, :, None]).astype(np.int8)


# ---------------------------------------------------------------------------
# Device generator (HIP).  Built by __graft_entry__.build() into libsynth.so.
# ---------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_dlib = None


def _device_lib():
    global _dlib
    if _dlib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"device generator not built: {LIB_PATH} is missing")
        lib = ctypes.CDLL(LIB_PATH)
        lib.synth_gaussian_volts.argtypes = [
            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
            ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_double,
            ctypes.c_double, ctypes.c_void_p]
        lib.synth_gaussian_volts.restype = ctypes.c_int
        _dlib = lib
    return _dlib


def device_volts(out, sigma: float = 8.0, seed: int = MWAX_SEED, sources=(), L: int = 128,
                 nu_c: float = NU_C, max_delay: float = 50e-9, s0: int = 0, stream=None):
    """Fill a device int8 tensor ``out`` [n_inputs][n_samples][2] on the GPU.

    ``out`` may be a row-strided view (rows ``ld`` samples apart).  Enqueued on
    ``stream`` (default: torch's current stream).
    """
    import torch
    assert out.dtype == torch.int8 and out.is_cuda and out.dim() == 3 and out.shape[2] == 2
    assert out.stride(2) == 1 and out.stride(1) == 2
    n_in, S = out.shape[0], out.shape[1]
    ld = out.stride(0) // 2
    amps = np.array([s.amp for s in sources] or [0.0], np.float64)
    k0s = np.array([s.k0 for s in sources] or [0], np.int32)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    rc = _device_lib().synth_gaussian_volts(
        ctypes.c_void_p(out.data_ptr()), n_in, S, ld, s0, sigma, seed & 0xFFFFFFFFFFFFFFFF,
        len(sources), amps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        k0s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), L, nu_c, max_delay,
        ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"synth_gaussian_volts failed ({rc})")
    return out
