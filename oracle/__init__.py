"""FP64 CPU oracle of the MWAX FX correlation hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA contraction); this
module only marshals numpy arrays.  Conventions (Morrison et al. 2023):

* F step (Sec. 2.5.1): unnormalised forward DFT of contiguous frames of L
  samples, channels fftshifted so DC sits at c = L/2 (Sec. 2.6).
* X step (Sec. 2.5.2): V_j[c][n1,n2] = sum_{m in j} X_n1[m,c] conj(X_n2[m,c])
  for n1 >= n2, packed at n1 (n1+1)/2 + n2 (Sec. 2.7).
* Channel averaging (Sec. 2.6): centre-symmetric means of F fine channels
  (F + 1 with half-weight ends for even F), DC left out of the centre one.
* Weights (Sec. 4.1): fraction of an integration's 50 ms sub-blocks populated
  in both inputs of a pair; optional normalisation V / w.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_i8p = ctypes.POINTER(ctypes.c_int8)
_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_f32p = ctypes.POINTER(ctypes.c_float)
_c_f64p = ctypes.POINTER(ctypes.c_double)

_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
            _SRC, "-lm", "-lpthread", "-o", tmp,
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_dft.argtypes = [ctypes.c_int, _c_f64p, _c_f64p]
        lib.orc_fft.argtypes = [ctypes.c_int, _c_f64p, _c_f64p]
        lib.orc_channelise.argtypes = [_c_i8p, ctypes.c_int64, _c_i32p, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, _c_f64p]
        lib.orc_correlate.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int64, ctypes.c_int, _c_f64p]
        lib.orc_correlate_full.argtypes = lib.orc_correlate.argtypes
        lib.orc_correlate_i64.argtypes = [_c_i8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int64, _c_i64p]
        lib.orc_requantise.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       _c_f32p, _c_i8p]
        lib.orc_calibrate.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      _c_f64p, _c_f32p, _c_f32p, _c_i64p]
        lib.orc_round_fp16.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_double, _c_f64p]
        lib.orc_pack_tilebl.argtypes = [_c_f64p, ctypes.c_int, ctypes.c_int, _c_f64p]
        lib.orc_vis_weights.argtypes = [ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, _c_f64p]
        lib.orc_apply_weights.argtypes = [_c_f64p, _c_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_fscrunch.argtypes = [_c_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_f64p]
        lib.orc_delay_correct.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                          _c_f64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_double]
        lib.orc_beamform.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _c_f64p,
                                     ctypes.c_int, _c_f64p]
        lib.orc_incoherent.argtypes = [_c_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _c_f64p]
        for f in ("orc_dft", "orc_fft", "orc_channelise", "orc_correlate", "orc_correlate_full",
                  "orc_correlate_i64", "orc_requantise", "orc_calibrate", "orc_round_fp16",
                  "orc_pack_tilebl", "orc_vis_weights", "orc_apply_weights", "orc_fscrunch",
                  "orc_delay_correct", "orc_beamform", "orc_incoherent"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctype)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _as_pairs(x) -> np.ndarray:
    """complex array -> contiguous float64 [..., 2]."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        out = np.empty(x.shape + (2,), np.float64)
        out[..., 0] = x.real
        out[..., 1] = x.imag
        return out
    return np.ascontiguousarray(x, dtype=np.float64)


def _to_complex(a: np.ndarray) -> np.ndarray:
    return a[..., 0] + 1j * a[..., 1]


def pair_index(n1, n2):
    """Packed lower-triangle index of pair (n1 >= n2)  (Sec. 2.7 reading)."""
    n1 = np.asarray(n1, dtype=np.int64)
    n2 = np.asarray(n2, dtype=np.int64)
    return n1 * (n1 + 1) // 2 + n2


def n_pairs(n_in: int) -> int:
    return n_in * (n_in + 1) // 2


def dft(x) -> np.ndarray:
    """Forward DFT by its definition, O(L^2): complex [L] -> complex [L]."""
    xp = _as_pairs(np.asarray(x, dtype=np.complex128))
    L = xp.shape[0]
    X = np.empty_like(xp)
    _check(_load().orc_dft(L, _ptr(xp, _c_f64p), _ptr(X, _c_f64p)), "dft")
    return _to_complex(X)


def fft(x) -> np.ndarray:
    """Forward FFT by recursive decimation in time (radix 2 for powers of two,
    mixed radix on the smallest prime factor otherwise): complex [L] -> [L]."""
    xp = _as_pairs(np.asarray(x, dtype=np.complex128))
    L = xp.shape[0]
    X = np.empty_like(xp)
    _check(_load().orc_fft(L, _ptr(xp, _c_f64p), _ptr(X, _c_f64p)), "fft")
    return _to_complex(X)


def channelise(volts: np.ndarray, L: int, inputs=None, m0: int = 0, nm: int | None = None,
               use_dft: bool = False) -> np.ndarray:
    """F step on int8 voltages [n_rows][S][2] -> complex128 spectra [nm][L][n_sel].

    Channel axis fftshifted: c = (k + L/2) mod L.  ``inputs`` picks rows.
    """
    v = np.ascontiguousarray(volts, dtype=np.int8)
    assert v.ndim == 3 and v.shape[2] == 2
    n_rows, S = v.shape[0], v.shape[1]
    sel = np.arange(n_rows, dtype=np.int32) if inputs is None else np.asarray(inputs, np.int32)
    sel = np.ascontiguousarray(sel)
    if nm is None:
        nm = S // L - m0
    if (m0 + nm) * L > S:
        raise ValueError("frames exceed the samples given")
    spec = np.empty((nm, L, len(sel), 2), np.float64)
    _check(_load().orc_channelise(_ptr(v, _c_i8p), S, _ptr(sel, _c_i32p), len(sel), m0, nm, L,
                                  int(use_dft), _ptr(spec, _c_f64p)), "channelise")
    return _to_complex(spec)


def correlate(spec: np.ndarray, T: int, threads: int = 1) -> np.ndarray:
    """X step on spectra [M][L][n] -> complex128 [M//T][L][P] (packed)."""
    sp = _as_pairs(spec.astype(np.complex128, copy=False))
    M, L, n = sp.shape[:3]
    vis = np.empty((M // T, L, n_pairs(n), 2), np.float64)
    _check(_load().orc_correlate(_ptr(sp, _c_f64p), M, L, n, T, threads, _ptr(vis, _c_f64p)),
           "correlate")
    return _to_complex(vis)


def correlate_full(spec: np.ndarray, T: int, threads: int = 1) -> np.ndarray:
    """Both triangles: complex128 [M//T][L][n][n], same summation order."""
    sp = _as_pairs(spec.astype(np.complex128, copy=False))
    M, L, n = sp.shape[:3]
    vis = np.empty((M // T, L, n, n, 2), np.float64)
    _check(_load().orc_correlate_full(_ptr(sp, _c_f64p), M, L, n, T, threads,
                                      _ptr(vis, _c_f64p)), "correlate_full")
    return _to_complex(vis)


def correlate_i64(q: np.ndarray, T: int) -> np.ndarray:
    """Exact X step on int8 channelised voltages [M][L][n][2] -> int64 [M//T][L][P][2]."""
    qq = np.ascontiguousarray(q, dtype=np.int8)
    M, L, n = qq.shape[:3]
    vis = np.empty((M // T, L, n_pairs(n), 2), np.int64)
    _check(_load().orc_correlate_i64(_ptr(qq, _c_i8p), M, L, n, T, _ptr(vis, _c_i64p)),
           "correlate_i64")
    return vis


def requantise(spec: np.ndarray, inv_s) -> np.ndarray:
    """q = clamp(round_half_even(x * inv_s[c]), -127, 127) -> int8 [M][L][n][2]."""
    sp = _as_pairs(spec.astype(np.complex128, copy=False))
    M, L, n = sp.shape[:3]
    inv = np.ascontiguousarray(inv_s, dtype=np.float32)
    assert inv.shape == (L,)
    q = np.empty((M, L, n, 2), np.int8)
    _check(_load().orc_requantise(_ptr(sp, _c_f64p), M, L, n, _ptr(inv, _c_f32p),
                                  _ptr(q, _c_i8p)), "requantise")
    return q


def calibrate(spec: np.ndarray, prev=None, return_populated: bool = False):
    """Per-channel (sigma^2 [L] f64, s [L] f32, inv_s [L] f32) from spectra [M][L][n].

    Frames (spectrum m of input n) whose L values are all zero are left out of
    the mean.  If no frame is populated the scales ``prev`` = (s, inv_s) of the
    previous integration are returned (ones if there is none)."""
    sp = _as_pairs(spec.astype(np.complex128, copy=False))
    M, L, n = sp.shape[:3]
    sig2 = np.empty(L, np.float64)
    s = np.empty(L, np.float32)
    inv = np.empty(L, np.float32)
    pop = np.zeros(1, np.int64)
    _check(_load().orc_calibrate(_ptr(sp, _c_f64p), M, L, n, _ptr(sig2, _c_f64p),
                                 _ptr(s, _c_f32p), _ptr(inv, _c_f32p), _ptr(pop, _c_i64p)), "calibrate")
    if pop[0] == 0 and prev is not None:
        s = np.array(prev[0], np.float32, copy=True)
        inv = np.array(prev[1], np.float32, copy=True)
    if return_populated:
        return sig2, s, inv, int(pop[0])
    return sig2, s, inv


def round_fp16(x, scale: float = 1.0) -> np.ndarray:
    """Round x*scale to the nearest binary16 value (ties to even), as float64."""
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    y = np.empty_like(xa)
    _check(_load().orc_round_fp16(_ptr(xa, _c_f64p), xa.size, float(scale), _ptr(y, _c_f64p)),
           "round_fp16")
    return y


def pack_tilebl(vis: np.ndarray, n_tiles: int) -> np.ndarray:
    """Packed input-level [L][P] -> tile-baseline view [B][L][4] (XX, XY, YX, YY)."""
    vp = _as_pairs(np.asarray(vis, dtype=np.complex128))
    L = vp.shape[0]
    B = n_tiles * (n_tiles + 1) // 2
    out = np.empty((B, L, 4, 2), np.float64)
    _check(_load().orc_pack_tilebl(_ptr(vp, _c_f64p), L, n_tiles, _ptr(out, _c_f64p)),
           "pack_tilebl")
    return _to_complex(out)


def fx_correlate(volts: np.ndarray, L: int, T: int, threads: int = 1) -> np.ndarray:
    """Whole FP64 chain: voltages [n][S][2] -> packed visibilities [S//L//T][L][P]."""
    spec = channelise(volts, L)
    return correlate(spec, T, threads)


def _inputs_of(P: int) -> int:
    """Number of inputs n with n (n + 1) / 2 = P pairs."""
    n = int(round(((8 * P + 1) ** 0.5 - 1) / 2))
    if n * (n + 1) // 2 != P:
        raise ValueError(f"{P} is not a pair count n (n + 1) / 2")
    return n


def vis_weights(flags: np.ndarray, subs_per_int: int) -> np.ndarray:
    """Occupancy weights (Sec. 4.1): flags [n][n_ints * subs] (nonzero = zeroed
    sub-block) -> [n_ints][P] fraction of sub-blocks populated in both inputs."""
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    n, nsub = f.shape
    if subs_per_int < 1 or nsub % subs_per_int:
        raise ValueError("flags must hold a whole number of integrations")
    n_ints = nsub // subs_per_int
    w = np.empty((n_ints, n_pairs(n)), np.float64)
    _check(_load().orc_vis_weights(f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), n,
                                   int(subs_per_int), n_ints, _ptr(w, _c_f64p)), "vis_weights")
    return w


def apply_weights(vis, w) -> np.ndarray:
    """Normalised visibilities (Sec. 4.1): [n_ints][L][P] / w [n_ints][P] where w > 0."""
    vp = _as_pairs(np.asarray(vis, dtype=np.complex128)).copy()
    n_ints, L, P = vp.shape[:3]
    wa = np.ascontiguousarray(w, dtype=np.float64)
    if wa.shape != (n_ints, P):
        raise ValueError("weights must be [n_ints][P]")
    n = _inputs_of(P)
    _check(_load().orc_apply_weights(_ptr(vp, _c_f64p), _ptr(wa, _c_f64p), n, L, n_ints),
           "apply_weights")
    return _to_complex(vp)


def fscrunch(vis, F: int) -> np.ndarray:
    """Channel averaging (Sec. 2.6): [n_ints][L][P] -> [n_ints][L/F][P]."""
    vp = _as_pairs(np.asarray(vis, dtype=np.complex128))
    n_ints, L, P = vp.shape[:3]
    if F < 1 or L % F:
        raise ValueError("F must divide L")
    n = _inputs_of(P)
    out = np.empty((n_ints, L // F, P, 2), np.float64)
    _check(_load().orc_fscrunch(_ptr(vp, _c_f64p), n, L, n_ints, int(F), _ptr(out, _c_f64p)), "fscrunch")
    return _to_complex(out)


def delay_correct(spec, delays, step_samples: int, nu_over_fs: float, m0: int = 0) -> np.ndarray:
    """Fractional delay and phase correction (Sec. 2.5.1, Sec. 4.3) of spectra
    [M][L][n] (frame m at stream samples (m0 + m) L ..): each sample of input k
    times exp(-2 pi i ((c - L/2) / L + nu_c / f_s) d) with d = delays[k][step]
    in samples, step = stream sample // step_samples."""
    sp = _as_pairs(np.asarray(spec, dtype=np.complex128)).copy()
    M, L, n = sp.shape[:3]
    d = np.ascontiguousarray(delays, dtype=np.float64)
    if d.ndim != 2 or d.shape[0] != n:
        raise ValueError("delays must be [n_inputs][n_steps]")
    _check(_load().orc_delay_correct(_ptr(sp, _c_f64p), M, L, n, int(m0), _ptr(d, _c_f64p), d.shape[1],
                                     int(step_samples), float(nu_over_fs)), "delay_correct")
    return _to_complex(sp)


def beamform(spec, weights) -> np.ndarray:
    """Coherent tied-array beams (Sec. 4.4): spectra [M][L][n] and complex
    weights [L][nb][n] -> beams [M][L][nb] = sum_n w spec."""
    sp = _as_pairs(np.asarray(spec, dtype=np.complex128))
    M, L, n = sp.shape[:3]
    w = _as_pairs(np.asarray(weights, dtype=np.complex128))
    if w.shape[0] != L or w.shape[2] != n:
        raise ValueError("weights must be [L][n_beams][n_inputs]")
    nb = w.shape[1]
    out = np.empty((M, L, nb, 2), np.float64)
    _check(_load().orc_beamform(_ptr(sp, _c_f64p), M, L, n, _ptr(w, _c_f64p), nb, _ptr(out, _c_f64p)),
           "beamform")
    return _to_complex(out)


def incoherent(spec, t_avg: int, f_avg: int) -> np.ndarray:
    """Incoherent beam (Sec. 4.4): detected power summed over the inputs of each
    polarisation, t_avg spectra and f_avg channels -> [M/t_avg][L/f_avg][2]."""
    sp = _as_pairs(np.asarray(spec, dtype=np.complex128))
    M, L, n = sp.shape[:3]
    out = np.empty((M // max(t_avg, 1), L // max(f_avg, 1), 2), np.float64)
    _check(_load().orc_incoherent(_ptr(sp, _c_f64p), M, L, n, int(t_avg), int(f_avg), _ptr(out, _c_f64p)),
           "incoherent")
    return out
