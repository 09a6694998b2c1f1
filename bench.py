#!/usr/bin/env python3
"""Benchmark of the FX correlation hot path on one MI355X.

Workload (one step = one pass of the whole hot path over one 8 s block):
256 tiles x 2 pols = 512 inputs, one 1.28 MHz coarse channel, 8 s of complex
int8 voltages (10.24 M samples per input, Gaussian sigma = 8 plus three point
sources, seeded, generated on the device), 128-point FFT (10 kHz channels),
one 8 s integration.  Per step: channelise (per-integration int8 scale
calibration, FFT, requantise, transpose) -> correlate (int8 MFMA X-engine) ->
integrate (pack the 131,328-pair lower triangle x 128 channels).

Printed: one JSON line with the X-engine CMAC/s of the whole step (value), the
real-time factor, the dominant kernel's roofline fraction (HIP-event timing on
the plan's stream), the FP16 / FP32-plain X-engines on the same block, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0,
    "int8_tops": 5000.0,
    "fp16_tflops": 2500.0,
    "fp32_vector_tflops": 157.3,
}
N_TILES, L, SECONDS, F_S = 256, 128, 8.0, 1.28e6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_channel_256tiles_8s.json")
TRAFFIC_WEIGHTS_FILE = os.path.join(ROOT, "profiles", "traffic_weights_256tiles_8s.json")


def measured_traffic(key, path=TRAFFIC_FILE):
    """HBM bytes per launch of kernel `key` from the committed counter summary, or
    None when there is none or the kernel's source has changed since it was taken."""
    from paper_2303_11557_amd import profiling
    try:
        ent = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not ent or ent.get("source_sha") != profiling.source_sha(key.split("_")[0]):
        return None
    return ent["hbm_bytes_per_launch"]


# Batch workload: 24 coarse channels as uneven instances (tile counts, FFT
# lengths, integration times cycled), each with 8 s of sigma = 8 voltages and
# one seeded point source; run as one batch in 1 s calls.
BATCH_TILES, BATCH_L, BATCH_TAU = (64, 128, 256), (32, 128, 1024), (0.5, 2.0, 8.0)
BATCH_CALL_S = 1.0


def batch_instances():
    return [(BATCH_TILES[i % 3], BATCH_L[(i // 3) % 3], BATCH_TAU[(i // 9) % 3]) for i in range(24)]


def cpu_baseline(volts, L, seconds, what, accuracy=None):
    """The FP64 oracle (channelise + packed-triangle X-engine) timed on the host
    cores over the first spectra of ``volts`` (a device int8 [n][S][2] tensor),
    the sample grown until it takes about ``seconds``; then on one thread over a
    smaller sample.  ``accuracy(n_spec, spec, vis)``, if given, receives the
    oracle's spectra and visibilities of the multi-threaded sample (one
    integration over its n_spec spectra) and returns the GPU paths' measured
    error against them, reported under "accuracy"."""
    import oracle
    n_in = volts.shape[0]
    P = n_in * (n_in + 1) // 2
    threads = max(1, min(16, os.cpu_count() or 1))
    max_spec = min(2048, volts.shape[1] // L)
    v_host = volts[:, : max_spec * L].cpu().numpy()
    kept = {}

    def oracle_rate(n_spec, th, keep=False):
        t0 = time.perf_counter()
        spec = oracle.channelise(v_host, L, nm=n_spec)
        vis = oracle.correlate(spec, n_spec, threads=th)
        dt = time.perf_counter() - t0
        if keep:
            kept.update(n_spec=n_spec, spec=spec, vis=vis)
        return dt

    def grow(th, target, keep=False):
        n_spec = 2
        dt = oracle_rate(n_spec, th, keep)
        while dt < 0.5 * target and n_spec < max_spec:
            n_spec = int(min(max_spec, max(2 * n_spec, n_spec * target / max(dt, 1e-3))))
            dt = oracle_rate(n_spec, th, keep)
        return n_spec, dt

    n_spec, dt = grow(threads, seconds, keep=accuracy is not None)
    acc = None
    if accuracy is not None:
        acc = accuracy(kept["n_spec"], kept["spec"], kept["vis"])
        kept.clear()
    n1, dt1 = grow(1, seconds / 3)
    out = {"value": P * n_spec * L / dt, "unit": "CMAC/s", "cores": threads, "kind": "oracle",
           "sample": f"all {n_in} inputs, all {L} channels, first {n_spec} spectra "
                     f"({n_spec * L} samples) of {what}; FP64 FFT + packed triangle; {dt:.1f} s wall",
           "value_1_thread": P * n1 * L / dt1, "sample_1_thread": f"first {n1} spectra, {dt1:.1f} s wall"}
    if acc is not None:
        out["accuracy"] = acc
    return out


def gpu_error_vs_oracle(volts, L, n_spec, spec, vis_ref):
    """Measured error of every X-engine precision against the FP64 oracle on one
    integration over the first n_spec spectra of the block, all pairs: the
    largest per-channel relative Frobenius error; for INT8 also the fraction of
    codes at the clip level +-127 and the codes that differ from the oracle's
    requantisation of its FP64 spectra (with its own scale calibration)."""
    import numpy as np
    import torch

    import oracle
    from paper_2303_11557_amd.mwax import Plan, make_config
    n_in = volts.shape[0]
    ref = vis_ref[0]
    den = np.linalg.norm(ref, axis=-1)
    out = {"integration_spectra": int(n_spec)}
    for prec in ("int8", "fp16", "fp32"):
        with Plan(make_config(n_in // 2, L=L, T=n_spec, xprec=prec, max_samples=n_spec * L)) as p:
            p.channelise(volts[:, : n_spec * L])
            codes = p.read_channelised().cpu().numpy() if prec == "int8" else None
            ncal = p.dims.cal_spectra
            p.correlate()
            got = p.integrate(1)[0].cpu().numpy().astype(np.complex128)
        err = np.linalg.norm(got - ref, axis=-1) / den
        ent = {"max_rel_frob_per_channel": float(err.max()), "median_rel_frob_per_channel": float(np.median(err))}
        if prec == "int8":
            _, _, inv_o = oracle.calibrate(spec[:ncal])
            qo = oracle.requantise(spec, inv_o)
            nd = int(np.count_nonzero(codes != qo))
            ent.update(codes=int(codes.size), codes_differing_from_fp64_requantisation=nd,
                       max_code_difference=int(np.abs(codes.astype(np.int16) - qo.astype(np.int16)).max()),
                       clip_fraction=float(np.count_nonzero(np.abs(codes.astype(np.int16)) == 127) / codes.size))
            del codes, qo
        out[prec] = ent
        torch.cuda.empty_cache()
    return out


def copy_bandwidth():
    """Device-to-device copy rate (bytes read + written per second) of a 4 GiB
    buffer, timed with HIP events: the practical HBM ceiling on this machine."""
    import torch
    src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="channel",
                    choices=["channel", "batch", "stream", "weights", "fscrunch", "ultrafine", "beamform"],
                    help="channel: one coarse channel, 256 tiles, 8 s (the headline metric); "
                         "batch: 24 uneven instances as one batch; stream: 24 channels streamed in 8 s blocks")
    ap.add_argument("--stream-rounds", type=int, default=15, help="8 s blocks per channel, flat out")
    ap.add_argument("--stream-paced-rounds", type=int, default=15,
                    help="8 s blocks per channel over the host link: flat out, then real-time paced (15 = 120 s)")
    ap.add_argument("--stream-budget-gb", type=float, default=64.0, help="HBM budget of the block pool")
    ap.add_argument("--batch-call-s", type=float, default=BATCH_CALL_S, help="seconds of voltages per batch call")
    ap.add_argument("--stream-call-s", type=float, default=2.0,
                    help="seconds of voltages per plan call (stream; 2 s = one integration)")
    ap.add_argument("--fft-len", type=int, default=L, help="channel workload: FFT length (default 128)")
    ap.add_argument("--ultra-modes", default="all", help="ultrafine: comma list of 40kHz_250ms,10kHz_1s,1kHz_8s")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--xprec", default="int8", choices=["int8", "fp16", "fp32"])
    ap.add_argument("--variants", default="fp16,fp32",
                    help="other X-engine precisions to time on the same block ('none' to skip)")
    ap.add_argument("--variant-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle CPU time")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 4 GiB device-to-device once (calibrates HBM byte counters)")
    return ap.parse_args()


def main_batch(args):
    import torch

    import synth
    from paper_2303_11557_amd import mwax
    from paper_2303_11557_amd.mwax import Batch, make_config

    torch.cuda.set_device(0)
    mwax.lib()
    S = int(SECONDS * F_S)
    chunk = int(args.batch_call_s * F_S)
    ncalls = S // chunk
    inst = batch_instances()
    cfgs = [make_config(t, L=Lc, int_time_s=tau, xprec=args.xprec, max_samples=chunk) for (t, Lc, tau) in inst]
    dims = [mwax.derive(c) for c in cfgs]
    cmac_per_step = sum(d.n_pairs * S for d in dims)
    volts = []
    for i, (t, Lc, tau) in enumerate(inst):
        v = torch.empty((2 * t, S, 2), dtype=torch.int8, device="cuda")
        synth.device_volts(v, seed=synth.MWAX_SEED + 3 + (i << 16),
                           sources=[synth.Source(3.0, (7 * i) % Lc - Lc // 2)], L=Lc)
        volts.append(v)
    torch.cuda.synchronize()
    outs = [torch.empty((-(-chunk // (d.spectra_per_int * d.fft_len)) + 1, d.fft_len, d.n_pairs),
                        dtype=torch.complex64, device="cuda") for d in dims]

    with Batch(cfgs) as b:
        t0 = time.perf_counter()
        kc, grid = b.autotune([v[:, :chunk] for v in volts], trials=3)
        tune_s = time.perf_counter() - t0
        tiles = b.tiles()

        def step():
            for k in range(ncalls):
                b.run([v[:, k * chunk:(k + 1) * chunk] for v in volts])
                for i, p in enumerate(b.plans):
                    p.integrate(outs[i].shape[0], out=outs[i])

        for _ in range(args.warmup):
            step()
        b.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        b.sync()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        # one more pass with the launches issued one by one, for per-kernel times
        b.set_graph(False)
        b.set_timing(True)
        for fam in range(5):
            b.kernel_time(fam)
        step()
        fam = {name: b.kernel_time(i) for i, name in
               ((0, "fengine"), (1, "xengine"), (3, "calib"), (4, "call"))}
        # the same eager pass with every instance on each tile edge, for the
        # record of what the tuner's tile choice is worth
        x_by_tile = {}
        for te in (128, 64):
            b.set_tiles([te] * len(cfgs))
            b.kernel_time(1)
            step()
            x_by_tile[te] = round(b.kernel_time(1)[0] / ncalls, 3)
        b.set_tiles(tiles)
        b.set_timing(False)
        b.set_graph(True)
        eager_ms = fam["call"][0]

    x_ms, x_n = fam["xengine"]
    x_ops_launch = 8.0 * cmac_per_step / max(x_n, 1)
    x_avg = x_ms / max(x_n, 1)
    x_ach = x_ops_launch / (x_avg / 1e3) / 1e12
    x_peak = PEAK["int8_tops"] if args.xprec == "int8" else PEAK["fp16_tflops"]
    b_out = 2 if args.xprec == "int8" else 4
    f_ms, f_n = fam["fengine"]
    f_bytes = sum(d.n_inputs * S * (2 + b_out) for d in dims)
    f_gbs = f_bytes / (f_ms / 1e3) / 1e9
    roof_x = {"kernel": f"xengine_batch_{args.xprec}", "bound": "mfma", "achieved": round(x_ach, 2),
              "peak": x_peak, "unit": "TFLOP/s", "frac": round(x_ach / x_peak, 4), "traffic": None,
              "avg_launch_ms": round(x_avg, 4), "launches": x_n, "ops_per_launch": x_ops_launch}
    roof_f = {"kernel": f"fengine_batch_{args.xprec}", "bound": "hbm", "achieved": round(f_gbs, 1),
              "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(f_gbs / PEAK["hbm_gbs"], 4),
              "traffic": None, "ms_per_step": round(f_ms, 3), "launches": f_n, "bytes_per_step": f_bytes}
    dominant, other = (roof_x, roof_f) if x_ms >= f_ms else (roof_f, roof_x)
    cpu = None if args.no_cpu_baseline else cpu_baseline(volts[2], BATCH_L[0], args.cpu_seconds,
                                                         "instance 2 (256 tiles, 32-pt FFT)")
    line = {
        "metric": "X-engine CMAC/s & real-time factor, 24 uneven instances in one batch",
        "value": cmac_per_step / (ms / 1e3), "unit": "CMAC/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.xprec,
        "data": "synthetic",
        "config": {"workload": "24 instances: tiles {64,128,256} x 2 pols, FFT {32,128,1024}, integrations "
                               "{0.5,2,8} s (cycled), 8 s of complex int8 sigma=8 voltages + 1 source each, "
                               f"one batch, {args.batch_call_s:g} s calls",
                   "instances": [list(x) for x in inst], "cmac_per_step": cmac_per_step,
                   "input_bytes": sum(v.numel() for v in volts)},
        "rtf": round(SECONDS / (ms / 1e3), 2),
        "graph_replay": True,
        "eager_ms_per_step": round(eager_ms, 3),
        "calibration_ms_per_step": round(fam["calib"][0], 3),
        "autotune": {"kchunk": kc, "tile": tiles, "grid": grid, "seconds": round(tune_s, 2),
                     "xengine_ms_per_call": {"tuned": round(x_ms / max(ncalls, 1), 3),
                                             "all_tile_128": x_by_tile[128], "all_tile_64": x_by_tile[64]}},
        "roofline": dominant, "roofline_other": other,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# Weights workload: one 8 s block of one coarse channel at 256 tiles, 2 s
# integrations (four visibility sets of 128 channels x 131,328 pairs), 50 ms
# zeroing flags (160 per input per block, 1 % lost, input 0 lost throughout).
WEIGHTS_INT_S, WEIGHTS_SUB_S, WEIGHTS_LOSS = 2.0, 0.05, 0.01


def main_weights(args):
    import numpy as np
    import torch

    import synth
    from paper_2303_11557_amd import mwax

    torch.cuda.set_device(0)
    mwax.lib()
    n_in = 2 * N_TILES
    P = n_in * (n_in + 1) // 2
    n_ints = int(round(SECONDS / WEIGHTS_INT_S))
    subs = int(round(WEIGHTS_INT_S / WEIGHTS_SUB_S))
    flags_h = synth.zero_flags(n_in, n_ints * subs, WEIGHTS_LOSS, seed=synth.MWAX_SEED + 7)
    flags_h[0, :] = 1
    flags = torch.from_numpy(flags_h).cuda()
    gen = torch.Generator(device="cuda").manual_seed(synth.MWAX_SEED + 8)
    vis = torch.randn((n_ints, L, P), dtype=torch.complex64, device="cuda", generator=gen)
    if args.copy_probe:
        copy_bandwidth()                 # a 4 GiB copy of known size scales the HBM counters
    w = torch.empty((n_ints, P), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        mwax.vis_weights(flags, subs, out=w, stream=stream)
        mwax.apply_weights(vis, w, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # per-kernel durations: HIP events on the stream the kernels run on
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for e in ev:
        e[0].record(stream)
        mwax.vis_weights(flags, subs, out=w, stream=stream)
        e[1].record(stream)
        mwax.apply_weights(vis, w, stream=stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    w_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / len(ev)
    a_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / len(ev)
    a_bytes = 2 * n_ints * L * P * 8 + n_ints * P * 4
    w_bytes = n_in * n_ints * subs + n_ints * P * 4
    a_gbs = a_bytes / (a_ms / 1e3) / 1e9
    w_gbs = w_bytes / (w_ms / 1e3) / 1e9
    step_bytes = a_bytes + w_bytes
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        vis_h = vis.cpu().numpy()
        t0 = time.perf_counter()
        reps = 0
        while True:
            wo = oracle.vis_weights(flags_h, subs)
            oracle.apply_weights(vis_h, wo)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= args.cpu_seconds or reps >= 32:
                break
        cpu = {"value": reps * step_bytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole step (weights of {n_in} inputs x {n_ints * subs} sub-blocks, normalisation "
                         f"of {n_ints} x {L} x {P} visibilities) {reps} times, {dt:.1f} s wall"}
    line = {
        "metric": "visibility weights + normalisation throughput (algorithmic HBM bytes/s)",
        "value": step_bytes / (ms / 1e3) / 1e9, "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256 tiles x 2 pols, 1 coarse channel, 128 fine channels, one 8 s block: "
                               "four 2 s visibility sets, 50 ms zeroing flags (1 % lost, input 0 lost)",
                   "n_inputs": n_in, "n_ints": n_ints, "subs_per_int": subs, "bytes_per_step": step_bytes},
        "rtf": round(SECONDS / (ms / 1e3), 1),
        "roofline": {"kernel": "apply_weights_kernel", "bound": "hbm", "achieved": round(a_gbs, 1),
                     "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(a_gbs / PEAK["hbm_gbs"], 4),
                     "traffic": measured_traffic("weights_apply", TRAFFIC_WEIGHTS_FILE),
                     "avg_launch_ms": round(a_ms, 4), "bytes_per_launch": a_bytes},
        "roofline_other": {"kernel": "vis_weights_kernel", "bound": "hbm", "achieved": round(w_gbs, 1),
                           "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(w_gbs / PEAK["hbm_gbs"], 4),
                           "traffic": measured_traffic("weights_occupancy", TRAFFIC_WEIGHTS_FILE),
                           "avg_launch_ms": round(w_ms, 4), "bytes_per_launch": w_bytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# Averaging workload: one 8 s integration of one coarse channel at 256 tiles
# with 1024 fine channels (1.25 kHz), averaged by 8 to 128 channels of 10 kHz.
AVG_L, AVG_F = 1024, 8
TRAFFIC_AVG_FILE = os.path.join(ROOT, "profiles", "traffic_fscrunch_256tiles_8s.json")


def main_fscrunch(args):
    import numpy as np
    import torch

    import synth
    from paper_2303_11557_amd import mwax

    torch.cuda.set_device(0)
    mwax.lib()
    n_in = 2 * N_TILES
    P = n_in * (n_in + 1) // 2
    N = AVG_L // AVG_F
    gen = torch.Generator(device="cuda").manual_seed(synth.MWAX_SEED + 10)
    vis = torch.randn((1, AVG_L, P), dtype=torch.complex64, device="cuda", generator=gen)
    out = torch.empty((1, N, P), dtype=torch.complex64, device="cuda")
    if args.copy_probe:
        copy_bandwidth()                 # a 4 GiB copy of known size scales the HBM counters
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        mwax.fscrunch(vis, AVG_F, out=out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mwax.fscrunch(vis, AVG_F, out=out, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in ev:
        e0.record(stream)
        mwax.fscrunch(vis, AVG_F, out=out, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    k_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)
    nbytes = AVG_L * P * 8 + N * P * 8
    gbs = nbytes / (k_ms / 1e3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n_s = 256                        # pairs of the first 256 inputs: the first 32,896 of the triangle
        P_s = n_s * (n_s + 1) // 2
        sample = np.ascontiguousarray(vis[:, :, :P_s].cpu().numpy())
        t0, reps = time.perf_counter(), 0
        while True:
            oracle.fscrunch(sample, AVG_F)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= args.cpu_seconds or reps >= 64:
                break
        s_bytes = AVG_L * P_s * 8 + N * P_s * 8
        cpu = {"value": reps * s_bytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the pairs of the first {n_s} inputs ({P_s} of {P}) x {AVG_L} channels, averaged by "
                         f"{AVG_F}, {reps} times, {dt:.1f} s wall"}
    line = {
        "metric": "channel averaging throughput (algorithmic HBM bytes/s)",
        "value": nbytes / (ms / 1e3) / 1e9, "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256 tiles x 2 pols, 1 coarse channel, one 8 s integration of 1024 fine channels "
                               "(1.25 kHz) averaged by 8 to 128 x 10 kHz",
                   "n_inputs": n_in, "fine_channels": AVG_L, "fscrunch": AVG_F, "bytes_per_step": nbytes},
        "rtf": round(SECONDS / (ms / 1e3), 1),
        "roofline": {"kernel": "fscrunch_kernel", "bound": "hbm", "achieved": round(gbs, 1),
                     "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(gbs / PEAK["hbm_gbs"], 4),
                     "traffic": measured_traffic("average_fscrunch", TRAFFIC_AVG_FILE),
                     "avg_launch_ms": round(k_ms, 4), "bytes_per_launch": nbytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# Ultra-fine workload: the paper's F-engine (Sec. 2.5.1: 6,400-point FFT, 200 Hz
# channels) at 256 tiles on one 8 s block, X-engine on the 6,400 channels, and
# the averaging of each integration to the output width (Sec. 2.6).  The three
# output modes the paper benchmarks (Table 2): 40 kHz / 250 ms, 10 kHz / 1 s,
# 1 kHz / 8 s.
ULTRA_MODES = {"40kHz_250ms": (200, 0.25), "10kHz_1s": (50, 1.0), "1kHz_8s": (5, 8.0)}
ULTRA_L = 6400


def main_ultrafine(args):
    import torch

    import synth
    from paper_2303_11557_amd import mwax
    from paper_2303_11557_amd.mwax import Plan, make_config

    torch.cuda.set_device(0)
    mwax.lib()
    S = int(SECONDS * F_S)
    n_in = 2 * N_TILES
    P = n_in * (n_in + 1) // 2
    cmac = P * S
    volts = torch.empty((n_in, S, 2), dtype=torch.int8, device="cuda")
    synth.device_volts(volts, seed=synth.MWAX_SEED + 2,
                       sources=[synth.Source(2.0, -370), synth.Source(3.0, 50), synth.Source(4.0, 2010)], L=ULTRA_L)
    torch.cuda.synchronize()
    modes = {}
    b_out = {"int8": 2, "fp16": 4, "fp32": 8}[args.xprec]
    x_peak = {"int8": PEAK["int8_tops"], "fp16": PEAK["fp16_tflops"], "fp32": PEAK["fp32_vector_tflops"]}[args.xprec]
    # where the averaging happens: inside the X-engine (mwax_set_averaging; the
    # fine-channel visibilities are never formed; INT8 and FP16) or at emission
    # (mwax_integrate_averaged over the fine-channel integrators)
    paths = ("xengine", "emission") if args.xprec != "fp32" else ("emission",)
    for name, (F, tau) in ULTRA_MODES.items():
        if args.ultra_modes != "all" and name not in args.ultra_modes.split(","):
            continue
        # calls of 1 s, or of the whole integration when it is longer (one
        # X-engine flush per integration); every completed integration is
        # emitted already averaged to the output width
        call = int(max(1.0, tau) * F_S)
        cfg = make_config(N_TILES, L=ULTRA_L, int_time_s=tau, xprec=args.xprec, max_samples=call)
        n_ints = int(round(SECONDS / tau))
        res = {}
        for path in paths:
            with Plan(cfg) as p:
                out = torch.empty((n_ints, ULTRA_L // F, P), dtype=torch.complex64, device="cuda")
                if path == "xengine":
                    p.set_averaging(F)

                def step():
                    j = 0
                    for off in range(0, S, call):
                        p.channelise(volts[:, off:off + call])
                        p.correlate()
                        if path == "xengine":
                            j += p.integrate(n_ints - j, out=out[j:]).shape[0]
                        else:
                            j += p.integrate_averaged(F, n_ints - j, out=out[j:]).shape[0]
                    return j

                for _ in range(args.warmup):
                    step()
                p.sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    assert step() == n_ints
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / args.steps
                # per-kernel durations (HIP events on the plan's stream) in one more step
                p.set_timing(True)
                for fam in range(4):
                    p.kernel_time(fam)
                step()
                p.sync()
                fam = {name_: p.kernel_time(i) for i, name_ in enumerate(("fengine", "xengine", "pack", "calib"))}
                p.set_timing(False)
            f_ms, f_n = fam["fengine"]
            x_ms, x_n = fam["xengine"]
            p_ms, p_n = fam["pack"]
            f_bytes = n_in * S * (2 + b_out)           # algorithmic: voltages in, channel-major spectra out
            x_ops = 8.0 * cmac
            if path == "xengine":                      # FP64 output-channel integrators in, averages out
                emit_bytes = n_ints * (ULTRA_L // F) * P * (16 + 8)
            else:                                      # fine-channel integrators in, averages out
                integ_b = 8 if args.xprec == "int8" and tau * F_S / ULTRA_L <= 65536 else 16
                emit_bytes = n_ints * (ULTRA_L * P * integ_b + (ULTRA_L // F) * P * 8)
            kern = {
                "fengine": {"bound": "hbm", "ms": round(f_ms, 3), "launches": f_n, "bytes": f_bytes,
                            "achieved": round(f_bytes / (f_ms / 1e3) / 1e9, 1), "unit": "GB/s",
                            "frac": round(f_bytes / (f_ms / 1e3) / 1e9 / PEAK["hbm_gbs"], 4)},
                "xengine": {"bound": "mfma", "ms": round(x_ms, 3), "launches": x_n, "ops": x_ops,
                            "achieved": round(x_ops / (x_ms / 1e3) / 1e12, 2), "unit": "TFLOP/s",
                            "frac": round(x_ops / (x_ms / 1e3) / 1e12 / x_peak, 4)},
                "emit": {"bound": "hbm", "ms": round(p_ms, 3), "launches": p_n, "bytes": emit_bytes,
                         "achieved": round(emit_bytes / (p_ms / 1e3) / 1e9, 1), "unit": "GB/s",
                         "frac": round(emit_bytes / (p_ms / 1e3) / 1e9 / PEAK["hbm_gbs"], 4)},
                "calib_ms": round(fam["calib"][0], 3),
            }
            dom = max(("fengine", "xengine", "emit"), key=lambda k: kern[k]["ms"])
            res[path] = {"ms_per_8s": round(ms, 3), "rtf_per_channel": round(SECONDS / (ms / 1e3), 2),
                         "rtf_24_channels": round(SECONDS / (ms / 1e3) / 24.0, 3),
                         "cmac_per_s": cmac / (ms / 1e3), "dominant": dom, "kernels": kern}
            torch.cuda.empty_cache()
        best = min(res, key=lambda k: res[k]["ms_per_8s"])
        modes[name] = {"fscrunch": F, "int_time_s": tau, "call_s": call / F_S, "integrations": n_ints,
                       "output_channels": ULTRA_L // F, "averaging": best, **res[best], "paths": res}
    cpu = None if args.no_cpu_baseline else cpu_baseline(volts, ULTRA_L, args.cpu_seconds,
                                                         "the same 8 s block at 6,400 channels")
    head = modes.get("10kHz_1s") or next(iter(modes.values()))
    dk = head["kernels"][head["dominant"]]
    line = {
        "metric": "real-time factor of the paper's output modes, 6,400-point F-engine, 256 tiles",
        "value": head["cmac_per_s"], "unit": "CMAC/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_8s"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.xprec, "data": "synthetic",
        "config": {"workload": "256 tiles x 2 pols, 1 coarse channel, 8 s block of complex int8 sigma=8 "
                               "voltages + 3 sources, 6,400-pt FFT (200 Hz), plan calls of max(1 s, integration), "
                               "every integration averaged to the output width inside the X-engine or at emission "
                               "(the faster is the mode's figure, both are reported; modes: 40 kHz/250 ms, "
                               "10 kHz/1 s, 1 kHz/8 s)",
                   "fft_len": ULTRA_L, "samples": S, "cmac_per_8s": cmac},
        "roofline": {"kernel": head["dominant"], "bound": dk["bound"], "achieved": dk["achieved"],
                     "peak": PEAK["hbm_gbs"] if dk["bound"] == "hbm" else PEAK[{"int8": "int8_tops", "fp16": "fp16_tflops", "fp32": "fp32_vector_tflops"}[args.xprec]],
                     "unit": dk["unit"], "frac": dk["frac"], "traffic": None, "ms_per_step": dk["ms"]},
        "modes": modes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# Beamformer workload: 256 tiles, one coarse channel, 1 s of voltages through
# the INT8 F-engine at 128 channels (10 kHz), then BEAMS coherent beams (Sec.
# 4.4: many pointings at the full coarse-channel bandwidth) and one incoherent
# beam at 1 ms x 40 kHz resolution (t_avg 10 spectra, f_avg 4 channels).
BEAMS = 32


def main_beamform(args):
    import numpy as np
    import torch

    import synth
    from paper_2303_11557_amd import mwax
    from paper_2303_11557_amd.mwax import Plan, make_config

    torch.cuda.set_device(0)
    mwax.lib()
    S = int(F_S)
    n_in = 2 * N_TILES
    M = S // L
    volts = torch.empty((n_in, S, 2), dtype=torch.int8, device="cuda")
    synth.device_volts(volts, seed=synth.MWAX_SEED + 11, sources=[synth.Source(3.0, 17)], L=L)
    taus = synth.source_delays(n_in, synth.MWAX_SEED + 11)
    nu = synth.NU_C + (np.arange(L) - L // 2) * F_S / L
    # beam 0 phases every path up for the source's delays; the others point elsewhere
    tau_b = np.stack([taus] + [taus * np.cos(0.3 * k) for k in range(1, BEAMS)])    # [BEAMS][n_in]
    w = np.exp(2j * np.pi * nu[:, None, None] * tau_b[None, :, :]).astype(np.complex64)   # [L][BEAMS][n_in]
    d_w = torch.from_numpy(w).cuda()
    stream = torch.cuda.current_stream()
    with Plan(make_config(N_TILES, L=L, T=M, xprec=args.xprec, max_samples=S)) as p:
        beams = torch.empty((M, L, BEAMS), dtype=torch.complex64, device="cuda")
        inc = torch.empty((M // 10, L // 4, 2), dtype=torch.float32, device="cuda")
        p.channelise(volts)
        p.correlate()
        p.sync()

        def step():
            p.beamform(d_w, out=beams)
            p.beamform_incoherent(10, 4, out=inc)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        for e in ev:
            e[0].record(stream)
            p.beamform(d_w, out=beams)
            e[1].record(stream)
            p.beamform_incoherent(10, 4, out=inc)
            e[2].record(stream)
        torch.cuda.synchronize()
        b_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / len(ev)
        i_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / len(ev)
        g = beams[:, (17 + L // 2) % L, :].abs().pow(2).mean(0).cpu().numpy()
    cmac = float(n_in) * BEAMS * M * L
    flops = 8.0 * cmac
    b_out = {"int8": 2, "fp16": 4, "fp32": 8}[args.xprec]
    b_tf = flops / (b_ms / 1e3) / 1e12
    i_bytes = n_in * S * b_out + (M // 10) * (L // 4) * 2 * 4
    i_gbs = i_bytes / (i_ms / 1e3) / 1e9
    peak = PEAK["fp32_vector_tflops"]         # the FP32 matrix-core peak is the same 157.3 TFLOP/s
    line = {
        "metric": "tied-array beamformer: coherent beams TFLOP/s and incoherent GB/s, 256 tiles",
        "value": cmac / (b_ms / 1e3), "unit": "CMAC/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"256 tiles x 2 pols, 1 s of complex int8 sigma=8 voltages + 1 source, "
                               f"{args.xprec} F-engine at 128 channels, {BEAMS} coherent beams, incoherent beam "
                               "over 10 spectra x 4 channels", "beams": BEAMS, "spectra": M, "channels": L},
        "roofline": {"kernel": "beamform_kernel", "bound": "mfma", "achieved": round(b_tf, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(b_tf / peak, 4), "traffic": None,
                     "avg_launch_ms": round(b_ms, 4), "flops_per_launch": flops},
        "incoherent": {"kernel": "incoherent_kernel", "bound": "hbm", "achieved": round(i_gbs, 1),
                       "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(i_gbs / PEAK["hbm_gbs"], 4),
                       "avg_launch_ms": round(i_ms, 4), "bytes_per_launch": i_bytes},
        "phased_beam_gain": round(float(g[0] / np.median(g[1:])), 2),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        import oracle
        # the oracle on a bounded sample: all inputs and beams, first spectra
        n_spec = 256
        with Plan(make_config(N_TILES, L=L, T=n_spec, xprec="fp32", max_samples=n_spec * L)) as p2:
            p2.channelise(volts[:, : n_spec * L])
            spec = p2.read_channelised().cpu().numpy().astype(np.float64)
        spec = spec[..., 0] + 1j * spec[..., 1]
        t0 = time.perf_counter()
        oracle.beamform(spec, w)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": float(n_in) * BEAMS * n_spec * L / dt, "unit": "CMAC/s", "cores": 1,
                                "kind": "oracle", "sample": f"all {n_in} inputs, {BEAMS} beams, {L} channels, "
                                f"first {n_spec} spectra; FP64 sums; {dt:.1f} s wall"}
    print(json.dumps(line), flush=True)


def main_stream(args):
    """Streaming: 24 coarse channels x 256 tiles, continuous 8 s blocks, 2 s
    integrations on the device, int8 X-engine, admission by HBM budget.
    (i) blocks resident in the pool (made once by the device generator): the
    compute real-time factor; (ii) every block copied from a pinned host buffer
    (replayed at shifting offsets): end to end over the host link; a paced run
    of (ii) releases each round of 24 blocks every 8 s and gives the latency
    from a block's arrival (its last sample) to its visibilities on the device."""
    import numpy as np
    import torch

    import synth
    from paper_2303_11557_amd import mwax
    from paper_2303_11557_amd.mwax import Stream, device_view, make_config

    torch.cuda.set_device(0)
    mwax.lib()
    n_ch, n_tiles, Lc, tau = 24, 256, 128, 2.0
    block = int(SECONDS * F_S)
    call = int(args.stream_call_s * F_S)
    cfg = make_config(n_tiles, L=Lc, int_time_s=tau, xprec=args.xprec, max_samples=call)
    d = mwax.derive(cfg)
    n_in, P = d.n_inputs, d.n_pairs
    budget = int(args.stream_budget_gb * 1e9)
    pad = 1 << 16
    out = {}
    with Stream(cfg, n_ch, block, budget, out_depth=6) as s:
        slots = s.info.pool_slots
        # (i) pre-fill every pool buffer once with distinct generated blocks
        for k in range(slots):
            slot, ptr = s.acquire(0)
            v = device_view(ptr, (n_in, block, 2), torch.int8)
            synth.device_volts(v, seed=synth.MWAX_SEED + 4, L=Lc, s0=k * block,
                               sources=[synth.Source(2.0, 17)], stream=s.info.ingest_stream)
        torch.cuda.synchronize()
        free = list(range(slots))            # acquired, holding data

        def run(rounds, variant, paced, host=None):
            recs = []
            t_start = s.now()
            nonlocal free
            for r in range(rounds):
                print(f"stream {variant}{' paced' if paced else ''}: round {r + 1} of {rounds}", file=sys.stderr,
                      flush=True)
                t_arr = t_start + SECONDS * (r + 1) if paced else None
                if paced:
                    while s.now() < t_arr:
                        recs.extend(s.poll(0))
                        time.sleep(0.002)
                for ch in range(n_ch):
                    slot = free.pop() if free else s.acquire(-1)[0]
                    if variant == "ii":
                        off = ((r * n_ch + ch) * 4096) % pad
                        s.copy_in(slot, host[:, off:off + block])
                    s.submit(slot, ch, t_arr if paced else s.now())
                    recs.extend(s.poll(0))
            while len(recs) < rounds * n_ch:
                recs.extend(s.poll(-1))
            wall = max(r["t_ready_s"] for r in recs) - t_start
            lat = np.array([r["t_ready_s"] - r["t_arrival_s"] for r in recs])
            data_s = rounds * SECONDS
            return {"blocks": len(recs), "wall_s": round(wall, 3), "rtf": round(data_s / wall, 3),
                    "cmac_per_s": n_ch * rounds * P * block / wall,
                    "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                    "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
                    "latency_max_s": round(float(lat.max()), 4),
                    "integrations": int(sum(r["n_ints"] for r in recs))}

        out["warmup"] = run(1, "i", False)
        out["device_resident"] = run(args.stream_rounds, "i", False)
        # (ii) pinned host pool: one block plus a margin, filled from the device generator
        host = torch.empty((n_in, block + pad, 2), dtype=torch.int8, pin_memory=True)
        gen = torch.empty((n_in, block + pad, 2), dtype=torch.int8, device="cuda")
        synth.device_volts(gen, seed=synth.MWAX_SEED + 4 + 1, L=Lc, sources=[synth.Source(2.0, 17)])
        host.copy_(gen)
        del gen
        torch.cuda.empty_cache()
        out["host_link"] = run(max(1, args.stream_paced_rounds), "ii", False, host)
        out["paced_host_link"] = run(args.stream_paced_rounds, "ii", True, host)
        info = s.info

    dr = out["device_resident"]
    line = {
        "metric": "real-time factor & block latency, 24 coarse channels x 256 tiles streamed in 8 s blocks",
        "value": dr["cmac_per_s"], "unit": "CMAC/s", "n_gpus": 1, "steps": args.stream_rounds, "warmup": 1,
        "ms_per_step": round(dr["wall_s"] * 1e3 / args.stream_rounds, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.xprec, "data": "synthetic",
        "config": {"workload": "24 channels x 256 tiles x 2 pols, continuous 8 s blocks of complex int8 "
                               "sigma=8 voltages + 1 source, 128-pt FFT, 2 s integrations on device, "
                               f"{args.stream_call_s:g} s plan calls, admission by HBM budget",
                   "channels": n_ch, "block_samples": block, "pool_slots": info.pool_slots,
                   "hbm_budget_bytes": budget, "device_bytes": info.device_bytes},
        "rtf": dr["rtf"],
        "latency_p50_s": out["paced_host_link"]["latency_p50_s"],
        "latency_p99_s": out["paced_host_link"]["latency_p99_s"],
        "runs": out,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(coarse channels would shard across GPUs with no exchange between them)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return main_batch(args)
    if args.workload == "stream":
        return main_stream(args)
    if args.workload == "weights":
        return main_weights(args)
    if args.workload == "fscrunch":
        return main_fscrunch(args)
    if args.workload == "ultrafine":
        return main_ultrafine(args)
    if args.workload == "beamform":
        return main_beamform(args)

    import torch

    import synth
    from paper_2303_11557_amd import mwax
    from paper_2303_11557_amd.mwax import Plan, make_config

    torch.cuda.set_device(0)
    mwax.lib()
    L = args.fft_len
    S = int(SECONDS * F_S)
    n_in = 2 * N_TILES
    T = S // L
    P = n_in * (n_in + 1) // 2
    cmac_per_step = P * S                   # distinct Hermitian entries x samples
    sources = [synth.Source(2.0, -37), synth.Source(3.0, 5), synth.Source(4.0, 41)]
    volts = torch.empty((n_in, S, 2), dtype=torch.int8, device="cuda")
    synth.device_volts(volts, seed=synth.MWAX_SEED + 2, sources=sources, L=L)
    torch.cuda.synchronize()
    if args.copy_probe:
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")   # 4 GiB read + 4 GiB written
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    def run_variant(prec, steps, warmup):
        with Plan(make_config(N_TILES, L=L, T=T, xprec=prec, max_samples=S)) as p:
            out = torch.empty((1, L, P), dtype=torch.complex64, device="cuda")

            def step():
                p.channelise(volts)
                p.correlate()
                p.integrate(1, out=out)

            for _ in range(warmup):
                step()
            p.sync()
            p.set_timing(True)
            for fam in range(4):
                p.kernel_time(fam)               # clear
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            p.sync()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            fam = {name: p.kernel_time(i) for i, name in enumerate(("fengine", "xengine", "pack", "calib"))}
            p.set_timing(False)
        ms = (t1 - t0) * 1e3 / steps
        return ms, fam, out

    ms, fam, out = run_variant(args.xprec, args.steps, args.warmup)
    torch.cuda.synchronize()
    value = cmac_per_step / (ms / 1e3)

    # ---- roofline of the kernels (algorithmic work per launch / event-timed duration)
    f_ms, f_n = fam["fengine"]
    x_ms, x_n = fam["xengine"]
    p_ms, p_n = fam["pack"]
    b_out = {"int8": 2, "fp16": 4, "fp32": 8}[args.xprec]
    x_peak = {"int8": PEAK["int8_tops"], "fp16": PEAK["fp16_tflops"], "fp32": PEAK["fp32_vector_tflops"]}[args.xprec]
    x_ops_launch = 8.0 * cmac_per_step * args.steps / max(x_n, 1)
    x_avg_ms = x_ms / max(x_n, 1)
    x_achieved = x_ops_launch / (x_avg_ms / 1e3) / 1e12
    # F-engine main pass: int8 in + channelised out per sample of every input.  The
    # int8 scale calibration (a statistics pass over the first 1024 spectra of each
    # integration and its reduction) is timed and reported on its own.
    f_bytes_launch = n_in * S * (2 + b_out) * args.steps / max(f_n, 1)
    f_avg_ms = f_ms / max(f_n, 1)
    f_gbs = f_bytes_launch / (f_avg_ms / 1e3) / 1e9 if f_ms > 0 else 0.0
    c_ms, _ = fam["calib"]

    roof_x = {"kernel": f"xengine_{args.xprec}", "bound": "mfma" if args.xprec != "fp32" else "alu",
              "achieved": round(x_achieved, 2), "peak": x_peak, "unit": "TFLOP/s",
              "frac": round(x_achieved / x_peak, 4), "traffic": measured_traffic(f"xengine_{args.xprec}"),
              "avg_launch_ms": round(x_avg_ms, 4), "launches": x_n,
              "ops_per_launch": x_ops_launch}
    copy_gbs = copy_bandwidth()
    roof_f = {"kernel": f"fengine_{args.xprec}", "bound": "hbm", "achieved": round(f_gbs, 1),
              "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(f_gbs / copy_gbs, 4),
              "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(f_gbs / PEAK["hbm_gbs"], 4),
              "traffic": measured_traffic(f"fengine_{args.xprec}"),
              "avg_launch_ms": round(f_avg_ms, 4), "launches": f_n,
              "bytes_per_launch": f_bytes_launch}
    dominant, other = (roof_x, roof_f) if x_ms >= f_ms else (roof_f, roof_x)

    # ---- other X-engine precisions on the same block
    variants = {}
    if args.variants != "none":
        for prec in [v for v in args.variants.split(",") if v and v != args.xprec]:
            vms, vfam, _ = run_variant(prec, args.variant_steps, 1)
            vx_ms, vx_n = vfam["xengine"]
            vpeak = {"int8": PEAK["int8_tops"], "fp16": PEAK["fp16_tflops"],
                     "fp32": PEAK["fp32_vector_tflops"]}[prec]
            vach = 8.0 * cmac_per_step * args.variant_steps / (vx_ms / 1e3) / 1e12
            variants[prec] = {
                "ms_per_step": round(vms, 3), "cmac_per_s": cmac_per_step / (vms / 1e3),
                "xengine_ms_per_step": round(vx_ms / args.variant_steps, 3),
                "xengine_tflops": round(vach, 2), "xengine_peak": vpeak,
                "xengine_frac": round(vach / vpeak, 4), "rtf_per_channel": round(SECONDS / (vms / 1e3), 2),
            }
            torch.cuda.empty_cache()
        if "fp32" in variants:
            variants["speedup_vs_fp32_plain"] = round(variants["fp32"]["ms_per_step"] / ms, 2)

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same block
    cpu = None if args.no_cpu_baseline else cpu_baseline(
        volts, L, args.cpu_seconds, "the same 8 s block",
        accuracy=lambda n, spec, vis: gpu_error_vs_oracle(volts, L, n, spec, vis))
    if cpu and "accuracy" in cpu:
        for prec, ent in cpu["accuracy"].items():
            if prec in variants:
                variants[prec]["err_vs_fp64"] = ent

    rtf = SECONDS / (ms / 1e3)
    line = {
        "metric": "X-engine CMAC/s & real-time factor at 256 tiles: int8/FP16 MFMA vs FP32 plain",
        "value": value,
        "unit": "CMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.xprec,
        "data": "synthetic",
        "config": {
            "workload": "256 tiles x 2 pols, 1 coarse channel, 8 s (10.24 M samples) complex int8 "
                        f"Gaussian sigma=8 + 3 point sources, {L}-pt FFT, one 8 s integration, "
                        f"{args.xprec} X-engine",
            "n_inputs": n_in, "samples": S, "fft_len": L, "spectra_per_integration": T,
            "pairs": P, "cmac_per_step": cmac_per_step,
        },
        "rtf_per_channel": round(rtf, 2),
        "rtf_24_channels": round(rtf / 24.0, 2),
        "roofline": dominant,
        "roofline_other": other,
        "pack_ms_per_step": round(p_ms / max(args.steps, 1), 4),
        "calibration_ms_per_step": round(c_ms / max(args.steps, 1), 4),
        "variants": variants,
        "err_vs_fp64": (cpu or {}).get("accuracy", {}).get(args.xprec),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
