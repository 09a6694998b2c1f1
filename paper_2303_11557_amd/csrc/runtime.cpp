// Host runtime of libmwax: plan derivation, workspace, stream position and
// integration bookkeeping, kernel launches, error reporting.  Implements the C
// ABI declared in mwax.h.
//
// Stream model (Sec. 2.5.2: integrations are whole numbers of spectra of a
// continuous stream).  The voltage stream is cut into spectra of L samples;
// integration j covers stream spectra [jT, (j+1)T).  A channelise call covering
// stream spectra [g, g+M) is split into segments at integration boundaries;
// each segment is laid out in the channel-major buffer from a fresh row group,
// so no row group mixes two integrations.  Integration j accumulates in device
// slot j mod n_slots until mwax_integrate emits it.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <mutex>

#include "plan.h"

namespace mwax {

namespace {
thread_local std::string g_last_error;
}  // namespace

mwax_status fail(mwax_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

mwax_status ok() {
    g_last_error.clear();
    return MWAX_OK;
}

mwax_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? MWAX_E_NOMEM : MWAX_E_DEVICE,
                "%s: %s", what, hipGetErrorString(e));
}

}  // namespace mwax

using namespace mwax;

namespace {
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

mwax_status mwax::derive(const mwax_config *cfg, mwax_dims *o) {
    if (!cfg || !o) return fail(MWAX_E_INVAL, "null configuration or output");
    if (cfg->n_pols != 2) return fail(MWAX_E_INVAL, "n_pols must be 2 (got %d)", cfg->n_pols);
    if (cfg->n_tiles < 1 || cfg->n_tiles > 1024)
        return fail(MWAX_E_INVAL, "n_tiles must be in 1..1024 (got %d)", cfg->n_tiles);
    if (!(cfg->coarse_bw_hz > 0) || !std::isfinite(cfg->coarse_bw_hz))
        return fail(MWAX_E_INVAL, "coarse_bw_hz must be positive");
    if (!(cfg->fine_chan_hz > 0) || !std::isfinite(cfg->fine_chan_hz))
        return fail(MWAX_E_INVAL, "fine_chan_hz must be positive");
    const double lf = cfg->coarse_bw_hz / cfg->fine_chan_hz;
    const int64_t L = llround(lf);
    if (L < 1 || std::fabs(lf - (double)L) > 1e-9 * lf)
        return fail(MWAX_E_INVAL, "coarse_bw/fine_chan = %.9g is not a whole number of channels", lf);
    if ((!is_pow2(L) || L > 1024) && L != kUltraFineL)
        return fail(MWAX_E_UNSUPPORTED, "FFT length %lld: powers of two 1..1024 and 6400 are implemented",
                    (long long)L);
    if (!(cfg->int_time_s > 0) || !std::isfinite(cfg->int_time_s))
        return fail(MWAX_E_INVAL, "int_time_s must be positive");
    const double tf = cfg->int_time_s * cfg->coarse_bw_hz / (double)L;
    const int64_t T = llround(tf);
    if (T < 1 || std::fabs(tf - (double)T) > 1e-9 * std::max(1.0, tf))
        return fail(MWAX_E_INVAL, "int_time * coarse_bw / L = %.9g must be a whole number of spectra >= 1", tf);
    if (cfg->xprec < MWAX_X_FP32 || cfg->xprec > MWAX_X_INT8)
        return fail(MWAX_E_INVAL, "unknown xprec %d", cfg->xprec);
    if (cfg->reserved != 0 || cfg->flags != 0) return fail(MWAX_E_INVAL, "reserved fields and flags must be 0");
    if (cfg->max_samples < L || cfg->max_samples % L != 0)
        return fail(MWAX_E_INVAL, "max_samples must be a positive multiple of L = %lld", (long long)L);

    std::memset(o, 0, sizeof *o);
    const int64_t n_in = 2 * (int64_t)cfg->n_tiles;
    o->n_inputs = (int32_t)n_in;
    o->fft_len = (int32_t)L;
    o->spectra_per_int = T;
    o->n_pairs = n_in * (n_in + 1) / 2;
    o->n_baselines = (int64_t)cfg->n_tiles * (cfg->n_tiles + 1) / 2;
    o->max_spectra = cfg->max_samples / L;
    const int64_t segs = (o->max_spectra + T - 1) / T + 1;     // integrations one call can touch
    o->n_slots = (int32_t)(segs + 1);
    o->group = group_of(cfg->xprec);
    o->vis_per_int = L * o->n_pairs;
    o->cal_spectra = std::min<int64_t>(T, (kCalSamples + L - 1) / L);
    const int64_t NG = (o->max_spectra + o->group - 1) / o->group + segs;
    const uint64_t chan_b = (uint64_t)L * NG * n_in * kRowBytes;
    const uint64_t integ_b = (uint64_t)o->n_slots * integ_slot_bytes(cfg->xprec, T, L, o->n_pairs);
    const uint64_t small_b = (uint64_t)o->n_slots * 2 * L * 4 + 6 * L * 4 + L * 8 + (uint64_t)kStatsMaxWG * (L + 1) * 8;
    const uint64_t esize = cfg->xprec == MWAX_X_INT8 ? 1 : (cfg->xprec == MWAX_X_FP16 ? 2 : 4);
    const uint64_t mid_b = L == kUltraFineL ? (uint64_t)n_in * cfg->max_samples * 2 * esize : 0;
    o->workspace_bytes = chan_b + integ_b + small_b + mid_b;
    o->sample_time_s = 1.0 / cfg->coarse_bw_hz;
    o->fine_chan_hz = cfg->coarse_bw_hz / (double)L;
    o->int_time_s = (double)T * (double)L / cfg->coarse_bw_hz;
    return MWAX_OK;
}

// ---------------------------------------------------------------------------
// Static workspace for plans created by mwax_plan_create_noalloc: a file-scope
// device array (each device that loads the library holds its own copy until the
// process ends).  Host code never uses the array's name as an address: the
// device address of each device's copy is looked up once, with that device
// current, and kept in g_scratch_ptr.  At most one such plan lives on a device
// at a time (they would share the array).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kScratchMaxDevices] = {};
bool g_scratch_live[kScratchMaxDevices] = {};
}  // namespace

__device__ __align__(256) uint8_t scratch[kScratchBytes];

void mwax::free_plan(mwax_plan p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    for (auto &e : p->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto e : p->pool) (void)hipEventDestroy(e);
    if (p->static_ws) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (p->device >= 0 && p->device < kScratchMaxDevices) g_scratch_live[p->device] = false;
    } else {
        (void)hipFree(p->chan);
        (void)hipFree(p->integ);
        (void)hipFree(p->scales);
        (void)hipFree(p->fixed);
        (void)hipFree(p->ones);
        (void)hipFree(p->last);
        (void)hipFree(p->tw);
        (void)hipFree(p->stats);
        (void)hipFree(p->mid);
    }
    delete p;
}

mwax_status mwax::plan_segments(mwax_plan p, int64_t M, std::vector<Segment> &out) {
    out.clear();
    int64_t g = p->g_chan, done = 0, grp = 0;
    while (done < M) {
        Segment s;
        s.j = g / p->T;
        s.local0 = g - s.j * p->T;
        s.nframes = std::min(p->T - s.local0, M - done);
        s.slot = (int)(s.j % p->nslots);
        s.frame0 = done;
        s.grp0 = grp;
        s.ngrp = (s.nframes + p->G - 1) / p->G;
        grp += s.ngrp;
        g += s.nframes;
        done += s.nframes;
        out.push_back(s);
    }
    if (grp > p->NG) return fail(MWAX_E_INVAL, "block needs %lld row groups, buffer holds %lld",
                                 (long long)grp, (long long)p->NG);
    for (const Segment &s : out) {
        const int64_t owner = p->slot_owner[s.slot];
        if (s.local0 == 0) {
            if (owner != -1)
                return fail(MWAX_E_STATE,
                            "integration %lld needs device slot %d, still held by integration %lld: "
                            "call mwax_integrate first", (long long)s.j, s.slot, (long long)owner);
        } else if (owner != s.j) {
            return fail(MWAX_E_STATE, "integration %lld lost its slot", (long long)s.j);
        }
    }
    return MWAX_OK;
}

FArgs mwax::calib_args(mwax_plan p, const Segment &s, const int8_t *volts, int64_t ld) {
    const int64_t ncal = std::min(p->d.cal_spectra, s.nframes);
    FArgs a{};
    a.volts = volts;
    a.ld = ld;
    a.frame0 = s.frame0;
    a.nframes = ncal;
    a.n_in = p->n_in;
    a.R = p->R;
    a.ngrp = (int32_t)((ncal + p->G - 1) / p->G);
    a.stats_mode = 1;
    a.tw = p->tw;
    a.stats = p->stats;
    return a;
}

FArgs mwax::fengine_args(mwax_plan p, const Segment &s, const int8_t *volts, int64_t ld) {
    FArgs a{};
    a.volts = volts;
    a.ld = ld;
    a.frame0 = s.frame0;
    a.nframes = s.nframes;
    a.chan = p->chan;
    a.NG = p->NG;
    a.grp0 = s.grp0;
    a.n_in = p->n_in;
    a.R = p->R;
    a.ngrp = (int32_t)s.ngrp;
    a.stats_mode = 0;
    a.tw = p->tw;
    a.inv_s = p->scales + (size_t)s.slot * 2 * p->L + p->L;
    a.half_scale = std::ldexp(1.0f, -fp16_exponent(p->L));
    a.mid = p->mid;
    a.mid_frames = p->d.max_spectra;
    if (p->dl) {
        a.dl = p->dl;
        a.dl_ld = p->dl_steps;
        a.dl_f0 = p->g_chan + s.frame0 - p->dl_pos0;   // g_chan: stream frame of the call's start
        a.dl_fps = p->dl_fps;
        a.dl_nu = p->dl_nu;
    }
    return a;
}

int mwax::stats_grid(mwax_plan p, const FArgs &a) {
    return p->L == kUltraFineL ? fft6400_grid(p->n_in, a.nframes, true) : fengine_grid(p->n_in, p->R, a.ngrp, true);
}

hipError_t mwax::launch_fengine_segment(mwax_plan p, const Segment &s, const FArgs &a) {
    if (p->L != kUltraFineL) return launch_fengine(p->L, p->xprec, a, p->stream);
    hipError_t e = launch_fft6400(p->xprec, a, p->stream);
    if (e != hipSuccess) return e;
    CornerArgs c{};
    c.mid = p->mid;
    c.mid_frames = p->d.max_spectra;
    c.frame0 = s.frame0;
    c.nframes = s.nframes;
    c.chan = p->chan;
    c.NG = p->NG;
    c.grp0 = s.grp0;
    c.n_in = p->n_in;
    c.L = p->L;
    return launch_corner_turn(p->xprec == MWAX_X_INT8 ? 1 : (p->xprec == MWAX_X_FP16 ? 2 : 4), c, p->stream);
}

XArgs mwax::xengine_args(mwax_plan p, const Segment &s) {
    XArgs a{};
    a.chan = p->chan;
    a.NG = p->NG;
    a.grp0 = s.grp0;
    a.ngrp = (int32_t)s.ngrp;
    a.n_in = p->n_in;
    a.L = p->L;
    a.ntiles = p->ntiles;
    a.tile = xengine_tile(p->xprec);
    a.integ = (uint8_t *)p->integ + (size_t)s.slot * p->slot_bytes;
    a.P = p->P;
    a.first = s.local0 == 0;
    a.i32 = p->integ32;
    a.nks = p->whole_segments ? 1 : 0;   // 0: launch_xengine chooses
    return a;
}

namespace {

// Set the scales of the integrations that begin in this block (INT8 plans).
mwax_status begin_integrations(mwax_plan p, const int8_t *volts, int64_t ld, bool from_voltages) {
    for (const Segment &s : p->segs) {
        if (s.local0 != 0) continue;
        p->slot_owner[s.slot] = s.j;
        p->slot_count[s.slot] = 0;
        p->last_slot = s.slot;
        if (p->xprec != MWAX_X_INT8) continue;
        float *dst = p->scales + (size_t)s.slot * 2 * p->L;
        hipError_t e;
        if (p->fixed_mode || !from_voltages) {
            e = launch_copy_scales(p->fixed_mode ? p->fixed : p->ones, dst, 2 * p->L, p->stream);
        } else {
            const FArgs a = calib_args(p, s, volts, ld);
            e = timed(p, 3, [&] {
                return p->L == kUltraFineL ? launch_fft6400(p->xprec, a, p->stream)
                                           : launch_fengine(p->L, p->xprec, a, p->stream);
            });
            if (e == hipSuccess) {
                const int nwg = stats_grid(p, a);
                e = timed(p, 3, [&] { return launch_calib_finish(p->stats, nwg, p->L, dst, p->last, p->stream); });
            }
        }
        if (e != hipSuccess) return hip_fail(e, "scale calibration launch");
    }
    return MWAX_OK;
}

mwax_status check_plan(mwax_plan p) {
    if (!p) return fail(MWAX_E_INVAL, "null plan");
    return MWAX_OK;
}

}  // namespace

extern "C" {

const char *mwax_last_error(void) { return g_last_error.c_str(); }

mwax_status mwax_plan_derive(const mwax_config *cfg, mwax_dims *out) {
    mwax_status s = derive(cfg, out);
    return s == MWAX_OK ? ok() : s;
}

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Create a plan whose workspace is allocated with hipMalloc (ws == NULL) or
// carved out of ws[0 .. cap) (no allocation; MWAX_E_INVAL if it does not fit).
mwax_status create_plan(const mwax_config *cfg, void *hip_stream, mwax_plan *out, uint8_t *ws, size_t cap) {
    if (!out) return fail(MWAX_E_INVAL, "null output handle");
    *out = nullptr;
    mwax_dims d;
    mwax_status st = derive(cfg, &d);
    if (st != MWAX_OK) return st;

    mwax_plan p = new (std::nothrow) mwax_plan_s;
    if (!p) return fail(MWAX_E_NOMEM, "host allocation failed");
    p->cfg = *cfg;
    p->d = d;
    p->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&p->device);
    p->L = d.fft_len;
    p->G = d.group;
    p->n_in = d.n_inputs;
    p->xprec = cfg->xprec;
    p->T = d.spectra_per_int;
    p->P = d.n_pairs;
    p->nslots = d.n_slots;
    int lds_limit = 0;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess ||
        lds_limit <= 0)
        lds_limit = 65536;
    if (lds_limit > kMaxLds) lds_limit = kMaxLds;
    p->R = p->L == kUltraFineL ? 1 : fengine_pick_R(p->L, p->xprec, p->n_in, lds_limit);
    if (p->L == kUltraFineL ? fft6400_lds_bytes() > lds_limit
                            : (fengine_lds_bytes(p->L, p->xprec, p->R, false) > lds_limit ||
                               fengine_lds_bytes(p->L, p->xprec, p->R, true) > lds_limit)) {
        mwax_status r = fail(MWAX_E_UNSUPPORTED, "F-engine for L = %d needs %d bytes of LDS, device allows %d",
                             p->L, fengine_lds_bytes(p->L, p->xprec, p->R, false), lds_limit);
        delete p;
        return r;
    }
    const int nt = (p->n_in + xengine_tile(p->xprec) - 1) / xengine_tile(p->xprec);
    p->ntiles = nt * (nt + 1) / 2;
    const int64_t segs = (d.max_spectra + p->T - 1) / p->T + 1;
    p->NG = (d.max_spectra + p->G - 1) / p->G + segs;
    p->integ32 = integ_elem_bytes(p->xprec, p->T) == 8;
    p->slot_bytes = (size_t)integ_slot_bytes(p->xprec, p->T, p->L, p->P);
    p->slot_owner.assign(p->nslots, -1);
    p->slot_count.assign(p->nslots, 0);
    // 6,400 channels: an integration's first X-engine flush overwrites its slot,
    // so slots are not cleared when emitted (mwax_correlate clears one itself
    // before a launch that would add into it)
    if (p->L == kUltraFineL) p->clear_on_emit = false;

    // workspace buffers, in order
    const size_t esize = p->xprec == MWAX_X_INT8 ? 1 : (p->xprec == MWAX_X_FP16 ? 2 : 4);
    void **ptrs[] = {(void **)&p->chan, &p->integ, (void **)&p->scales, (void **)&p->fixed, (void **)&p->ones,
                     (void **)&p->last, (void **)&p->tw, (void **)&p->stats, (void **)&p->mid};
    const size_t sizes[] = {(size_t)p->L * p->NG * p->n_in * kRowBytes, p->slot_bytes * p->nslots,
                            (size_t)p->nslots * 2 * p->L * sizeof(float), (size_t)2 * p->L * sizeof(float),
                            (size_t)2 * p->L * sizeof(float), (size_t)2 * p->L * sizeof(float),
                            (size_t)p->L * sizeof(float2), (size_t)kStatsMaxWG * stats_row(p->L) * sizeof(double),
                            p->L == kUltraFineL ? (size_t)p->n_in * d.max_spectra * p->L * 2 * esize : 0};
    constexpr int nbuf = (int)(sizeof(sizes) / sizeof(sizes[0]));
    hipError_t e = hipSuccess;
    if (ws) {
        size_t total = 0;
        for (int k = 0; k < nbuf; ++k) total += align256(sizes[k]);
        if (total > cap) {
            mwax_status r = fail(MWAX_E_INVAL, "plan workspace of %zu bytes exceeds the %zu-byte static workspace",
                                 total, cap);
            delete p;
            return r;
        }
        size_t off = 0;
        for (int k = 0; k < nbuf; ++k) {
            *ptrs[k] = sizes[k] > 0 ? ws + off : nullptr;
            off += align256(sizes[k]);
        }
        p->static_ws = true;
    } else {
        for (int k = 0; k < nbuf && e == hipSuccess; ++k)
            if (sizes[k] > 0) e = hipMalloc(ptrs[k], sizes[k]);
        if (e != hipSuccess) {
            mwax_status r = hip_fail(e, "workspace allocation");
            free_plan(p);
            return r;
        }
    }
    // initial state, written by kernels on the plan's stream
    e = launch_fill_f32(p->ones, 1.0f, 2 * p->L, p->stream);
    if (e == hipSuccess) e = launch_fill_f32(p->fixed, 1.0f, 2 * p->L, p->stream);
    if (e == hipSuccess) e = launch_twiddles(p->tw, p->L, p->stream);
    if (e == hipSuccess) e = launch_fill_zero(p->integ, p->slot_bytes * p->nslots, p->stream);
    if (e == hipSuccess) e = launch_copy_scales(p->ones, p->scales, 2 * p->L, p->stream);
    if (e == hipSuccess) e = launch_copy_scales(p->ones, p->last, 2 * p->L, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        mwax_status r = hip_fail(e, "plan initialisation");
        if (p->static_ws) delete p;   // nothing allocated; the caller holds the workspace lock
        else free_plan(p);
        return r;
    }
    *out = p;
    return ok();
}

}  // namespace

mwax_status mwax_plan_create(const mwax_config *cfg, void *hip_stream, mwax_plan *out) {
    return create_plan(cfg, hip_stream, out, nullptr, 0);
}

mwax_status mwax_plan_create_noalloc(const mwax_config *cfg, void *hip_stream, mwax_plan *out) {
    if (!out) return fail(MWAX_E_INVAL, "null output handle");
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= kScratchMaxDevices) return fail(MWAX_E_UNSUPPORTED, "device %d: no static workspace", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // once per device, with that device current: the address of its copy
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "static workspace address");
        if (!ptr) return fail(MWAX_E_DEVICE, "static workspace address: null");
        g_scratch_ptr[dev] = (uint8_t *)ptr;
    }
    if (g_scratch_live[dev])
        return fail(MWAX_E_STATE, "device %d already has a plan in the static workspace: destroy it first", dev);
    mwax_status st = create_plan(cfg, hip_stream, out, g_scratch_ptr[dev], kScratchBytes);
    if (st == MWAX_OK) g_scratch_live[dev] = true;
    return st;
}

mwax_status mwax_plan_destroy(mwax_plan p) {
    if (p && p->in_batch) return fail(MWAX_E_INVAL, "this plan belongs to a batch or stream: destroy that instead");
    free_plan(p);
    return ok();
}

mwax_status mwax_plan_get_dims(mwax_plan p, mwax_dims *out) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!out) return fail(MWAX_E_INVAL, "null output");
    *out = p->d;
    return ok();
}

mwax_status mwax_channelise(mwax_plan p, const int8_t *d_volts, int64_t n_samples, int64_t ld_samples) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!d_volts) return fail(MWAX_E_INVAL, "null voltage pointer");
    if ((uintptr_t)d_volts & 15) return fail(MWAX_E_INVAL, "voltages must be 16-byte aligned");
    if (n_samples <= 0 || n_samples % p->L != 0 || n_samples > p->cfg.max_samples)
        return fail(MWAX_E_INVAL, "n_samples = %lld must be a positive multiple of L = %d and <= max_samples = %lld",
                    (long long)n_samples, p->L, (long long)p->cfg.max_samples);
    if (ld_samples < n_samples || ld_samples % 8 != 0)
        return fail(MWAX_E_INVAL, "ld_samples = %lld must be >= n_samples and a multiple of 8", (long long)ld_samples);
    if (p->pending) return fail(MWAX_E_STATE, "the previous channelised block has not been correlated");
    const int64_t M = n_samples / p->L;
    if (p->dl) {
        const int64_t last_step = (p->g_chan + M - 1 - p->dl_pos0) / p->dl_fps;
        if (last_step >= p->dl_steps)
            return fail(MWAX_E_INVAL, "the delay table covers %lld steps; this call reaches step %lld",
                        (long long)p->dl_steps, (long long)last_step);
    }
    std::vector<Segment> segs;
    mwax_status st = plan_segments(p, M, segs);
    if (st != MWAX_OK) return st;
    p->segs = segs;
    st = begin_integrations(p, d_volts, ld_samples, true);
    if (st != MWAX_OK) return st;
    for (const Segment &s : p->segs) {
        const FArgs a = fengine_args(p, s, d_volts, ld_samples);
        hipError_t e = timed(p, 0, [&] { return launch_fengine_segment(p, s, a); });
        if (e != hipSuccess) return hip_fail(e, "F-engine launch");
    }
    p->pending = true;
    p->have_block = true;
    p->block_spectra = M;
    p->g_chan += M;
    return ok();
}

mwax_status mwax_load_channelised(mwax_plan p, const void *d_chan, int64_t n_spectra) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!d_chan) return fail(MWAX_E_INVAL, "null channelised pointer");
    if (n_spectra <= 0 || n_spectra > p->d.max_spectra)
        return fail(MWAX_E_INVAL, "n_spectra = %lld must be in 1..max_spectra = %lld", (long long)n_spectra,
                    (long long)p->d.max_spectra);
    const int esize = p->xprec == MWAX_X_INT8 ? 1 : (p->xprec == MWAX_X_FP16 ? 2 : 4);
    if ((uintptr_t)d_chan % esize) return fail(MWAX_E_INVAL, "channelised data misaligned");
    if (p->pending) return fail(MWAX_E_STATE, "the previous channelised block has not been correlated");
    std::vector<Segment> segs;
    mwax_status st = plan_segments(p, n_spectra, segs);
    if (st != MWAX_OK) return st;
    p->segs = segs;
    st = begin_integrations(p, nullptr, 0, false);
    if (st != MWAX_OK) return st;
    for (const Segment &s : p->segs) {
        RepackArgs a{};
        a.canon = const_cast<void *>(d_chan);
        a.m0 = s.frame0;
        a.nframes = s.nframes;
        a.chan = p->chan;
        a.NG = p->NG;
        a.grp0 = s.grp0;
        a.n_in = p->n_in;
        a.L = p->L;
        a.G = p->G;
        a.esize = esize;
        a.to_internal = 1;
        hipError_t e = launch_repack(a, p->stream);
        if (e != hipSuccess) return hip_fail(e, "load launch");
    }
    p->pending = true;
    p->have_block = true;
    p->block_spectra = n_spectra;
    p->g_chan += n_spectra;
    return ok();
}

mwax_status mwax_read_channelised(mwax_plan p, void *d_out, int64_t max_spectra, int64_t *n_spectra) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!d_out || !n_spectra) return fail(MWAX_E_INVAL, "null output");
    if (!p->have_block) return fail(MWAX_E_STATE, "nothing has been channelised");
    if (p->block_spectra > max_spectra)
        return fail(MWAX_E_INVAL, "block holds %lld spectra, output room for %lld", (long long)p->block_spectra,
                    (long long)max_spectra);
    const int esize = p->xprec == MWAX_X_INT8 ? 1 : (p->xprec == MWAX_X_FP16 ? 2 : 4);
    for (const Segment &s : p->segs) {
        RepackArgs a{};
        a.canon = d_out;
        a.m0 = s.frame0;
        a.nframes = s.nframes;
        a.chan = p->chan;
        a.NG = p->NG;
        a.grp0 = s.grp0;
        a.n_in = p->n_in;
        a.L = p->L;
        a.G = p->G;
        a.esize = esize;
        a.to_internal = 0;
        hipError_t e = launch_repack(a, p->stream);
        if (e != hipSuccess) return hip_fail(e, "read launch");
    }
    *n_spectra = p->block_spectra;
    return ok();
}

mwax_status mwax_beamform(mwax_plan p, const void *d_weights, int32_t n_beams, void *d_out, int64_t max_spectra,
                          int64_t *n_spectra) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!d_weights || !d_out || !n_spectra) return fail(MWAX_E_INVAL, "null argument");
    if (((uintptr_t)d_weights & 7) || ((uintptr_t)d_out & 7)) return fail(MWAX_E_INVAL, "weights and output must be 8-byte aligned");
    if (n_beams < 1 || n_beams > 65535 * 64) return fail(MWAX_E_INVAL, "n_beams = %d out of range", n_beams);
    if (!p->have_block) return fail(MWAX_E_STATE, "nothing has been channelised");
    if (p->block_spectra > max_spectra)
        return fail(MWAX_E_INVAL, "block holds %lld spectra, output room for %lld", (long long)p->block_spectra,
                    (long long)max_spectra);
    const int esize = p->xprec == MWAX_X_INT8 ? 1 : (p->xprec == MWAX_X_FP16 ? 2 : 4);
    for (const Segment &s : p->segs) {
        BeamArgs a{};
        a.chan = p->chan;
        a.NG = p->NG;
        a.grp0 = s.grp0;
        a.nframes = s.nframes;
        a.m0 = s.frame0;
        a.scales = p->xprec == MWAX_X_INT8 ? p->scales + (size_t)s.slot * 2 * p->L : nullptr;
        a.post = p->xprec == MWAX_X_FP16 ? std::ldexp(1.0f, fp16_exponent(p->L)) : 1.0f;
        a.n_in = p->n_in;
        a.L = p->L;
        a.nb = n_beams;
        a.w = (const float2 *)d_weights;
        a.out = (float2 *)d_out;
        hipError_t e = launch_beamform(esize, a, p->stream);
        if (e != hipSuccess) return hip_fail(e, "beamformer launch");
    }
    *n_spectra = p->block_spectra;
    return ok();
}

mwax_status mwax_beamform_incoherent(mwax_plan p, int32_t t_avg, int32_t f_avg, float *d_out, int64_t max_bins,
                                     int64_t *n_time_bins) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!d_out || !n_time_bins) return fail(MWAX_E_INVAL, "null argument");
    if ((uintptr_t)d_out & 3) return fail(MWAX_E_INVAL, "output must be 4-byte aligned");
    if (!p->have_block) return fail(MWAX_E_STATE, "nothing has been channelised");
    if (t_avg < 1 || p->block_spectra % t_avg != 0)
        return fail(MWAX_E_INVAL, "t_avg = %d must divide the block's %lld spectra", t_avg, (long long)p->block_spectra);
    if (f_avg < 1 || p->L % f_avg != 0) return fail(MWAX_E_INVAL, "f_avg = %d must divide L = %d", f_avg, p->L);
    if ((int)p->segs.size() > kIncohMaxSeg)
        return fail(MWAX_E_UNSUPPORTED, "block spans %zu integration segments, at most %d", p->segs.size(), kIncohMaxSeg);
    const int64_t nj = p->block_spectra / t_avg;
    if (nj * (p->L / f_avg) > max_bins)
        return fail(MWAX_E_INVAL, "output needs %lld bins, room for %lld", (long long)(nj * (p->L / f_avg)),
                    (long long)max_bins);
    IncohArgs a{};
    a.chan = p->chan;
    a.NG = p->NG;
    a.n_in = p->n_in;
    a.L = p->L;
    a.t_avg = t_avg;
    a.f_avg = f_avg;
    a.n_o = p->L / f_avg;
    a.n_j = nj;
    a.post = p->xprec == MWAX_X_FP16 ? std::ldexp(1.0f, fp16_exponent(p->L)) : 1.0f;
    a.nseg = (int32_t)p->segs.size();
    for (int k = 0; k < a.nseg; ++k) {
        const Segment &s = p->segs[k];
        a.seg_m0[k] = s.frame0;
        a.seg_grp0[k] = s.grp0;
        a.seg_scales[k] = p->xprec == MWAX_X_INT8 ? p->scales + (size_t)s.slot * 2 * p->L : nullptr;
    }
    a.out = d_out;
    hipError_t e = launch_incoherent(p->xprec == MWAX_X_INT8 ? 1 : (p->xprec == MWAX_X_FP16 ? 2 : 4), a, p->stream);
    if (e != hipSuccess) return hip_fail(e, "incoherent beam launch");
    *n_time_bins = nj;
    return ok();
}

mwax_status mwax_correlate(mwax_plan p) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!p->pending) return fail(MWAX_E_STATE, "no fresh channelised block to correlate");
    for (const Segment &s : p->segs) {
        if (p->favg > 1) {
            // averaging X-engine: whole segments, the first one of an integration stores
            XAvgArgs v{};
            v.chan = p->chan;
            v.NG = p->NG;
            v.grp0 = s.grp0;
            v.ngrp = (int32_t)s.ngrp;
            v.n_in = p->n_in;
            v.L = p->L;
            v.F = p->favg;
            v.N = p->L / p->favg;
            v.ntiles = xengine_tile_count(p->n_in, kXTileSmall);
            v.scales = p->xprec == MWAX_X_INT8 ? p->scales + (size_t)s.slot * 2 * p->L : nullptr;
            v.integ = (uint8_t *)p->integ + (size_t)s.slot * p->slot_bytes;
            v.P = p->P;
            v.first = s.local0 == 0;
            hipError_t e = timed(p, 1, [&] { return launch_xengine_avg(p->xprec, v, p->stream); });
            if (e != hipSuccess) return hip_fail(e, "X-engine launch");
            p->slot_count[s.slot] += s.nframes;
            continue;
        }
        const XArgs a = xengine_args(p, s);
        if (s.local0 == 0 && !p->clear_on_emit && xengine_accumulates(p->xprec, a)) {
            // this launch adds into a slot that was not cleared when it was last emitted
            hipError_t e = launch_fill_zero(a.integ, p->slot_bytes, p->stream);
            if (e != hipSuccess) return hip_fail(e, "slot clear");
        }
        hipError_t e = timed(p, 1, [&] { return launch_xengine(p->xprec, a, p->stream); });
        if (e != hipSuccess) return hip_fail(e, "X-engine launch");
        p->slot_count[s.slot] += s.nframes;
    }
    p->pending = false;
    return ok();
}

static mwax_status emit(mwax_plan p, void *d_vis, float *d_scales, int32_t max_ints, int32_t *n_emitted,
                        int32_t order, int32_t F = 1, const float *avg_w = nullptr) {
    int32_t n = 0;
    const double post = p->xprec == MWAX_X_FP16 ? std::ldexp(1.0, 2 * fp16_exponent(p->L)) : 1.0;
    const int Lout = p->L / p->favg;   // channels held by the integrators as emitted
    const size_t per_int = order == MWAX_ORDER_TILE_BL ? (size_t)p->d.n_baselines * Lout * 4
                           : order == 3                ? (size_t)(p->L / F) * p->P
                                                       : (size_t)Lout * p->P;
    const size_t esz = order == 2 ? 16 : 8;
    const bool pre = p->favg > 1;   // averaged in the X-engine: FP64 integrators [L / favg][P]
    while (n < max_ints) {
        const int64_t j = p->next_emit;
        const int slot = (int)(j % p->nslots);
        if (p->slot_owner[slot] != j || p->slot_count[slot] < p->T) break;
        PackArgs a{};
        a.integ = (uint8_t *)p->integ + (size_t)slot * p->slot_bytes;
        a.is_int = p->xprec == MWAX_X_INT8 && !pre;
        a.scales = p->scales + (size_t)slot * 2 * p->L;
        a.post = post;
        a.out = (uint8_t *)d_vis + (size_t)n * per_int * esz;
        a.scales_out = d_scales ? d_scales + (size_t)n * p->L : nullptr;
        a.order = order;
        a.clear = p->clear_on_emit && !pre;
        a.i32 = p->integ32;
        a.L = pre ? p->L / p->favg : p->L;
        a.n_in = p->n_in;
        a.P = p->P;
        a.F = F;
        a.avg_w = avg_w ? avg_w + (size_t)n * p->P : nullptr;
        hipError_t e = timed(p, 2, [&] { return launch_pack(a, p->stream); });
        if (e != hipSuccess) return hip_fail(e, "pack launch");
        p->slot_owner[slot] = -1;
        p->slot_count[slot] = 0;
        ++p->next_emit;
        ++n;
    }
    *n_emitted = n;
    return ok();
}

mwax_status mwax_integrate(mwax_plan p, void *d_vis, int32_t max_ints, int32_t *n_emitted, int32_t order) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!n_emitted) return fail(MWAX_E_INVAL, "null n_emitted");
    *n_emitted = 0;
    if (max_ints < 0 || (max_ints > 0 && !d_vis)) return fail(MWAX_E_INVAL, "bad output buffer");
    if (order != MWAX_ORDER_CHAN_TRI && order != MWAX_ORDER_TILE_BL) return fail(MWAX_E_INVAL, "unknown order %d", order);
    if (((uintptr_t)d_vis & 7) != 0) return fail(MWAX_E_INVAL, "output must be 8-byte aligned");
    return emit(p, d_vis, nullptr, max_ints, n_emitted, order);
}

mwax_status mwax_integrate_averaged(mwax_plan p, int32_t fscrunch, const float *d_weights, void *d_vis,
                                    int32_t max_ints, int32_t *n_emitted) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!n_emitted) return fail(MWAX_E_INVAL, "null n_emitted");
    *n_emitted = 0;
    if (fscrunch < 1 || p->L % fscrunch != 0)
        return fail(MWAX_E_INVAL, "fscrunch = %d must divide L = %d", fscrunch, p->L);
    if (p->favg > 1)
        return fail(MWAX_E_STATE, "the plan averages in its X-engine (mwax_set_averaging): use mwax_integrate");
    if (max_ints < 0 || (max_ints > 0 && !d_vis)) return fail(MWAX_E_INVAL, "bad output buffer");
    if (((uintptr_t)d_vis & 7) != 0 || ((uintptr_t)d_weights & 3) != 0)
        return fail(MWAX_E_INVAL, "output must be 8-byte and weights 4-byte aligned");
    return emit(p, d_vis, nullptr, max_ints, n_emitted, 3, fscrunch, d_weights);
}

mwax_status mwax_integrate_raw_i64(mwax_plan p, int64_t *d_vis, float *d_scales, int32_t max_ints,
                                   int32_t *n_emitted) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (!n_emitted) return fail(MWAX_E_INVAL, "null n_emitted");
    *n_emitted = 0;
    if (p->xprec != MWAX_X_INT8) return fail(MWAX_E_UNSUPPORTED, "raw int64 output exists for INT8 plans only");
    if (p->favg > 1)
        return fail(MWAX_E_STATE, "the plan averages in its X-engine (mwax_set_averaging): no integer sums are kept");
    if (max_ints < 0 || (max_ints > 0 && !d_vis)) return fail(MWAX_E_INVAL, "bad output buffer");
    if (((uintptr_t)d_vis & 15) != 0) return fail(MWAX_E_INVAL, "output must be 16-byte aligned");
    return emit(p, d_vis, d_scales, max_ints, n_emitted, 2);
}

static bool integration_in_progress(mwax_plan p) {
    if (p->pending) return true;
    for (int s = 0; s < p->nslots; ++s)
        if (p->slot_owner[s] != -1 && p->slot_count[s] < p->T) return true;
    return false;
}

mwax_status mwax_set_scales(mwax_plan p, const float *h_scales) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (p->xprec != MWAX_X_INT8) return fail(MWAX_E_UNSUPPORTED, "scales exist for INT8 plans only");
    if (!h_scales) return fail(MWAX_E_INVAL, "null scales");
    if (integration_in_progress(p)) return fail(MWAX_E_STATE, "an integration is in progress");
    std::vector<float> v(2 * p->L);
    for (int c = 0; c < p->L; ++c) {
        const float s = h_scales[c];
        if (!(s > 0.0f) || !std::isfinite(s)) return fail(MWAX_E_INVAL, "scale %d must be finite and > 0", c);
        v[c] = s;
        v[p->L + c] = 1.0f / s;
    }
    hipError_t e = hipMemcpyAsync(p->fixed, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "scale upload");
    p->fixed_mode = true;
    return ok();
}

mwax_status mwax_get_scales(mwax_plan p, float *d_scales) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (p->xprec != MWAX_X_INT8) return fail(MWAX_E_UNSUPPORTED, "scales exist for INT8 plans only");
    if (!d_scales || ((uintptr_t)d_scales & 3) != 0) return fail(MWAX_E_INVAL, "null or misaligned output");
    if (p->last_slot < 0) return fail(MWAX_E_STATE, "no integration has begun");
    hipError_t e = launch_copy_scales(p->scales + (size_t)p->last_slot * 2 * p->L, d_scales, p->L, p->stream);
    if (e != hipSuccess) return hip_fail(e, "scale copy");
    return ok();
}

mwax_status mwax_auto_scales(mwax_plan p) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (p->xprec != MWAX_X_INT8) return fail(MWAX_E_UNSUPPORTED, "scales exist for INT8 plans only");
    if (integration_in_progress(p)) return fail(MWAX_E_STATE, "an integration is in progress");
    p->fixed_mode = false;
    return ok();
}

mwax_status mwax_set_delays(mwax_plan p, const float *d_delays, int64_t n_steps, int64_t step_samples,
                            double sky_freq_hz) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (p->batched) return fail(MWAX_E_UNSUPPORTED, "delay correction is not applied by batches");
    if (p->pending) return fail(MWAX_E_STATE, "the previous channelised block has not been correlated");
    if (!d_delays) {
        p->dl = nullptr;
        p->dl_steps = 0;
        return ok();
    }
    if (((uintptr_t)d_delays & 3) != 0) return fail(MWAX_E_INVAL, "delay table must be 4-byte aligned");
    if (n_steps < 1) return fail(MWAX_E_INVAL, "n_steps must be >= 1");
    if (step_samples < p->L || step_samples % p->L != 0 || step_samples / p->L > 0x7fffffff)
        return fail(MWAX_E_INVAL, "step_samples = %lld must be a positive multiple of L = %d",
                    (long long)step_samples, p->L);
    if (!std::isfinite(sky_freq_hz)) return fail(MWAX_E_INVAL, "sky frequency must be finite");
    p->dl = d_delays;
    p->dl_steps = n_steps;
    p->dl_fps = (int32_t)(step_samples / p->L);
    p->dl_pos0 = p->g_chan;
    p->dl_nu = sky_freq_hz / p->cfg.coarse_bw_hz;
    return ok();
}

mwax_status mwax_reset(mwax_plan p) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    hipError_t e = launch_fill_zero(p->integ, p->slot_bytes * p->nslots, p->stream);
    if (e == hipSuccess) e = launch_copy_scales(p->ones, p->last, 2 * p->L, p->stream);
    if (e != hipSuccess) return hip_fail(e, "reset");
    p->last_slot = -1;
    std::fill(p->slot_owner.begin(), p->slot_owner.end(), -1);
    std::fill(p->slot_count.begin(), p->slot_count.end(), 0);
    p->g_chan = 0;
    p->next_emit = 0;
    p->dl = nullptr;
    p->dl_steps = 0;
    p->pending = false;
    p->have_block = false;
    p->segs.clear();
    return ok();
}

mwax_status mwax_set_averaging(mwax_plan p, int32_t fscrunch) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (fscrunch < 1 || p->L % fscrunch != 0)
        return fail(MWAX_E_INVAL, "fscrunch = %d must divide L = %d", fscrunch, p->L);
    if (fscrunch > 1 && p->xprec == MWAX_X_FP32)
        return fail(MWAX_E_UNSUPPORTED, "averaging in the X-engine runs on the matrix cores (INT8 or FP16 plans)");
    if (p->in_batch) return fail(MWAX_E_UNSUPPORTED, "batch and stream instances do not average in their X-engine");
    if (fscrunch > 1 && xengine_tile_count(p->n_in, kXTileSmall) * (int64_t)(p->L / fscrunch) > INT32_MAX)
        return fail(MWAX_E_UNSUPPORTED, "too many work items");
    // the FP64 output-channel integrators must fit a slot
    if (fscrunch > 1 && (size_t)(p->L / fscrunch) * (size_t)p->P * 16 > p->slot_bytes)
        return fail(MWAX_E_UNSUPPORTED, "averaged integrators (%d channels) exceed the plan's slots", p->L / fscrunch);
    const bool fresh = p->g_chan == 0 && !p->pending &&
                       std::all_of(p->slot_owner.begin(), p->slot_owner.end(), [](int64_t o) { return o == -1; });
    if (!fresh) return fail(MWAX_E_STATE, "averaging is chosen before the first block (or after mwax_reset)");
    p->favg = fscrunch;
    return ok();
}

mwax_status mwax_sync(mwax_plan p) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronisation");
    return ok();
}

mwax_status mwax_set_timing(mwax_plan p, int32_t enable) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    p->timing = enable != 0;
    return ok();
}

mwax_status mwax_kernel_time(mwax_plan p, int32_t family, double *total_ms, int64_t *launches) {
    if (check_plan(p) != MWAX_OK) return MWAX_E_INVAL;
    if (family < 0 || family > 3 || !total_ms || !launches) return fail(MWAX_E_INVAL, "bad arguments");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronisation");
    for (auto &ev : p->events) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
            p->t_ms[ev.fam] += ms;
            p->t_n[ev.fam] += 1;
        }
        p->pool.push_back(ev.a);
        p->pool.push_back(ev.b);
    }
    p->events.clear();
    *total_ms = p->t_ms[family];
    *launches = p->t_n[family];
    p->t_ms[family] = 0.0;
    p->t_n[family] = 0;
    return ok();
}

}  // extern "C"
