// Host-side state of a plan, shared by the single-plan and batch runtimes of
// libmwax (not part of the C ABI).
#pragma once

#include <string>
#include <vector>

#include "mwax_internal.h"

namespace mwax {

// Error reporting: set the calling thread's last-error message and return s.
mwax_status fail(mwax_status s, const char *fmt, ...);
mwax_status ok();
mwax_status hip_fail(hipError_t e, const char *what);

constexpr int64_t kCalSamples = 131072;   // calibration window: 0.1024 s at 1.28 Msps

struct Segment {
    int64_t j;        // integration index
    int slot;         // device slot
    int64_t frame0;   // first spectrum of the segment within the call
    int64_t nframes;  // spectra in the segment
    int64_t grp0;     // first row group in the channel-major buffer
    int64_t ngrp;     // row groups
    int64_t local0;   // offset of the first spectrum within integration j
};

}  // namespace mwax

struct mwax_plan_s {
    mwax_config cfg{};
    mwax_dims d{};
    hipStream_t stream = nullptr;
    int device = 0;
    int L = 0, G = 0, n_in = 0, xprec = 0, R = 1, ntiles = 0;
    int64_t T = 0, P = 0;

    uint8_t *chan = nullptr;
    int64_t NG = 0;
    void *integ = nullptr;
    size_t slot_bytes = 0;
    bool integ32 = false;           // INT8 integrators are int32 pairs (T <= kInt32MaxSpectra)
    int nslots = 0;
    float *scales = nullptr;        // [nslots][2][L] (s, inv_s)
    float *fixed = nullptr;         // [2][L] user scales
    float *ones = nullptr;          // [2][L] = 1
    float *last = nullptr;          // [2][L] scales of the most recent calibrated integration
    int last_slot = -1;             // slot of the most recently begun integration
    float2 *tw = nullptr;
    double *stats = nullptr;        // [kStatsMaxWG][L + 1]
    uint8_t *mid = nullptr;         // L = 6400: frame-major spectra of a call [n_in][max_spectra][L][2]

    int64_t g_chan = 0;             // stream spectra channelised (incl. the pending block)
    bool pending = false;           // a channelised block awaits mwax_correlate
    bool have_block = false;        // the buffer holds a block (for read-back)
    int64_t block_spectra = 0;
    std::vector<mwax::Segment> segs;
    std::vector<int64_t> slot_owner, slot_count;
    int64_t next_emit = 0;
    bool fixed_mode = false;
    bool in_batch = false;          // owned by a batch or stream (destroyed with it)
    bool static_ws = false;         // workspace lives in the library's static device array
    bool batched = false;           // an instance of a batch (its F-engine runs from batch tables)
    // fractional delay and phase correction (mwax_set_delays): caller's table
    // [n_in][dl_steps] of delays in samples; step s covers stream frames
    // dl_pos0 + s dl_fps .. dl_pos0 + (s + 1) dl_fps - 1
    const float *dl = nullptr;
    int64_t dl_steps = 0;
    int32_t dl_fps = 0;
    int64_t dl_pos0 = 0;
    double dl_nu = 0.0;             // sky frequency / coarse bandwidth
    // Clear a slot's integrators when its integration is emitted.  Off only where
    // every integration's first X-engine flush overwrites the whole slot
    // (whole-segment INT8/FP16 work of a batch); mwax_correlate clears a slot
    // itself before accumulating into one that was not cleared.
    bool clear_on_emit = true;
    // X-engine launches run whole segments (no K-chunks with atomic flushes).
    // Chunks fill the resident slots of a launch running alone; the stream
    // runtime sets this, because its two lanes fill each other's launch tails.
    bool whole_segments = false;
    int favg = 1;                   // mwax_set_averaging: fine channels per emitted channel

    bool timing = false;
    struct Ev { hipEvent_t a, b; int fam; };
    std::vector<Ev> events;
    std::vector<hipEvent_t> pool;
    double t_ms[4] = {0, 0, 0, 0};
    int64_t t_n[4] = {0, 0, 0, 0};
};

namespace mwax {

inline hipEvent_t get_event(mwax_plan p) {
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Wraps a launch with timing events when timing is on.
template <class F>
hipError_t timed(mwax_plan p, int fam, F &&launch) {
    if (!p->timing) return launch();
    hipEvent_t a = get_event(p), b = get_event(p);
    if (!a || !b) return hipErrorOutOfMemory;
    (void)hipEventRecord(a, p->stream);
    hipError_t e = launch();
    (void)hipEventRecord(b, p->stream);
    p->events.push_back({a, b, fam});
    return e;
}

mwax_status derive(const mwax_config *cfg, mwax_dims *o);
void free_plan(mwax_plan p);
// Split a block of M spectra at integration boundaries and check slot use.
mwax_status plan_segments(mwax_plan p, int64_t M, std::vector<Segment> &out);
// Per-integration scale calibration launch arguments of a segment that begins an
// integration (INT8, automatic scales).
FArgs calib_args(mwax_plan p, const Segment &s, const int8_t *volts, int64_t ld);
// F-engine main-pass launch arguments of a segment.
FArgs fengine_args(mwax_plan p, const Segment &s, const int8_t *volts, int64_t ld);
// Statistics-pass workgroups of a calibration launch (rows of its partial sums).
int stats_grid(mwax_plan p, const FArgs &a);
// The F-engine main pass of one segment: the fused single-kernel transform, or
// for L = 6400 the frame-major transform followed by the corner-turn.
hipError_t launch_fengine_segment(mwax_plan p, const Segment &s, const FArgs &a);
// X-engine launch arguments of a segment.
XArgs xengine_args(mwax_plan p, const Segment &s);

}  // namespace mwax
