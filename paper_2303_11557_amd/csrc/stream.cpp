// Real-time streaming runtime of libmwax (Sec. 2.4: 8 s sub-observation blocks
// per coarse channel arrive continuously; Sec. 3.4: each must be correlated in
// less than its own duration).
//
// A pool of device block buffers, sized by an HBM budget, is the admission
// control: a producer acquires a free buffer, writes a block into it on the
// ingest stream and submits it for a channel.  The channel's lane stream waits
// for the ingest, runs that channel's plan over the block and emits its
// completed integrations into the channel's device output ring.  Channels
// alternate between two lane streams, so the launches of neighbouring channels
// overlap and fill each other's drain tails (a 1 s call at 256 tiles is a pair
// of ~1 ms launches); the compute stream then waits for the block's lane, so
// blocks complete, and work a caller enqueues on the compute stream runs, in
// submission order.  A buffer returns to the pool when the event recorded after
// its block's work has completed.  Ready
// times are event timestamps converted to the stream clock through a reference
// event recorded (and waited for) at creation.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "plan.h"

using namespace mwax;

namespace {

constexpr int kMaxChannels = 64;
constexpr int kLanes = 2;   // per-channel work streams (with ingest and compute: 4 hardware queues)

enum SlotState { kFree = 0, kAcquired = 1, kBusy = 2 };

struct InFlight {
    mwax_block_done rec;
    hipEvent_t done;    // on the compute stream, after the block's work
    hipEvent_t join;    // on the block's lane stream (waited for by the compute stream)
};

}  // namespace

struct mwax_stream_s {
    mwax_stream_config cfg{};
    int device = 0;
    hipStream_t ingest = nullptr, compute = nullptr;
    hipStream_t lanes[kLanes] = {};
    std::vector<mwax_plan> plans;
    std::vector<int64_t> blocks_seen;       // per channel
    std::vector<int64_t> reported_end;      // per channel: integrations [0, end) returned by poll
    int n_in = 0, L = 0;
    int64_t P = 0;
    uint64_t block_bytes = 0;
    std::vector<int8_t *> pool;
    std::vector<int> state;
    std::vector<hipEvent_t> ingest_ev;
    std::deque<InFlight> inflight;
    std::vector<mwax_block_done> finished;  // retired, not yet reported by poll
    std::vector<hipEvent_t> ev_pool;
    std::vector<void *> ring;               // per channel [out_depth][L][P] complex64
    uint64_t device_bytes = 0;
    hipEvent_t ev_ref = nullptr;
    std::chrono::steady_clock::time_point t0;
    double t_ref = 0.0;                     // stream-clock time of ev_ref
};

namespace {

double now_s(mwax_stream s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

void free_stream(mwax_stream s) {
    if (!s) return;
    for (auto l : s->lanes)
        if (l) (void)hipStreamSynchronize(l);
    if (s->compute) (void)hipStreamSynchronize(s->compute);
    if (s->ingest) (void)hipStreamSynchronize(s->ingest);
    for (auto &f : s->inflight) {
        (void)hipEventDestroy(f.done);
        (void)hipEventDestroy(f.join);
    }
    for (auto e : s->ev_pool) (void)hipEventDestroy(e);
    for (auto e : s->ingest_ev) (void)hipEventDestroy(e);
    if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
    for (auto p : s->pool) (void)hipFree(p);
    for (auto r : s->ring) (void)hipFree(r);
    for (auto p : s->plans) free_plan(p);
    if (s->ingest) (void)hipStreamDestroy(s->ingest);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    for (auto l : s->lanes)
        if (l) (void)hipStreamDestroy(l);
    delete s;
}

hipEvent_t stream_event(mwax_stream s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Retire the oldest in-flight block if its work has finished (or, with wait,
// once it has).  Returns 1 if a block was retired, 0 if not, < 0 on error.
int retire_front(mwax_stream s, bool wait, mwax_block_done *out) {
    if (s->inflight.empty()) return 0;
    InFlight &f = s->inflight.front();
    hipError_t e = wait ? hipEventSynchronize(f.done) : hipEventQuery(f.done);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) {
        hip_fail(e, "stream block completion");
        return -1;
    }
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, s->ev_ref, f.done);
    if (e != hipSuccess) {
        hip_fail(e, "stream event timing");
        return -1;
    }
    f.rec.t_ready_s = s->t_ref + (double)ms * 1e-3;
    if (out) *out = f.rec;
    s->state[f.rec.slot] = kFree;
    s->ev_pool.push_back(f.done);
    s->ev_pool.push_back(f.join);
    s->inflight.pop_front();
    return 1;
}

// Wait for a finished block for up to wait_ms (< 0: without limit); its record
// goes to *done.
int wait_one(mwax_stream s, int32_t wait_ms, std::vector<mwax_block_done> *done) {
    mwax_block_done rec{};
    int r = retire_front(s, false, &rec);
    if (r != 0 || s->inflight.empty() || wait_ms == 0) {
        if (r > 0 && done) done->push_back(rec);
        return r;
    }
    if (wait_ms < 0) {
        r = retire_front(s, true, &rec);
    } else {
        const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(wait_ms);
        while ((r = retire_front(s, false, &rec)) == 0 && std::chrono::steady_clock::now() < until)
            std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    if (r > 0 && done) done->push_back(rec);
    return r;
}

}  // namespace

extern "C" {

mwax_status mwax_stream_create(const mwax_stream_config *cfg, mwax_stream *out) {
    if (!out) return fail(MWAX_E_INVAL, "null output handle");
    *out = nullptr;
    if (!cfg) return fail(MWAX_E_INVAL, "null configuration");
    if (cfg->n_channels < 1 || cfg->n_channels > kMaxChannels)
        return fail(MWAX_E_INVAL, "n_channels must be in 1..%d", kMaxChannels);
    if (cfg->out_depth < 1) return fail(MWAX_E_INVAL, "out_depth must be >= 1");
    mwax_dims d;
    mwax_status st = derive(&cfg->cfg, &d);
    if (st != MWAX_OK) return st;
    if (cfg->block_samples <= 0 || cfg->block_samples % cfg->cfg.max_samples != 0)
        return fail(MWAX_E_INVAL, "block_samples must be a positive multiple of max_samples = %lld",
                    (long long)cfg->cfg.max_samples);
    if (cfg->cfg.max_samples % 8 != 0) return fail(MWAX_E_INVAL, "max_samples must be a multiple of 8");
    const uint64_t block_bytes = (uint64_t)d.n_inputs * (uint64_t)cfg->block_samples * 2;
    const uint64_t slots = cfg->hbm_budget_bytes / block_bytes;
    if (slots < 1)
        return fail(MWAX_E_INVAL, "an HBM budget of %llu bytes holds no %llu-byte block",
                    (unsigned long long)cfg->hbm_budget_bytes, (unsigned long long)block_bytes);

    mwax_stream s = new (std::nothrow) mwax_stream_s;
    if (!s) return fail(MWAX_E_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    (void)hipGetDevice(&s->device);
    s->n_in = d.n_inputs;
    s->L = d.fft_len;
    s->P = d.n_pairs;
    s->block_bytes = block_bytes;
    hipError_t e = hipStreamCreateWithFlags(&s->ingest, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
    for (int l = 0; l < kLanes && e == hipSuccess; ++l) e = hipStreamCreateWithFlags(&s->lanes[l], hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_stream(s);
        return hip_fail(e, "stream creation");
    }
    for (int k = 0; k < cfg->n_channels; ++k) {
        mwax_plan p = nullptr;
        st = mwax_plan_create(&cfg->cfg, s->lanes[k % kLanes], &p);
        if (st != MWAX_OK) {
            std::string m = mwax_last_error();
            free_stream(s);
            return fail(st, "channel %d: %s", k, m.c_str());
        }
        p->in_batch = true;
        p->whole_segments = true;                       // the lanes fill each other's tails
        p->clear_on_emit = p->xprec == MWAX_X_FP32;     // whole segments overwrite a slot
        s->plans.push_back(p);
        s->device_bytes += d.workspace_bytes;
        void *r = nullptr;
        const size_t rb = (size_t)cfg->out_depth * s->L * s->P * 8;
        e = hipMalloc(&r, rb);
        if (e != hipSuccess) {
            free_stream(s);
            return hip_fail(e, "output ring allocation");
        }
        s->ring.push_back(r);
        s->device_bytes += rb;
    }
    s->blocks_seen.assign(cfg->n_channels, 0);
    s->reported_end.assign(cfg->n_channels, 0);
    for (uint64_t k = 0; k < slots; ++k) {
        void *b = nullptr;
        e = hipMalloc(&b, block_bytes);
        if (e != hipSuccess) {
            free_stream(s);
            return hip_fail(e, "block pool allocation");
        }
        s->pool.push_back((int8_t *)b);
        s->state.push_back(kFree);
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_stream(s);
            return hip_fail(e, "event creation");
        }
        s->ingest_ev.push_back(ev);
        s->device_bytes += block_bytes;
    }
    e = hipEventCreate(&s->ev_ref);
    if (e == hipSuccess) e = hipEventRecord(s->ev_ref, s->compute);
    if (e == hipSuccess) e = hipEventSynchronize(s->ev_ref);
    s->t_ref = now_s(s);
    if (e != hipSuccess) {
        free_stream(s);
        return hip_fail(e, "stream clock reference");
    }
    *out = s;
    return ok();
}

mwax_status mwax_stream_destroy(mwax_stream s) {
    free_stream(s);
    return ok();
}

mwax_status mwax_stream_get_info(mwax_stream s, mwax_stream_info *out) {
    if (!s || !out) return fail(MWAX_E_INVAL, "null argument");
    out->pool_slots = (int32_t)s->pool.size();
    out->n_inputs = s->n_in;
    out->block_bytes = s->block_bytes;
    out->block_ld = s->cfg.block_samples;
    out->ingest_stream = s->ingest;
    out->compute_stream = s->compute;
    out->device_bytes = s->device_bytes;
    return ok();
}

mwax_status mwax_stream_plan(mwax_stream s, int32_t channel, mwax_plan *out) {
    if (!s || !out) return fail(MWAX_E_INVAL, "null argument");
    if (channel < 0 || channel >= s->cfg.n_channels) return fail(MWAX_E_INVAL, "channel %d out of range", channel);
    *out = s->plans[channel];
    return ok();
}

mwax_status mwax_stream_now(mwax_stream s, double *t) {
    if (!s || !t) return fail(MWAX_E_INVAL, "null argument");
    *t = now_s(s);
    return ok();
}

mwax_status mwax_stream_acquire(mwax_stream s, int32_t wait_ms, int32_t *slot, int8_t **d_block) {
    if (!s || !slot || !d_block) return fail(MWAX_E_INVAL, "null argument");
    auto &pend = s->finished;
    for (;;) {
        for (size_t k = 0; k < s->pool.size(); ++k)
            if (s->state[k] == kFree) {
                s->state[k] = kAcquired;
                *slot = (int32_t)k;
                *d_block = s->pool[k];
                return ok();
            }
        // every buffer is acquired or in flight: wait for the oldest block
        const int r = wait_one(s, wait_ms, &pend);
        if (r < 0) return MWAX_E_DEVICE;
        if (r == 0) return fail(MWAX_E_STATE, "HBM budget exhausted: all %zu block buffers are in use",
                                s->pool.size());
    }
}

mwax_status mwax_stream_copy_in(mwax_stream s, int32_t slot, const int8_t *h_block, int64_t h_ld) {
    if (!s || !h_block) return fail(MWAX_E_INVAL, "null argument");
    if (slot < 0 || slot >= (int32_t)s->pool.size() || s->state[slot] != kAcquired)
        return fail(MWAX_E_STATE, "slot %d is not acquired", slot);
    if (h_ld < s->cfg.block_samples) return fail(MWAX_E_INVAL, "h_ld must be >= block_samples");
    const size_t row = (size_t)s->cfg.block_samples * 2;
    hipError_t e = hipMemcpy2DAsync(s->pool[slot], row, h_block, (size_t)h_ld * 2, row, (size_t)s->n_in,
                                    hipMemcpyHostToDevice, s->ingest);
    if (e != hipSuccess) return hip_fail(e, "block copy");
    return ok();
}

mwax_status mwax_stream_submit(mwax_stream s, int32_t slot, int32_t channel, double t_arrival_s) {
    if (!s) return fail(MWAX_E_INVAL, "null stream");
    if (channel < 0 || channel >= s->cfg.n_channels) return fail(MWAX_E_INVAL, "channel %d out of range", channel);
    if (slot < 0 || slot >= (int32_t)s->pool.size() || s->state[slot] != kAcquired)
        return fail(MWAX_E_STATE, "slot %d is not acquired", slot);
    mwax_plan p = s->plans[channel];
    if (p->pending) return fail(MWAX_E_STATE, "channel %d has a pending block", channel);
    // the emitted integrations must fit the ring without overwriting each other
    const int64_t max_new = (s->cfg.block_samples / s->L + p->T - 1) / p->T + 1;
    if (max_new > s->cfg.out_depth)
        return fail(MWAX_E_INVAL, "a block can complete %lld integrations; out_depth is %d", (long long)max_new,
                    s->cfg.out_depth);
    // Back-pressure on the output ring: integration j overwrites the entry of
    // j - out_depth.  Every entry this block overwrites must belong to an
    // integration that poll has already returned (the caller has been told it
    // is ready, and its reads of it come before this submit).  The block
    // completes integrations next_emit .. end_int - 1 (every earlier completed
    // one has been emitted: the lane emits after each call).
    const int64_t end_int = (p->g_chan + s->cfg.block_samples / s->L) / p->T;
    const int64_t newest_victim = end_int - 1 - s->cfg.out_depth;
    if (newest_victim >= 0 && newest_victim >= s->reported_end[channel])
        return fail(MWAX_E_STATE,
                    "channel %d: this block could overwrite integration %lld in the output ring, which "
                    "mwax_stream_poll has not returned yet (poll first, or raise out_depth)",
                    channel, (long long)newest_victim);
    hipEvent_t done = stream_event(s);
    if (!done) return fail(MWAX_E_NOMEM, "event creation");
    hipEvent_t join = stream_event(s);
    if (!join) {
        s->ev_pool.push_back(done);
        return fail(MWAX_E_NOMEM, "event creation");
    }
    mwax_block_done rec{};
    rec.channel = channel;
    rec.slot = slot;
    rec.block = s->blocks_seen[channel];
    rec.first_int = p->next_emit;
    rec.t_arrival_s = t_arrival_s;
    rec.t_submit_s = now_s(s);

    hipStream_t lane = s->lanes[channel % kLanes];
    hipError_t e = hipEventRecord(s->ingest_ev[slot], s->ingest);
    if (e == hipSuccess) e = hipStreamWaitEvent(lane, s->ingest_ev[slot], 0);
    if (e != hipSuccess) {
        s->ev_pool.push_back(done);
        s->ev_pool.push_back(join);
        return hip_fail(e, "ingest ordering");
    }
    const int64_t chunk = s->cfg.cfg.max_samples, ld = s->cfg.block_samples;
    const size_t per_int = (size_t)s->L * s->P * 8;
    int32_t n_ints = 0;
    mwax_status st = MWAX_OK;
    for (int64_t off = 0; off < s->cfg.block_samples && st == MWAX_OK; off += chunk) {
        st = mwax_channelise(p, s->pool[slot] + off * 2, chunk, ld);
        if (st == MWAX_OK) st = mwax_correlate(p);
        // emit after every call: completed integrations free their device slots
        while (st == MWAX_OK) {
            const int64_t j = p->next_emit;
            const int32_t room = (int32_t)(s->cfg.out_depth - j % s->cfg.out_depth);
            int32_t n = 0;
            st = mwax_integrate(p, (uint8_t *)s->ring[channel] + (size_t)(j % s->cfg.out_depth) * per_int, room,
                                &n, MWAX_ORDER_CHAN_TRI);
            if (st != MWAX_OK || n == 0) break;
            n_ints += n;
        }
    }
    // The plan calls validated their arguments up front, so a failure here is a
    // device error; the buffer still stays busy until the work enqueued on it ends.
    // The compute stream joins the lane.
    e = hipEventRecord(join, lane);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->compute, join, 0);
    if (e == hipSuccess) e = hipEventRecord(done, s->compute);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(lane);
        (void)hipStreamSynchronize(s->compute);
        s->ev_pool.push_back(done);
        s->ev_pool.push_back(join);
        s->state[slot] = kFree;
        return hip_fail(e, "completion event");
    }
    rec.n_ints = n_ints;
    s->state[slot] = kBusy;
    s->blocks_seen[channel] += 1;
    s->inflight.push_back({rec, done, join});
    return st == MWAX_OK ? ok() : st;
}

mwax_status mwax_stream_poll(mwax_stream s, int32_t wait_ms, mwax_block_done *out, int32_t max, int32_t *n) {
    if (!s || !n || (max > 0 && !out)) return fail(MWAX_E_INVAL, "null argument");
    *n = 0;
    auto &pend = s->finished;
    if (pend.empty()) {
        const int r = wait_one(s, wait_ms, &pend);
        if (r < 0) return MWAX_E_DEVICE;
    }
    for (;;) {   // everything else already finished
        mwax_block_done rec{};
        const int r = retire_front(s, false, &rec);
        if (r < 0) return MWAX_E_DEVICE;
        if (r == 0) break;
        pend.push_back(rec);
    }
    const int32_t k = std::min<int32_t>(max, (int32_t)pend.size());
    for (int32_t i = 0; i < k; ++i) {
        out[i] = pend[i];
        s->reported_end[pend[i].channel] = pend[i].first_int + pend[i].n_ints;
    }
    pend.erase(pend.begin(), pend.begin() + k);
    *n = k;
    return ok();
}

mwax_status mwax_stream_vis(mwax_stream s, int32_t channel, int64_t j, void **d_vis) {
    if (!s || !d_vis) return fail(MWAX_E_INVAL, "null argument");
    if (channel < 0 || channel >= s->cfg.n_channels) return fail(MWAX_E_INVAL, "channel %d out of range", channel);
    mwax_plan p = s->plans[channel];
    if (j < 0 || j >= s->reported_end[channel] || j < p->next_emit - s->cfg.out_depth)
        return fail(MWAX_E_STATE, "integration %lld of channel %d is not in the output ring (not yet returned "
                    "by mwax_stream_poll, or overwritten)", (long long)j, channel);
    *d_vis = (uint8_t *)s->ring[channel] + (size_t)(j % s->cfg.out_depth) * s->L * s->P * 8;
    return ok();
}

}  // extern "C"
