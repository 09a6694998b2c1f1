// Batch runtime of libmwax: many per-coarse-channel plans (Sec. 2.1: one
// coarse channel per server, up to 24) driven as one unit of device work.
//
// Per call the host splits every instance's block into segments exactly as a
// single plan does, then writes three kinds of device work tables:
//   F-engine descriptors (one table per distinct L, for the calibration
//     statistics pass and for the main pass), each with the range of workgroups
//     of the fixed-size launch that serve it;
//   calibration-finish descriptors, one per integration that begins;
//   X-engine descriptors (one per segment) and work items (tile x channel x
//     chunk of row groups) in 8 per-XCD queues, balanced by longest-first
//     assignment of (segment, channel, chunk) units, the tiles of a unit kept
//     together in one queue so they share that XCD's L2.
// The tables go to the device in one copy from pinned host memory; then the
// fixed launch sequence runs, captured once as a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "plan.h"

using namespace mwax;

namespace {

constexpr int kMaxInstances = 64;
constexpr int kMainGridCap = 8192;    // F-engine workgroups per launch: tens of items each
constexpr int kUnitOverheadGroups = 16;   // setup + flush of a tile item, in row-group units

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct FTable {        // one batched F-engine launch
    size_t off_n = 0, off_b0 = 0, off_desc = 0;
    int max_desc = 0;
    int grid = 0;
};

struct LGroup {
    int L = 0;
    std::vector<int> members;
    FTable stats, main;
    size_t stats_off = 0;   // doubles into the batch statistics buffer
};

}  // namespace

struct mwax_batch_s {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int n = 0;
    int xprec = 0;
    std::vector<mwax_plan> inst;
    std::vector<int> max_segs;      // per instance: segments one call can hold
    std::vector<LGroup> groups;
    std::vector<int> group_of;

    // tuning
    std::vector<int> kchunk;        // row groups per X item, 0 = whole segment
    std::vector<int> tile;          // X-engine tile edge per instance (128 or 64)
    int xgrid = 0, xgrid_max = 0;
    std::string cache_path;         // autotuner's on-disk cache ("" = none)

    // tables
    size_t bytes = 0, off_upload = 0;
    size_t off_counters = 0, off_cal_n = 0, off_cal = 0, off_xq = 0, off_xdesc = 0, off_items = 0;
    int max_cal = 0, max_L = 1, max_xdesc = 0;
    int64_t max_items = 0;
    uint8_t *d_tab = nullptr;
    uint8_t *h_tab[2] = {nullptr, nullptr};
    hipEvent_t up_ev[2] = {nullptr, nullptr};
    int stage = 0;
    double *d_stats = nullptr;
    size_t stats_doubles = 0;

    // graph
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    // timing
    bool timing = false;
    struct Ev { hipEvent_t a, b; int fam; };
    std::vector<Ev> events;
    std::vector<hipEvent_t> pool;
    double t_ms[5] = {0, 0, 0, 0, 0};
    int64_t t_n[5] = {0, 0, 0, 0, 0};
};

namespace {

hipEvent_t batch_event(mwax_batch b) {
    if (!b->pool.empty()) {
        hipEvent_t e = b->pool.back();
        b->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <class F>
hipError_t btimed(mwax_batch b, int fam, bool on, F &&launch) {
    if (!on) return launch();
    hipEvent_t a = batch_event(b), c = batch_event(b);
    if (!a || !c) return hipErrorOutOfMemory;
    (void)hipEventRecord(a, b->stream);
    hipError_t e = launch();
    (void)hipEventRecord(c, b->stream);
    b->events.push_back({a, c, fam});
    return e;
}

void drop_graph(mwax_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void free_tables(mwax_batch b) {
    drop_graph(b);
    (void)hipFree(b->d_tab);
    (void)hipFree(b->d_stats);
    for (int k = 0; k < 2; ++k) {
        (void)hipHostFree(b->h_tab[k]);
        b->h_tab[k] = nullptr;
    }
    b->d_tab = nullptr;
    b->d_stats = nullptr;
}

void free_batch(mwax_batch b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_tables(b);
    for (int k = 0; k < 2; ++k)
        if (b->up_ev[k]) (void)hipEventDestroy(b->up_ev[k]);
    for (auto &e : b->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto e : b->pool) (void)hipEventDestroy(e);
    for (mwax_plan p : b->inst) free_plan(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Effective chunk of instance i: 0 (whole segments) or at least enough row
// groups that a segment has at most kXBatchMaxSplit chunks.
int64_t eff_chunk(mwax_batch b, int i) {
    const int kc = b->kchunk[i];
    if (kc <= 0) return 0;
    const int64_t need = ceil_div(b->inst[i]->NG, kXBatchMaxSplit);
    return std::max<int64_t>(kc, need);
}

int nblk_of(mwax_plan p) { return (p->n_in + p->R - 1) / p->R; }

// X-engine tiles per channel of instance i at its tile edge.
int ntiles_of(mwax_batch b, int i) { return xengine_tile_count(b->inst[i]->n_in, b->tile[i]); }
// Tile edges instance i may take: a work item names its tile in 8 bits.
bool tile_allowed(mwax_batch b, int i, int te) {
    return (te == kXTile || te == kXTileSmall) && xengine_tile_count(b->inst[i]->n_in, te) <= kXBatchMaxTiles;
}

// Whole-segment work items overwrite a slot with the first flush of each
// integration, so emitting an integration need not clear its slot; chunked INT8
// items add atomically and need cleared slots.  Slots emitted without clearing
// are cleared when an instance switches to chunked items.
mwax_status apply_clear_policy(mwax_batch b) {
    for (int i = 0; i < b->n; ++i) {
        mwax_plan p = b->inst[i];
        const bool clear = b->kchunk[i] > 0;
        if (clear && !p->clear_on_emit) {
            for (int s = 0; s < p->nslots; ++s) {
                if (p->slot_owner[s] != -1) continue;
                hipError_t e = launch_fill_zero((uint8_t *)p->integ + (size_t)s * p->slot_bytes, p->slot_bytes, p->stream);
                if (e != hipSuccess) return hip_fail(e, "slot clear");
            }
        }
        p->clear_on_emit = clear;
    }
    return MWAX_OK;
}

// Table layout and buffers for the current tuning.
mwax_status layout(mwax_batch b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);   // old tables may still be read
    free_tables(b);
    size_t off = (size_t)kXQueues * kXCounterStride * 4;   // queue counters (not uploaded)
    b->off_counters = 0;
    b->off_upload = off;
    size_t stats_d = 0;
    b->max_cal = 0;
    b->max_L = 1;
    b->max_xdesc = 0;
    b->max_items = 0;
    for (LGroup &g : b->groups) {
        int sdesc = 0, mdesc = 0;
        int64_t mitems = 0;
        for (int i : g.members) {
            mwax_plan p = b->inst[i];
            mdesc += b->max_segs[i];
            mitems += (int64_t)(p->NG) * nblk_of(p);
            if (p->xprec == MWAX_X_INT8) sdesc += b->max_segs[i];
        }
        g.stats.max_desc = sdesc;
        g.stats.grid = sdesc * kStatsMaxWG;
        g.main.max_desc = mdesc;
        g.main.grid = (int)std::min<int64_t>(kMainGridCap, std::max<int64_t>(mitems, mdesc));
        g.stats_off = stats_d;
        stats_d += (size_t)sdesc * kStatsMaxWG * stats_row(g.L);
        for (FTable *t : {&g.stats, &g.main}) {
            t->off_n = off;
            off += 16;
            t->off_b0 = off;
            off = align_up(off + (size_t)(t->max_desc + 1) * 4, 16);
            t->off_desc = off;
            off = align_up(off + (size_t)t->max_desc * sizeof(FArgs), 16);
        }
        b->max_L = std::max(b->max_L, g.L);
    }
    for (int i = 0; i < b->n; ++i) {
        mwax_plan p = b->inst[i];
        if (p->xprec == MWAX_X_INT8) b->max_cal += b->max_segs[i];
        b->max_xdesc += b->max_segs[i];
        const int64_t kc = eff_chunk(b, i);
        const int64_t chunks = kc ? ceil_div(p->NG, kc) + b->max_segs[i] : b->max_segs[i];
        b->max_items += (int64_t)p->L * ntiles_of(b, i) * chunks;
    }
    if (b->max_xdesc > kXBatchMaxDesc)
        return fail(MWAX_E_UNSUPPORTED, "batch needs %d segment descriptors per call, at most %d are supported",
                    b->max_xdesc, kXBatchMaxDesc);
    b->off_cal_n = off;
    off += 16;
    b->off_cal = off;
    off = align_up(off + (size_t)b->max_cal * sizeof(CalDesc), 16);
    b->off_xq = off;
    off = align_up(off + (kXQueues + 1) * 4, 16);
    b->off_xdesc = off;
    off = align_up(off + (size_t)b->max_xdesc * sizeof(XDesc), 16);
    b->off_items = off;
    off = align_up(off + (size_t)b->max_items * 4, 256);
    b->bytes = off;
    b->stats_doubles = stats_d;

    hipError_t e = hipMalloc((void **)&b->d_tab, b->bytes);
    if (e == hipSuccess && stats_d) e = hipMalloc((void **)&b->d_stats, stats_d * sizeof(double));
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipHostMalloc((void **)&b->h_tab[k], b->bytes, 0);
    if (e != hipSuccess) {
        free_tables(b);
        return hip_fail(e, "batch table allocation");
    }
    for (int k = 0; k < 2; ++k) std::memset(b->h_tab[k], 0, b->bytes);
    e = hipMemcpyAsync(b->d_tab, b->h_tab[0], b->bytes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch table initialisation");
    return MWAX_OK;
}

template <class T>
T *tab(uint8_t *base, size_t off) { return reinterpret_cast<T *>(base + off); }

// The fixed launch sequence of one batch step.  x_only: just the X-engine (the
// autotuner's trials).
hipError_t launch_sequence(mwax_batch b, bool per_kernel_timing, bool x_only) {
    uint8_t *d = b->d_tab;
    hipError_t e = launch_zero_i32(tab<int32_t>(d, b->off_counters), kXQueues * kXCounterStride, b->stream);
    if (!x_only) {
        for (LGroup &g : b->groups) {
            if (e != hipSuccess || g.stats.grid == 0) continue;
            FBatchArgs a{tab<FArgs>(d, g.stats.off_desc), tab<int32_t>(d, g.stats.off_b0), tab<int32_t>(d, g.stats.off_n)};
            e = btimed(b, 3, per_kernel_timing,
                       [&] { return launch_fengine_batch(g.L, b->xprec, true, a, g.stats.grid, b->stream); });
        }
        if (e == hipSuccess && b->max_cal > 0)
            e = btimed(b, 3, per_kernel_timing, [&] {
                return launch_calib_batch(tab<CalDesc>(d, b->off_cal), tab<int32_t>(d, b->off_cal_n), b->max_cal,
                                          b->max_L, b->stream);
            });
        for (LGroup &g : b->groups) {
            if (e != hipSuccess) break;
            FBatchArgs a{tab<FArgs>(d, g.main.off_desc), tab<int32_t>(d, g.main.off_b0), tab<int32_t>(d, g.main.off_n)};
            e = btimed(b, 0, per_kernel_timing,
                       [&] { return launch_fengine_batch(g.L, b->xprec, false, a, g.main.grid, b->stream); });
        }
    }
    if (e == hipSuccess) {
        XBatchArgs a{tab<XDesc>(d, b->off_xdesc), tab<uint32_t>(d, b->off_items), tab<int32_t>(d, b->off_xq),
                     tab<int32_t>(d, b->off_counters)};
        e = btimed(b, 1, per_kernel_timing, [&] { return launch_xengine_batch(b->xprec, a, b->xgrid, b->stream); });
    }
    return e;
}

mwax_status capture(mwax_batch b) {
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    hipError_t le = launch_sequence(b, false, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le != hipSuccess ? le : e, "graph capture");
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return hip_fail(e, "graph instantiation");
    }
    return MWAX_OK;
}

struct Unit {
    int d, c, k, ntiles;
    int64_t cost;
};

// Host tables of one call, written into staging buffer h.
struct CallTables {
    std::vector<std::vector<FArgs>> fs, fm;     // per group
    std::vector<std::vector<int32_t>> fs_b0, fm_b0;
    std::vector<CalDesc> cal;
    std::vector<XDesc> xd;
    std::vector<int> xd_inst;
    std::vector<int32_t> qbeg;
    std::vector<uint32_t> items;
};

void build_x_tables(mwax_batch b, const std::vector<std::vector<Segment>> &segs, const std::vector<int> &active,
                    CallTables &t) {
    t.xd.clear();
    t.xd_inst.clear();
    std::vector<Unit> units;
    for (int i : active) {
        mwax_plan p = b->inst[i];
        const int64_t kc = eff_chunk(b, i);
        for (const Segment &s : segs[i]) {
            const XArgs xa = xengine_args(p, s);
            XDesc x{};
            x.chan = xa.chan;
            x.NG = xa.NG;
            x.grp0 = xa.grp0;
            x.integ = xa.integ;
            x.P = xa.P;
            x.ngrp = xa.ngrp;
            x.n_in = xa.n_in;
            x.kchunk = (int32_t)(kc ? std::min<int64_t>(kc, s.ngrp) : s.ngrp);
            x.ksplit = (int32_t)ceil_div(s.ngrp, x.kchunk);
            x.first = xa.first;
            x.i32 = xa.i32;
            x.te = b->tile[i];
            const int nt = ntiles_of(b, i);
            const int d = (int)t.xd.size();
            t.xd.push_back(x);
            t.xd_inst.push_back(i);
            for (int c = 0; c < p->L; ++c)
                for (int k = 0; k < x.ksplit; ++k) {
                    const int64_t g = std::min<int64_t>(x.kchunk, s.ngrp - (int64_t)k * x.kchunk);
                    units.push_back({d, c, k, nt, (int64_t)nt * (g + kUnitOverheadGroups)});
                }
        }
    }
    // longest first, each unit to the least-loaded queue
    std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &c) { return a.cost > c.cost; });
    std::vector<std::vector<uint32_t>> q(kXQueues);
    int64_t load[kXQueues] = {0};
    for (const Unit &u : units) {
        int best = 0;
        for (int k = 1; k < kXQueues; ++k)
            if (load[k] < load[best]) best = k;
        load[best] += u.cost;
        for (int tt = 0; tt < u.ntiles; ++tt) q[best].push_back(xitem_pack(u.d, u.c, tt, u.k));
    }
    t.qbeg.assign(kXQueues + 1, 0);
    t.items.clear();
    for (int k = 0; k < kXQueues; ++k) {
        t.qbeg[k] = (int32_t)t.items.size();
        t.items.insert(t.items.end(), q[k].begin(), q[k].end());
    }
    t.qbeg[kXQueues] = (int32_t)t.items.size();
}

// Workgroup ranges proportional to work, at least one each, within grid.
std::vector<int32_t> block_ranges(const std::vector<int64_t> &work, int grid) {
    std::vector<int32_t> b0(work.size() + 1, 0);
    const int64_t total = std::accumulate(work.begin(), work.end(), (int64_t)0);
    const int64_t spare = std::max<int64_t>(0, grid - (int64_t)work.size());
    for (size_t d = 0; d < work.size(); ++d) {
        int64_t nb = 1 + (total > 0 ? spare * work[d] / total : 0);
        nb = std::min<int64_t>(nb, std::max<int64_t>(1, work[d]));
        // whole rounds of the 8 XCDs: the F-engine then hands each XCD one
        // contiguous range of items per round, so the output lines that adjacent
        // items share are completed in one L2
        if (nb >= 8) nb &= ~(int64_t)7;
        b0[d + 1] = (int32_t)(b0[d] + nb);
    }
    return b0;
}

mwax_status write_tables(mwax_batch b, const CallTables &t, size_t *upload_bytes) {
    if ((int64_t)t.items.size() > b->max_items || (int)t.xd.size() > b->max_xdesc || (int)t.cal.size() > b->max_cal)
        return fail(MWAX_E_INVAL, "batch tables overflow (internal bound)");
    // make sure the staging buffer's previous copy has been consumed
    const int k = b->stage;
    if (b->up_ev[k]) {
        hipError_t e = hipEventSynchronize(b->up_ev[k]);
        if (e != hipSuccess) return hip_fail(e, "batch staging");
    }
    uint8_t *h = b->h_tab[k];
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const LGroup &g = b->groups[gi];
        const std::vector<FArgs> *lists[2] = {&t.fs[gi], &t.fm[gi]};
        const std::vector<int32_t> *b0s[2] = {&t.fs_b0[gi], &t.fm_b0[gi]};
        const FTable *tabs[2] = {&g.stats, &g.main};
        for (int w = 0; w < 2; ++w) {
            const FTable &ft = *tabs[w];
            if ((int)lists[w]->size() > ft.max_desc) return fail(MWAX_E_INVAL, "batch F tables overflow (internal bound)");
            *tab<int32_t>(h, ft.off_n) = (int32_t)lists[w]->size();
            std::memcpy(h + ft.off_b0, b0s[w]->data(), b0s[w]->size() * 4);
            if (!lists[w]->empty()) std::memcpy(h + ft.off_desc, lists[w]->data(), lists[w]->size() * sizeof(FArgs));
        }
    }
    *tab<int32_t>(h, b->off_cal_n) = (int32_t)t.cal.size();
    if (!t.cal.empty()) std::memcpy(h + b->off_cal, t.cal.data(), t.cal.size() * sizeof(CalDesc));
    std::memcpy(h + b->off_xq, t.qbeg.data(), t.qbeg.size() * 4);
    if (!t.xd.empty()) std::memcpy(h + b->off_xdesc, t.xd.data(), t.xd.size() * sizeof(XDesc));
    if (!t.items.empty()) std::memcpy(h + b->off_items, t.items.data(), t.items.size() * 4);
    *upload_bytes = b->off_items + t.items.size() * 4 - b->off_upload;
    return MWAX_OK;
}

mwax_status upload(mwax_batch b, size_t nbytes) {
    const int k = b->stage;
    hipError_t e = hipMemcpyAsync(b->d_tab + b->off_upload, b->h_tab[k] + b->off_upload, nbytes,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) {
        if (!b->up_ev[k]) e = hipEventCreateWithFlags(&b->up_ev[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b->up_ev[k], b->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    b->stage ^= 1;
    return MWAX_OK;
}

mwax_status check_batch(mwax_batch b) {
    if (!b) return fail(MWAX_E_INVAL, "null batch");
    return MWAX_OK;
}

// Validate a call and plan its segments without changing any state.
mwax_status prepare_call(mwax_batch b, const int8_t *const *d_volts, const int64_t *n_samples,
                         const int64_t *ld_samples, std::vector<std::vector<Segment>> &segs,
                         std::vector<int> &active) {
    if (!d_volts || !n_samples || !ld_samples) return fail(MWAX_E_INVAL, "null argument array");
    segs.assign(b->n, {});
    active.clear();
    for (int i = 0; i < b->n; ++i) {
        mwax_plan p = b->inst[i];
        const int64_t ns = n_samples[i], ld = ld_samples[i];
        if (ns == 0) continue;
        if (!d_volts[i]) return fail(MWAX_E_INVAL, "instance %d: null voltage pointer", i);
        if ((uintptr_t)d_volts[i] & 15) return fail(MWAX_E_INVAL, "instance %d: voltages must be 16-byte aligned", i);
        if (ns < 0 || ns % p->L != 0 || ns > p->cfg.max_samples)
            return fail(MWAX_E_INVAL, "instance %d: n_samples = %lld must be a multiple of L = %d and <= %lld", i,
                        (long long)ns, p->L, (long long)p->cfg.max_samples);
        if (ld < ns || ld % 8 != 0)
            return fail(MWAX_E_INVAL, "instance %d: ld_samples = %lld must be >= n_samples and a multiple of 8", i,
                        (long long)ld);
        if (p->pending)
            return fail(MWAX_E_STATE, "instance %d: a block channelised by mwax_channelise awaits mwax_correlate", i);
        mwax_status st = plan_segments(p, ns / p->L, segs[i]);
        if (st != MWAX_OK) {
            std::string m = mwax_last_error();
            return fail(st, "instance %d: %s", i, m.c_str());
        }
        if ((int)segs[i].size() > b->max_segs[i]) return fail(MWAX_E_INVAL, "instance %d: too many segments", i);
        active.push_back(i);
    }
    return MWAX_OK;
}

// Build every table of a call and update the instances' bookkeeping.
void build_call(mwax_batch b, const int8_t *const *d_volts, const int64_t *ld_samples,
                const std::vector<std::vector<Segment>> &segs, const std::vector<int> &active, CallTables &t) {
    const size_t ng = b->groups.size();
    t.fs.assign(ng, {});
    t.fm.assign(ng, {});
    t.fs_b0.assign(ng, {});
    t.fm_b0.assign(ng, {});
    t.cal.clear();
    std::vector<std::vector<int64_t>> mwork(ng);
    std::vector<int> stats_count(ng, 0);
    for (int i : active) {
        mwax_plan p = b->inst[i];
        const int gi = b->group_of[i];
        LGroup &g = b->groups[gi];
        p->segs = segs[i];
        const size_t chain0 = t.cal.size();   // this instance's calibration descriptors start here
        for (const Segment &s : p->segs) {
            if (s.local0 == 0) {
                p->slot_owner[s.slot] = s.j;
                p->slot_count[s.slot] = 0;
                p->last_slot = s.slot;
                if (p->xprec == MWAX_X_INT8) {
                    CalDesc cd{};
                    cd.scales = p->scales + (size_t)s.slot * 2 * p->L;
                    cd.last = p->last;
                    cd.L = p->L;
                    if (p->fixed_mode) {
                        cd.copy_src = p->fixed;
                    } else {
                        FArgs a = calib_args(p, s, d_volts[i], ld_samples[i]);
                        const int nwg = fengine_grid(p->n_in, p->R, a.ngrp, true);
                        a.stats = b->d_stats + g.stats_off + (size_t)stats_count[gi] * kStatsMaxWG * stats_row(g.L);
                        ++stats_count[gi];
                        cd.stats = a.stats;
                        cd.nwg = nwg;
                        t.fs[gi].push_back(a);
                        const int32_t last = t.fs_b0[gi].empty() ? 0 : t.fs_b0[gi].back();
                        if (t.fs_b0[gi].empty()) t.fs_b0[gi].push_back(0);
                        t.fs_b0[gi].push_back(last + nwg);
                    }
                    t.cal.push_back(cd);
                }
            }
            t.fm[gi].push_back(fengine_args(p, s, d_volts[i], ld_samples[i]));
            mwork[gi].push_back((int64_t)s.ngrp * nblk_of(p));
        }
        if (t.cal.size() > chain0) t.cal[chain0].n_chain = (int32_t)(t.cal.size() - chain0);
    }
    for (size_t gi = 0; gi < ng; ++gi) {
        if (t.fs_b0[gi].empty()) t.fs_b0[gi].push_back(0);
        t.fm_b0[gi] = block_ranges(mwork[gi], b->groups[gi].main.grid);
    }
    build_x_tables(b, segs, active, t);
}

void finish_call(mwax_batch b, const std::vector<int> &active) {
    for (int i : active) {
        mwax_plan p = b->inst[i];
        int64_t M = 0;
        for (const Segment &s : p->segs) {
            p->slot_count[s.slot] += s.nframes;
            M += s.nframes;
        }
        p->pending = false;
        p->have_block = true;
        p->block_spectra = M;
        p->g_chan += M;
    }
}

mwax_status run_tables(mwax_batch b, const CallTables &t, bool x_only, bool allow_graph) {
    size_t nbytes = 0;
    mwax_status st = write_tables(b, t, &nbytes);
    if (st != MWAX_OK) return st;
    st = upload(b, nbytes);
    if (st != MWAX_OK) return st;
    const bool graph = allow_graph && b->use_graph && !x_only;
    if (graph && !b->exec) {
        st = capture(b);
        if (st != MWAX_OK) return st;
    }
    hipError_t e = btimed(b, 4, b->timing, [&] {
        return graph ? hipGraphLaunch(b->exec, b->stream) : launch_sequence(b, b->timing, x_only);
    });
    if (e != hipSuccess) return hip_fail(e, graph ? "batch graph launch" : "batch launch");
    return MWAX_OK;
}

// The autotuner's on-disk cache, a text file of one entry per line:
//   shape <arch> <n_in> <L> <xprec> <tile> <kchunk>   the choice for a shape class
//   grid <arch> <classes> <xprec> <grid>               the persistent grid of a batch
// (<classes>: the batch's shape classes as n_in x L x count, comma-separated).
// Lines that do not parse are dropped when the file is rewritten.
struct TuneCache {
    struct Entry {
        std::string arch;
        int n_in, L, xprec, tile, kchunk;
    };
    struct GridEntry {
        std::string arch, sig;
        int xprec, grid;
    };
    std::vector<Entry> shapes;
    std::vector<GridEntry> grids;

    void read(const std::string &path) {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            std::istringstream in(line);
            std::string kind;
            in >> kind;
            if (kind == "shape") {
                Entry e;
                if (in >> e.arch >> e.n_in >> e.L >> e.xprec >> e.tile >> e.kchunk) put(e.arch, e.n_in, e.L, e.xprec, e.tile, e.kchunk);
            } else if (kind == "grid") {
                GridEntry g;
                if (in >> g.arch >> g.sig >> g.xprec >> g.grid && g.grid > 0) put_grid(g.arch, g.sig, g.xprec, g.grid);
            }
        }
    }
    const Entry *find(const std::string &arch, int n_in, int L, int xprec) const {
        for (const Entry &e : shapes)
            if (e.arch == arch && e.n_in == n_in && e.L == L && e.xprec == xprec) return &e;
        return nullptr;
    }
    int grid(const std::string &arch, const std::string &sig, int xprec) const {
        for (const GridEntry &g : grids)
            if (g.arch == arch && g.sig == sig && g.xprec == xprec) return g.grid;
        return 0;
    }
    void put(const std::string &arch, int n_in, int L, int xprec, int tile, int kchunk) {
        for (Entry &e : shapes)
            if (e.arch == arch && e.n_in == n_in && e.L == L && e.xprec == xprec) {
                e.tile = tile;
                e.kchunk = kchunk;
                return;
            }
        shapes.push_back({arch, n_in, L, xprec, tile, kchunk});
    }
    void put_grid(const std::string &arch, const std::string &sig, int xprec, int grid_) {
        for (GridEntry &g : grids)
            if (g.arch == arch && g.sig == sig && g.xprec == xprec) {
                g.grid = grid_;
                return;
            }
        grids.push_back({arch, sig, xprec, grid_});
    }
    // written to a temporary file, then renamed over the old one
    bool write(const std::string &path) const {
        const std::string tmp = path + ".tmp";
        {
            std::ofstream f(tmp, std::ios::trunc);
            if (!f) return false;
            for (const Entry &e : shapes)
                f << "shape " << e.arch << ' ' << e.n_in << ' ' << e.L << ' ' << e.xprec << ' ' << e.tile << ' '
                  << e.kchunk << '\n';
            for (const GridEntry &g : grids)
                f << "grid " << g.arch << ' ' << g.sig << ' ' << g.xprec << ' ' << g.grid << '\n';
            if (!f) return false;
        }
        return std::rename(tmp.c_str(), path.c_str()) == 0;
    }
};

// The device's architecture name without its feature suffixes (e.g. gfx950).
std::string device_arch(int dev) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    if (c != std::string::npos) a.resize(c);
    return a.empty() ? "unknown" : a;
}

void collect_times(mwax_batch b) {
    for (auto &ev : b->events) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
            b->t_ms[ev.fam] += ms;
            b->t_n[ev.fam] += 1;
        }
        b->pool.push_back(ev.a);
        b->pool.push_back(ev.b);
    }
    b->events.clear();
}

}  // namespace

extern "C" {

mwax_status mwax_batch_create(const mwax_config *cfgs, int32_t n, void *hip_stream, mwax_batch *out) {
    if (!out) return fail(MWAX_E_INVAL, "null output handle");
    *out = nullptr;
    if (!cfgs || n < 1 || n > kMaxInstances)
        return fail(MWAX_E_INVAL, "a batch holds 1..%d instances (got %d)", kMaxInstances, n);
    for (int i = 0; i < n; ++i) {
        mwax_dims d;
        mwax_status st = derive(&cfgs[i], &d);
        if (st != MWAX_OK) {
            std::string m = mwax_last_error();
            return fail(st, "instance %d: %s", i, m.c_str());
        }
        if (cfgs[i].xprec != cfgs[0].xprec)
            return fail(MWAX_E_UNSUPPORTED, "instance %d: every instance of a batch must use the same xprec", i);
        if (d.fft_len > 1024)
            return fail(MWAX_E_UNSUPPORTED, "instance %d: batches take FFT lengths up to 1024 (got %d); run the "
                        "6,400-point transform as a plan", i, d.fft_len);
    }
    if (cfgs[0].xprec == MWAX_X_FP32)
        return fail(MWAX_E_UNSUPPORTED, "FP32 plans run on the vector ALUs and are not batched (use INT8 or FP16)");

    mwax_batch b = new (std::nothrow) mwax_batch_s;
    if (!b) return fail(MWAX_E_NOMEM, "host allocation failed");
    b->n = n;
    b->xprec = cfgs[0].xprec;
    (void)hipGetDevice(&b->device);
    hipError_t e = hipSuccess;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&b->stream);
        b->own_stream = e == hipSuccess;
        if (e != hipSuccess) {
            delete b;
            return hip_fail(e, "stream creation");
        }
    }
    for (int i = 0; i < n; ++i) {
        mwax_plan p = nullptr;
        mwax_status st = mwax_plan_create(&cfgs[i], b->stream, &p);
        if (st != MWAX_OK) {
            std::string m = mwax_last_error();
            free_batch(b);
            return fail(st, "instance %d: %s", i, m.c_str());
        }
        p->in_batch = true;
        p->batched = true;
        b->inst.push_back(p);
        b->max_segs.push_back((int)(ceil_div(p->d.max_spectra, p->T) + 1));
        int gi = -1;
        for (size_t k = 0; k < b->groups.size(); ++k)
            if (b->groups[k].L == p->L) gi = (int)k;
        if (gi < 0) {
            LGroup g;
            g.L = p->L;
            b->groups.push_back(g);
            gi = (int)b->groups.size() - 1;
            e = fengine_prepare_batch(p->L, b->xprec);
            if (e != hipSuccess) {
                free_batch(b);
                return hip_fail(e, "F-engine set-up");
            }
        }
        b->groups[gi].members.push_back(i);
        b->group_of.push_back(gi);
    }
    b->kchunk.assign(n, 0);
    b->tile.assign(n, kXTile);
    b->xgrid_max = xengine_batch_max_grid(b->xprec, b->device);
    b->xgrid = b->xgrid_max;
    mwax_status st = layout(b);
    if (st == MWAX_OK) st = apply_clear_policy(b);
    if (st != MWAX_OK) {
        free_batch(b);
        return st;
    }
    *out = b;
    return ok();
}

mwax_status mwax_batch_destroy(mwax_batch b) {
    free_batch(b);
    return ok();
}

mwax_status mwax_batch_plan(mwax_batch b, int32_t i, mwax_plan *out) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (!out || i < 0 || i >= b->n) return fail(MWAX_E_INVAL, "instance index %d out of range", i);
    *out = b->inst[i];
    return ok();
}

mwax_status mwax_batch_run(mwax_batch b, const int8_t *const *d_volts, const int64_t *n_samples,
                           const int64_t *ld_samples) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    std::vector<std::vector<Segment>> segs;
    std::vector<int> active;
    mwax_status st = prepare_call(b, d_volts, n_samples, ld_samples, segs, active);
    if (st != MWAX_OK) return st;
    if (active.empty()) return ok();
    CallTables t;
    build_call(b, d_volts, ld_samples, segs, active, t);
    st = run_tables(b, t, false, true);
    if (st != MWAX_OK) return st;
    finish_call(b, active);
    return ok();
}

mwax_status mwax_batch_autotune(mwax_batch b, const int8_t *const *d_volts, const int64_t *n_samples,
                                const int64_t *ld_samples, int32_t trials) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (trials < 1 || trials > 100) return fail(MWAX_E_INVAL, "trials must be in 1..100");
    for (int i = 0; i < b->n; ++i) {
        mwax_plan p = b->inst[i];
        bool fresh = p->g_chan == 0 && !p->pending;
        for (int s = 0; s < p->nslots; ++s) fresh = fresh && p->slot_owner[s] == -1;
        if (!fresh) return fail(MWAX_E_STATE, "instance %d is not at stream position 0 (mwax_reset it)", i);
        if (!n_samples || n_samples[i] <= 0)
            return fail(MWAX_E_INVAL, "the autotuner needs a block for every instance (instance %d)", i);
    }
    std::vector<std::vector<Segment>> segs;
    std::vector<int> active;
    mwax_status st = prepare_call(b, d_volts, n_samples, ld_samples, segs, active);
    if (st != MWAX_OK) return st;

    // candidates: tile edge x row groups per work item (chunks: INT8 only)
    const std::vector<int> chunks = b->xprec == MWAX_X_INT8 ? std::vector<int>{0, 4096, 2048, 1024, 512, 256, 128}
                                                            : std::vector<int>{0};
    const std::vector<int> tiles = {kXTile, kXTileSmall};
    const std::vector<int> saved_kc = b->kchunk, saved_tile = b->tile;
    const int saved_grid = b->xgrid;

    // instance shape classes (inputs, L), heaviest first
    std::vector<std::pair<int64_t, std::vector<int>>> classes;
    for (int i = 0; i < b->n; ++i) {
        mwax_plan p = b->inst[i];
        bool placed = false;
        for (auto &c : classes) {
            mwax_plan q = b->inst[c.second[0]];
            if (q->n_in == p->n_in && q->L == p->L) {
                c.second.push_back(i);
                c.first += p->P * n_samples[i];
                placed = true;
            }
        }
        if (!placed) classes.push_back({p->P * n_samples[i], {i}});
    }
    std::stable_sort(classes.begin(), classes.end(), [](const auto &a, const auto &c) { return a.first > c.first; });

    // the on-disk cache: a shape class found there keeps its entry untimed
    TuneCache cache;
    const std::string arch = device_arch(b->device);
    if (!b->cache_path.empty()) cache.read(b->cache_path);
    std::vector<bool> cached(classes.size(), false);
    for (size_t k = 0; k < classes.size(); ++k) {
        mwax_plan p = b->inst[classes[k].second[0]];
        const TuneCache::Entry *e = cache.find(arch, p->n_in, p->L, b->xprec);
        if (!e || !tile_allowed(b, classes[k].second[0], e->tile) || (e->kchunk > 0 && b->xprec != MWAX_X_INT8))
            continue;
        for (int i : classes[k].second) {
            b->tile[i] = e->tile;
            b->kchunk[i] = e->kchunk;
        }
        cached[k] = true;
    }
    std::string sig = "";
    for (auto &c : classes) {
        mwax_plan p = b->inst[c.second[0]];
        sig += std::to_string(p->n_in) + "x" + std::to_string(p->L) + "x" + std::to_string(c.second.size()) + ",";
    }
    const int cached_grid = cache.grid(arch, sig, b->xprec);
    const bool all_cached = std::all_of(cached.begin(), cached.end(), [](bool v) { return v; });
    if (all_cached && cached_grid > 0) {
        b->xgrid = std::min(cached_grid, b->xgrid_max);
        st = layout(b);
        if (st == MWAX_OK) st = apply_clear_policy(b);
        return st == MWAX_OK ? ok() : st;
    }

    // tables sized for the largest candidate (the smallest chunk, the small tile)
    const std::vector<int> cur_kc = b->kchunk, cur_tile = b->tile;
    b->kchunk.assign(b->n, chunks.back());
    for (int i = 0; i < b->n; ++i)
        if (tile_allowed(b, i, kXTileSmall) && xengine_tile_count(b->inst[i]->n_in, kXTileSmall) >
                                                  xengine_tile_count(b->inst[i]->n_in, b->tile[i]))
            b->tile[i] = kXTileSmall;
    st = layout(b);
    if (st != MWAX_OK) return st;
    b->kchunk = cur_kc;
    b->tile = cur_tile;

    CallTables t;
    build_call(b, d_volts, ld_samples, segs, active, t);
    st = run_tables(b, t, false, false);     // channelise once (and a first X pass)
    if (st != MWAX_OK) return st;
    finish_call(b, active);

    const bool saved_timing = b->timing;
    b->timing = false;
    auto time_x = [&](double *ms_out) -> mwax_status {
        build_x_tables(b, segs, active, t);
        std::vector<double> v;
        for (int r = 0; r < trials; ++r) {
            hipEvent_t e0 = batch_event(b), e1 = batch_event(b);
            if (!e0 || !e1) return fail(MWAX_E_NOMEM, "event creation");
            size_t nbytes = 0;
            mwax_status s2 = write_tables(b, t, &nbytes);
            if (s2 == MWAX_OK) s2 = upload(b, nbytes);
            if (s2 != MWAX_OK) return s2;
            (void)hipEventRecord(e0, b->stream);
            hipError_t e = launch_sequence(b, false, true);
            (void)hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            b->pool.push_back(e0);
            b->pool.push_back(e1);
            if (e != hipSuccess) return hip_fail(e, "autotune trial");
            v.push_back(ms);
        }
        std::sort(v.begin(), v.end());
        *ms_out = v[v.size() / 2];
        return MWAX_OK;
    };

    double best = 0.0;
    st = time_x(&best);
    for (int pass = 0; pass < 2 && st == MWAX_OK; ++pass) {
        for (size_t k = 0; k < classes.size() && st == MWAX_OK; ++k) {
            if (cached[k]) continue;
            const std::vector<int> &members = classes[k].second;
            const int i0 = members[0];
            int pick_kc = b->kchunk[i0], pick_te = b->tile[i0];
            for (int te : tiles) {
                if (!tile_allowed(b, i0, te)) continue;
                for (int kc : chunks) {
                    if (te == b->tile[i0] && kc == b->kchunk[i0]) continue;
                    if (kc > 0 && kc >= b->inst[i0]->NG) continue;   // same as whole segments
                    for (int i : members) {
                        b->kchunk[i] = kc;
                        b->tile[i] = te;
                    }
                    double ms = 0.0;
                    st = time_x(&ms);
                    if (st != MWAX_OK) break;
                    if (ms < 0.99 * best) {
                        best = ms;
                        pick_kc = kc;
                        pick_te = te;
                    }
                }
                if (st != MWAX_OK) break;
            }
            for (int i : members) {
                b->kchunk[i] = pick_kc;
                b->tile[i] = pick_te;
            }
        }
    }
    if (st == MWAX_OK) {
        int pick = b->xgrid;
        for (int gsz : {b->xgrid_max / 2, (3 * b->xgrid_max) / 4, b->xgrid_max}) {
            if (gsz == b->xgrid || gsz < 8) continue;
            b->xgrid = gsz;
            double ms = 0.0;
            st = time_x(&ms);
            if (st != MWAX_OK) break;
            if (ms < 0.99 * best) {
                best = ms;
                pick = gsz;
            }
        }
        b->xgrid = pick;
    }
    b->timing = saved_timing;
    if (st != MWAX_OK) {
        b->kchunk = saved_kc;
        b->tile = saved_tile;
        b->xgrid = saved_grid;
    } else if (!b->cache_path.empty()) {
        for (auto &c : classes) {
            mwax_plan p = b->inst[c.second[0]];
            cache.put(arch, p->n_in, p->L, b->xprec, b->tile[c.second[0]], b->kchunk[c.second[0]]);
        }
        cache.put_grid(arch, sig, b->xprec, b->xgrid);
        if (!cache.write(b->cache_path)) st = fail(MWAX_E_INVAL, "cannot write the tuning cache %s", b->cache_path.c_str());
    }
    mwax_status st2 = layout(b);
    for (int i = 0; i < b->n; ++i) {
        mwax_status r = mwax_reset(b->inst[i]);
        if (st2 == MWAX_OK) st2 = r;
    }
    if (st2 == MWAX_OK) st2 = apply_clear_policy(b);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (st != MWAX_OK) return st;
    if (st2 != MWAX_OK) return st2;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    return ok();
}

mwax_status mwax_batch_get_tiles(mwax_batch b, int32_t *tile) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (!tile) return fail(MWAX_E_INVAL, "null tile array");
    for (int i = 0; i < b->n; ++i) tile[i] = b->tile[i];
    return ok();
}

mwax_status mwax_batch_set_tiles(mwax_batch b, const int32_t *tile) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (!tile) return fail(MWAX_E_INVAL, "null tile array");
    for (int i = 0; i < b->n; ++i)
        if (!tile_allowed(b, i, tile[i]))
            return fail(MWAX_E_INVAL, "tile[%d] = %d: the tile edge is %d or %d (at most %d tiles per channel)", i,
                        tile[i], kXTile, kXTileSmall, kXBatchMaxTiles);
    for (int i = 0; i < b->n; ++i)
        if (b->inst[i]->pending) return fail(MWAX_E_STATE, "instance %d has a pending block", i);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(MWAX_E_DEVICE, "stream synchronisation");
    b->tile.assign(tile, tile + b->n);
    mwax_status st = layout(b);
    return st == MWAX_OK ? ok() : st;
}

mwax_status mwax_batch_set_tuning_cache(mwax_batch b, const char *path) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    b->cache_path = path ? path : "";
    return ok();
}

mwax_status mwax_batch_get_tuning(mwax_batch b, int32_t *kchunk, int32_t *grid) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (kchunk)
        for (int i = 0; i < b->n; ++i) kchunk[i] = b->kchunk[i];
    if (grid) *grid = b->xgrid;
    return ok();
}

mwax_status mwax_batch_set_tuning(mwax_batch b, const int32_t *kchunk, int32_t grid) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (grid < 0) return fail(MWAX_E_INVAL, "grid must be >= 0");
    if (kchunk)
        for (int i = 0; i < b->n; ++i) {
            if (kchunk[i] < 0) return fail(MWAX_E_INVAL, "kchunk[%d] must be >= 0", i);
            if (kchunk[i] > 0 && b->xprec != MWAX_X_INT8)
                return fail(MWAX_E_UNSUPPORTED, "chunked X-engine items need exact (INT8) partial sums");
        }
    for (int i = 0; i < b->n; ++i)
        if (b->inst[i]->pending) return fail(MWAX_E_STATE, "instance %d has a pending block", i);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(MWAX_E_DEVICE, "stream synchronisation");
    if (kchunk) b->kchunk.assign(kchunk, kchunk + b->n);
    b->xgrid = grid == 0 ? b->xgrid_max : std::min(grid, 65535);
    mwax_status st = layout(b);
    if (st == MWAX_OK) st = apply_clear_policy(b);
    return st == MWAX_OK ? ok() : st;
}

mwax_status mwax_batch_set_graph(mwax_batch b, int32_t enable) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    b->use_graph = enable != 0;
    return ok();
}

mwax_status mwax_batch_set_timing(mwax_batch b, int32_t enable) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    b->timing = enable != 0;
    return ok();
}

mwax_status mwax_batch_kernel_time(mwax_batch b, int32_t family, double *total_ms, int64_t *launches) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    if (family < 0 || family > 4 || !total_ms || !launches) return fail(MWAX_E_INVAL, "bad arguments");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronisation");
    collect_times(b);
    *total_ms = b->t_ms[family];
    *launches = b->t_n[family];
    b->t_ms[family] = 0.0;
    b->t_n[family] = 0;
    return ok();
}

mwax_status mwax_batch_sync(mwax_batch b) {
    if (check_batch(b) != MWAX_OK) return MWAX_E_INVAL;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronisation");
    return ok();
}

}  // extern "C"
