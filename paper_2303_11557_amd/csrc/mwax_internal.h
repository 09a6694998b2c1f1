// Internal declarations shared by the runtime and the kernel files of libmwax.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mwax.h"

namespace mwax {

// Every row of the channel-major buffer is 32 bytes: G spectra of one input in
// one channel, real parts first then imaginary parts (int8: 16 + 16 bytes,
// binary16: 8 + 8 halves, float32: 4 + 4 floats).  This is the operand order
// the matrix cores read: one 16-byte half row per lane.
constexpr int kRowBytes = 32;

// INT8 integrators are int32 pairs when an integration holds at most this many
// spectra: |Re V| <= 2 * 127^2 * T and |Im V - sum re| <= 2 * 127^2 * T + 127 T
// stay below 2^31 (2.122e9 at T = 65536); int64 pairs otherwise.
constexpr int64_t kInt32MaxSpectra = 65536;
inline int integ_elem_bytes(int xprec, int64_t T) {
    return xprec == MWAX_X_INT8 && T <= kInt32MaxSpectra ? 8 : 16;
}
// Bytes of one integrator slot [L][P] (padded to 256 so every slot is aligned
// and can be cleared in 16-byte units).
inline uint64_t integ_slot_bytes(int xprec, int64_t T, int64_t L, int64_t P) {
    return ((uint64_t)L * P * integ_elem_bytes(xprec, T) + 255) / 256 * 256;
}

// Layout of one 32-byte row (G frames of one channel and input, elements of es
// bytes).  INT8 (G = 16) and binary16 (G = 8): bytes 0..7 hold the real parts of
// frames 0 .. G/2-1, bytes 8..15 their imaginary parts, bytes 16..31 the same for
// frames G/2 .. G-1, so that each 16-byte half is one matrix-core operand that
// carries both parts of its frames.  FP32 (G = 4): real parts 0..15, imaginary
// parts 16..31.
__host__ __device__ constexpr int row_re_off(int f, int es) {
    return es == 4 ? f * 4 : f * es + (f * es >= 8 ? 8 : 0);
}
__host__ __device__ constexpr int row_im_gap(int es) { return es == 4 ? 16 : 8; }

inline int group_of(int xprec) {
    return xprec == MWAX_X_INT8 ? 16 : (xprec == MWAX_X_FP16 ? 8 : 4);
}

// Binary16 scaling exponent e = ceil(log2(L) / 2): |X| 2^-e <= 127 sqrt(2 L) 2^-e
// stays far below 65504 for every supported L.
inline int fp16_exponent(int L) {
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    return (lg + 1) / 2;
}

// ---------------------------------------------------------------------------
// F-engine
// ---------------------------------------------------------------------------
struct FArgs {
    const int8_t *volts;    // [N_in][ld][2]
    int64_t ld;             // samples between input rows
    int64_t frame0;         // first source frame (call-local) of the segment
    int64_t nframes;        // frames in the segment
    uint8_t *chan;          // channel-major buffer [L][NG][N_in][32 B]
    int64_t NG;             // row groups per channel in the buffer
    int64_t grp0;           // first destination group of the segment
    int32_t n_in;           // inputs
    int32_t R;              // inputs per workgroup
    int32_t ngrp;           // destination groups of the segment (or calibration groups)
    int32_t stats_mode;     // 1: accumulate per-channel power instead of writing
    const float2 *tw;       // W_L^k = exp(-2 pi i k / L), k < L
    const float *inv_s;     // [L] INT8 inverse scales of the segment's integration
    float half_scale;       // 2^-e for FP16
    double *stats;          // stats mode: [n_workgroups][L + 1] partial power sums
                            // per channel, then the count of populated frames
    uint8_t *mid;           // L = 6400: frame-major spectra [N_in][mid_frames][L][2]
    int64_t mid_frames;     // frames per input row of mid
    // fractional delay and phase correction (NULL dl: none): frame f of the
    // segment uses the delay dl[n * dl_ld + (dl_f0 + f) / dl_fps] (samples)
    const float *dl;
    int64_t dl_ld;          // steps per input row of dl
    int64_t dl_f0;          // table frame index of the segment's first frame
    int32_t dl_fps;         // frames per delay step
    double dl_nu;           // sky frequency of the coarse channel centre / f_s
};

constexpr int kStatsMaxWG = 1024;   // calibration partial rows per launch (max)
int fengine_lds_bytes(int L, int xprec, int R, bool stats);
int fengine_grid(int n_in, int R, int ngrp, bool stats);
constexpr int kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950
int fengine_pick_R(int L, int xprec, int n_in, int lds_limit);
hipError_t launch_fengine(int L, int xprec, const FArgs &a, hipStream_t s);
hipError_t launch_twiddles(float2 *tw, int L, hipStream_t s);
// Rows of the statistics buffer: L channel sums + the populated-frame count.
inline int64_t stats_row(int L) { return (int64_t)L + 1; }
// stats: [nwg][L + 1] partial sums -> scales [2][L] (s, inv_s) for one slot; a
// window without populated frames takes last [2][L] (the most recent calibrated
// scales), which every other calibration updates
hipError_t launch_calib_finish(const double *stats, int nwg, int L, float *scales, float *last, hipStream_t s);
hipError_t launch_copy_scales(const float *src, float *dst, int L, hipStream_t s);
hipError_t launch_fill_f32(float *dst, float v, int n, hipStream_t s);

// The 6,400-point transform of Sec. 2.5.1 (fft6400.hip): a frame-major main
// pass into FArgs::mid, then the corner-turn into the channel-major buffer.
constexpr int kUltraFineL = 6400;
struct CornerArgs {
    const uint8_t *mid;     // [N_in][mid_frames][L][2] elements
    int64_t mid_frames;
    int64_t frame0;         // first frame of the segment in mid
    int64_t nframes;        // frames of the segment
    uint8_t *chan;          // channel-major buffer [L][NG][N_in][32 B]
    int64_t NG;
    int64_t grp0;           // first destination group of the segment
    int32_t n_in;
    int32_t L;
};
int fft6400_grid(int n_in, int64_t nframes, bool stats);
int fft6400_lds_bytes();
hipError_t launch_fft6400(int xprec, const FArgs &a, hipStream_t s);
hipError_t launch_corner_turn(int esize, const CornerArgs &a, hipStream_t s);

// Tied-array beamforming (Sec. 4.4) from the channel-major buffer, one
// segment (one integration's spectra, one scale per channel) per launch.
struct BeamArgs {
    const uint8_t *chan;    // [L][NG][N_in][32 B]
    int64_t NG;
    int64_t grp0;           // first row group of the segment
    int64_t nframes;        // spectra of the segment
    int64_t m0;             // output index of the segment's first spectrum
    const float *scales;    // INT8: s_c [L] of the segment's integration; else NULL
    float post;             // FP16: 2^e; else 1
    int32_t n_in;
    int32_t L;
    int32_t nb;             // beams
    const float2 *w;        // [L][nb][N_in] weights
    float2 *out;            // [M][L][nb]
};
hipError_t launch_beamform(int esize, const BeamArgs &a, hipStream_t s);
constexpr int kIncohMaxSeg = 64;
struct IncohArgs {
    const uint8_t *chan;
    int64_t NG;
    int32_t n_in;
    int32_t L;
    int32_t t_avg, f_avg;   // spectra and channels per output bin
    int32_t n_o;            // L / f_avg
    int64_t n_j;            // block spectra / t_avg
    float post;
    int32_t nseg;
    int64_t seg_m0[kIncohMaxSeg];          // block index of each segment's first spectrum
    int64_t seg_grp0[kIncohMaxSeg];
    const float *seg_scales[kIncohMaxSeg]; // INT8 s_c per segment; else NULL
    float *out;             // [n_j][n_o][2]
};
hipError_t launch_incoherent(int esize, const IncohArgs &a, hipStream_t s);

// Reads a workgroup-uniform table entry through the constant address space: the
// compiler may then reload its fields where they are used (as it does for kernel
// arguments) instead of holding them in registers for the whole kernel.
template <class T>
__device__ __forceinline__ T load_uniform(const T *p) {
    T v;
    __builtin_memcpy(&v, (const __attribute__((address_space(4))) void *)p, sizeof(T));
    return v;
}

// Batched F-engine: one launch covers the segments of many plans with the same
// L and precision.  The tables live in device memory (they change per call while
// the launch itself, grid included, is fixed and can be replayed from a graph).
struct FBatchArgs {
    const FArgs *desc;      // [ndesc] segments
    const int32_t *block0;  // [ndesc + 1] first workgroup of each descriptor
    const int32_t *ndesc;   // number of descriptors this call
};
hipError_t launch_fengine_batch(int L, int xprec, bool stats, const FBatchArgs &b, int grid, hipStream_t s);
hipError_t fengine_prepare_batch(int L, int xprec);   // LDS attribute, once, outside graph capture

// Batched scale calibration finish (or copy of fixed scales), one descriptor per
// integration that begins in the call.
struct CalDesc {
    const double *stats;    // [nwg][L + 1] partial power sums and counts (NULL in copy mode)
    const float *copy_src;  // copy mode: [2][L] scales to install
    float *scales;          // [2][L] destination (s, inv_s)
    float *last;            // [2][L] the instance's most recent calibrated scales
    int32_t nwg;
    int32_t L;
    int32_t n_chain;        // first descriptor of an instance: its descriptors in
                            // this call (consecutive, processed in order); else 0
    int32_t pad;
};
hipError_t launch_calib_batch(const CalDesc *desc, const int32_t *ndesc, int max_desc, int max_L, hipStream_t s);

// Canonical [M][L][N_in][2] <-> internal layout, one segment at a time.
struct RepackArgs {
    void *canon;            // [M][L][N_in][2] elements
    int64_t m0;             // first canonical spectrum of the segment
    int64_t nframes;        // spectra in the segment
    uint8_t *chan;
    int64_t NG, grp0;
    int32_t n_in, L, G, esize;  // elements per row half = G; element bytes
    int32_t to_internal;    // 1: canon -> chan (load), 0: chan -> canon (read)
};
hipError_t launch_repack(const RepackArgs &a, hipStream_t s);

// ---------------------------------------------------------------------------
// X-engine
// ---------------------------------------------------------------------------
struct XArgs {
    const uint8_t *chan;    // [L][NG][N_in][32 B]
    int64_t NG;
    int64_t grp0;           // first group of the segment
    int32_t ngrp;           // groups in the segment
    int32_t n_in;
    int32_t L;
    int32_t ntiles;         // lower-triangle tiles per channel
    int32_t tile;           // tile edge (rows)
    void *integ;            // this slot's integrators [L][P][2] (int64 or double)
    int64_t P;
    int32_t nks;            // chunks of row groups per tile (set by launch_xengine;
                            // 1 on entry: whole segments)
    int32_t kchunk;         // row groups per chunk
    int32_t first;          // the segment starts its integration: a tile's first
                            // non-atomic flush stores instead of adding
    int32_t i32;            // INT8 integrators are int32 pairs (else int64)
};
// Averaging X-engine (plans with mwax_set_averaging): one segment of F-channel
// output channels, accumulated straight into FP64 integrators [N][P][2].
struct XAvgArgs {
    const uint8_t *chan;    // [L][NG][N_in][32 B]
    int64_t NG;
    int64_t grp0;           // first group of the segment
    int32_t ngrp;           // groups in the segment
    int32_t n_in;
    int32_t L;
    int32_t F;              // fine channels per output channel
    int32_t N;              // output channels, L / F
    int32_t ntiles;         // 64-edge lower-triangle tiles per channel
    const float *scales;    // INT8: s_c [L] of the segment's integration; else NULL
    void *integ;            // this slot's integrators [N][P] (double2)
    int64_t P;
    int32_t first;          // the segment starts its integration: store, not add
};
hipError_t launch_xengine_avg(int xprec, const XAvgArgs &a, hipStream_t s);

// INT8 launches split every tile's row groups into chunks when that fills the
// device's resident workgroup slots more evenly (chunks flush with exact int64
// atomic adds); other precisions run whole segments.
hipError_t launch_xengine(int xprec, const XArgs &a, hipStream_t s);
// True if launch_xengine adds every partial sum into the integrators (FP32, or
// INT8 split into chunks); false if the first flush of a segment that starts
// its integration overwrites them.
bool xengine_accumulates(int xprec, const XArgs &a);
int xengine_tile(int xprec);
// Tile edges of the MFMA X-engine: single plans use kXTile; a batch instance
// may use either (the autotuner picks).  Lower-triangle tiles per channel:
constexpr int kXTile = 128, kXTileSmall = 64;
int xengine_tile_count(int n_in, int te);

// Persistent batched X-engine.  A work item is one 128 x 128 tile of one channel
// of one segment over a chunk of its row groups, packed in 32 bits:
//   desc (8 bits) | channel (10) | tile (8) | chunk (6)
// Items sit in 8 queues, one per XCD (workgroup b runs on XCD b mod 8); a
// workgroup drains its own queue, then takes work from the others.  Chunks of
// one (channel, tile) run concurrently only in segments with ksplit > 1, whose
// flushes are int64 atomic adds (exact and order-free); otherwise every
// integrator element has one writer per launch.
struct XDesc {
    const uint8_t *chan;
    int64_t NG;
    int64_t grp0;
    void *integ;            // segment's slot integrators [L][P][2]
    int64_t P;
    int32_t ngrp;           // row groups of the segment
    int32_t n_in;
    int32_t kchunk;         // row groups per chunk
    int32_t ksplit;         // chunks = ceil(ngrp / kchunk)
    int32_t first;          // as XArgs::first
    int32_t i32;            // as XArgs::i32
    int32_t te;             // tile edge: kXTile or kXTileSmall
};
constexpr int kXBatchMaxDesc = 256;
constexpr int kXBatchMaxTiles = 256;
constexpr int kXBatchMaxSplit = 64;
constexpr int kXQueues = 8;
constexpr int kXCounterStride = 64;   // ints between queue counters (256 bytes)
__host__ __device__ inline uint32_t xitem_pack(int d, int c, int t, int k) {
    return ((uint32_t)d << 24) | ((uint32_t)c << 14) | ((uint32_t)t << 6) | (uint32_t)k;
}
struct XBatchArgs {
    const XDesc *desc;
    const uint32_t *items;  // queue q holds items[qbeg[q] .. qbeg[q+1])
    const int32_t *qbeg;    // [kXQueues + 1]
    int32_t *counters;      // [kXQueues * kXCounterStride], zero at launch
};
hipError_t launch_xengine_batch(int xprec, const XBatchArgs &b, int grid, hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int n, hipStream_t s);
int xengine_batch_max_grid(int xprec, int device);   // resident workgroups on the device

// ---------------------------------------------------------------------------
// Integrate / pack
// ---------------------------------------------------------------------------
struct PackArgs {
    void *integ;            // slot integrators [L][P][2], cleared after reading if clear
    int32_t is_int;         // int64 (1) or double (0) integrators
    const float *scales;    // INT8: s_c [L]; else NULL
    double post;            // FP16/FP32: multiply by this (2^(2e) or 1)
    void *out;              // complex64 or int64 output of this integration
    float *scales_out;      // raw mode: copy of s_c, may be NULL
    int32_t order;          // mwax_order; 2 = raw int64; 3 = averaged by F (CHAN_TRI)
    int32_t clear;          // zero the integrators after reading them
    int32_t i32;            // INT8 integrators are int32 pairs (else int64)
    int32_t L;
    int32_t n_in;
    int64_t P;
    int32_t F;              // order 3: channels averaged into one (Sec. 2.6)
    const float *avg_w;     // order 3: occupancy weights [P] of this integration, or NULL
};
hipError_t launch_pack(const PackArgs &a, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace mwax
