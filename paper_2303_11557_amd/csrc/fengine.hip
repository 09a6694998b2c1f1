// F-engine of the FX correlator (Morrison et al. 2023, Sec. 2.5 and 2.5.1):
// per input and per contiguous frame of L complex int8 samples, an
// unnormalised forward FFT in FP32, channels re-ordered so DC sits at
// c = L/2 (centre-symmetric channels, Sec. 2.6), then requantised (INT8 /
// binary16) or kept (FP32) and transposed through LDS into the channel-major
// layout the X-engine reads (the transpose of Sec. 2.5.1).
//
// One workgroup owns R inputs x G consecutive frames of one integration
// segment = one 32-byte row group per (channel, input).  The raw int8 frames
// are staged in LDS with coalesced 16-byte loads (INT8 at L = 1024: loaded by
// the FFT lanes themselves, see FCfg::DIRECT); each FFT is computed by a
// group of L2 lanes holding L1 = L / L2 points each:
//   X[k1 + L1 k2] = sum_r W_L2^(r k2) W_L^(r k1) sum_n1 x[r + L2 n1] W_L1^(n1 k1)
// (a two-pass Cooley-Tukey split): pass 1 in registers per lane, twiddle,
// exchange of the L1 x L2 block through LDS, pass 2 in registers.  The
// quantised outputs are written to an LDS image of the workgroup's output rows,
// which is then stored with coalesced 16-byte writes.
#include <algorithm>
#include <type_traits>

#include "fft_common.h"
#include "mwax_internal.h"

namespace mwax {
namespace {

using namespace fft;

// Two-pass split L = L1 * L2 over an FFT group of L2 lanes.  Pass 2 (length L2)
// is done by each lane on U columns when L2 <= L1.  At L >= 512 a lane keeps 16
// points (L2 = 32 or 64 > L1 = 16): each pass-2 transform is shared by
// P = L2 / 16 neighbouring lanes, an in-lane 16-point DFT, a second exchange and
// in-lane P-point DFTs (see fengine_body).  Measured against 32 points per lane:
// 1.2x (L = 1024) and 1.1x (L = 512) for INT8, 1.12x / 1.13x for binary16,
// 1.06x / 1.12x for FP32 (about 150 instead of 230-280 VGPRs).
template <int L, int XP>
struct FftShape {
    static constexpr bool kLaneSplit = L >= 512;
    static constexpr int L2 = L <= 16 ? 1
                              : (L == 32 ? 4
                              : (L <= 128 ? 8 : (L == 256 ? 16 : (kLaneSplit ? L / 16 : (L == 512 ? 16 : 32)))));
    static constexpr int L1 = L / L2;
    static constexpr int P = L2 > L1 ? L2 / L1 : 1;
    static constexpr int U = (L2 > 1 && P == 1) ? L1 / L2 : 1;
};

template <int XP>
struct PrecTraits;
template <>
struct PrecTraits<MWAX_X_INT8> { static constexpr int G = 16, ES = 1; };
template <>
struct PrecTraits<MWAX_X_FP16> { static constexpr int G = 8, ES = 2; };
template <>
struct PrecTraits<MWAX_X_FP32> { static constexpr int G = 4, ES = 4; };

// Channel of output slot i of lane r (see the kernel comment): bin
// k = (r U + u) + L1 k2 with i = u L2 + k2; with P lanes per pass-2 transform,
// lane r = k1 P + g holds k = k1 + L1 (g + P j + L1 q) in slot i = j P + q.
// Channel (k + L/2) mod L.
template <int L, int XP>
__device__ __forceinline__ int bin_of(int r, int i) {
    using SH = FftShape<L, XP>;
    if constexpr (SH::P > 1) return r / SH::P + SH::L1 * (r % SH::P + SH::P * (i / SH::P) + SH::L1 * (i % SH::P));
    else if constexpr (SH::L2 > 1) return (r * SH::U + i / SH::L2) + SH::L1 * (i % SH::L2);
    else return i;
}
template <int L, int XP>
__device__ __forceinline__ int chan_of(int r, int i) {
    return (bin_of<L, XP>(r, i) + L / 2) & (L - 1);
}

// Gain of the fractional delay correction for signed bin ks (channel offset
// c - L/2): exp(-2 pi i (ks alpha + phi)), alpha = d / L, phi = the frame's
// phase offset (nu_c / f_s) d reduced to [-1/2, 1/2] revolutions.
__device__ __forceinline__ float2 delay_gain(int ks, float alpha, float phi) {
    float sn, cs;
    sincospif(-2.0f * fmaf((float)ks, alpha, phi), &sn, &cs);
    return make_float2(cs, sn);
}

constexpr int kThreads = 256;   // default workgroup size (see FCfg::THREADS)

// Output-image padding per channel (bytes beyond R * 32), chosen so the packed
// output writes of a wave fall in distinct LDS banks.
constexpr int cp_pad(int L, int XP) {
    return L <= 16 ? 4 : (L == 32 ? (XP == MWAX_X_INT8 ? 8 : 4)
                       : (L == 64 ? (XP == MWAX_X_INT8 ? 8 : 16)
                       : (L <= 256 ? (XP == MWAX_X_INT8 ? 4 : 8) : 4)));
}

// Work decomposition of one workgroup (THREADS threads) for length L and
// output precision XP.  An FFT group is L2 lanes; a wave holds GPW groups.
// Each group transforms FPG consecutive frames of one input, so that the
// results of FPG frames leave in one packed LDS write; the workgroup covers
// R inputs x G frames (one 32-byte row group per channel and input).
template <int L, int XP>
struct FCfg {
    using SH = FftShape<L, XP>;
    static constexpr int L1 = SH::L1, L2 = SH::L2, U = SH::U;
    static constexpr int G = PrecTraits<XP>::G, ES = PrecTraits<XP>::ES;
    // INT8 at 16 <= L <= 256: one frame per group (byte writes) holds fewer
    // registers than packing two frames' codes, for more waves per SIMD.  At
    // L >= 512 (32 or 64 lanes per FFT) an INT8 group transforms two frames,
    // so that a workgroup still covers the 16 frames of a row group, and
    // L = 1024 (one FFT per wave) takes eight waves at every precision (two
    // inputs per item for FP32: 64-byte runs per channel).  Binary16 keeps one
    // frame per group (two would need 86 KB of LDS at L = 128, one workgroup per CU).
    static constexpr int FPG = XP == MWAX_X_INT8 ? (L >= 16 && L <= 256 ? 1 : 2) : 1;
    // INT8 at L = 1024: four waves, each transforming two packs of an item in
    // turn, its lanes loading their own samples straight from HBM (a lane's
    // samples r + 64 n1 of a frame are one 128-byte line per load instruction).
    // Without the staging area a workgroup needs 71 KB of LDS, so two fit a CU
    // and one workgroup's barriers and image store overlap the other's FFTs:
    // 2.34 instead of 1.86 TB/s.  (At L = 512, two 32-lane groups per wave,
    // the same scheme ran at 2.04 instead of 2.37 TB/s.)
    static constexpr bool DIRECT = XP == MWAX_X_INT8 && L == 1024;
    static constexpr int THREADS = DIRECT ? kThreads : (L == 1024 ? 512 : kThreads);
    static constexpr int P = SH::P;
    static constexpr int GPW = 64 / L2;
    static constexpr int NGWG = THREADS / 64 * GPW;   // FFT groups per workgroup
    static constexpr int PACKS = G / FPG;         // frame packs per input
    static constexpr int R = NGWG >= PACKS ? NGWG / PACKS : 1;   // inputs per workgroup item
    static constexpr int PPG = PACKS * R / NGWG;  // packs per group and item
    static constexpr int CP = R * kRowBytes + cp_pad(L, XP);
    static constexpr int SP = 2 * L + 16;         // staged frame pitch (bytes)
    // exchange area per group (float2): L + 8, or L1 rows of L2 + P (P > 1)
    static constexpr int EXR = L2 + P;
    static constexpr int EXG = P > 1 ? L1 * EXR : L + 8;
    static constexpr int OUT_BYTES = L * CP;
    static constexpr int STAGE_BYTES = L2 > 1 && !DIRECT ? R * G * SP : 0;
    static constexpr int EX_BYTES = L2 > 1 ? NGWG * EXG * 8 : 0;
    // statistics pass: per-lane channel sums (L1 floats) and populated-frame counts
    static constexpr int RED_BYTES = THREADS * (L1 + 1) * 4;
    // load the next item's frames while transforming the current one (where the
    // extra registers keep the occupancy)
    static constexpr bool PREFETCH = XP != MWAX_X_FP32 && L2 > 1 && (L <= 256 || XP == MWAX_X_INT8) && !DIRECT;
    static_assert(R >= 1 && NGWG * PPG == PACKS * R && (PPG == 1 || GPW == 1), "bad decomposition");
    // workgroups of a single-plan launch (each takes items in rounds): enough that
    // the workgroups holding adjacent items stay in step (their rows share output
    // lines), few enough that each one's set-up is spread over tens of items.
    // Measured at 256 tiles, 8 s: 65,536 at every length but 256, where 131,072
    // is 10 % faster (32,768 - 262,144 swept).
    static constexpr int64_t GRID_CAP = L == 256 ? 131072 : 65536;
};

// One complex int8 sample, converted exactly.  Written with arithmetic shifts of
// the halfword placed in the upper half of a word so that each component is one
// sign-extending byte-select convert (the int8_t casts of a 16-bit load compile
// to a separate extract per component).
__device__ __forceinline__ float2 load_pair(const uint8_t *p) {
    const int32_t w = (int32_t)((uint32_t)*reinterpret_cast<const uint16_t *>(p) << 16);
    return make_float2((float)((w << 8) >> 24), (float)(w >> 24));
}

// The work of workgroup wg of nwg workgroups on the segment described by a;
// DELAY: apply the fractional delay and phase correction before requantising.
template <int L, int XP, bool STATS, bool DELAY = false>
__device__ __forceinline__ void fengine_body(const FArgs &a, const int wg, const int nwg, const int xoff,
                                             uint8_t *smem) {
    using C = FCfg<L, XP>;
    constexpr int L1 = C::L1, L2 = C::L2, U = C::U, G = C::G, ES = C::ES, FPG = C::FPG;
    constexpr int GPW = C::GPW, PACKS = C::PACKS, R = C::R, CP = C::CP, SP = C::SP, EXG = C::EXG;
    uint8_t *outbuf = smem;
    uint8_t *stage = smem + (STATS ? 0 : C::OUT_BYTES);
    float2 *ex = reinterpret_cast<float2 *>(stage + C::STAGE_BYTES);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gi = lane / L2, r = lane % L2;
    const int gg = wave * GPW + gi;            // FFT group within the workgroup
    constexpr int PPG = C::PPG;                // packs gg PPG + pp of the item are group gg's
    const int nblk = (a.n_in + R - 1) / R;
    const int items = a.ngrp * nblk;

    // Per-lane constants.  Output slot i of a lane (i = u * L2 + k2 for the
    // two-pass split) holds FFT bin k = (r U + u) + L1 k2, channel (k + L/2) mod L.
    constexpr bool kTwReg = L1 <= 16;
    constexpr int P = C::P;
    float2 twr[kTwReg && L2 > 1 ? L1 : 1];
    if constexpr (kTwReg && L2 > 1) {
#pragma unroll
        for (int i = 1; i < L1; ++i) twr[i] = a.tw[(r * i) % L];        // W_L^(r k1)
    }
    // W_L2^(q m2) for the values q = 1 .. P-1 of the columns m2 = g + P j that
    // lane (k1, g) = (r / P, r % P) transforms after the second exchange
    constexpr int kTw2 = P > 1 ? (P - 1) * (L1 / P) : 1;
    float2 tw2[kTw2];
    if constexpr (P > 1) {
#pragma unroll
        for (int q = 1; q < P; ++q)
#pragma unroll
            for (int j = 0; j < L1 / P; ++j)
                tw2[(q - 1) * (L1 / P) + j] = a.tw[((q * (r % P + P * j)) % L2) * (L / L2)];
    }
    float sc[XP == MWAX_X_INT8 && kTwReg && !STATS ? L1 : 1];
    if constexpr (XP == MWAX_X_INT8 && kTwReg && !STATS) {
#pragma unroll
        for (int i = 0; i < L1; ++i) sc[i] = a.inv_s[chan_of<L, XP>(r, i)];
    }
    float acc[STATS ? L1 : 1];
#pragma unroll
    for (int i = 0; i < (STATS ? L1 : 1); ++i) acc[i] = 0.0f;
    int popc = 0;   // statistics pass: populated frames this lane counted

    // Staging of the raw frames (two-pass split) through registers; with
    // PREFETCH the global loads of the next item are issued before the current
    // item is transformed, so their latency hides behind the FFT work.
    constexpr int UPF = 2 * L / 16;                      // 16-byte units per frame
    constexpr int NUNITS = L2 > 1 && !C::DIRECT ? R * G * UPF : 0;
    constexpr int NU = (NUNITS + C::THREADS - 1) / C::THREADS;
    uint4 pre[NU > 0 ? NU : 1];
    auto fetch = [&](int it) {
        if constexpr (NU > 0) {
            const int gs = it / nblk;
            const int m0 = (it - gs * nblk) * R;
            const int nr = min(R, a.n_in - m0);
            const int64_t l0 = (int64_t)gs * G;
            const int fv = (int)min((int64_t)G, a.nframes - l0);
            // the item's first sample (uniform); a unit adds its row and offset
            const int8_t *ib = a.volts + ((int64_t)m0 * a.ld + (a.frame0 + l0) * L) * 2;
#pragma unroll
            for (int j = 0; j < NU; ++j) {
                const int u = tid + j * C::THREADS;
                const int sl = u / (G * UPF);
                const int rem = u - sl * G * UPF;
                const int f = rem / UPF;
                pre[j] = make_uint4(0u, 0u, 0u, 0u);     // frames past the end are zero
                if (u < NUNITS && sl < nr && f < fv)
                    pre[j] = *reinterpret_cast<const uint4 *>(ib + (int64_t)sl * (2 * a.ld) + rem * 16);
            }
        }
    };
    // Item of round t.  Workgroup b of a launch runs on XCD b mod 8, and each
    // XCD has its own L2.  The output rows of consecutive items (adjacent inputs
    // of one row group) share cache lines, so a round hands each XCD one
    // contiguous range of items: a line is then completed in one L2 instead of
    // leaving several L2s as partial 32- or 64-byte writes.  xoff: the XCD of
    // workgroup 0 of this work (batched launches).
    const bool xmap = (nwg & 7) == 0;
    auto item_at = [&](int t) {
        return t * nwg + (xmap ? ((wg + xoff) & 7) * (nwg >> 3) + (wg >> 3) : wg);
    };
    const int rounds = (items + nwg - 1) / nwg;
    if constexpr (C::PREFETCH) {
        if (item_at(0) < items) fetch(item_at(0));
    }
    // DIRECT: the 16-bit samples of the group's next frame (q = pp FPG + t of
    // item it), loaded while the current frame is transformed; zeros past the
    // segment or the inputs
    uint32_t raw[C::DIRECT ? L1 : 1];
    auto fetch_frame = [&](int it, int q) {
        if constexpr (C::DIRECT) {
            const int gs = it / nblk;
            const int pg = gg * PPG + q / FPG;
            const int ni = (it - gs * nblk) * R + pg / PACKS;
            const int f = (pg % PACKS) * FPG + q % FPG;
            const int64_t l0 = (int64_t)gs * G;
            if (ni < a.n_in && f < (int)min((int64_t)G, a.nframes - l0)) {
                const uint16_t *src = reinterpret_cast<const uint16_t *>(
                                          a.volts + ((int64_t)ni * a.ld + (a.frame0 + l0 + f) * L) * 2) + r;
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) raw[n1] = src[L2 * n1];
            } else {
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) raw[n1] = 0u;
            }
        }
    };
    if constexpr (C::DIRECT) {
        if (item_at(0) < items) fetch_frame(item_at(0), 0);
    }

    for (int round = 0; round < rounds; ++round) {
        const int item = item_at(round);
        if (item >= items) continue;   // the last round's tail (uniform per workgroup)
        const int gsel = item / nblk;
        const int n0 = (item - gsel * nblk) * R;
        const int nrows = min(R, a.n_in - n0);

        __syncthreads();  // LDS of the previous item fully consumed
        if constexpr (L2 > 1 && !C::DIRECT) {
            if constexpr (!C::PREFETCH) fetch(item);
#pragma unroll
            for (int j = 0; j < NU; ++j) {
                const int u = tid + j * C::THREADS;
                if (u < NUNITS) {
                    const int sl = u / (G * UPF);
                    const int rem = u - sl * G * UPF;
                    const int f = rem / UPF, o = rem - f * UPF;
                    *reinterpret_cast<uint4 *>(stage + (sl * G + f) * SP + o * 16) = pre[j];
                }
            }
            __syncthreads();
            if constexpr (C::PREFETCH) {
                if (round + 1 < rounds && item_at(round + 1) < items) fetch(item_at(round + 1));
            }
        }
        const int64_t lf0 = (int64_t)gsel * G;
        const int fvalid = (int)min((int64_t)G, a.nframes - lf0);
        const int64_t src_frame = a.frame0 + lf0;

        for (int pp = 0; pp < PPG; ++pp) {
        const int nl = (gg * PPG + pp) / PACKS;           // the pack's input within the item
        const int pk = (gg * PPG + pp) - nl * PACKS;      // and its frames pk FPG + t
        // first frame of the pack: binary16 bits per slot, or int8 codes packed four
        // to a word (re words, then im words)
        constexpr int kQ0 = XP == MWAX_X_INT8 ? 2 * ((L1 + 3) / 4) : 2 * L1;
        uint32_t q0[XP != MWAX_X_FP32 && FPG == 2 && !STATS ? kQ0 : 1];
        if constexpr (XP == MWAX_X_INT8 && FPG == 2 && !STATS) {
#pragma unroll
            for (int w = 0; w < kQ0; ++w) q0[w] = 0u;
        }
        for (int t = 0; t < FPG; ++t) {
            const int f = pk * FPG + t;
            float2 v[L1];
            if constexpr (C::DIRECT) {
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) {
                    const int32_t w = (int32_t)(raw[n1] << 16);
                    v[n1] = make_float2((float)((w << 8) >> 24), (float)(w >> 24));
                }
                // start the loads of the group's next frame (in this item or the next)
                const int q = pp * FPG + t + 1;
                if (q < PPG * FPG) fetch_frame(item, q);
                else if (round + 1 < rounds && item_at(round + 1) < items) fetch_frame(item_at(round + 1), 0);
            } else if constexpr (L2 == 1) {
                if (nl < nrows && f < fvalid) {
                    const uint8_t *src = reinterpret_cast<const uint8_t *>(a.volts) +
                                         ((int64_t)(n0 + nl) * a.ld + (src_frame + f) * L) * 2;
                    if constexpr (L == 1) {
                        v[0] = load_pair(src);
                    } else {
#pragma unroll
                        for (int q = 0; q < L / 2; ++q) {
                            const uint32_t wv = *reinterpret_cast<const uint32_t *>(src + 4 * q);
                            v[2 * q] = make_float2((float)(int8_t)wv, (float)(int8_t)(wv >> 8));
                            v[2 * q + 1] = make_float2((float)(int8_t)(wv >> 16), (float)(int8_t)(wv >> 24));
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < L; ++q) v[q] = make_float2(0.0f, 0.0f);
                }
            } else {
                const uint8_t *fr = stage + (nl * G + f) * SP;
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) v[n1] = load_pair(fr + 2 * (r + L2 * n1));
            }
            if constexpr (STATS) {
                // a frame is populated if any of its samples is nonzero (zeroed
                // frames, from lost packets, are left out of the calibration);
                // frames past the segment or input range were loaded as zeros
                bool nz = false;
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) nz = nz || v[n1].x != 0.0f || v[n1].y != 0.0f;
                if constexpr (L2 == 1) {
                    popc += nz ? 1 : 0;
                } else {
                    const uint64_t m = __ballot(nz);
                    const uint64_t gm = L2 == 64 ? m : (m >> (gi * L2)) & ((1ull << (L2 & 63)) - 1ull);
                    popc += (r == 0 && gm != 0ull) ? 1 : 0;
                }
            }
            dft_regs<L1>(v);

            // this frame's delay (signal path n0 + nl) and phase offset
            float dl_alpha = 0.0f, dl_phi = 0.0f;
            if constexpr (DELAY) {
                float d = 0.0f;
                if (nl < nrows && f < fvalid)
                    d = a.dl[(int64_t)(n0 + nl) * a.dl_ld + (a.dl_f0 + lf0 + f) / a.dl_fps];
                const double ph = (double)d * a.dl_nu;
                dl_phi = (float)(ph - rint(ph));
                dl_alpha = d * (1.0f / (float)L);
            }

            // consume output slot i (FFT bin of this lane) with value X; tc: the
            // frame's place in its pack as a compile-time constant (see emit_frame)
            auto emit = [&](int i, float2 X, auto tc) {
                constexpr int T = decltype(tc)::value;
                if constexpr (DELAY) {
                    const int k = bin_of<L, XP>(r, i);
                    const float2 g = delay_gain(k < L / 2 ? k : k - L, dl_alpha, dl_phi);
                    X = make_float2(X.x * g.x - X.y * g.y, X.x * g.y + X.y * g.x);
                }
                if constexpr (STATS) {
                    acc[i] += X.x * X.x + X.y * X.y;
                } else {
                    const int c = chan_of<L, XP>(r, i);
                    uint8_t *row = outbuf + c * CP + nl * kRowBytes + row_re_off(pk * FPG, ES);
                    constexpr int IM = row_im_gap(ES);
                    if constexpr (XP == MWAX_X_INT8) {
                        float s;
                        if constexpr (kTwReg) s = sc[i];
                        else s = a.inv_s[c];
                        const uint32_t br = quant8_bits(X.x, s), bi = quant8_bits(X.y, s);
                        if constexpr (FPG == 1) {
                            // one frame per group: the code's low byte goes straight out
                            row[0] = (uint8_t)br;
                            row[IM] = (uint8_t)bi;
                        } else {
                            // frame 0: keep the code's low byte in byte i % 4 of a word;
                            // frame 1: pair it with the new code, one 16-bit write per half
                            constexpr int kW = (L1 + 3) / 4;
                            const int w = i / 4, p = i % 4;
                            if constexpr (T == 0) {
                                const uint32_t ins = (0x03020100u & ~(0xffu << (8 * p))) | (0x04u << (8 * p));
                                q0[w] = __builtin_amdgcn_perm(br, q0[w], ins);
                                q0[kW + w] = __builtin_amdgcn_perm(bi, q0[kW + w], ins);
                            } else {
                                const uint32_t pair = 0x0c0c0400u | (uint32_t)p;
                                *reinterpret_cast<uint16_t *>(row) = (uint16_t)__builtin_amdgcn_perm(br, q0[w], pair);
                                *reinterpret_cast<uint16_t *>(row + IM) = (uint16_t)__builtin_amdgcn_perm(bi, q0[kW + w], pair);
                            }
                        }
                    } else if constexpr (XP == MWAX_X_FP16) {
                        const _Float16 hr = (_Float16)(X.x * a.half_scale), hi = (_Float16)(X.y * a.half_scale);
                        const uint32_t br = (uint32_t)__builtin_bit_cast(uint16_t, hr);
                        const uint32_t bi = (uint32_t)__builtin_bit_cast(uint16_t, hi);
                        if constexpr (FPG == 2) {
                            if constexpr (T == 0) {
                                q0[2 * i] = br;
                                q0[2 * i + 1] = bi;
                            } else {
                                *reinterpret_cast<uint32_t *>(row) = q0[2 * i] | (br << 16);
                                *reinterpret_cast<uint32_t *>(row + IM) = q0[2 * i + 1] | (bi << 16);
                            }
                        } else {
                            *reinterpret_cast<uint16_t *>(row) = (uint16_t)br;
                            *reinterpret_cast<uint16_t *>(row + IM) = (uint16_t)bi;
                        }
                    } else {
                        *reinterpret_cast<float *>(row) = X.x;
                        *reinterpret_cast<float *>(row + IM) = X.y;
                    }
                }
            };
            // run body(tc) with the frame's place in the pack as a constant, so that
            // the emission of a two-frame pack has no per-slot branch on t
            auto emit_frame = [&](auto body) {
                if (FPG == 1 || t == 0) body(std::integral_constant<int, 0>{});
                else body(std::integral_constant<int, 1>{});
            };

            if constexpr (L2 == 1) {
                emit_frame([&](auto tc) {
#pragma unroll
                    for (int k = 0; k < L1; ++k) emit(k, v[k], tc);
                });
            } else {
#pragma unroll
                for (int k1 = 1; k1 < L1; ++k1) {      // W_L^0 = 1
                    float2 w;
                    if constexpr (kTwReg) w = twr[k1];
                    else w = a.tw[(r * k1) % L];
                    v[k1] = make_float2(v[k1].x * w.x - v[k1].y * w.y, v[k1].x * w.y + v[k1].y * w.x);
                }
                if constexpr (P > 1) {
                    // lane r writes its column of the L1 x L2 block (row pitch
                    // L2 + P keeps the writes and the strided reads below free of
                    // bank conflicts); lane (k1, h) = (r / P, r % P) then takes
                    // rows h + P m of column k1 and an in-lane 16-point DFT over m.
                    // A second exchange hands lane (k1, g) the P values over h of the
                    // columns m2 = g + P j; each takes the twiddle W_L2^(h m2) (none
                    // for h = 0) and their P-point DFTs complete the column's
                    // transform: slot j P + q of the lane holds bin k1 + L1 (g + P j + L1 q)
                    float2 *eg = ex + gg * EXG;
#pragma unroll
                    for (int k1 = 0; k1 < L1; ++k1) eg[k1 * C::EXR + r] = v[k1];
                    wave_sync();
                    const int k1 = r / P, h = r % P;
                    float2 w[L1];
#pragma unroll
                    for (int m = 0; m < L1; ++m) w[m] = eg[k1 * C::EXR + h + P * m];
                    dft_regs<L1>(w);
                    // lane rows of L1 + 1 float2: writes (fixed m) and reads (fixed
                    // h, j) both fall in distinct banks
                    constexpr int XR = L1 + 1;
                    static_assert(C::L2 * XR <= EXG, "second exchange exceeds the group's area");
                    wave_sync();   // the first exchange has been read
#pragma unroll
                    for (int m = 0; m < L1; ++m) eg[r * XR + m] = w[m];
                    wave_sync();
#pragma unroll
                    for (int j = 0; j < L1 / P; ++j) {
#pragma unroll
                        for (int q = 0; q < P; ++q) {
                            float2 y = eg[(k1 * P + q) * XR + h + P * j];
                            if (q > 0) {
                                const float2 t = tw2[(q - 1) * (L1 / P) + j];
                                y = make_float2(y.x * t.x - y.y * t.y, y.x * t.y + y.y * t.x);
                            }
                            w[j * P + q] = y;
                        }
                        dft_regs<P>(w + j * P);
                    }
                    emit_frame([&](auto tc) {
#pragma unroll
                        for (int i = 0; i < L1; ++i) emit(i, w[i], tc);
                    });
                } else {
                    // exchange through LDS; column swizzle r ^ (k1 / U) keeps both the
                    // writes (fixed k1) and the reads (fixed r2) free of bank conflicts
                    float2 *eg = ex + gg * EXG;
#pragma unroll
                    for (int k1 = 0; k1 < L1; ++k1) eg[k1 * L2 + (r ^ (k1 / U))] = v[k1];
                    wave_sync();
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int k1 = r * U + u;
                        float2 w[L2];
#pragma unroll
                        for (int r2 = 0; r2 < L2; ++r2) w[r2] = eg[k1 * L2 + (r2 ^ r)];
                        dft_regs<L2>(w);
                        emit_frame([&](auto tc) {
#pragma unroll
                            for (int k2 = 0; k2 < L2; ++k2) emit(u * L2 + k2, w[k2], tc);
                        });
                    }
                }
                wave_sync();
            }
        }
        }   // packs of the group

        if constexpr (!STATS) {
            __syncthreads();
            // store the image: per channel, nrows rows of 32 bytes, 16 bytes per
            // thread; unit u = (c, 16-byte piece e of the channel's nrows rows)
            const int64_t cstride = a.NG * a.n_in * kRowBytes;    // bytes per channel
            uint8_t *db = a.chan + ((a.grp0 + gsel) * a.n_in + n0) * kRowBytes;
            auto store_unit = [&](int c, int e) {
                const uint32_t *src = reinterpret_cast<const uint32_t *>(outbuf + c * CP + e * 16);
                *reinterpret_cast<uint4 *>(db + c * cstride + e * 16) = make_uint4(src[0], src[1], src[2], src[3]);
            };
            constexpr int SU = L * R * 2, NJ = (SU + C::THREADS - 1) / C::THREADS;
            if (nrows == R && NJ <= 2) {
                // unrolled (more units per thread would hold their loads in registers)
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const int u = tid + j * C::THREADS;
                    if (SU % C::THREADS == 0 || u < SU) store_unit(u / (2 * R), u % (2 * R));
                }
            } else if (nrows == R) {
                for (int u = tid; u < SU; u += C::THREADS) store_unit(u / (2 * R), u % (2 * R));
            } else {
                for (int u = tid; u < L * nrows * 2; u += C::THREADS) store_unit(u / (nrows * 2), u % (nrows * 2));
            }
        }
    }

    if constexpr (STATS) {
        // Deterministic reduction of the per-lane channel sums: lanes with the same r
        // hold the same channel set; sum them in a fixed order.
        __syncthreads();
        float *red = reinterpret_cast<float *>(smem);   // [THREADS / L2 slots][L2][L1]
        int *redp = reinterpret_cast<int *>(red + C::THREADS * L1);
#pragma unroll
        for (int i = 0; i < L1; ++i) red[(gg * L2 + r) * L1 + i] = acc[i];
        redp[tid] = popc;
        __syncthreads();
        constexpr int NSLOT = C::THREADS / L2;
        // partial row of this workgroup: L channel sums, then the populated count
        double *row = a.stats + (int64_t)wg * (L + 1);
        for (int t = tid; t < L; t += C::THREADS) {
            const int rr = t / L1, i = t - rr * L1;
            double sum = 0.0;
            for (int sl = 0; sl < NSLOT; ++sl) sum += (double)red[(sl * L2 + rr) * L1 + i];
            row[chan_of<L, XP>(rr, i)] = sum;
        }
        if (tid == 0) {
            int64_t n = 0;
            for (int t = 0; t < C::THREADS; ++t) n += redp[t];
            row[L] = (double)n;
        }
    }
}

template <int L, int XP, bool STATS, bool DELAY>
__global__ __launch_bounds__((FCfg<L, XP>::THREADS)) void fengine_kernel(FArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    fengine_body<L, XP, STATS, DELAY>(a, blockIdx.x, gridDim.x, 0, smem);
}

// Batched form: workgroups [block0[d], block0[d+1]) of the launch work on
// descriptor d (a segment of one plan of the batch); the rest return at once.
template <int L, int XP, bool STATS>
__global__ __launch_bounds__((FCfg<L, XP>::THREADS)) void fengine_batch_kernel(FBatchArgs b) {
    extern __shared__ __align__(16) uint8_t smem[];
    // the tables are read through the constant address space (scalar loads)
    const int nd = load_uniform(b.ndesc);
    const int blk = blockIdx.x;
    if (blk >= load_uniform(b.block0 + nd)) return;
    int d = 0;
    while (load_uniform(b.block0 + d + 1) <= blk) ++d;
    const FArgs a = load_uniform(b.desc + d);
    const int first = load_uniform(b.block0 + d), count = load_uniform(b.block0 + d + 1) - first;
    fengine_body<L, XP, STATS>(a, blk - first, count, first & 7, smem);
}

template <int L, int XP>
constexpr int cfg_value_lds(bool stats) {
    using C = FCfg<L, XP>;
    return stats ? (C::STAGE_BYTES + C::EX_BYTES > C::RED_BYTES ? C::STAGE_BYTES + C::EX_BYTES : C::RED_BYTES)
                 : C::OUT_BYTES + C::STAGE_BYTES + C::EX_BYTES;
}

template <int L, int XP>
hipError_t launch_L(const FArgs &a, hipStream_t s) {
    using C = FCfg<L, XP>;
    const bool stats = a.stats_mode != 0;
    if (a.R != C::R) return hipErrorInvalidValue;
    const int lds = fengine_lds_bytes(L, XP, a.R, stats);
    int grid = fengine_grid(a.n_in, a.R, a.ngrp, stats);
    if (!stats) grid = (int)std::min<int64_t>((int64_t)a.ngrp * ((a.n_in + C::R - 1) / C::R), C::GRID_CAP);
    if (grid < 1) return hipSuccess;
    // allow dynamic LDS beyond the default limit (once per instantiation)
    const int variant = stats ? 1 : (a.dl ? 2 : 0);
    const void *fns[3] = {reinterpret_cast<const void *>(&fengine_kernel<L, XP, false, false>),
                          reinterpret_cast<const void *>(&fengine_kernel<L, XP, true, false>),
                          reinterpret_cast<const void *>(&fengine_kernel<L, XP, false, true>)};
    static bool attr_done[3] = {false, false, false};
    if (!attr_done[variant]) {
        (void)hipFuncSetAttribute(fns[variant], hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
        attr_done[variant] = true;
    }
    if (variant == 1)
        hipLaunchKernelGGL((fengine_kernel<L, XP, true, false>), dim3((unsigned)grid), dim3(C::THREADS), lds, s, a);
    else if (variant == 2)
        hipLaunchKernelGGL((fengine_kernel<L, XP, false, true>), dim3((unsigned)grid), dim3(C::THREADS), lds, s, a);
    else
        hipLaunchKernelGGL((fengine_kernel<L, XP, false, false>), dim3((unsigned)grid), dim3(C::THREADS), lds, s, a);
    return hipGetLastError();
}

template <int L, int XP>
hipError_t prepare_batch_L() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&fengine_batch_kernel<L, XP, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&fengine_batch_kernel<L, XP, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    return e;
}

template <int L, int XP>
hipError_t launch_batch_L(bool stats, const FBatchArgs &b, int grid, hipStream_t s) {
    const int lds = cfg_value_lds<L, XP>(stats);
    if (stats)
        hipLaunchKernelGGL((fengine_batch_kernel<L, XP, true>), dim3((unsigned)grid), dim3(FCfg<L, XP>::THREADS), lds, s, b);
    else
        hipLaunchKernelGGL((fengine_batch_kernel<L, XP, false>), dim3((unsigned)grid), dim3(FCfg<L, XP>::THREADS), lds, s, b);
    return hipGetLastError();
}

#define MWAX_L_SWITCH(CALL)                         \
    switch (L) {                                    \
        case 1: return CALL(1);                     \
        case 2: return CALL(2);                     \
        case 4: return CALL(4);                     \
        case 8: return CALL(8);                     \
        case 16: return CALL(16);                   \
        case 32: return CALL(32);                   \
        case 64: return CALL(64);                   \
        case 128: return CALL(128);                 \
        case 256: return CALL(256);                 \
        case 512: return CALL(512);                 \
        case 1024: return CALL(1024);               \
        default: return hipErrorInvalidValue;       \
    }

template <int XP>
hipError_t launch_batch_xp(int L, bool stats, const FBatchArgs &b, int grid, hipStream_t s) {
#define MWAX_CALL(LL) launch_batch_L<LL, XP>(stats, b, grid, s)
    MWAX_L_SWITCH(MWAX_CALL)
#undef MWAX_CALL
}

template <int XP>
hipError_t prepare_batch_xp(int L) {
#define MWAX_CALL(LL) prepare_batch_L<LL, XP>()
    MWAX_L_SWITCH(MWAX_CALL)
#undef MWAX_CALL
}

template <int XP>
hipError_t launch_xp(int L, const FArgs &a, hipStream_t s) {
    switch (L) {
        case 1: return launch_L<1, XP>(a, s);
        case 2: return launch_L<2, XP>(a, s);
        case 4: return launch_L<4, XP>(a, s);
        case 8: return launch_L<8, XP>(a, s);
        case 16: return launch_L<16, XP>(a, s);
        case 32: return launch_L<32, XP>(a, s);
        case 64: return launch_L<64, XP>(a, s);
        case 128: return launch_L<128, XP>(a, s);
        case 256: return launch_L<256, XP>(a, s);
        case 512: return launch_L<512, XP>(a, s);
        case 1024: return launch_L<1024, XP>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
__global__ void twiddle_kernel(float2 *tw, int L) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L) return;
    // exp(-2 pi i k / L) in FP64, rounded to FP32; quarter turns exact.
    const int q4 = (4 * k) % L == 0 ? (4 * k) / L : -1;
    if (q4 >= 0) {
        const float re[4] = {1.0f, 0.0f, -1.0f, 0.0f};
        const float im[4] = {0.0f, -1.0f, 0.0f, 1.0f};
        tw[k] = make_float2(re[q4], im[q4]);
        return;
    }
    double sn, cs;
    sincospi(-2.0 * (double)k / (double)L, &sn, &cs);
    tw[k] = make_float2((float)cs, (float)sn);
}

// Scales of channel c from its power sum and populated-frame count over the
// calibration window:
//   sigma^2 = power / (2 populated),  s = 5 sigma / 127,  inv_s = 127 / (5 sigma)
// (s = inv_s = 1 for a channel of zero power).  With no populated frame the
// window holds only zeroed samples: the channel keeps last[] (the scales of the
// plan's most recent calibrated integration).  Otherwise last[] is updated.
__device__ __forceinline__ void finish_scale(double sum, double count, int L, float *scales, float *last, int c) {
    float s = last[c], inv = last[L + c];
    if (count > 0.0) {
        const double var = sum / (2.0 * count);
        s = 1.0f;
        inv = 1.0f;
        if (var > 0.0) {
            const double sd = sqrt(var);
            s = (float)(5.0 * sd / 127.0);
            inv = (float)(127.0 / (5.0 * sd));
        }
        last[c] = s;
        last[L + c] = inv;
    }
    scales[c] = s;
    scales[L + c] = inv;
}

// Scales of channel c from the partial rows of nwg workgroups ([nwg][L + 1]: L
// power sums, then the populated-frame count), reduced in a fixed order so the
// result is bitwise reproducible.
__device__ void calib_finish_channel(const double *stats, int nwg, int L, float *scales, float *last, int c) {
    __shared__ double part[256], cnt[256];
    __syncthreads();   // part/cnt of a previous call on this workgroup fully read
    double t = 0.0, n = 0.0;
    for (int w = threadIdx.x; w < nwg; w += 256) {
        t += stats[(int64_t)w * (L + 1) + c];
        n += stats[(int64_t)w * (L + 1) + L];
    }
    part[threadIdx.x] = t;
    cnt[threadIdx.x] = n;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            part[threadIdx.x] += part[threadIdx.x + h];
            cnt[threadIdx.x] += cnt[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    finish_scale(part[0], cnt[0], L, scales, last, c);
}

__global__ void calib_finish_kernel(const double *stats, int nwg, int L, float *scales, float *last) {
    calib_finish_channel(stats, nwg, L, scales, last, blockIdx.x);
}

// Wide transforms (L = 6400): one workgroup per 16 channels.  Thread (channel
// cl, slice sl) sums the partial rows sl, sl + 16, ... into eight running sums
// (row sl + 16 (8 k + i) into sum i, so eight loads are in flight); the eight
// sums, then the sixteen slices (and the frame counts) are added in a fixed
// order.
constexpr int kWideCh = 16, kWideSl = 256 / kWideCh;
__global__ __launch_bounds__(256) void calib_finish_wide_kernel(const double *stats, int nwg, int L, float *scales,
                                                                float *last) {
    constexpr int kAcc = 8;
    __shared__ double part[kWideSl][kWideCh], cnt[kWideSl];
    const int cl = threadIdx.x % kWideCh, sl = threadIdx.x / kWideCh, c = blockIdx.x * kWideCh + cl;
    const int cc = c < L ? c : L;   // channels past L read the count column instead
    double ts[kAcc] = {}, ns[kAcc] = {};
    int w = sl;
    for (; w + kWideSl * (kAcc - 1) < nwg; w += kWideSl * kAcc) {
#pragma unroll
        for (int i = 0; i < kAcc; ++i) {
            ts[i] += stats[(int64_t)(w + kWideSl * i) * (L + 1) + cc];
            ns[i] += stats[(int64_t)(w + kWideSl * i) * (L + 1) + L];
        }
    }
#pragma unroll
    for (int i = 0; i < kAcc; ++i) {
        if (w + kWideSl * i < nwg) {
            ts[i] += stats[(int64_t)(w + kWideSl * i) * (L + 1) + cc];
            ns[i] += stats[(int64_t)(w + kWideSl * i) * (L + 1) + L];
        }
    }
    double t = 0.0, n = 0.0;
#pragma unroll
    for (int i = 0; i < kAcc; ++i) {
        t += ts[i];
        n += ns[i];
    }
    part[sl][cl] = t;
    if (cl == 0) cnt[sl] = n;
    __syncthreads();
    if (sl != 0 || c >= L) return;
    t = 0.0;
    n = 0.0;
    for (int k = 0; k < kWideSl; ++k) {
        t += part[k][cl];
        n += cnt[k];
    }
    finish_scale(t, n, L, scales, last, c);
}

// One workgroup per (channel, descriptor).  The descriptors of one instance are
// consecutive and its first one carries their number (n_chain); that workgroup
// processes them in order, so an integration whose window holds no populated
// frame takes the scales of the instance's previous calibrated integration,
// also within one call.  Other descriptors and channels past L return at once.
__global__ void calib_batch_kernel(const CalDesc *desc, const int32_t *ndesc) {
    const int d = blockIdx.y, c = blockIdx.x;
    if (d >= *ndesc) return;
    const CalDesc head = desc[d];
    if (head.n_chain == 0 || c >= head.L) return;
    for (int k = 0; k < head.n_chain; ++k) {
        const CalDesc cd = desc[d + k];
        if (cd.copy_src) {
            if (threadIdx.x == 0) {
                cd.scales[c] = cd.copy_src[c];
                cd.scales[cd.L + c] = cd.copy_src[cd.L + c];
            }
        } else {
            calib_finish_channel(cd.stats, cd.nwg, cd.L, cd.scales, cd.last, c);
        }
    }
}

__global__ void copy_scales_kernel(const float *src, float *dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void fill_f32_kernel(float *dst, float v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

template <int ES>
__global__ void repack_kernel(RepackArgs a) {
    using E = typename std::conditional<ES == 1, int8_t, typename std::conditional<ES == 2, uint16_t, float>::type>::type;
    const int64_t per_m = (int64_t)a.L * a.n_in;
    const int64_t span = a.to_internal ? (int64_t)((a.nframes + a.G - 1) / a.G) * a.G : a.nframes;
    const int64_t total = span * per_m;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = t / per_m;
        const int64_t rem = t - m * per_m;
        const int c = (int)(rem / a.n_in);
        const int n = (int)(rem - (int64_t)c * a.n_in);
        const int64_t g = a.grp0 + m / a.G;
        const int f = (int)(m % a.G);
        E *row = reinterpret_cast<E *>(a.chan + (((int64_t)c * a.NG + g) * a.n_in + n) * kRowBytes);
        E *cv = reinterpret_cast<E *>(a.canon) + (((a.m0 + m) * a.L + c) * (int64_t)a.n_in + n) * 2;
        const int ire = row_re_off(f, ES) / ES, iim = ire + row_im_gap(ES) / ES;
        if (a.to_internal) {
            E re = E(0), im = E(0);
            if (m < a.nframes) {
                re = cv[0];
                im = cv[1];
                if constexpr (ES == 1) {
                    if (re == (E)-128) re = (E)-127;
                    if (im == (E)-128) im = (E)-127;
                }
            }
            row[ire] = re;
            row[iim] = im;
        } else {
            cv[0] = row[ire];
            cv[1] = row[iim];
        }
    }
}

}  // namespace

template <int XP>
static int cfg_value(int L, int what) {
#define MWAX_CFG_CASE(LL)                                                                     \
    case LL:                                                                                  \
        return what == 0 ? FCfg<LL, XP>::R                                                    \
                         : (what == 1 ? FCfg<LL, XP>::OUT_BYTES + FCfg<LL, XP>::STAGE_BYTES + \
                                            FCfg<LL, XP>::EX_BYTES                            \
                                      : std::max(FCfg<LL, XP>::STAGE_BYTES + FCfg<LL, XP>::EX_BYTES, \
                                                 FCfg<LL, XP>::RED_BYTES));
    switch (L) {
        MWAX_CFG_CASE(1) MWAX_CFG_CASE(2) MWAX_CFG_CASE(4) MWAX_CFG_CASE(8) MWAX_CFG_CASE(16)
        MWAX_CFG_CASE(32) MWAX_CFG_CASE(64) MWAX_CFG_CASE(128) MWAX_CFG_CASE(256)
        MWAX_CFG_CASE(512) MWAX_CFG_CASE(1024)
        default: return -1;
    }
#undef MWAX_CFG_CASE
}

static int cfg_of(int L, int xprec, int what) {
    switch (xprec) {
        case MWAX_X_INT8: return cfg_value<MWAX_X_INT8>(L, what);
        case MWAX_X_FP16: return cfg_value<MWAX_X_FP16>(L, what);
        default: return cfg_value<MWAX_X_FP32>(L, what);
    }
}

int fengine_grid(int n_in, int R, int ngrp, bool stats) {
    const int64_t items = (int64_t)ngrp * ((n_in + R - 1) / R);
    // stats mode writes one partial row per workgroup: keep that buffer small
    const int64_t cap = stats ? kStatsMaxWG : 65536;
    return (int)(items < cap ? items : cap);
}

int fengine_pick_R(int L, int xprec, int /*n_in*/, int /*lds_limit*/) { return cfg_of(L, xprec, 0); }

int fengine_lds_bytes(int L, int xprec, int /*R*/, bool stats) { return cfg_of(L, xprec, stats ? 2 : 1); }

hipError_t launch_fengine(int L, int xprec, const FArgs &a, hipStream_t s) {
    switch (xprec) {
        case MWAX_X_INT8: return launch_xp<MWAX_X_INT8>(L, a, s);
        case MWAX_X_FP16: return launch_xp<MWAX_X_FP16>(L, a, s);
        case MWAX_X_FP32: return launch_xp<MWAX_X_FP32>(L, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fengine_batch(int L, int xprec, bool stats, const FBatchArgs &b, int grid, hipStream_t s) {
    if (grid < 1) return hipSuccess;
    switch (xprec) {
        case MWAX_X_INT8: return launch_batch_xp<MWAX_X_INT8>(L, stats, b, grid, s);
        case MWAX_X_FP16: return launch_batch_xp<MWAX_X_FP16>(L, stats, b, grid, s);
        case MWAX_X_FP32: return launch_batch_xp<MWAX_X_FP32>(L, stats, b, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t fengine_prepare_batch(int L, int xprec) {
    switch (xprec) {
        case MWAX_X_INT8: return prepare_batch_xp<MWAX_X_INT8>(L);
        case MWAX_X_FP16: return prepare_batch_xp<MWAX_X_FP16>(L);
        case MWAX_X_FP32: return prepare_batch_xp<MWAX_X_FP32>(L);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_calib_batch(const CalDesc *desc, const int32_t *ndesc, int max_desc, int max_L, hipStream_t s) {
    if (max_desc < 1) return hipSuccess;
    hipLaunchKernelGGL(calib_batch_kernel, dim3((unsigned)max_L, (unsigned)max_desc), dim3(256), 0, s, desc, ndesc);
    return hipGetLastError();
}

hipError_t launch_twiddles(float2 *tw, int L, hipStream_t s) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
    return hipGetLastError();
}

hipError_t launch_calib_finish(const double *stats, int nwg, int L, float *scales, float *last, hipStream_t s) {
    if (L == kUltraFineL)
        hipLaunchKernelGGL(calib_finish_wide_kernel, dim3((L + kWideCh - 1) / kWideCh), dim3(256), 0, s, stats, nwg, L,
                           scales, last);
    else
        hipLaunchKernelGGL(calib_finish_kernel, dim3(L), dim3(256), 0, s, stats, nwg, L, scales, last);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *dst, float v, int n, hipStream_t s) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dst, v, n);
    return hipGetLastError();
}

hipError_t launch_copy_scales(const float *src, float *dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(copy_scales_kernel, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_repack(const RepackArgs &a, hipStream_t s) {
    const int64_t span = a.to_internal ? (int64_t)((a.nframes + a.G - 1) / a.G) * a.G : a.nframes;
    const int64_t total = span * a.L * a.n_in;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    switch (a.esize) {
        case 1: hipLaunchKernelGGL(repack_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(repack_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(repack_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mwax
