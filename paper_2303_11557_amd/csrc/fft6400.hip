// F-engine for the 6,400-point transform of Sec. 2.5.1: every 5 ms frame of
// 6,400 complex samples of every signal path is transformed into 6,400
// ultra-fine channels of 200 Hz (unnormalised forward FFT in FP32, channels
// centre-symmetric with DC at c = 3200, Sec. 2.6), then requantised (INT8 /
// binary16) or kept (FP32).
//
// A workgroup of 256 lanes transforms one frame at a time,
// 6400 = 25 x 256 = 25 x 16 x 16:
//   pass 1  lane r holds x[r + 256 n1] (n1 < 25, loaded straight from HBM, the
//           lanes of a wave reading 128 contiguous bytes per load) and computes
//           the 25-point DFT in registers as 5 x 5 radix-5 butterflies, then
//           multiplies bin k1 by W_6400^(r k1);
//   pass 2  the 25 x 256 block goes through LDS; 400 16-point DFTs over
//           r = ra + 16 rb (for each k1, ra), times W_256^(ra k2a), in place;
//   pass 3  400 16-point DFTs over ra (for each k1, k2a), giving bin
//           k = k1 + 25 k2a + 400 k2b.  Lane d = 25 k2a + k1 holds bins
//           d + 400 k2b, so the lanes of a wave write 64 consecutive channels.
// The output is frame-major, [input][frame][channel] (the order a transform
// produces); corner_turn_kernel then moves it into the channel-major row
// groups the X-engine reads ([channel][group][input][32 B]): a 6,400-channel
// row group of one input is 200 KB, beyond the LDS of a workgroup, so the
// transpose of Sec. 2.5.1 is its own HBM pass at this length.
#include "fft_common.h"
#include "mwax_internal.h"

namespace mwax {
namespace {

using namespace fft;

constexpr int kL = 6400;
constexpr int kT = 256;          // lanes per workgroup (one frame at a time)
constexpr int kN1 = 25;          // pass-1 points per lane
constexpr int kPitch = 273;      // float2 per row of the 25 x 256 exchange block
                                 // (273 = 17 mod 32 keeps passes 2 and 3 nearly
                                 // free of bank conflicts)
constexpr int kNd = 400;         // 16-point DFTs in passes 2 and 3

// cos and sin of 2 pi j / 25 (j < 25), rounded to FP32 from their FP64 values
struct W25 {
    static constexpr float c[25] = {
        1.0f, 0.9685831665992737f, 0.8763066530227661f, 0.728968620300293f, 0.5358268022537231f,
        0.30901700258255005f, 0.06279052048921585f, -0.187381312251091f, -0.4257792830467224f,
        -0.6374239921569824f, -0.80901700258255f, -0.9297764897346497f, -0.9921147227287292f,
        -0.9921147227287292f, -0.9297764897346497f, -0.80901700258255f, -0.6374239921569824f,
        -0.4257792830467224f, -0.187381312251091f, 0.06279052048921585f, 0.30901700258255005f,
        0.5358268022537231f, 0.728968620300293f, 0.8763066530227661f, 0.9685831665992737f};
    static constexpr float s[25] = {
        0.0f, 0.24868988990783691f, 0.4817536771297455f, 0.6845471262931824f, 0.8443279266357422f,
        0.9510565400123596f, 0.9980267286300659f, 0.9822872281074524f, 0.9048270583152771f,
        0.7705132365226746f, 0.5877852439880371f, 0.3681245446205139f, 0.12533323466777802f,
        -0.12533323466777802f, -0.3681245446205139f, -0.5877852439880371f, -0.7705132365226746f,
        -0.9048270583152771f, -0.9822872281074524f, -0.9980267286300659f, -0.9510565400123596f,
        -0.8443279266357422f, -0.6845471262931824f, -0.4817536771297455f, -0.24868988990783691f};
};

__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// Forward 5-point DFT in place (W = exp(-2 pi i / 5)):
//   t1 = a1 + a4, t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3
//   X0 = a0 + t1 + t2
//   X1, X4 = (a0 + c1 t1 + c2 t2) -+ i (s1 t3 + s2 t4)
//   X2, X3 = (a0 + c2 t1 + c1 t2) -+ i (s2 t3 - s1 t4)
// with c_j = cos(2 pi j / 5), s_j = sin(2 pi j / 5).
__device__ __forceinline__ void radix5(float2 &a0, float2 &a1, float2 &a2, float2 &a3, float2 &a4) {
    constexpr float c1 = W25::c[5], c2 = W25::c[10], s1 = W25::s[5], s2 = W25::s[10];
    const float2 t1 = make_float2(a1.x + a4.x, a1.y + a4.y), t2 = make_float2(a2.x + a3.x, a2.y + a3.y);
    const float2 t3 = make_float2(a1.x - a4.x, a1.y - a4.y), t4 = make_float2(a2.x - a3.x, a2.y - a3.y);
    const float2 b1 = make_float2(fmaf(c2, t2.x, fmaf(c1, t1.x, a0.x)), fmaf(c2, t2.y, fmaf(c1, t1.y, a0.y)));
    const float2 b2 = make_float2(fmaf(c1, t2.x, fmaf(c2, t1.x, a0.x)), fmaf(c1, t2.y, fmaf(c2, t1.y, a0.y)));
    const float2 u = make_float2(fmaf(s2, t4.x, s1 * t3.x), fmaf(s2, t4.y, s1 * t3.y));
    const float2 w = make_float2(fmaf(-s1, t4.x, s2 * t3.x), fmaf(-s1, t4.y, s2 * t3.y));
    a0 = make_float2(a0.x + t1.x + t2.x, a0.y + t1.y + t2.y);
    a1 = make_float2(b1.x + u.y, b1.y - u.x);
    a4 = make_float2(b1.x - u.y, b1.y + u.x);
    a2 = make_float2(b2.x + w.y, b2.y - w.x);
    a3 = make_float2(b2.x - w.y, b2.y + w.x);
}

// 25-point DFT of v (natural order in and out) as 5 x 5: with n = a + 5 b and
// k = c + 5 d,  X[c + 5 d] = sum_a W_5^(a d) W_25^(a c) sum_b x[a + 5 b] W_5^(b c).
__device__ __forceinline__ void dft25(float2 *v) {
    float2 y[25];   // y[5 a + c]
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        float2 p0 = v[a], p1 = v[a + 5], p2 = v[a + 10], p3 = v[a + 15], p4 = v[a + 20];
        radix5(p0, p1, p2, p3, p4);
        y[5 * a] = p0;
        y[5 * a + 1] = p1;
        y[5 * a + 2] = p2;
        y[5 * a + 3] = p3;
        y[5 * a + 4] = p4;
    }
#pragma unroll
    for (int a = 1; a < 5; ++a)
#pragma unroll
        for (int c = 1; c < 5; ++c) y[5 * a + c] = cmul(y[5 * a + c], make_float2(W25::c[a * c], -W25::s[a * c]));
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        float2 q0 = y[c], q1 = y[5 + c], q2 = y[10 + c], q3 = y[15 + c], q4 = y[20 + c];
        radix5(q0, q1, q2, q3, q4);
        v[c] = q0;
        v[c + 5] = q1;
        v[c + 10] = q2;
        v[c + 15] = q3;
        v[c + 20] = q4;
    }
}

template <int XP>
struct Elem;
template <>
struct Elem<MWAX_X_INT8> { static constexpr int ES = 1; };
template <>
struct Elem<MWAX_X_FP16> { static constexpr int ES = 2; };
template <>
struct Elem<MWAX_X_FP32> { static constexpr int ES = 4; };

// Main pass (STATS = false): spectra of frames frame0 .. frame0 + nframes - 1 of
// every input, written to a.mid[n][frame][channel][re, im].  Statistics pass:
// per-channel power sums and the populated-frame count of those frames, one
// row [L + 1] per workgroup in a.stats (see calib_finish_channel).
// DELAY: the fractional delay and phase correction of the frame's step, in the
// epilogue: lane d holds the signed bins d + 400 j (j = -8 .. 7), so its gains
// exp(-2 pi i ((d + 400 j) d_s / L + phi)) are b w^j with b, w from two sincos.
template <int XP, bool STATS, bool DELAY>
__global__ __launch_bounds__(kT, 2) void fft6400_kernel(FArgs a) {
    __shared__ float2 blk[kN1 * kPitch];
    constexpr int ES = Elem<XP>::ES;
    const int r = threadIdx.x;
    const int64_t items = (int64_t)a.n_in * a.nframes;

    // Per-lane twiddles, the same for every frame this lane transforms:
    // W_6400^(r k1) (k1 = 1 .. 24) after pass 1 and W_256^(ra k) = W_6400^(25 ra k)
    // (k = 1 .. 15) after the DFTs of pass 2, one complex multiply per bin.
    float2 t1[kN1];
#pragma unroll
    for (int k1 = 1; k1 < kN1; ++k1) t1[k1] = a.tw[r * k1];           // r k1 < 6400
    const int ra = r & 15;            // pass-2 column of both of this lane's DFTs
    float2 t2[16];
#pragma unroll
    for (int k = 1; k < 16; ++k) t2[k] = a.tw[25 * ra * k];           // 25 ra k < 6400

    float acc[STATS ? 32 : 1];
#pragma unroll
    for (int i = 0; i < (STATS ? 32 : 1); ++i) acc[i] = 0.0f;
    int64_t popc = 0;

    // raw samples of an item, x[r + 256 n1] as 16-bit (re, im) words
    uint32_t raw[kN1];
    auto fetch = [&](int64_t it) {
        const int64_t n = it / a.nframes, m = it - n * a.nframes;
        const uint16_t *src = reinterpret_cast<const uint16_t *>(a.volts + (n * a.ld + (a.frame0 + m) * kL) * 2);
#pragma unroll
        for (int n1 = 0; n1 < kN1; ++n1) raw[n1] = src[r + 256 * n1];
    };
    if ((int64_t)blockIdx.x < items) fetch(blockIdx.x);

    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t n = it / a.nframes, m = it - n * a.nframes;
        float2 v[kN1];
#pragma unroll
        for (int n1 = 0; n1 < kN1; ++n1)
            v[n1] = make_float2((float)(int8_t)raw[n1], (float)(int8_t)(raw[n1] >> 8));
        if constexpr (STATS) {
            // a frame is populated if any sample is nonzero (zeroed frames, from
            // lost packets, are left out of the calibration)
            bool nz = false;
#pragma unroll
            for (int n1 = 0; n1 < kN1; ++n1) nz = nz || (raw[n1] & 0xffffu) != 0u;
            if (__syncthreads_or(nz ? 1 : 0) && r == 0) ++popc;
        }
        if (it + gridDim.x < items) fetch(it + gridDim.x);   // next frame's loads in flight

        // pass 1
        dft25(v);
#pragma unroll
        for (int k1 = 1; k1 < kN1; ++k1) {
            v[k1] = cmul(v[k1], t1[k1]);
        }
        __syncthreads();   // the previous frame's pass 3 has read blk
#pragma unroll
        for (int k1 = 0; k1 < kN1; ++k1) blk[k1 * kPitch + r] = v[k1];
        __syncthreads();

        // pass 2: DFTs d = 16 k1 + ra over rb, in place
        for (int d = r; d < kNd; d += kT) {
            float2 *col = blk + (d >> 4) * kPitch + ra;
            float2 w[16];
#pragma unroll
            for (int rb = 0; rb < 16; ++rb) w[rb] = col[16 * rb];
            dft_regs<16>(w);
#pragma unroll
            for (int k = 1; k < 16; ++k) {
                w[k] = cmul(w[k], t2[k]);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) col[16 * k] = w[k];
        }
        __syncthreads();

        // this frame's delay: w^j = exp(-2 pi i 400 j d_s / L), j = 0 .. 8
        float dl_alpha = 0.0f, dl_phi = 0.0f;
        float2 pw[DELAY ? 9 : 1];
        if constexpr (DELAY) {
            const float dly = a.dl[n * a.dl_ld + (a.dl_f0 + m) / a.dl_fps];
            const double ph = (double)dly * a.dl_nu;
            dl_phi = (float)(ph - rint(ph));
            dl_alpha = dly / (float)kL;
            float sn, cs;
            sincospif(-2.0f * dly * (400.0f / (float)kL), &sn, &cs);
            pw[0] = make_float2(1.0f, 0.0f);
            pw[1] = make_float2(cs, sn);
#pragma unroll
            for (int j = 2; j <= 8; ++j) pw[j] = cmul(pw[j - 1], pw[1]);
        }

        // pass 3: DFTs d = 25 k2a + k1 over ra; bins d + 400 k2b
#pragma unroll
        for (int slot = 0; slot < 2; ++slot) {
            const int d = r + slot * kT;
            if (d < kNd) {
                const int k1 = d % kN1, k2a = d / kN1;
                const float2 *row = blk + k1 * kPitch + 16 * k2a;
                uint8_t *drow = a.mid + (((n * a.mid_frames) + a.frame0 + m) * kL + d) * 2 * ES;
                const float *srow = a.inv_s + d;
                float2 z[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) z[q] = row[q];
                dft_regs<16>(z);
                float2 gb = make_float2(1.0f, 0.0f);
                if constexpr (DELAY) {
                    float sn, cs;
                    sincospif(-2.0f * fmaf((float)d, dl_alpha, dl_phi), &sn, &cs);
                    gb = make_float2(cs, sn);
                }
#pragma unroll
                for (int k2b = 0; k2b < 16; ++k2b) {
                    float2 X = z[k2b];
                    if constexpr (DELAY) {
                        // bins past L/2 are the negative frequencies d + 400 (k2b - 16)
                        const float2 wj = k2b < 8 ? pw[k2b] : make_float2(pw[16 - k2b].x, -pw[16 - k2b].y);
                        X = cmul(X, cmul(gb, wj));
                    }
                    if constexpr (STATS) {
                        acc[slot * 16 + k2b] += X.x * X.x + X.y * X.y;
                    } else {
                        // channel (d + 400 k2b + L/2) mod L = d + 400 ((k2b + 8) mod 16), as
                        // d < 400: a compile-time offset from the lane's first channel
                        const int co = 400 * ((k2b + 8) & 15);
                        uint8_t *dst = drow + co * 2 * ES;
                        if constexpr (XP == MWAX_X_INT8) {
                            const float s = srow[co];
                            const uint32_t br = quant8_bits(X.x, s) & 0xffu, bi = quant8_bits(X.y, s) & 0xffu;
                            *reinterpret_cast<uint16_t *>(dst) = (uint16_t)(br | (bi << 8));
                        } else if constexpr (XP == MWAX_X_FP16) {
                            const _Float16 hr = (_Float16)(X.x * a.half_scale), hi = (_Float16)(X.y * a.half_scale);
                            *reinterpret_cast<uint32_t *>(dst) = (uint32_t)__builtin_bit_cast(uint16_t, hr) |
                                                                 ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
                        } else {
                            *reinterpret_cast<float2 *>(dst) = X;
                        }
                    }
                }
            }
        }
    }

    if constexpr (STATS) {
        // every channel belongs to exactly one (lane, slot, k2b) of the workgroup
        double *row = a.stats + (int64_t)blockIdx.x * (kL + 1);
#pragma unroll
        for (int slot = 0; slot < 2; ++slot) {
            const int d = r + slot * kT;
            if (d < kNd) {
#pragma unroll
                for (int k2b = 0; k2b < 16; ++k2b) row[(d + 400 * k2b + kL / 2) % kL] = (double)acc[slot * 16 + k2b];
            }
        }
        if (r == 0) row[kL] = (double)popc;
    }
}

// Frame-major spectra [input][frame][channel][re, im] (elements of ES bytes) ->
// channel-major row groups [channel][group][input][32 B] (the row layout of
// row_re_off / row_im_gap).  A workgroup moves one row group (G frames) x 64
// channels x 32 inputs = 64 KB.  Loads: 16 bytes per lane along the channels of
// one (input, frame), stored as they are into an LDS image [input][frame]
// [channel] (each input's block padded by 16 bytes).  Then lane (input, channel
// quad) reads the G x 4 samples of its quad, regroups them in registers into the
// four 32-byte rows of (channel, input) and stores them; the 32 lanes of a
// half-wave hold 32 consecutive inputs, so the rows of a channel go out as 1 KB
// runs.  Frames past the segment and inputs past n_in read as zeros; rows of
// inputs past n_in are not written.
constexpr int kCtChannels = 64, kCtInputs = 32;

// Bytes of {hi, lo} picked by sel (v_perm_b32: selector 0-3 picks bytes of lo,
// 4-7 bytes of hi).
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

template <int ES>
__global__ __launch_bounds__(256) void corner_turn_kernel(CornerArgs a) {
    constexpr int G = 16 / ES, CB = kCtChannels, NB = kCtInputs;
    constexpr int FB = CB * 2 * ES;            // bytes of one (input, frame)
    constexpr int NPITCH = G * FB + 16;        // bytes of one input's block
    constexpr int UPF = FB / 16;               // 16-byte units per (input, frame)
    __shared__ __align__(16) uint8_t img[NB * NPITCH];
    const int g = blockIdx.x, c0 = blockIdx.y * CB, n0 = blockIdx.z * NB;
    const int tid = threadIdx.x;
    const int fvalid = (int)min((int64_t)G, a.nframes - (int64_t)g * G);
    const int64_t fstride = (int64_t)a.L * 2 * ES;   // bytes between frames of an input
    // unit tid + 256 j: (input nl0 + 2 j, frame f, unit cu), since 256 units span
    // two inputs' G frames.  Every load is issued (from a clamped, valid address)
    // and its value dropped afterwards when it lies past the inputs or frames, so
    // that no load waits behind a branch for the one before it.
    static_assert(256 / UPF == 2 * G, "a pass of the workgroup covers two inputs");
    const int cu = tid % UPF, f = (tid / UPF) % G, nl0 = tid / (UPF * G);
    const int fr = min(f, fvalid - 1);
    uint4 val[NB / 2];
#pragma unroll
    for (int j = 0; j < NB / 2; ++j) {
        const int n = min(n0 + nl0 + 2 * j, a.n_in - 1);
        val[j] = *reinterpret_cast<const uint4 *>(
            a.mid + ((int64_t)n * a.mid_frames + a.frame0 + (int64_t)g * G + fr) * fstride + (int64_t)c0 * 2 * ES +
            cu * 16);
    }
    uint8_t *ldst = img + nl0 * NPITCH + f * FB + cu * 16;
#pragma unroll
    for (int j = 0; j < NB / 2; ++j) {
        const bool in = n0 + nl0 + 2 * j < a.n_in && f < fvalid;
        *reinterpret_cast<uint4 *>(ldst + j * 2 * NPITCH) = in ? val[j] : make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    const int nl = tid & 31;
    if (n0 + nl >= a.n_in) return;
#pragma unroll
    for (int t = 0; t < CB / 4 / 8; ++t) {
        const int q = (tid >> 5) + 8 * t;      // channel quad of this lane
        const uint8_t *src = img + nl * NPITCH + q * 8 * ES;
        uint32_t w[4][8];                      // the four rows, as dwords
        if constexpr (ES == 1) {
            // frame f: (re, im) of channels 4q .. 4q + 3 in two dwords
            uint2 r[16];
#pragma unroll
            for (int f = 0; f < 16; ++f) r[f] = *reinterpret_cast<const uint2 *>(src + f * FB);
#pragma unroll
            for (int fb = 0; fb < 4; ++fb) {
                const int wre = (fb >> 1) * 4 + (fb & 1), wim = wre + 2;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // frames 4 fb .. 4 fb + 3 (A .. D) of channels 2h (bytes 0 = re,
                    // 1 = im) and 2h + 1 (bytes 2, 3): a 4 x 4 byte transpose
                    const uint32_t A = h ? r[4 * fb].y : r[4 * fb].x, B = h ? r[4 * fb + 1].y : r[4 * fb + 1].x;
                    const uint32_t C = h ? r[4 * fb + 2].y : r[4 * fb + 2].x, D = h ? r[4 * fb + 3].y : r[4 * fb + 3].x;
                    const uint32_t P = perm(B, A, 0x05010400u), Q = perm(B, A, 0x07030602u);   // A0 B0 A1 B1, A2 B2 A3 B3
                    const uint32_t R = perm(D, C, 0x05010400u), S = perm(D, C, 0x07030602u);   // C0 D0 C1 D1, C2 D2 C3 D3
                    w[2 * h][wre] = perm(R, P, 0x05040100u);
                    w[2 * h][wim] = perm(R, P, 0x07060302u);
                    w[2 * h + 1][wre] = perm(S, Q, 0x05040100u);
                    w[2 * h + 1][wim] = perm(S, Q, 0x07060302u);
                }
            }
        } else if constexpr (ES == 2) {
            // frame f: one dword (re | im << 16) per channel
            uint4 r[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) r[f] = *reinterpret_cast<const uint4 *>(src + f * FB);
#pragma unroll
            for (int pp = 0; pp < 4; ++pp) {
                const int wre = (pp >> 1) * 4 + (pp & 1), wim = wre + 2;
                const uint32_t X[4] = {r[2 * pp].x, r[2 * pp].y, r[2 * pp].z, r[2 * pp].w};
                const uint32_t Y[4] = {r[2 * pp + 1].x, r[2 * pp + 1].y, r[2 * pp + 1].z, r[2 * pp + 1].w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    w[k][wre] = (X[k] & 0xffffu) | (Y[k] << 16);
                    w[k][wim] = (X[k] >> 16) | (Y[k] & 0xffff0000u);
                }
            }
        } else {
            // frame f: (re, im) of the four channels in eight dwords
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const uint4 lo = *reinterpret_cast<const uint4 *>(src + f * FB);
                const uint4 hi = *reinterpret_cast<const uint4 *>(src + f * FB + 16);
                w[0][f] = lo.x; w[0][4 + f] = lo.y;
                w[1][f] = lo.z; w[1][4 + f] = lo.w;
                w[2][f] = hi.x; w[2][4 + f] = hi.y;
                w[3][f] = hi.z; w[3][4 + f] = hi.w;
            }
        }
        uint8_t *dst = a.chan + (((int64_t)(c0 + 4 * q) * a.NG + a.grp0 + g) * a.n_in + n0 + nl) * kRowBytes;
        const int64_t cstep = a.NG * a.n_in * kRowBytes;   // bytes between channels
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint4 *row = reinterpret_cast<uint4 *>(dst + k * cstep);
            row[0] = make_uint4(w[k][0], w[k][1], w[k][2], w[k][3]);
            row[1] = make_uint4(w[k][4], w[k][5], w[k][6], w[k][7]);
        }
    }
}

template <int XP>
hipError_t launch_fft_xp(const FArgs &a, bool stats, int grid, hipStream_t s) {
    if (stats) hipLaunchKernelGGL((fft6400_kernel<XP, true, false>), dim3((unsigned)grid), dim3(kT), 0, s, a);
    else if (a.dl) hipLaunchKernelGGL((fft6400_kernel<XP, false, true>), dim3((unsigned)grid), dim3(kT), 0, s, a);
    else hipLaunchKernelGGL((fft6400_kernel<XP, false, false>), dim3((unsigned)grid), dim3(kT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int fft6400_grid(int n_in, int64_t nframes, bool stats) {
    const int64_t items = (int64_t)n_in * nframes;
    // main pass: two rounds of the resident workgroups (two per CU, 256 CUs), so a
    // workgroup loads its twiddles once for tens of frames; statistics pass: one
    // round, so that the partial rows (6,401 doubles each) stay few
    const int64_t cap = stats ? kStatsMaxWG / 2 : 1024;
    return (int)(items < cap ? items : cap);
}

int fft6400_lds_bytes() { return kN1 * kPitch * 8; }

hipError_t launch_fft6400(int xprec, const FArgs &a, hipStream_t s) {
    const bool stats = a.stats_mode != 0;
    const int grid = fft6400_grid(a.n_in, a.nframes, stats);
    if (grid < 1) return hipSuccess;
    switch (xprec) {
        case MWAX_X_INT8: return launch_fft_xp<MWAX_X_INT8>(a, stats, grid, s);
        case MWAX_X_FP16: return launch_fft_xp<MWAX_X_FP16>(a, stats, grid, s);
        case MWAX_X_FP32: return launch_fft_xp<MWAX_X_FP32>(a, stats, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_corner_turn(int esize, const CornerArgs &a, hipStream_t s) {
    const int64_t G = 16 / esize;
    const int64_t ngrp = (a.nframes + G - 1) / G;
    if (ngrp < 1) return hipSuccess;
    if (a.L % kCtChannels != 0 || ngrp > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)ngrp, (unsigned)(a.L / kCtChannels), (unsigned)((a.n_in + kCtInputs - 1) / kCtInputs));
    switch (esize) {
        case 1: hipLaunchKernelGGL(corner_turn_kernel<1>, grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(corner_turn_kernel<2>, grid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(corner_turn_kernel<4>, grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mwax
