// Tied-array beamforming (Sec. 4.4) from the channelised voltages a plan holds
// in its channel-major buffer (the F-engine output the X-engine reads).
//
// Coherent beams: per channel c, the beams of a block are the complex product
// B_c = W_c X_c (W_c: [beams][inputs] weights that phase the signal paths up
// for each pointing; X_c: [inputs][spectra]).  It runs on the FP32 matrix
// cores as two real products with K = (input, re/im):
//   Re B = [Re W, -Im W] . [Re X; Im X],   Im B = [Im W, Re W] . [Re X; Im X]
// with v_mfma_f32_32x32x2_f32: lanes 0..31 carry the re/re and lanes 32..63 the
// im parts of one input per instruction.  A workgroup owns 64 beams x 64
// spectra of one channel (four waves of 32 x 32); inputs are staged through LDS
// 32 at a time, the int8 codes / binary16 values decoded to FP32 there.  The
// channel's scale (INT8 s_c, FP16 2^e) is common to all inputs of the channel
// and is applied to the sums.
//
// Incoherent beam: the detected power of the inputs of each polarisation,
// summed over t_avg spectra and f_avg channels (FP64 sums, fixed reduction
// order).
#include "mwax_internal.h"

namespace mwax {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kKC = 32;     // inputs per LDS stage
constexpr int kWP = kKC + 1;   // float2 pitch of a beam's weights in LDS

// Spectrum t (0 .. G-1) of a 32-byte row, decoded to FP32 (before the scale).
template <int ES>
__device__ __forceinline__ float2 row_value(const uint8_t *row, int t) {
    const int re = row_re_off(t, ES), im = re + row_im_gap(ES);
    if constexpr (ES == 1) return make_float2((float)(int8_t)row[re], (float)(int8_t)row[im]);
    else if constexpr (ES == 2)
        return make_float2((float)__builtin_bit_cast(_Float16, *reinterpret_cast<const uint16_t *>(row + re)),
                           (float)__builtin_bit_cast(_Float16, *reinterpret_cast<const uint16_t *>(row + im)));
    else return make_float2(*reinterpret_cast<const float *>(row + re), *reinterpret_cast<const float *>(row + im));
}

// WB waves along the beams, 4 / WB along the spectra: a tile of 32 WB beams x
// 128 / WB spectra (WB = 1 when a launch has at most 32 beams, so that no wave
// multiplies empty beams).
template <int ES, int WB>
__global__ __launch_bounds__(256) void beamform_kernel(BeamArgs a) {
    constexpr int G = 16 / ES;
    constexpr int kBT = 32 * WB, kMT = 128 / WB;
    // one LDS block: the stage (weights [beam][input], voltages [input][spectrum])
    // and, after the K loop, the output tile [spectrum][beam] (pitch kBT + 1)
    constexpr int kStage = kBT * kWP + kKC * kMT, kOut = kMT * (kBT + 1);
    __shared__ float2 lds[kStage > kOut ? kStage : kOut];
    float2 *ws = lds, *xs = lds + kBT * kWP;
    const int c = blockIdx.z;
    const int m0 = blockIdx.x * kMT, b0 = blockIdx.y * kBT;
    const int tid = threadIdx.x, lane = tid & 63, half = lane >> 5, l32 = lane & 31;
    const int wave = tid >> 6, wb = wave / (4 / WB), wm = wave % (4 / WB);
    v16f acc_r, acc_i;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc_r[r] = acc_i[r] = 0.0f;

    for (int n0 = 0; n0 < a.n_in; n0 += kKC) {
        __syncthreads();   // the previous stage has been read
        // weights: thread -> beam tid / 4, inputs (tid % 4) * 8 .. + 7 (WB = 2), or
        // beam tid / 8, inputs (tid % 8) * 4 .. + 3 (WB = 1)
        {
            constexpr int PER = kBT * kKC / 256;
            const int bl = tid / (kKC / PER), nl0 = (tid % (kKC / PER)) * PER;
            const int b = b0 + bl;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int n = n0 + nl0 + e;
                float2 w = make_float2(0.0f, 0.0f);
                if (b < a.nb && n < a.n_in) w = a.w[((int64_t)c * a.nb + b) * a.n_in + n];
                ws[bl * kWP + nl0 + e] = w;
            }
        }
        // voltages: the kMT spectra of the tile for kKC inputs, decoded
        for (int u = tid; u < kKC * (kMT / G); u += 256) {
            const int nl = u % kKC, gl = u / kKC;
            const int n = n0 + nl;
            const int64_t tloc = (int64_t)m0 + gl * G;          // first spectrum of this row group
            float2 v[G];
            if (n < a.n_in && tloc < a.nframes) {
                const uint8_t *row = a.chan + (((int64_t)c * a.NG + a.grp0 + tloc / G) * a.n_in + n) * kRowBytes;
                uint4 h0 = *reinterpret_cast<const uint4 *>(row), h1 = *reinterpret_cast<const uint4 *>(row + 16);
                uint8_t buf[kRowBytes];
                __builtin_memcpy(buf, &h0, 16);
                __builtin_memcpy(buf + 16, &h1, 16);
#pragma unroll
                for (int t = 0; t < G; ++t) v[t] = row_value<ES>(buf, t);
            } else {
#pragma unroll
                for (int t = 0; t < G; ++t) v[t] = make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int t = 0; t < G; ++t) xs[nl * kMT + gl * G + t] = v[t];
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < kKC; ++k) {
            const float2 w = ws[(wb * 32 + l32) * kWP + k];
            const float2 x = xs[k * kMT + wm * 32 + l32];
            const float ar = half ? -w.y : w.x, ai = half ? w.x : w.y, bx = half ? x.y : x.x;
            acc_r = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bx, acc_r, 0, 0, 0);
            acc_i = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bx, acc_i, 0, 0, 0);
        }
    }

    // out[m][c][b]: stage the tile [spectrum][beam] through LDS, store rows of beams
    __syncthreads();
    float2 *os = lds;
    const float sc = a.scales ? a.scales[c] * a.post : a.post;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = (r >> 2) * 8 + half * 4 + (r & 3);   // beam within the wave's block
        const int j = l32;                                 // spectrum within the wave's block
        os[(wm * 32 + j) * (kBT + 1) + wb * 32 + i] = make_float2(acc_r[r] * sc, acc_i[r] * sc);
    }
    __syncthreads();
    for (int u = tid; u < kMT * kBT; u += 256) {
        const int ml = u / kBT, bl = u % kBT;
        const int64_t t = (int64_t)m0 + ml;
        if (t < a.nframes && b0 + bl < a.nb)
            a.out[((a.m0 + t) * a.L + c) * (int64_t)a.nb + b0 + bl] = os[ml * (kBT + 1) + bl];
    }
}

// Power of the frames [f0, f1) of one 32-byte row (G frames of one input):
// sum over those frames of re^2 + im^2.  INT8: exact, with signed 4-byte dot
// products on the bytes kept by a per-dword mask (a dword holds the re or the
// im parts of 4 frames); binary16 / FP32: FP64 sums of the exact squares.
template <int ES>
__device__ __forceinline__ double row_power(uint4 h0, uint4 h1, int f0, int f1) {
    const uint32_t w[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
    if constexpr (ES == 1) {
        // dword k: frames (k >> 2) * 8 + (k & 1) * 4 + 0 .. 3, re (k & 2 == 0) or im
        int acc = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int fb = (k >> 2) * 8 + (k & 1) * 4;
            uint32_t m = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) m |= (fb + e >= f0 && fb + e < f1) ? (0xffu << (8 * e)) : 0u;
            const int v = (int)(w[k] & m);
            acc = __builtin_amdgcn_sdot4(v, v, acc, false);
        }
        return (double)acc;
    } else if constexpr (ES == 2) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t >= f0 && t < f1) {
                const float2 v = row_value<2>(reinterpret_cast<const uint8_t *>(w), t);
                acc += (double)v.x * v.x + (double)v.y * v.y;
            }
        }
        return acc;
    } else {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= f0 && t < f1) {
                const float2 v = row_value<4>(reinterpret_cast<const uint8_t *>(w), t);
                acc += (double)v.x * v.x + (double)v.y * v.y;
            }
        }
        return acc;
    }
}

// One workgroup per output bin (o, j): channels o f_avg .. and spectra j t_avg
// .. of the block.  The bin's spectra are walked segment by segment and row
// group by row group; for each (row group, channel) the threads read whole
// 32-byte rows of consecutive inputs (thread tid takes inputs tid, tid + 256,
// .., all of one polarisation, so a wave reads 2 KB contiguous) and sum the
// power of the frames inside the bin; each (row group, channel) sum is scaled
// by the square of its channel's scale (INT8 s_c of the segment; binary16
// 2^e) and added to the thread's FP64 total.  The totals are reduced per
// polarisation in a fixed order.
template <int ES>
__global__ __launch_bounds__(256) void incoherent_kernel(IncohArgs a) {
    constexpr int G = 16 / ES;
    __shared__ double red[256];
    const int o = blockIdx.x;
    const int64_t j = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t m_lo = j * a.t_avg, m_hi = m_lo + a.t_avg;   // block spectra of the bin
    const int64_t m_end = a.n_j * a.t_avg;                       // block spectra
    const int64_t rstride = (int64_t)a.n_in * kRowBytes;         // bytes between row groups
    double acc = 0.0;
    for (int s = 0; s < a.nseg; ++s) {
        const int64_t s0 = a.seg_m0[s], s1 = s + 1 < a.nseg ? a.seg_m0[s + 1] : m_end;
        const int64_t lo = m_lo > s0 ? m_lo : s0, hi = m_hi < s1 ? m_hi : s1;
        if (lo >= hi) continue;
        const int64_t t0 = lo - s0, t1 = hi - s0;                 // spectra of the segment
        for (int64_t g = t0 / G; g * G < t1; ++g) {
            const int f0 = (int)(t0 > g * G ? t0 - g * G : 0), f1 = (int)(t1 - g * G < G ? t1 - g * G : G);
            for (int ci = 0; ci < a.f_avg; ++ci) {
                const int c = o * a.f_avg + ci;
                const uint8_t *rows = a.chan + ((int64_t)c * a.NG + a.seg_grp0[s] + g) * rstride;
                double pw = 0.0;
                for (int n = tid; n < a.n_in; n += 256) {
                    const uint4 *r = reinterpret_cast<const uint4 *>(rows + (int64_t)n * kRowBytes);
                    pw += row_power<ES>(r[0], r[1], f0, f1);
                }
                const double f = a.seg_scales[s] ? (double)a.seg_scales[s][c] * a.post : (double)a.post;
                acc += pw * f * f;
            }
        }
    }
    // inputs tid + 256 k have the polarisation tid & 1: even strides keep it
    red[tid] = acc;
    __syncthreads();
    for (int h = 128; h > 1; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid < 2) a.out[(j * a.n_o + o) * 2 + tid] = (float)red[tid];
}

}  // namespace

template <int WB>
hipError_t launch_beamform_wb(int esize, const BeamArgs &a, hipStream_t s) {
    constexpr int kBT = 32 * WB, kMT = 128 / WB;
    const dim3 grid((unsigned)((a.nframes + kMT - 1) / kMT), (unsigned)((a.nb + kBT - 1) / kBT), (unsigned)a.L);
    switch (esize) {
        case 1: hipLaunchKernelGGL((beamform_kernel<1, WB>), grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL((beamform_kernel<2, WB>), grid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL((beamform_kernel<4, WB>), grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_beamform(int esize, const BeamArgs &a, hipStream_t s) {
    if (a.nframes <= 0 || a.nb <= 0) return hipSuccess;
    return a.nb <= 32 ? launch_beamform_wb<1>(esize, a, s) : launch_beamform_wb<2>(esize, a, s);
}

hipError_t launch_incoherent(int esize, const IncohArgs &a, hipStream_t s) {
    if (a.n_o <= 0 || a.n_j <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.n_o, (unsigned)a.n_j);
    switch (esize) {
        case 1: hipLaunchKernelGGL(incoherent_kernel<1>, grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(incoherent_kernel<2>, grid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(incoherent_kernel<4>, grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mwax
