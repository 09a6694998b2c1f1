// F-engine of the FX correlator (Morrison et al. 2023, Sec. 2.5 and 2.5.1):
// per input and per contiguous frame of L complex int8 samples, an
// unnormalised forward FFT in FP32, channels re-ordered so DC sits at
// c = L/2 (centre-symmetric channels, Sec. 2.6), then requantised (INT8 /
// binary16) or kept (FP32) and transposed through LDS into the channel-major
// layout the X-engine reads (the transpose of Sec. 2.5.1).
//
// One workgroup owns R inputs x G consecutive frames of one integration
// segment = one 32-byte row group per (channel, input).  The raw int8 frames
// are staged in LDS with coalesced 16-byte loads; each FFT is computed by a
// group of L2 lanes holding L1 = L / L2 points each:
//   X[k1 + L1 k2] = sum_r W_L2^(r k2) W_L^(r k1) sum_n1 x[r + L2 n1] W_L1^(n1 k1)
// (a two-pass Cooley-Tukey split): pass 1 in registers per lane, twiddle,
// exchange of the L1 x L2 block through LDS, pass 2 in registers.  The
// quantised outputs are written to an LDS image of the workgroup's output rows,
// which is then stored with coalesced 16-byte writes.
#include "mwax_internal.h"

namespace mwax {
namespace {

template <int L>
struct FftShape {
    static constexpr int L2 = L <= 16 ? 1 : (L == 32 ? 4 : (L <= 128 ? 8 : (L <= 512 ? 16 : 32)));
    static constexpr int L1 = L / L2;
    static constexpr int U = (L2 > 1) ? L1 / L2 : 1;
};

template <int N>
__host__ __device__ constexpr int ilog2c() {
    int l = 0;
    while ((1 << l) < N) ++l;
    return l;
}

template <int N>
__device__ constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 1; b < N; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// b * W_N^e with W_N^e read from the W_L table at index e * TS (TS = L / N).
// e = 0 and e = N/4 are exact (1 and -i).
template <int N, int TS>
__device__ __forceinline__ float2 tw_mul(float2 b, int e, const float2 *__restrict__ tw) {
    if (e == 0) return b;
    if (4 * e == N) return make_float2(b.y, -b.x);
    const float2 w = tw[e * TS];
    return make_float2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
}

// In-register radix-2 decimation-in-time DFT of N points, natural order in and out.
template <int N, int TS>
__device__ __forceinline__ void dft_regs(float2 *v, const float2 *__restrict__ tw) {
    if constexpr (N > 1) {
        float2 t[N];
#pragma unroll
        for (int i = 0; i < N; ++i) t[i] = v[bitrev<N>(i)];
#pragma unroll
        for (int s = 0; s < ilog2c<N>(); ++s) {
            const int h = 1 << s;
#pragma unroll
            for (int base = 0; base < N; base += 2 * h) {
#pragma unroll
                for (int j = 0; j < h; ++j) {
                    const float2 b = tw_mul<N, TS>(t[base + j + h], j * (N / (2 * h)), tw);
                    const float2 a = t[base + j];
                    t[base + j] = make_float2(a.x + b.x, a.y + b.y);
                    t[base + j + h] = make_float2(a.x - b.x, a.y - b.y);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = t[i];
    }
}

template <int XP>
struct PrecTraits;
template <>
struct PrecTraits<MWAX_X_INT8> { static constexpr int G = 16, ES = 1; };
template <>
struct PrecTraits<MWAX_X_FP16> { static constexpr int G = 8, ES = 2; };
template <>
struct PrecTraits<MWAX_X_FP32> { static constexpr int G = 4, ES = 4; };

// Channel of output slot i of lane r (see the kernel comment): bin
// k = (r U + u) + L1 k2 with i = u L2 + k2, channel (k + L/2) mod L.
template <int L>
__device__ __forceinline__ int chan_of(int r, int i) {
    using SH = FftShape<L>;
    int k;
    if constexpr (SH::L2 > 1) k = (r * SH::U + i / SH::L2) + SH::L1 * (i % SH::L2);
    else k = i;
    return (k + L / 2) & (L - 1);
}

// Requantisation rule of the INT8 X-engine: q = clamp(rne(x), -127, 127).
__device__ __forceinline__ int8_t quant8(float x) {
    return (int8_t)(int)fminf(fmaxf(rintf(x), -127.0f), 127.0f);
}

template <int XP>
__device__ __forceinline__ void put_out(uint8_t *row, int f, float2 X, float sc) {
    if constexpr (XP == MWAX_X_INT8) {
        row[f] = (uint8_t)quant8(X.x * sc);
        row[16 + f] = (uint8_t)quant8(X.y * sc);
    } else if constexpr (XP == MWAX_X_FP16) {
        *reinterpret_cast<_Float16 *>(row + 2 * f) = (_Float16)(X.x * sc);
        *reinterpret_cast<_Float16 *>(row + 16 + 2 * f) = (_Float16)(X.y * sc);
    } else {
        *reinterpret_cast<float *>(row + 4 * f) = X.x;
        *reinterpret_cast<float *>(row + 16 + 4 * f) = X.y;
    }
}

constexpr int kThreads = 256;

template <int L>
__host__ __device__ constexpr int ex_group_pitch() {  // float2 units per FFT group
    return FftShape<L>::L1 * (FftShape<L>::L2 + 1) + 8;
}

template <int L, int XP, bool STATS>
__global__ __launch_bounds__(kThreads) void fengine_kernel(FArgs a) {
    using SH = FftShape<L>;
    constexpr int L1 = SH::L1, L2 = SH::L2, U = SH::U;
    constexpr int G = PrecTraits<XP>::G;
    constexpr int GPW = 64 / L2;            // FFTs per wave per iteration
    constexpr int FPI = 4 * GPW;            // FFTs per workgroup per iteration
    constexpr int EXK = L2 + 1;             // exchange: float2 pitch of a k1 row
    constexpr int EXG = ex_group_pitch<L>();
    constexpr int SP = 2 * L + 16;          // staged frame pitch (bytes)
    extern __shared__ __align__(16) uint8_t smem[];

    const int R = a.R;
    const int CP = R * kRowBytes + 16;      // output image: bytes per channel
    uint8_t *outbuf = smem;
    uint8_t *stage = smem + (STATS ? 0 : L * CP);
    float2 *ex = reinterpret_cast<float2 *>(stage + (L2 > 1 ? R * G * SP : 0));

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gi = lane / L2, r = lane % L2;
    const int nblk = (a.n_in + R - 1) / R;
    const int items = a.ngrp * nblk;
    const int nfft = R * G;

    // Per-lane constants.  Output slot i of a lane (i = u * L2 + k2 for the
    // two-pass split) holds FFT bin k = (r U + u) + L1 k2, channel (k + L/2) mod L.
    constexpr bool kTwReg = L1 <= 16;       // keep the inter-pass twiddles in registers
    constexpr bool kScReg = L1 <= 16;       // keep the INT8 scales in registers
    float2 twr[kTwReg ? L1 : 1];
    float sc[kScReg ? L1 : 1];
#pragma unroll
    for (int i = 0; i < L1; ++i) {
        if constexpr (L2 > 1 && kTwReg) twr[i] = a.tw[(r * i) % L];
        if constexpr (kScReg) {
            if constexpr (XP == MWAX_X_INT8 && !STATS) sc[i] = a.inv_s[chan_of<L>(r, i)];
            else if constexpr (XP == MWAX_X_FP16) sc[i] = a.half_scale;
            else sc[i] = 1.0f;
        }
    }
    float acc[STATS ? L1 : 1];
#pragma unroll
    for (int i = 0; i < (STATS ? L1 : 1); ++i) acc[i] = 0.0f;

    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int gsel = item / nblk;
        const int n0 = (item - gsel * nblk) * R;
        const int nrows = min(R, a.n_in - n0);
        const int64_t lf0 = (int64_t)gsel * G;
        const int fvalid = (int)min((int64_t)G, a.nframes - lf0);
        const int64_t src_frame = a.frame0 + lf0;

        __syncthreads();  // LDS of the previous item fully consumed
        if constexpr (L2 > 1) {
            constexpr int UPF = 2 * L / 16;
            const int units = R * G * UPF;
            for (int u = tid; u < units; u += kThreads) {
                const int nl = u / (G * UPF);
                const int rem = u - nl * G * UPF;
                const int f = rem / UPF, o = rem - f * UPF;
                uint4 val = make_uint4(0, 0, 0, 0);
                if (nl < nrows && f < fvalid)
                    val = *reinterpret_cast<const uint4 *>(
                        a.volts + ((int64_t)(n0 + nl) * a.ld + (src_frame + f) * L) * 2 + o * 16);
                *reinterpret_cast<uint4 *>(stage + (nl * G + f) * SP + o * 16) = val;
            }
            __syncthreads();
        }

        for (int it = 0; it < nfft; it += FPI) {
            const int fi = it + wave * GPW + gi;
            const bool live = fi < nfft;
            const int x = live ? fi / R : 0;
            const int nl = live ? fi - x * R : 0;
            const int f = (x & 3) * (G / 4) + (x >> 2);   // frames 4 apart share an instruction
            uint8_t *orow = outbuf + nl * kRowBytes;

            // consume output slot i (bin of this lane) with value X
            auto emit = [&](int i, float2 X) {
                if (!live) return;
                if constexpr (STATS) {
                    acc[i] += X.x * X.x + X.y * X.y;
                } else {
                    const int c = chan_of<L>(r, i);
                    float s;
                    if constexpr (kScReg) s = sc[i];
                    else if constexpr (XP == MWAX_X_INT8) s = a.inv_s[c];
                    else if constexpr (XP == MWAX_X_FP16) s = a.half_scale;
                    else s = 1.0f;
                    put_out<XP>(orow + c * CP, f, X, s);
                }
            };

            float2 v[L1];
            if constexpr (L2 == 1) {
                // whole frame per lane, straight from global memory
                if (live && nl < nrows && f < fvalid) {
                    const int8_t *src = a.volts + ((int64_t)(n0 + nl) * a.ld + (src_frame + f) * L) * 2;
                    if constexpr (L == 1) {
                        const char2 s2 = *reinterpret_cast<const char2 *>(src);
                        v[0] = make_float2((float)s2.x, (float)s2.y);
                    } else {
#pragma unroll
                        for (int q = 0; q < L / 2; ++q) {
                            const char4 s4 = *reinterpret_cast<const char4 *>(src + 4 * q);
                            v[2 * q] = make_float2((float)s4.x, (float)s4.y);
                            v[2 * q + 1] = make_float2((float)s4.z, (float)s4.w);
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < L; ++q) v[q] = make_float2(0.0f, 0.0f);
                }
                dft_regs<L1, 1>(v, a.tw);
#pragma unroll
                for (int k = 0; k < L1; ++k) emit(k, v[k]);
            } else {
                const uint8_t *fr = stage + (nl * G + f) * SP;
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) {
                    const char2 s2 = *reinterpret_cast<const char2 *>(fr + 2 * (r + L2 * n1));
                    v[n1] = make_float2((float)s2.x, (float)s2.y);
                }
                dft_regs<L1, L / L1>(v, a.tw);
#pragma unroll
                for (int k1 = 0; k1 < L1; ++k1) {
                    float2 w;
                    if constexpr (kTwReg) w = twr[k1];
                    else w = a.tw[(r * k1) % L];
                    v[k1] = make_float2(v[k1].x * w.x - v[k1].y * w.y, v[k1].x * w.y + v[k1].y * w.x);
                }
                float2 *eg = ex + (wave * GPW + gi) * EXG;
#pragma unroll
                for (int k1 = 0; k1 < L1; ++k1) eg[k1 * EXK + r] = v[k1];
                wave_sync();
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    float2 w[L2];
#pragma unroll
                    for (int r2 = 0; r2 < L2; ++r2) w[r2] = eg[(r * U + u) * EXK + r2];
                    dft_regs<L2, L / L2>(w, a.tw);
#pragma unroll
                    for (int k2 = 0; k2 < L2; ++k2) emit(u * L2 + k2, w[k2]);
                }
                wave_sync();
            }
        }

        if constexpr (!STATS) {
            __syncthreads();
            // store the image: per channel, nrows rows of 32 bytes, 16 bytes per thread
            const int units = L * nrows * 2;
            for (int u = tid; u < units; u += kThreads) {
                const int c = u / (nrows * 2);
                const int rem = u - c * nrows * 2;
                const int nl = rem >> 1, h = rem & 1;
                const uint4 val = *reinterpret_cast<const uint4 *>(outbuf + c * CP + nl * kRowBytes + h * 16);
                uint8_t *dst = a.chan + ((((int64_t)c * a.NG + a.grp0 + gsel) * a.n_in) + n0 + nl) * kRowBytes + h * 16;
                *reinterpret_cast<uint4 *>(dst) = val;
            }
        }
    }

    if constexpr (STATS) {
        // Deterministic reduction of the per-lane channel sums: lanes with the same r
        // hold the same channel set; sum them in a fixed order.
        __syncthreads();
        float *red = reinterpret_cast<float *>(smem);   // [kThreads / L2 slots][L2][L1]
        const int slot = wave * GPW + gi;
#pragma unroll
        for (int i = 0; i < L1; ++i) red[(slot * L2 + r) * L1 + i] = acc[i];
        __syncthreads();
        constexpr int NSLOT = kThreads / L2;
        for (int t = tid; t < L; t += kThreads) {
            const int rr = t / L1, i = t - rr * L1;
            double s = 0.0;
            for (int sl = 0; sl < NSLOT; ++sl) s += (double)red[(sl * L2 + rr) * L1 + i];
            a.stats[(int64_t)blockIdx.x * L + chan_of<L>(rr, i)] = s;
        }
    }
}

template <int L, int XP>
hipError_t launch_L(const FArgs &a, hipStream_t s) {
    const bool stats = a.stats_mode != 0;
    const int lds = fengine_lds_bytes(L, XP, a.R, stats);
    const int grid = fengine_grid(a.n_in, a.R, a.ngrp, stats);
    if (grid < 1) return hipSuccess;
    // allow dynamic LDS beyond the default limit (once per instantiation)
    static bool attr_done[2] = {false, false};
    if (!attr_done[stats]) {
        const void *fn = stats ? reinterpret_cast<const void *>(&fengine_kernel<L, XP, true>)
                               : reinterpret_cast<const void *>(&fengine_kernel<L, XP, false>);
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
        attr_done[stats] = true;
    }
    if (stats)
        hipLaunchKernelGGL((fengine_kernel<L, XP, true>), dim3((unsigned)grid), dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL((fengine_kernel<L, XP, false>), dim3((unsigned)grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
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

int l2_of(int L) {
    return L <= 16 ? 1 : (L == 32 ? 4 : (L <= 128 ? 8 : (L <= 512 ? 16 : 32)));
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

__global__ void calib_finish_kernel(const double *stats, int nwg, int L, double count, float *scales) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= L) return;
    double t = 0.0;
    for (int w = 0; w < nwg; ++w) t += stats[(int64_t)w * L + c];
    const double var = t / (2.0 * count);
    float s = 1.0f, inv = 1.0f;
    if (var > 0.0) {
        const double sd = sqrt(var);
        s = (float)(5.0 * sd / 127.0);
        inv = (float)(127.0 / (5.0 * sd));
    }
    scales[c] = s;
    scales[L + c] = inv;
}

__global__ void copy_scales_kernel(const float *src, float *dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
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
            row[f] = re;
            row[a.G + f] = im;
        } else {
            cv[0] = row[f];
            cv[1] = row[a.G + f];
        }
    }
}

}  // namespace

int fengine_pick_R(int L, int xprec, int n_in, int lds_limit) {
    const int G = group_of(xprec);
    const int L2 = l2_of(L);
    // at least one FFT per lane per iteration, and about 8 KiB of output image
    int R = (kThreads + G * L2 - 1) / (G * L2);
    while (R * L * kRowBytes < 8192 && R < 64) R *= 2;
    if (R > n_in) R = n_in;
    if (R < 1) R = 1;
    while (R > 1 && (fengine_lds_bytes(L, xprec, R, false) > lds_limit ||
                     fengine_lds_bytes(L, xprec, R, true) > lds_limit))
        R /= 2;
    return R;
}

int fengine_grid(int n_in, int R, int ngrp, bool stats) {
    const int64_t items = (int64_t)ngrp * ((n_in + R - 1) / R);
    // stats mode writes one partial row per workgroup: keep that buffer small
    const int64_t cap = stats ? kStatsMaxWG : 65536;
    return (int)(items < cap ? items : cap);
}

int fengine_lds_bytes(int L, int xprec, int R, bool stats) {
    const int G = group_of(xprec);
    const int L2 = l2_of(L);
    const int L1 = L / L2;
    const int CP = R * kRowBytes + 16;
    int bytes = stats ? 0 : L * CP;
    if (L2 > 1) {
        bytes += R * G * (2 * L + 16);
        bytes += (kThreads / L2) * (L1 * (L2 + 1) + 8) * 8;
    }
    if (stats) {
        const int red = kThreads * L1 * 4;
        if (bytes < red) bytes = red;
    }
    return bytes;
}

hipError_t launch_fengine(int L, int xprec, const FArgs &a, hipStream_t s) {
    switch (xprec) {
        case MWAX_X_INT8: return launch_xp<MWAX_X_INT8>(L, a, s);
        case MWAX_X_FP16: return launch_xp<MWAX_X_FP16>(L, a, s);
        case MWAX_X_FP32: return launch_xp<MWAX_X_FP32>(L, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_twiddles(float2 *tw, int L, hipStream_t s) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
    return hipGetLastError();
}

hipError_t launch_calib_finish(const double *stats, int nwg, int L, double count, float *scales,
                               hipStream_t s) {
    hipLaunchKernelGGL(calib_finish_kernel, dim3((L + 255) / 256), dim3(256), 0, s, stats, nwg, L,
                       count, scales);
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
