// X-engine of the FX correlator (Morrison et al. 2023, Sec. 2.5.2): for each
// fine channel c and every input pair n1 >= n2 (autos included),
//   V[c][n1,n2] += sum_m X_n1[m,c] conj(X_n2[m,c]),
// accumulated into per-integration device integrators (Sec. 2.5.2, time
// integration) in the packed lower-triangle order p = n1(n1+1)/2 + n2.
//
// The complex Hermitian rank-k update is run as two real GEMMs over the
// channel-major rows [re_0..re_{G-1} | im_0..im_{G-1}] of each input:
//   Re V[n1,n2] = sum (re1 re2 + im1 im2) = A_n1 . A_n2,   A = [re | im]
//   Im V[n1,n2] = sum (im1 re2 - re1 im2) = A_n1 . B_n2,   B = [-im | re]
// so every complex multiply-accumulate is four real ones and nothing is
// wasted on the real expansion.  B is built once per workgroup while staging
// (negating the imaginary half), so the matrix cores read A, A and B straight
// from LDS.  Work is split into 128 x 128 tiles of the lower triangle; waves
// skip 32 x 32 blocks that lie wholly above the diagonal or past the last
// input.
//
//   INT8: v_mfma_i32_32x32x32_i8, int32 partials flushed to int64 integrators
//         at most every 32768 spectra (|partial| <= 2 * 127^2 * 32768 < 2^31).
//   FP16: v_mfma_f32_32x32x16_f16, FP32 partials flushed to FP64 integrators.
//   FP32: vector ALUs, 4 x 8 complex outputs per thread, two-level FP32
//         partials (see xengine_f32) flushed to FP64 integrators every 2048
//         spectra.
#include "mwax_internal.h"

namespace mwax {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kTile = 128;          // tile edge in inputs
constexpr int kThreads = 256;       // 4 waves
constexpr int kKG = 4;              // row groups per LDS stage

// Lower-triangle tile index t -> (I, J), I >= J, t = I(I+1)/2 + J.
__device__ __forceinline__ void tile_ij(int t, int &I, int &J) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// Workgroups are handed to the 8 XCDs round-robin.  Renumber them so the
// workgroups one XCD receives carry consecutive logical indices: the tiles of a
// channel then share that XCD's L2 for the input panels they all read.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
    const int full = nb & ~7;
    if (b >= full) return b;
    return (b & 7) * (full >> 3) + (b >> 3);
}

// Per-byte two's-complement negation of four int8 values in [-127, 127].
__device__ __forceinline__ uint32_t neg_i8x4(uint32_t x) {
    const uint32_t nx = ~x;
    return ((nx & 0x7F7F7F7Fu) + 0x01010101u) ^ (nx & 0x80808080u);
}

template <int XP>
__device__ __forceinline__ uint4 negate16(uint4 v) {
    if constexpr (XP == MWAX_X_INT8) {
        return make_uint4(neg_i8x4(v.x), neg_i8x4(v.y), neg_i8x4(v.z), neg_i8x4(v.w));
    } else {
        return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
    }
}

template <int XP>
struct MfmaT;
template <>
struct MfmaT<MWAX_X_INT8> {
    using acc_t = v16i;
    static constexpr int G = 16;                 // spectra per row group
    static constexpr int kFlushGroups = 2048;    // 32768 spectra
    __device__ static acc_t mma(uint4 a, uint4 b, acc_t c) {
        v4i av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, c, 0, 0, 0);
    }
};
template <>
struct MfmaT<MWAX_X_FP16> {
    using acc_t = v16f;
    static constexpr int G = 8;
    static constexpr int kFlushGroups = 1 << 30;  // only at the end of the segment
    __device__ static acc_t mma(uint4 a, uint4 b, acc_t c) {
        v8h av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, c, 0, 0, 0);
    }
};

template <int XP>
__global__ __launch_bounds__(kThreads) void xengine_mfma(XArgs a) {
    using T = MfmaT<XP>;
    using acc_t = typename T::acc_t;
    // LDS: three panels, each [kKG][2 halves][128 rows][16 B]
    constexpr int kPanel = kKG * 2 * kTile * 16;
    __shared__ __align__(16) uint8_t lds[3 * kPanel];
    uint8_t *ldsA = lds, *ldsB = lds + kPanel, *ldsB2 = lds + 2 * kPanel;

    const int nb = gridDim.x;
    const int lin = xcd_logical(blockIdx.x, nb);
    const int c = lin / a.ntiles;
    int I, J;
    tile_ij(lin - c * a.ntiles, I, J);
    const int rowA0 = I * kTile, rowB0 = J * kTile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;

    // which 32 x 32 blocks this wave computes
    bool act[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb2 = 0; nb2 < 2; ++nb2) {
            const int RB = wr * 2 + mb, CB = wc * 2 + nb2;
            bool on = (rowA0 + RB * 32 < a.n_in) && (rowB0 + CB * 32 < a.n_in);
            if (I == J && RB < CB) on = false;
            act[mb][nb2] = on;
        }
    const bool any = act[0][0] || act[0][1] || act[1][0] || act[1][1];

    acc_t re[2][2], im[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb2 = 0; nb2 < 2; ++nb2) {
            re[mb][nb2] = acc_t{};
            im[mb][nb2] = acc_t{};
        }

    const uint8_t *base = a.chan + ((int64_t)c * a.NG + a.grp0) * (int64_t)a.n_in * kRowBytes;
    const int64_t gstride = (int64_t)a.n_in * kRowBytes;   // bytes between row groups

    // staging registers: kKG units of 16 B for each of the two panels
    uint4 ra[kKG], rb[kKG];
    auto load_stage = [&](int g0) {
#pragma unroll
        for (int k = 0; k < kKG; ++k) {
            const int row = tid >> 1, h = tid & 1;
            const bool gok = g0 + k < a.ngrp;
            ra[k] = make_uint4(0, 0, 0, 0);
            rb[k] = make_uint4(0, 0, 0, 0);
            if (gok && rowA0 + row < a.n_in)
                ra[k] = *reinterpret_cast<const uint4 *>(base + (g0 + k) * gstride + (int64_t)(rowA0 + row) * kRowBytes + h * 16);
            if (gok && rowB0 + row < a.n_in)
                rb[k] = *reinterpret_cast<const uint4 *>(base + (g0 + k) * gstride + (int64_t)(rowB0 + row) * kRowBytes + h * 16);
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int k = 0; k < kKG; ++k) {
            const int row = tid >> 1, h = tid & 1;
            const int off = ((k * 2 + h) * kTile + row) * 16;
            *reinterpret_cast<uint4 *>(ldsA + off) = ra[k];
            *reinterpret_cast<uint4 *>(ldsB + off) = rb[k];
            // B2 = [-im | re]: the re half goes to half 1, the negated im half to half 0
            const int off2 = ((k * 2 + (1 - h)) * kTile + row) * 16;
            *reinterpret_cast<uint4 *>(ldsB2 + off2) = h ? negate16<XP>(rb[k]) : rb[k];
        }
    };
    auto flush = [&]() {
        if (!any) return;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb2 = 0; nb2 < 2; ++nb2) {
                if (!act[mb][nb2]) continue;
                const int n2 = rowB0 + (wc * 2 + nb2) * 32 + l32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int n1 = rowA0 + (wr * 2 + mb) * 32 + (r >> 2) * 8 + half * 4 + (r & 3);
                    if (n1 < a.n_in && n2 <= n1) {
                        const int64_t p = (int64_t)n1 * (n1 + 1) / 2 + n2;
                        if constexpr (XP == MWAX_X_INT8) {
                            longlong2 *dst = reinterpret_cast<longlong2 *>(a.integ) + (int64_t)c * a.P + p;
                            longlong2 v = *dst;
                            v.x += re[mb][nb2][r];
                            v.y += im[mb][nb2][r];
                            *dst = v;
                        } else {
                            double2 *dst = reinterpret_cast<double2 *>(a.integ) + (int64_t)c * a.P + p;
                            double2 v = *dst;
                            v.x += (double)re[mb][nb2][r];
                            v.y += (double)im[mb][nb2][r];
                            *dst = v;
                        }
                    }
                }
                re[mb][nb2] = acc_t{};
                im[mb][nb2] = acc_t{};
            }
    };

    int since_flush = 0;
    load_stage(0);
    for (int g0 = 0; g0 < a.ngrp; g0 += kKG) {
        __syncthreads();
        store_stage();
        __syncthreads();
        if (g0 + kKG < a.ngrp) load_stage(g0 + kKG);
        if (any) {
#pragma unroll
            for (int k = 0; k < kKG; ++k) {
                uint4 fa[2], fb[2], fb2[2];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    fa[mb] = *reinterpret_cast<const uint4 *>(ldsA + ((k * 2 + half) * kTile + wr * 64 + mb * 32 + l32) * 16);
#pragma unroll
                for (int nb2 = 0; nb2 < 2; ++nb2) {
                    const int off = ((k * 2 + half) * kTile + wc * 64 + nb2 * 32 + l32) * 16;
                    fb[nb2] = *reinterpret_cast<const uint4 *>(ldsB + off);
                    fb2[nb2] = *reinterpret_cast<const uint4 *>(ldsB2 + off);
                }
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int nb2 = 0; nb2 < 2; ++nb2) {
                        // blocks of an active wave are all computed (a wave's time is set by
                        // its busiest sibling anyway); inactive ones are dropped at flush
                        re[mb][nb2] = T::mma(fa[mb], fb[nb2], re[mb][nb2]);
                        im[mb][nb2] = T::mma(fa[mb], fb2[nb2], im[mb][nb2]);
                    }
            }
        }
        since_flush += kKG;
        if (since_flush >= T::kFlushGroups) {
            flush();
            since_flush = 0;
        }
    }
    if (since_flush > 0) flush();
}

// ---------------------------------------------------------------------------
// FP32 X-engine on the vector ALUs.  512 threads, 4 x 8 complex outputs each.
//
// Two-level FP32 accumulation: each 16-spectrum stage is summed into an inner
// accumulator, which is then added to an outer one; the outer one is flushed
// to the FP64 integrator every 2048 spectra.  A single FP32 running sum is
// biased: in the channels whose bin is a multiple of L/4 the spectra of
// integer voltages are exact integers, their squares are 0 or 1 mod 4, and
// once the running sum passes 2^24 every addition rounds the same way.  The
// inner sums stay far below 2^24 (exact for those channels) and have evenly
// spread low bits, so the outer additions round without a bias.
// ---------------------------------------------------------------------------
constexpr int kF32Threads = 512;
constexpr int kF32FlushGroups = 512;   // 2048 spectra per FP32 outer partial

__global__ __launch_bounds__(kF32Threads) void xengine_f32(XArgs a) {
    constexpr int S = kKG * 4;   // spectra per stage
    __shared__ __align__(16) float sAr[S][kTile], sAi[S][kTile], sBr[S][kTile], sBi[S][kTile];

    const int nb = gridDim.x;
    const int lin = xcd_logical(blockIdx.x, nb);
    const int c = lin / a.ntiles;
    int I, J;
    tile_ij(lin - c * a.ntiles, I, J);
    const int rowA0 = I * kTile, rowB0 = J * kTile;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;        // rows ty*4 + i, cols tx*8 + j
    const bool active = !(I == J && tx * 8 > ty * 4 + 3) && (rowA0 + ty * 4 < a.n_in) &&
                        (rowB0 + tx * 8 < a.n_in);

    float inr[4][8], ini[4][8], outr[4][8], outi[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) inr[i][j] = ini[i][j] = outr[i][j] = outi[i][j] = 0.0f;

    const uint8_t *base = a.chan + ((int64_t)c * a.NG + a.grp0) * (int64_t)a.n_in * kRowBytes;
    const int64_t gstride = (int64_t)a.n_in * kRowBytes;

    auto flush = [&]() {
        if (!active) return;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n1 = rowA0 + ty * 4 + i;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int n2 = rowB0 + tx * 8 + j;
                if (n1 < a.n_in && n2 <= n1) {
                    double2 *dst = reinterpret_cast<double2 *>(a.integ) + (int64_t)c * a.P +
                                   (int64_t)n1 * (n1 + 1) / 2 + n2;
                    double2 v = *dst;
                    v.x += (double)outr[i][j];
                    v.y += (double)outi[i][j];
                    *dst = v;
                }
                outr[i][j] = outi[i][j] = 0.0f;
            }
        }
    };

    int since_flush = 0;
    for (int g0 = 0; g0 < a.ngrp; g0 += kKG) {
        __syncthreads();
        // stage kKG groups of both panels: 16-byte units, transposed to [spectrum][row]
        for (int u = tid; u < kKG * kTile * 2; u += kF32Threads) {
            const int k = u / (kTile * 2);
            const int row = (u >> 1) & (kTile - 1), h = u & 1;
            const bool gok = g0 + k < a.ngrp;
            float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
            if (gok && rowA0 + row < a.n_in)
                va = *reinterpret_cast<const float4 *>(base + (g0 + k) * gstride + (int64_t)(rowA0 + row) * kRowBytes + h * 16);
            if (gok && rowB0 + row < a.n_in)
                vb = *reinterpret_cast<const float4 *>(base + (g0 + k) * gstride + (int64_t)(rowB0 + row) * kRowBytes + h * 16);
            float (*da)[kTile] = h ? sAi : sAr;
            float (*db)[kTile] = h ? sBi : sBr;
            da[k * 4 + 0][row] = va.x; da[k * 4 + 1][row] = va.y; da[k * 4 + 2][row] = va.z; da[k * 4 + 3][row] = va.w;
            db[k * 4 + 0][row] = vb.x; db[k * 4 + 1][row] = vb.y; db[k * 4 + 2][row] = vb.z; db[k * 4 + 3][row] = vb.w;
        }
        __syncthreads();
        if (active) {
#pragma unroll 2
            for (int s = 0; s < S; ++s) {
                const float4 a0 = *reinterpret_cast<const float4 *>(&sAr[s][ty * 4]);
                const float4 a1 = *reinterpret_cast<const float4 *>(&sAi[s][ty * 4]);
                const float4 b0 = *reinterpret_cast<const float4 *>(&sBr[s][tx * 8]);
                const float4 b1 = *reinterpret_cast<const float4 *>(&sBr[s][tx * 8 + 4]);
                const float4 b2 = *reinterpret_cast<const float4 *>(&sBi[s][tx * 8]);
                const float4 b3 = *reinterpret_cast<const float4 *>(&sBi[s][tx * 8 + 4]);
                const float ar[4] = {a0.x, a0.y, a0.z, a0.w};
                const float ai[4] = {a1.x, a1.y, a1.z, a1.w};
                const float br[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
                const float bi[8] = {b2.x, b2.y, b2.z, b2.w, b3.x, b3.y, b3.z, b3.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        inr[i][j] = fmaf(ar[i], br[j], inr[i][j]);
                        inr[i][j] = fmaf(ai[i], bi[j], inr[i][j]);
                        ini[i][j] = fmaf(ai[i], br[j], ini[i][j]);
                        ini[i][j] = fmaf(-ar[i], bi[j], ini[i][j]);
                    }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    outr[i][j] += inr[i][j];
                    outi[i][j] += ini[i][j];
                    inr[i][j] = ini[i][j] = 0.0f;
                }
        }
        since_flush += kKG;
        if (since_flush >= kF32FlushGroups) {
            flush();
            since_flush = 0;
        }
    }
    if (since_flush > 0) flush();
}

}  // namespace

int xengine_tile(int) { return kTile; }

hipError_t launch_xengine(int xprec, const XArgs &a, hipStream_t s) {
    const int64_t blocks = (int64_t)a.ntiles * a.L;
    if (blocks <= 0 || a.ngrp <= 0) return hipSuccess;
    switch (xprec) {
        case MWAX_X_INT8:
            hipLaunchKernelGGL(xengine_mfma<MWAX_X_INT8>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
            break;
        case MWAX_X_FP16:
            hipLaunchKernelGGL(xengine_mfma<MWAX_X_FP16>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
            break;
        case MWAX_X_FP32:
            hipLaunchKernelGGL(xengine_f32, dim3((unsigned)blocks), dim3(kF32Threads), 0, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mwax
