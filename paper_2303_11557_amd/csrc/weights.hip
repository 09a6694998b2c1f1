// Visibility weights (Sec. 4.1, with the zeroing flags of Sec. 2.4 and the
// weight table of Sec. 2.7): the occupancy of each input pair over an
// integration, and the optional normalisation of the visibilities by it.
//
// Occupancy.  Flags mark, per input and per 50 ms sub-block, the sub-blocks
// whose samples were zeroed.  The weight of pair (n1, n2) in integration j is
// the fraction of j's sub-blocks populated in both inputs.  Each workgroup
// owns a 64 x 64 block of the pair triangle: it packs the populated flags of
// its 64 + 64 inputs into 32-bit masks in LDS, 1024 sub-blocks at a time, and
// every thread counts 4 x 4 pairs with AND + popcount.  No workspace.
//
// Normalisation.  V[j][c][p] /= w[j][p] where w > 0; where w == 0 every
// product in the sum had a zeroed factor, so V is already 0 and is left as it
// is.  One read and one write of the visibilities: HBM-bound.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.h"

namespace mwax {
namespace {

constexpr int kWBlock = 64;          // inputs per side of a pair block
constexpr int kWWords = 32;          // mask words per LDS pass (1024 sub-blocks)
constexpr int kMaxInputs = 2048;     // n_inputs of a 1024-tile array
constexpr int kRowBatch = 8;         // flag rows a wave loads before their ballots
static_assert(2 * kWBlock % (4 * kRowBatch) == 0, "row batches must tile the 128 rows");

__global__ __launch_bounds__(256) void vis_weights_kernel(const uint8_t *__restrict__ flags, int n_in,
                                                          int subs, int n_ints, float *__restrict__ w) {
    __shared__ uint32_t mask[2 * kWBlock][kWWords + 2];
    // lower-triangle block (bi >= bj) of this workgroup
    const int blk = blockIdx.x;
    int bi = (int)((sqrtf(8.0f * blk + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
    while (bi * (bi + 1) / 2 > blk) --bi;
    const int bj = blk - bi * (bi + 1) / 2;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t row_len = (int64_t)n_ints * subs;
    const int W = (subs + 31) / 32;
    const int64_t P = (int64_t)n_in * (n_in + 1) / 2;

    for (int j = blockIdx.y; j < n_ints; j += gridDim.y) {
        int cnt[4][4] = {};
        for (int w0 = 0; w0 < W; w0 += kWWords) {
            __syncthreads();
            // one wave per input row: 64 lanes read 64 consecutive flags and a
            // ballot of "populated" is two mask words.  A wave owns the rows
            // r = wave (mod 4) and loads 8 of them before their ballots, so the
            // loads overlap; addresses are clamped into the flag array.
            const int nw = min(kWWords, W - w0);
            const int lane = tid & 63, wave = tid >> 6;
            for (int k = 0; k < nw; k += 2) {
                const int b = (w0 + k) * 32 + lane;
                const int bc = min(b, subs - 1);
                for (int r0 = wave; r0 < 2 * kWBlock; r0 += 4 * kRowBatch) {
                    bool pop[kRowBatch];
#pragma unroll
                    for (int u = 0; u < kRowBatch; ++u) {
                        const int r = r0 + 4 * u;
                        const int n = r < kWBlock ? bi * kWBlock + r : bj * kWBlock + (r - kWBlock);
                        const uint8_t v = flags[(int64_t)min(n, n_in - 1) * row_len + (int64_t)j * subs + bc];
                        pop[u] = (n < n_in) & (b < subs) & (v == 0);
                    }
#pragma unroll
                    for (int u = 0; u < kRowBatch; ++u) {
                        const uint64_t m = __ballot(pop[u]);
                        if (lane == 0) mask[r0 + 4 * u][k] = (uint32_t)m;
                        if (lane == 1) mask[r0 + 4 * u][k + 1] = (uint32_t)(m >> 32);
                    }
                }
            }
            __syncthreads();
            for (int k = 0; k < nw; ++k) {
                uint32_t a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = mask[ty * 4 + i][k];
                    b[i] = mask[kWBlock + tx * 4 + i][k];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) cnt[i][jj] += __popc(a[i] & b[jj]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n1 = bi * kWBlock + ty * 4 + i;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int n2 = bj * kWBlock + tx * 4 + jj;
                if (n1 < n_in && n2 <= n1)
                    w[(int64_t)j * P + (int64_t)n1 * (n1 + 1) / 2 + n2] = (float)cnt[i][jj] / (float)subs;
            }
        }
    }
}

constexpr int kApplyPerThread = 4;
constexpr int kApplyChunk = 256 * kApplyPerThread;

__global__ __launch_bounds__(256) void apply_weights_kernel(float2 *__restrict__ vis, const float *__restrict__ w,
                                                            int64_t P, int L, int64_t rows, int64_t chunks) {
    const int64_t nblk = rows * chunks;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t row = b / chunks;          // j * L + c
        const int64_t p0 = (b - row * chunks) * kApplyChunk + threadIdx.x;
        float2 *v = vis + row * P;
        const float *wr = w + (row / L) * P;
        float2 x[kApplyPerThread];
        float s[kApplyPerThread];
#pragma unroll
        for (int e = 0; e < kApplyPerThread; ++e) {
            const int64_t p = p0 + e * 256;
            if (p < P) {
                x[e] = v[p];
                s[e] = wr[p];
            }
        }
#pragma unroll
        for (int e = 0; e < kApplyPerThread; ++e) {
            const int64_t p = p0 + e * 256;
            if (p < P && s[e] > 0.0f) v[p] = make_float2(x[e].x / s[e], x[e].y / s[e]);
        }
    }
}

}  // namespace
}  // namespace mwax

using namespace mwax;

extern "C" {

mwax_status mwax_vis_weights(const uint8_t *d_flags, int32_t n_inputs, int32_t subs_per_int, int32_t n_ints,
                             float *d_weights, void *hip_stream) {
    if (n_inputs < 1 || n_inputs > kMaxInputs)
        return fail(MWAX_E_INVAL, "n_inputs must be in 1..%d (got %d)", kMaxInputs, n_inputs);
    if (subs_per_int < 1) return fail(MWAX_E_INVAL, "subs_per_int must be >= 1 (got %d)", subs_per_int);
    if (n_ints < 0) return fail(MWAX_E_INVAL, "n_ints must be >= 0 (got %d)", n_ints);
    if (n_ints == 0) return ok();
    if (!d_flags || !d_weights) return fail(MWAX_E_INVAL, "null flags or weights pointer");
    if ((uintptr_t)d_weights & 3) return fail(MWAX_E_INVAL, "weights must be 4-byte aligned");
    const int nb = (n_inputs + kWBlock - 1) / kWBlock;
    const dim3 grid((unsigned)(nb * (nb + 1) / 2), (unsigned)std::min(n_ints, 65535));
    hipLaunchKernelGGL(vis_weights_kernel, grid, dim3(256), 0, (hipStream_t)hip_stream, d_flags, n_inputs,
                       subs_per_int, n_ints, d_weights);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "weights launch");
    return ok();
}

mwax_status mwax_apply_weights(void *d_vis, const float *d_weights, int32_t n_inputs, int32_t n_chan,
                               int32_t n_ints, void *hip_stream) {
    if (n_inputs < 1 || n_inputs > kMaxInputs)
        return fail(MWAX_E_INVAL, "n_inputs must be in 1..%d (got %d)", kMaxInputs, n_inputs);
    if (n_chan < 1) return fail(MWAX_E_INVAL, "n_chan must be >= 1 (got %d)", n_chan);
    if (n_ints < 0) return fail(MWAX_E_INVAL, "n_ints must be >= 0 (got %d)", n_ints);
    if (n_ints == 0) return ok();
    if (!d_vis || !d_weights) return fail(MWAX_E_INVAL, "null visibility or weights pointer");
    if (((uintptr_t)d_vis & 7) || ((uintptr_t)d_weights & 3))
        return fail(MWAX_E_INVAL, "visibilities must be 8-byte and weights 4-byte aligned");
    const int64_t P = (int64_t)n_inputs * (n_inputs + 1) / 2;
    const int64_t rows = (int64_t)n_ints * n_chan;
    const int64_t chunks = (P + kApplyChunk - 1) / kApplyChunk;
    const int64_t nblk = rows * chunks;
    const unsigned grid = (unsigned)std::min<int64_t>(nblk, 1 << 20);
    hipLaunchKernelGGL(apply_weights_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream,
                       (float2 *)d_vis, d_weights, P, n_chan, rows, chunks);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "weight normalisation launch");
    return ok();
}

}  // extern "C"
