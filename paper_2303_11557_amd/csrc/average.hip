// Channel averaging of visibilities (Sec. 2.6).  L fine channels, DC at
// c = L/2, are averaged by F into N = L / F output channels arranged
// centre-symmetrically: output channel o is centred (o - N/2) * F channels from
// DC (N/2 rounded down) and takes the channels at offsets d around its centre,
//   F odd : d = -(F-1)/2 .. (F-1)/2, weight 1;
//   F even: d = -F/2 .. F/2, the two outermost at weight 1/2 (a boundary falls
//           on a fine channel shared half and half by the two neighbours).
// The centre output channel leaves the DC channel out and is divided by the
// weight left (F - 1), every other by F.  With N even the outermost output
// channel is the half channel at the coarse-channel edges: its fine channels
// wrap round +-f_s/2.  F = 1 copies.  Optionally each pair's mean is divided by
// its occupancy weight while averaging (Sec. 2.6 allows a weight here; the
// weights are those of Sec. 4.1), where the weight is positive.
//
// One thread per pair and run of 4 consecutive output channels, produced in
// order: for even F the boundary channel a channel shares with the next is
// kept in a register, so each fine channel is read from HBM once (once more
// per run).  The sum runs in FP64 in ascending d: the weights are 1 and 1/2,
// so every product is exact and the value is the FP64 mean rounded once to
// FP32.  HBM-bound.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.h"

namespace mwax {
namespace {

constexpr int kAvgMaxInputs = 2048;
constexpr int kSegOut = 4;   // output channels one thread produces in order

__global__ __launch_bounds__(256) void fscrunch_kernel(const float2 *__restrict__ vis,
                                                       const float *__restrict__ weights, float2 *__restrict__ out,
                                                       int64_t P, int L, int F, int N, int nseg, int64_t rows,
                                                       int64_t chunks) {
    const int half = F / 2, oc = N / 2;
    const bool even = (F & 1) == 0;
    const int64_t nblk = rows * chunks;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t row = b / chunks;  // j * nseg + segment
        const int64_t p = (b - row * chunks) * 256 + threadIdx.x;
        if (p >= P) continue;
        const int64_t j = row / nseg;
        const int o0 = (int)(row - j * nseg) * kSegOut;
        const int o1 = min(N, o0 + kSegOut);
        const float2 *vj = vis + j * L * P + p;
        // occupancy weight of the pair (1 when none is given; 0 leaves the mean)
        const double wp = weights ? (double)weights[j * P + p] : 1.0;
        const double scale = wp > 0.0 ? wp : 1.0;
        float2 carry = make_float2(0.0f, 0.0f);
        bool have = false;
        for (int o = o0; o < o1; ++o) {
            const int base = L / 2 + (o - oc) * F;
            const bool centre = F > 1 && o == oc;
            double re = 0.0, im = 0.0;
#pragma unroll 4
            for (int d = -half; d <= half; ++d) {
                if (centre && d == 0) continue;
                const bool edge = even && (d == -half || d == half);
                const double w = edge ? 0.5 : 1.0;
                float2 v;
                if (even && d == -half && have) {
                    v = carry;  // the previous channel's upper boundary
                } else {
                    const int c = ((base + d) % L + L) % L;
                    v = vj[(int64_t)c * P];
                }
                re += w * (double)v.x;
                im += w * (double)v.y;
                if (even && d == half) {
                    carry = v;
                    have = true;
                }
            }
            const double wsum = centre ? (double)(F - 1) : (double)F;
            double yr = re / wsum, yi = im / wsum;
            if (weights) {
                yr /= scale;
                yi /= scale;
            }
            out[(j * N + o) * P + p] = make_float2((float)yr, (float)yi);
        }
    }
}

}  // namespace
}  // namespace mwax

using namespace mwax;

extern "C" {

mwax_status mwax_fscrunch(const void *d_vis, const float *d_weights, int32_t n_inputs, int32_t n_chan,
                          int32_t n_ints, int32_t fscrunch, void *d_out, void *hip_stream) {
    if (n_inputs < 1 || n_inputs > kAvgMaxInputs)
        return fail(MWAX_E_INVAL, "n_inputs must be in 1..%d (got %d)", kAvgMaxInputs, n_inputs);
    if (n_chan < 1) return fail(MWAX_E_INVAL, "n_chan must be >= 1 (got %d)", n_chan);
    if (fscrunch < 1 || n_chan % fscrunch)
        return fail(MWAX_E_INVAL, "fscrunch = %d must be >= 1 and divide n_chan = %d", fscrunch, n_chan);
    if (n_ints < 0) return fail(MWAX_E_INVAL, "n_ints must be >= 0 (got %d)", n_ints);
    if (n_ints == 0) return ok();
    if (!d_vis || !d_out) return fail(MWAX_E_INVAL, "null visibility pointer");
    if (((uintptr_t)d_vis & 7) || ((uintptr_t)d_out & 7))
        return fail(MWAX_E_INVAL, "visibilities must be 8-byte aligned");
    if ((uintptr_t)d_weights & 3) return fail(MWAX_E_INVAL, "weights must be 4-byte aligned");
    const int64_t P = (int64_t)n_inputs * (n_inputs + 1) / 2;
    const int N = n_chan / fscrunch;
    const uintptr_t in0 = (uintptr_t)d_vis, in1 = in0 + (uintptr_t)((int64_t)n_ints * n_chan * P * 8);
    const uintptr_t out0 = (uintptr_t)d_out, out1 = out0 + (uintptr_t)((int64_t)n_ints * N * P * 8);
    if (in0 < out1 && out0 < in1) return fail(MWAX_E_INVAL, "output overlaps the input visibilities");
    const int nseg = (N + kSegOut - 1) / kSegOut;
    const int64_t rows = (int64_t)n_ints * nseg;
    const int64_t chunks = (P + 255) / 256;
    const unsigned grid = (unsigned)std::min<int64_t>(rows * chunks, 1 << 20);
    hipLaunchKernelGGL(fscrunch_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream,
                       (const float2 *)d_vis, d_weights, (float2 *)d_out, P, n_chan, fscrunch, N, nseg, rows,
                       chunks);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "channel averaging launch");
    return ok();
}

}  // extern "C"
