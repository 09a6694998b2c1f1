// Integration output (Morrison et al. 2023, Sec. 2.5.2 and 2.7): turn one
// completed integration's device integrators into the output visibilities and
// (unless the next integration in the slot overwrites them anyway) clear them
// for reuse.  Done on the device rather than on the host CPU.
//
//   CHAN_TRI: out[c][p] = complex64(scale(V[c][p])), p = n1(n1+1)/2 + n2
//   TILE_BL : out[bl][c][pp] for tile baselines a >= b (bl = a(a+1)/2 + b) and
//             products pp = 2 p1 + p2 in the order XX, XY, YX, YY, taken from
//             input pair (2a+p1, 2b+p2); above the diagonal (auto-tile XY) the
//             conjugate of the mirrored entry.
//   raw     : out[c][p] = the exact int64 sums (INT8 integrators).
// scale: INT8 V_int * s_c * s_c (computed in FP64), FP16 and FP32 V * post.
//
// INT8 integrators hold Im V[n1,n2] - sum_m re_n1[m] (the X-engine forms its
// imaginary operand from one's complements); the autos, whose imaginary parts
// are zero, therefore hold -sum_m re_n1[m], and every entry of row n1 is
// corrected exactly by subtracting its auto's imaginary part.  So INT8 slots are
// cleared by a separate fill after the pack, never while it reads them.
#include "mwax_internal.h"

namespace mwax {
namespace {

__device__ __forceinline__ int64_t tri_row(int64_t t) {
    int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    return i;
}

// Exact INT8 sums of entry p = n1(n1+1)/2 + n2 of channel c (int32 or int64
// integrators; int32 ones are within range, see kInt32MaxSpectra).
__device__ __forceinline__ longlong2 int_vis(const PackArgs &a, int c, int64_t n1, int64_t p) {
    const int64_t d = n1 * (n1 + 1) / 2 + n1;
    if (a.i32) {
        const int2 *integ = reinterpret_cast<const int2 *>(a.integ) + (int64_t)c * a.P;
        const int2 v = integ[p];
        return make_longlong2(v.x, (long long)v.y - integ[d].y);
    }
    const longlong2 *integ = reinterpret_cast<const longlong2 *>(a.integ) + (int64_t)c * a.P;
    longlong2 v = integ[p];
    v.y -= integ[d].y;
    return v;
}

__device__ __forceinline__ float2 scaled(const PackArgs &a, int64_t p, int64_t n1, int c) {
    if (a.is_int) {
        const longlong2 v = int_vis(a, c, n1, p);
        const double s = (double)a.scales[c];
        return make_float2((float)((double)v.x * s * s), (float)((double)v.y * s * s));
    }
    const double2 v = reinterpret_cast<const double2 *>(a.integ)[(int64_t)c * a.P + p];
    return make_float2((float)(v.x * a.post), (float)(v.y * a.post));
}

__global__ void pack_tri_kernel(PackArgs a) {
    const int64_t total = (int64_t)a.L * a.P;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / a.P);
        const int64_t p = t - (int64_t)c * a.P;
        if (a.order == 2) {
            reinterpret_cast<longlong2 *>(a.out)[t] = int_vis(a, c, tri_row(p), p);
        } else if (a.is_int) {
            reinterpret_cast<float2 *>(a.out)[t] = scaled(a, p, tri_row(p), c);
        } else {
            reinterpret_cast<float2 *>(a.out)[t] = scaled(a, p, 0, c);
            if (a.clear) reinterpret_cast<double2 *>(a.integ)[t] = make_double2(0.0, 0.0);
        }
    }
    if (a.scales_out) {
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.L;
             c += (int64_t)gridDim.x * blockDim.x)
            a.scales_out[c] = a.scales[c];
    }
}

// Emission with channel averaging in the same pass (Sec. 2.6): output channel o
// of N = L / F holds the weighted mean of its fine channels' scaled integrator
// values (the rule of average.hip: offsets |d| <= F/2 around its centre, the
// outermost two at weight 1/2 for even F, DC left out of the centre channel),
// optionally divided by the pair's occupancy weight; FP64 sums, one rounding.
// Reading the integrators once replaces a pack to 6,400-channel visibilities
// and a second pass over them.
__global__ void pack_avg_kernel(PackArgs a) {
    const int N = a.L / a.F, oc = N / 2, half = a.F / 2;
    const bool even = (a.F & 1) == 0;
    const int64_t total = (int64_t)N * a.P;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(t / a.P);
        const int64_t p = t - (int64_t)o * a.P;
        const int64_t n1 = a.is_int ? tri_row(p) : 0;
        const bool centre = a.F > 1 && o == oc;
        double re = 0.0, im = 0.0, wsum = 0.0;
        for (int d = -half; d <= half; ++d) {
            if (centre && d == 0) continue;
            const double w = even && (d == -half || d == half) ? 0.5 : 1.0;
            const int c = ((a.L / 2 + (o - oc) * a.F + d) % a.L + a.L) % a.L;
            double vr, vi;
            if (a.is_int) {
                const longlong2 v = int_vis(a, c, n1, p);
                const double sc = (double)a.scales[c];
                vr = (double)v.x * sc * sc;
                vi = (double)v.y * sc * sc;
            } else {
                const double2 v = reinterpret_cast<const double2 *>(a.integ)[(int64_t)c * a.P + p];
                vr = v.x * a.post;
                vi = v.y * a.post;
            }
            re += w * vr;
            im += w * vi;
            wsum += w;
        }
        double div = wsum;
        if (a.avg_w) {
            const double wp = (double)a.avg_w[p];
            if (wp > 0.0) div *= wp;
        }
        reinterpret_cast<float2 *>(a.out)[t] = make_float2((float)(re / div), (float)(im / div));
    }
}

// gather pass of the tile-baseline order (integrators cleared afterwards)
__global__ void pack_tilebl_kernel(PackArgs a) {
    const int64_t nt = a.n_in / 2;
    const int64_t total = nt * (nt + 1) / 2 * a.L * 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int pp = (int)(t & 3);
        const int64_t rest = t >> 2;
        const int c = (int)(rest % a.L);
        const int64_t bl = rest / a.L;
        const int64_t ta = tri_row(bl);
        const int64_t tb = bl - ta * (ta + 1) / 2;
        const int64_t r = 2 * ta + (pp >> 1), s = 2 * tb + (pp & 1);
        float2 v;
        if (r >= s) {
            v = scaled(a, r * (r + 1) / 2 + s, r, c);
        } else {
            v = scaled(a, s * (s + 1) / 2 + r, s, c);
            v.y = -v.y;
        }
        reinterpret_cast<float2 *>(a.out)[t] = v;
    }
}

__global__ void fill_zero_kernel(uint4 *p, int64_t n16) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n16;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = make_uint4(0, 0, 0, 0);
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if ((bytes & 15) || ((uintptr_t)p & 15)) return hipErrorInvalidValue;
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n16)), dim3(256), 0, s, (uint4 *)p, n16);
    return hipGetLastError();
}

// integrator bytes of the slot, rounded up to whole 16-byte units (slots are
// padded to 256 bytes)
static size_t clear_bytes(const PackArgs &a) {
    return ((size_t)a.L * a.P * (a.i32 ? 8 : 16) + 15) / 16 * 16;
}

hipError_t launch_pack(const PackArgs &a, hipStream_t s) {
    if (a.order == 3) {
        if (a.F < 1 || a.L % a.F != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(pack_avg_kernel, dim3(grid_for((int64_t)(a.L / a.F) * a.P)), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !a.clear) return e;
        return a.is_int ? launch_fill_zero(a.integ, clear_bytes(a), s)
                        : launch_fill_zero(a.integ, (size_t)a.L * a.P * 16, s);
    }
    if (a.order == MWAX_ORDER_TILE_BL) {
        const int64_t nt = a.n_in / 2;
        const int64_t total = nt * (nt + 1) / 2 * a.L * 4;
        hipLaunchKernelGGL(pack_tilebl_kernel, dim3(grid_for(total)), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !a.clear) return e;
        return launch_fill_zero(a.integ, clear_bytes(a), s);
    }
    hipLaunchKernelGGL(pack_tri_kernel, dim3(grid_for((int64_t)a.L * a.P)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.clear || !a.is_int) return e;
    return launch_fill_zero(a.integ, clear_bytes(a), s);
}

}  // namespace mwax
