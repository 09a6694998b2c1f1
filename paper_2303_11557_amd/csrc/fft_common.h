// In-register FFT building blocks shared by the F-engine kernels of libmwax:
// constant twiddles of small transforms, the radix-2 decimation-in-time DFT of
// N <= 32 points held by one lane, and the int8 requantisation rule.
#pragma once

#include <hip/hip_runtime.h>

namespace mwax {
namespace fft {

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

// cos(2 pi e / N) and tan(2 pi e / N) for e < N/2 (N <= 32), rounded to FP32
// from their FP64 values; the tangent at e = N/4 is unused (that twiddle is -i).
template <int N>
struct TwConst;
template <>
struct TwConst<2> {
    static constexpr float c[1] = {1.0f}, t[1] = {0.0f};
};
template <>
struct TwConst<4> {
    static constexpr float c[2] = {1.0f, 0.0f}, t[2] = {0.0f, 0.0f};
};
template <>
struct TwConst<8> {
    static constexpr float c[4] = {1.0f, 0.70710677f, 0.0f, -0.70710677f};
    static constexpr float t[4] = {0.0f, 1.0f, 0.0f, -1.0f};
};
template <>
struct TwConst<16> {
    static constexpr float c[8] = {1.0f, 0.92387950f, 0.70710677f, 0.38268343f,
                                   0.0f, -0.38268343f, -0.70710677f, -0.92387950f};
    static constexpr float t[8] = {0.0f, 0.41421357f, 1.0f, 2.4142137f, 0.0f, -2.4142137f, -1.0f, -0.41421357f};
};
template <>
struct TwConst<32> {
    static constexpr float c[16] = {1.0f, 0.98078525f, 0.92387950f, 0.83146960f, 0.70710677f, 0.55557024f,
                                    0.38268343f, 0.19509032f, 0.0f, -0.19509032f, -0.38268343f, -0.55557024f,
                                    -0.70710677f, -0.83146960f, -0.92387950f, -0.98078525f};
    static constexpr float t[16] = {0.0f, 0.19891237f, 0.41421357f, 0.66817862f, 1.0f, 1.4966058f,
                                    2.4142137f, 5.0273395f, 0.0f, -5.0273395f, -2.4142137f, -1.4966058f,
                                    -1.0f, -0.66817862f, -0.41421357f, -0.19891237f};
};

// In-register radix-2 decimation-in-time DFT of N points, natural order in and
// out.  A butterfly a +- W b with W = W_N^e = cos(t) - i sin(t), t = 2 pi e/N:
// e = 0 and e = N/4 (W = -i) are exact; otherwise W b = cos(t) (b_x + b_y tan(t),
// b_y - b_x tan(t)), so the pair costs six FMAs (two for the bracket, one per
// output component) instead of a complex multiply and four additions.
template <int N>
__device__ __forceinline__ void dft_regs(float2 *v) {
    if constexpr (N > 1) {
        using TC = TwConst<N>;
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
                    const int e = j * (N / (2 * h));
                    const float2 a = t[base + j], b = t[base + j + h];
                    if (e == 0) {
                        t[base + j] = make_float2(a.x + b.x, a.y + b.y);
                        t[base + j + h] = make_float2(a.x - b.x, a.y - b.y);
                    } else if (4 * e == N) {               // W b = (b_y, -b_x)
                        t[base + j] = make_float2(a.x + b.y, a.y - b.x);
                        t[base + j + h] = make_float2(a.x - b.y, a.y + b.x);
                    } else {
                        const float c = TC::c[e], tn = TC::t[e];
                        const float u = fmaf(b.y, tn, b.x), w = fmaf(-b.x, tn, b.y);
                        t[base + j] = make_float2(fmaf(c, u, a.x), fmaf(c, w, a.y));
                        t[base + j + h] = make_float2(fmaf(-c, u, a.x), fmaf(-c, w, a.y));
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = t[i];
    }
}


// Magic-number rounding: fma(x, s, 1.5 * 2^23) rounds the exact product x * s to
// the nearest integer, ties to even, and keeps it in the low mantissa bits;
// clamping to 1.5 * 2^23 +- 127 then leaves the two's-complement int8 code in
// the low byte.  This is the requantisation rule q = clamp(rne(x s), -127, 127)
// evaluated on the FP32 spectrum x and FP32 scale s.
constexpr float kMagic = 12582912.0f;
__device__ __forceinline__ uint32_t quant8_bits(float x, float s) {
    const float r = fmaf(x, s, kMagic);
    return __float_as_uint(fminf(fmaxf(r, kMagic - 127.0f), kMagic + 127.0f));
}

}  // namespace fft
}  // namespace mwax
