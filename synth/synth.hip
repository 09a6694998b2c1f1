// Device twin of the seeded voltage generator in synth/__init__.py.
//
// Makes int8 complex voltages [n_inputs][ld][2] for samples s0 .. s0+S-1:
//   uniform  : SplitMix64 output function on seed + (idx+1) * 0x9E3779B97F4A7C15,
//              top 53 bits + 0.5, scaled by 2^-53
//   Gaussian : Box-Muller on draws 2*ctr and 2*ctr+1, ctr = n * 2^36 + s
//   sources  : amp * exp(2 pi i (((k0 s) mod L) / L - nu tau_n)), nu = nu_c + k0 f_s / L,
//              tau_n = max_delay * uniform(n, seed ^ 0xD1B54A32D192ED03)
//   sample   : clip(rint(sigma * gauss + sources), -127, 127)
// None of the correlator's arithmetic is here.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SYNTH_MAX_SOURCES 8

struct SynthSources {
    int32_t count;
    int32_t L;
    double nu_c;
    double max_delay;
    double amp[SYNTH_MAX_SOURCES];
    int32_t k0[SYNTH_MAX_SOURCES];
};

__device__ __forceinline__ uint64_t sm64(uint64_t idx, uint64_t seed) {
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unif(uint64_t idx, uint64_t seed) {
    return ((double)(sm64(idx, seed) >> 11) + 0.5) * 0x1p-53;
}

__global__ void synth_kernel(int8_t *out, int32_t n_in, int64_t S, int64_t ld, int64_t s0,
                             double sigma, uint64_t seed, SynthSources src) {
    const double two_pi = 6.283185307179586476925286766559;
    const double f_s = 1.28e6;
    int64_t total = (int64_t)n_in * S;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t n = t / S;
        int64_t s = s0 + (t - n * S);
        uint64_t ctr = (uint64_t)n * (1ull << 36) + (uint64_t)s;
        double u1 = unif(2 * ctr, seed);
        double u2 = unif(2 * ctr + 1, seed);
        double r = sqrt(-2.0 * log(u1));
        double th = two_pi * u2;
        double re = sigma * r * cos(th);
        double im = sigma * r * sin(th);
        if (src.count > 0) {
            double tau = src.max_delay * unif((uint64_t)n, seed ^ 0xD1B54A32D192ED03ull);
            for (int k = 0; k < src.count; ++k) {
                double nu = src.nu_c + src.k0[k] * f_s / src.L;
                int64_t ks = ((int64_t)src.k0[k] * s) % src.L;
                if (ks < 0) ks += src.L;
                double turns = (double)ks / src.L - nu * tau;
                re += src.amp[k] * cos(two_pi * turns);
                im += src.amp[k] * sin(two_pi * turns);
            }
        }
        re = fmin(fmax(rint(re), -127.0), 127.0);
        im = fmin(fmax(rint(im), -127.0), 127.0);
        char2 v;
        v.x = (int8_t)re;
        v.y = (int8_t)im;
        *reinterpret_cast<char2 *>(out + (n * ld + (s - s0)) * 2) = v;
    }
}

extern "C" int synth_gaussian_volts(void *d_out, int32_t n_in, int64_t S, int64_t ld, int64_t s0,
                                    double sigma, uint64_t seed, int32_t n_sources,
                                    const double *amps, const int32_t *k0s, int32_t L, double nu_c,
                                    double max_delay, void *stream) {
    if (!d_out || n_in < 1 || S < 0 || ld < S || s0 < 0 || n_sources < 0 ||
        n_sources > SYNTH_MAX_SOURCES || L < 1)
        return 1;
    if (S == 0) return 0;
    SynthSources src = {};
    src.count = n_sources;
    src.L = L;
    src.nu_c = nu_c;
    src.max_delay = max_delay;
    for (int k = 0; k < n_sources; ++k) {
        src.amp[k] = amps[k];
        src.k0[k] = k0s[k];
    }
    int64_t total = (int64_t)n_in * S;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (int8_t *)d_out, n_in, S, ld, s0, sigma, seed, src);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
