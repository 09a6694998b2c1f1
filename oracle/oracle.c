/*
 * oracle.c -- plain FP64 CPU reference of the MWAX FX correlation hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP library; the two meet only in the seeded input generators.
 *
 * What it computes (Morrison et al., "MWAX: A New Correlator for the
 * Murchison Widefield Array", PASA 2023):
 *
 *   F step   (Sec. 2.5, 2.5.1): each signal path's complex time series is cut
 *            into contiguous frames of L samples and each frame is Fourier
 *            transformed.  Forward sign, no normalisation (the paper names only
 *            cuFFT; the unnormalised forward transform is the reading taken).
 *              X_n[m,k] = sum_q x_n[mL+q] exp(-2 pi i k q / L)
 *            Output channel c = (k + L/2) mod L puts DC at the centre
 *            (centre-symmetric channels, Sec. 2.6).
 *   X step   (Sec. 2.5.2): for each channel, every input pair n1 >= n2
 *            (autos included) is cross-multiplied and summed over the spectra
 *            of an integration:
 *              V_j[c][n1,n2] = sum_{m in j} X_n1[m,c] conj(X_n2[m,c])
 *   Output   (Sec. 2.7): lower triangle packed row-major,
 *              index(n1,n2) = n1 (n1+1) / 2 + n2.
 *   Averaging (Sec. 2.6): centre-symmetric means of F fine channels (F + 1
 *            with half-weight ends for even F), DC left out of the centre.
 *   Weights  (Sec. 4.1): per pair and integration, the fraction of 50 ms
 *            sub-blocks populated in both inputs; optional V / w.
 *
 * Encodings the paper does not have (it computes in FP32 throughout,
 * Sec. 2.5.1 and 3.3) but the precision study needs, written out as rules:
 *   requantise: q = clamp(round_half_even(x * inv_s_c), -127, 127)
 *   calibrate : sigma_c^2 = mean over the populated (not all-zero) frames
 *               of (re^2+im^2)/2, s_c = 5 sigma_c / 127, inv_s_c = 127 /
 *               (5 sigma_c); no populated frame: the previous scales
 *   fp16      : round-half-even to the nearest binary16 value.
 *
 * Parity pins: every function here is pinned by tests against closed forms,
 * brute force, exact-integer special cases and invariants (see the tests).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared oracle.c -lm -lpthread
 * (-ffp-contract=off keeps every product and sum an individually rounded
 * IEEE double operation, so results do not depend on FMA contraction.)
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

/* exp(-2 pi i * num / den) with the angle reduced to [0, den) first, so large
 * products k*q do not lose precision.  Quarter turns are returned exactly
 * (1, -i, -1, i): then for L <= 4 every product with a twiddle is exact and
 * integer inputs give exact integer spectra. */
static void unit_root(int64_t num, int64_t den, double *re, double *im) {
    int64_t r = num % den;
    if (r < 0) r += den;
    if ((4 * r) % den == 0) {
        static const double qr[4] = {1.0, 0.0, -1.0, 0.0};
        static const double qi[4] = {0.0, -1.0, 0.0, 1.0};
        int quarter = (int)((4 * r) / den);
        *re = qr[quarter];
        *im = qi[quarter];
        return;
    }
    double ang = -2.0 * M_PI * (double)r / (double)den;
    *re = cos(ang);
    *im = sin(ang);
}

/* ---------------------------------------------------------------------------
 * Discrete Fourier transform by its definition (Sec. 2.5.1: one transform per
 * frame of L samples).  O(L^2).  x, X: [L][2] doubles.
 * ------------------------------------------------------------------------- */
int orc_dft(int L, const double *x, double *X) {
    if (L < 1) return ORC_EINVAL;
    for (int k = 0; k < L; ++k) {
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < L; ++q) {
            double wr, wi;
            unit_root((int64_t)k * q, L, &wr, &wi);
            double xr = x[2 * q], xi = x[2 * q + 1];
            sr += xr * wr - xi * wi;
            si += xr * wi + xi * wr;
        }
        X[2 * k] = sr;
        X[2 * k + 1] = si;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * The same transform by recursive radix-2 decimation in time (Cooley-Tukey):
 *   X[k]       = E[k] + w^k O[k]
 *   X[k + L/2] = E[k] - w^k O[k],   w = exp(-2 pi i / L),
 * with E, O the transforms of the even and odd samples.  L a power of two.
 * ------------------------------------------------------------------------- */
static void fft_rec(int L, const double *x, int stride, double *X, double *tmp) {
    if (L == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    int h = L / 2;
    double *E = tmp, *O = tmp + 2 * h, *sub = tmp + 2 * L;
    fft_rec(h, x, 2 * stride, E, sub);
    fft_rec(h, x + 2 * stride, 2 * stride, O, sub);
    for (int k = 0; k < h; ++k) {
        double wr, wi;
        unit_root(k, L, &wr, &wi);
        double tr = O[2 * k] * wr - O[2 * k + 1] * wi;
        double ti = O[2 * k] * wi + O[2 * k + 1] * wr;
        X[2 * k] = E[2 * k] + tr;
        X[2 * k + 1] = E[2 * k + 1] + ti;
        X[2 * (k + h)] = E[2 * k] - tr;
        X[2 * (k + h) + 1] = E[2 * k + 1] - ti;
    }
}

/* scratch needed by fft_rec for length L: 2L at this level + the child's. */
static size_t fft_scratch_doubles(int L) { return (size_t)8 * (size_t)(L > 0 ? L : 1) + 8; }

/* ---------------------------------------------------------------------------
 * The same transform for any L by recursive mixed-radix decimation in time
 * (the paper's 6,400-point transform, Sec. 2.5.1: 6400 = 2^8 * 5^2).  With p
 * the smallest prime factor of L and m = L / p, the p interleaved
 * subsequences x[p n + r] (r < p) are transformed (length m) and combined:
 *   X[k + m q] = sum_{r<p} W_L^(r (k + m q)) E_r[k],   k < m, q < p,
 * a direct p-term sum per output.  Powers of two take the radix-2 path above.
 * ------------------------------------------------------------------------- */
static int smallest_factor(int L) {
    for (int p = 2; p * p <= L; ++p)
        if (L % p == 0) return p;
    return L;
}

static void fft_mixed_rec(int L, const double *x, int stride, double *X, double *tmp) {
    if (L == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    const int p = smallest_factor(L), m = L / p;
    double *E = tmp, *sub = tmp + 2 * L;
    for (int r = 0; r < p; ++r) fft_mixed_rec(m, x + 2 * (int64_t)stride * r, stride * p, E + 2 * (int64_t)m * r, sub);
    for (int q = 0; q < p; ++q)
        for (int k = 0; k < m; ++k) {
            const int kk = k + m * q;
            double sr = 0.0, si = 0.0;
            for (int r = 0; r < p; ++r) {
                double wr, wi;
                unit_root((int64_t)r * kk, L, &wr, &wi);
                const double er = E[2 * ((int64_t)m * r + k)], ei = E[2 * ((int64_t)m * r + k) + 1];
                sr += er * wr - ei * wi;
                si += er * wi + ei * wr;
            }
            X[2 * kk] = sr;
            X[2 * kk + 1] = si;
        }
}

/* scratch of fft_mixed_rec: 2L at this level + the child's (2L/p + ...) */
static size_t fft_mixed_scratch_doubles(int L) { return (size_t)4 * (size_t)(L > 0 ? L : 1) + 8; }

static void fft_any(int L, const double *x, double *X, double *tmp) {
    if (is_pow2(L)) fft_rec(L, x, 1, X, tmp);
    else fft_mixed_rec(L, x, 1, X, tmp);
}

int orc_fft(int L, const double *x, double *X) {
    if (L < 1) return ORC_EINVAL;
    double *tmp = (double *)malloc(sizeof(double) * (fft_scratch_doubles(L) + fft_mixed_scratch_doubles(L)));
    if (!tmp) return ORC_ENOMEM;
    fft_any(L, x, X, tmp);
    free(tmp);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * F step for a chosen set of inputs and frames (Sec. 2.5.1).
 *   volts : int8 [n_rows][ld][2] (re, im), row n holds signal path n
 *           (n = 2*tile + pol, the [tile][polarisation] order of Sec. 2.5.1)
 *   inputs: the n_sel rows to transform
 *   frames: m0 .. m0+nm-1, frame m covers samples mL .. mL+L-1
 *   spec  : [nm][L][n_sel][2] doubles, channel axis fftshifted
 *           (the [time][channel][tile][pol] order of Sec. 2.5.1).
 * use_dft != 0 selects the O(L^2) definition instead of the FFT (radix-2 for
 * powers of two, mixed radix otherwise).
 * ------------------------------------------------------------------------- */
int orc_channelise(const int8_t *volts, int64_t ld, const int32_t *inputs, int n_sel,
                   int64_t m0, int64_t nm, int L, int use_dft, double *spec) {
    if (L < 1 || n_sel < 1 || nm < 0 || m0 < 0) return ORC_EINVAL;
    double *x = (double *)malloc(sizeof(double) * 2 * L);
    double *X = (double *)malloc(sizeof(double) * 2 * L);
    double *tmp = (double *)malloc(sizeof(double) * (fft_scratch_doubles(L) + fft_mixed_scratch_doubles(L)));
    if (!x || !X || !tmp) {
        free(x); free(X); free(tmp);
        return ORC_ENOMEM;
    }
    for (int s = 0; s < n_sel; ++s) {
        const int8_t *row = volts + (int64_t)inputs[s] * ld * 2;
        for (int64_t m = 0; m < nm; ++m) {
            const int8_t *fr = row + (m0 + m) * L * 2;
            for (int q = 0; q < L; ++q) {   /* promotion int8 -> double is exact */
                x[2 * q] = (double)fr[2 * q];
                x[2 * q + 1] = (double)fr[2 * q + 1];
            }
            if (use_dft) orc_dft(L, x, X);
            else fft_any(L, x, X, tmp);
            for (int k = 0; k < L; ++k) {
                int c = (k + L / 2) % L;
                double *dst = spec + (((m * L) + c) * (int64_t)n_sel + s) * 2;
                dst[0] = X[2 * k];
                dst[1] = X[2 * k + 1];
            }
        }
    }
    free(x); free(X); free(tmp);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * X step (Sec. 2.5.2) on FP64 spectra.
 *   spec : [M][L][n][2]   (as produced by orc_channelise)
 *   T    : spectra per integration; n_int = M / T integrations are produced
 *   vis  : [n_int][L][P][2], P = n(n+1)/2, packed lower triangle
 * For every output the sum runs over m in increasing order, starting from 0.
 * Threads split the channel axis; each output is owned by one thread.
 * ------------------------------------------------------------------------- */
typedef struct {
    const double *spec;
    int64_t M, T;
    int L, n, c0, c1, full;
    double *vis;
} corr_job;

static void *corr_worker(void *arg) {
    corr_job *J = (corr_job *)arg;
    const int64_t n = J->n, L = J->L;
    const int64_t P = J->full ? n * n : n * (n + 1) / 2;
    const int64_t n_int = J->M / J->T;
    for (int64_t j = 0; j < n_int; ++j) {
        for (int c = J->c0; c < J->c1; ++c) {
            double *acc = J->vis + ((j * L + c) * P) * 2;
            memset(acc, 0, sizeof(double) * 2 * P);
            for (int64_t m = j * J->T; m < (j + 1) * J->T; ++m) {
                const double *x = J->spec + ((m * L + c) * n) * 2;
                for (int64_t n1 = 0; n1 < n; ++n1) {
                    const double r1 = x[2 * n1], i1 = x[2 * n1 + 1];
                    const int64_t top = J->full ? n : n1 + 1;
                    double *row = acc + (J->full ? n1 * n : n1 * (n1 + 1) / 2) * 2;
                    for (int64_t n2 = 0; n2 < top; ++n2) {
                        const double r2 = x[2 * n2], i2 = x[2 * n2 + 1];
                        /* x1 * conj(x2) */
                        row[2 * n2] += r1 * r2 + i1 * i2;
                        row[2 * n2 + 1] += i1 * r2 - r1 * i2;
                    }
                }
            }
        }
    }
    return NULL;
}

static int run_corr(const double *spec, int64_t M, int L, int n, int64_t T, int threads,
                    int full, double *vis) {
    if (M < 0 || L < 1 || n < 1 || T < 1) return ORC_EINVAL;
    if (threads < 1) threads = 1;
    if (threads > L) threads = L;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    corr_job *jobs = (corr_job *)malloc(sizeof(corr_job) * threads);
    if (!tid || !jobs) {
        free(tid); free(jobs);
        return ORC_ENOMEM;
    }
    for (int t = 0; t < threads; ++t) {
        jobs[t].spec = spec; jobs[t].M = M; jobs[t].T = T; jobs[t].L = L; jobs[t].n = n;
        jobs[t].c0 = (int)((int64_t)L * t / threads);
        jobs[t].c1 = (int)((int64_t)L * (t + 1) / threads);
        jobs[t].full = full; jobs[t].vis = vis;
    }
    for (int t = 1; t < threads; ++t)
        if (pthread_create(&tid[t], NULL, corr_worker, &jobs[t]) != 0)
            jobs[t].c1 = -1;             /* could not start: run it below */
    corr_worker(&jobs[0]);
    for (int t = 1; t < threads; ++t) {
        if (jobs[t].c1 == -1) {
            jobs[t].c1 = (int)((int64_t)L * (t + 1) / threads);
            corr_worker(&jobs[t]);
        } else {
            pthread_join(tid[t], NULL);
        }
    }
    free(tid); free(jobs);
    return ORC_OK;
}

int orc_correlate(const double *spec, int64_t M, int L, int n, int64_t T, int threads,
                  double *vis) {
    return run_corr(spec, M, L, n, T, threads, 0, vis);
}

/* Full n x n matrix (both triangles) with the same summation order; used to
 * check the Hermitian invariant V[n2][n1] = conj(V[n1][n2]). */
int orc_correlate_full(const double *spec, int64_t M, int L, int n, int64_t T, int threads,
                       double *vis) {
    return run_corr(spec, M, L, n, T, threads, 1, vis);
}

/* ---------------------------------------------------------------------------
 * X step on int8 channelised voltages, exact in int64.
 *   q   : [M][L][n][2] int8;  vis: [n_int][L][P][2] int64
 * ------------------------------------------------------------------------- */
int orc_correlate_i64(const int8_t *q, int64_t M, int L, int n, int64_t T, int64_t *vis) {
    if (M < 0 || L < 1 || n < 1 || T < 1) return ORC_EINVAL;
    const int64_t P = (int64_t)n * (n + 1) / 2;
    const int64_t n_int = M / T;
    for (int64_t j = 0; j < n_int; ++j) {
        for (int c = 0; c < L; ++c) {
            int64_t *acc = vis + ((j * L + c) * P) * 2;
            memset(acc, 0, sizeof(int64_t) * 2 * P);
            for (int64_t m = j * T; m < (j + 1) * T; ++m) {
                const int8_t *x = q + ((m * L + c) * (int64_t)n) * 2;
                for (int64_t n1 = 0; n1 < n; ++n1) {
                    const int64_t r1 = x[2 * n1], i1 = x[2 * n1 + 1];
                    int64_t *row = acc + (n1 * (n1 + 1) / 2) * 2;
                    for (int64_t n2 = 0; n2 <= n1; ++n2) {
                        const int64_t r2 = x[2 * n2], i2 = x[2 * n2 + 1];
                        row[2 * n2] += r1 * r2 + i1 * i2;
                        row[2 * n2 + 1] += i1 * r2 - r1 * i2;
                    }
                }
            }
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Requantisation rule (not in the paper; the precision study's encoding):
 *   q = clamp(round_half_even(x * inv_s[c]), -127, 127), per component.
 * spec: [M][L][n][2] doubles; inv_s: [L] floats; q: [M][L][n][2] int8.
 * nearbyint() rounds half to even under the default rounding mode.
 * ------------------------------------------------------------------------- */
int orc_requantise(const double *spec, int64_t M, int L, int n, const float *inv_s, int8_t *q) {
    if (M < 0 || L < 1 || n < 1) return ORC_EINVAL;
    for (int64_t m = 0; m < M; ++m)
        for (int c = 0; c < L; ++c) {
            const double g = (double)inv_s[c];
            for (int64_t e = 0; e < 2 * (int64_t)n; ++e) {
                int64_t idx = (m * L + c) * 2 * (int64_t)n + e;
                double v = nearbyint(spec[idx] * g);
                if (v > 127.0) v = 127.0;
                if (v < -127.0) v = -127.0;
                q[idx] = (int8_t)v;
            }
        }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Per-channel scale from the first spectra of an integration (the calibration
 * rule of the int8 requantiser):
 *   a frame (spectrum m of input n) is populated if any of its L channel values
 *   is nonzero -- a frame of zeroed samples (lost packets are zeroed by the
 *   capture stage, Sec. 2.4) has an all-zero spectrum and is left out;
 *   sigma2[c] = sum over populated frames of (re^2 + im^2) / (2 * populated)
 *   s[c]      = 5 sqrt(sigma2) / 127        (clip level 127 <-> 5 sigma)
 *   inv_s[c]  = 127 / (5 sqrt(sigma2))
 * A channel with zero power gets s = inv_s = 1.  *populated receives the
 * count; with none populated sigma2 = 0 and s = inv_s = 1 (the caller keeps
 * the previous integration's scales then).
 * ------------------------------------------------------------------------- */
int orc_calibrate(const double *spec, int64_t M, int L, int n, double *sigma2, float *s,
                  float *inv_s, int64_t *populated) {
    if (M < 1 || L < 1 || n < 1) return ORC_EINVAL;
    int64_t pop = 0;
    for (int64_t m = 0; m < M; ++m)
        for (int64_t k = 0; k < n; ++k) {
            int any = 0;
            for (int c = 0; c < L && !any; ++c) {
                const double *x = spec + ((m * L + c) * n + k) * 2;
                any = x[0] != 0.0 || x[1] != 0.0;
            }
            pop += any;
        }
    if (populated) *populated = pop;
    for (int c = 0; c < L; ++c) {
        double acc = 0.0;
        for (int64_t m = 0; m < M; ++m)
            for (int64_t k = 0; k < n; ++k) {
                const double *x = spec + ((m * L + c) * n + k) * 2;
                acc += x[0] * x[0] + x[1] * x[1];
            }
        double v = pop > 0 ? acc / (2.0 * (double)pop) : 0.0;
        sigma2[c] = v;
        if (v > 0.0) {
            double sd = sqrt(v);
            s[c] = (float)(5.0 * sd / 127.0);
            inv_s[c] = (float)(127.0 / (5.0 * sd));
        } else {
            s[c] = 1.0f;
            inv_s[c] = 1.0f;
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Round y = x * scale to the nearest IEEE binary16 value (ties to even) and
 * return it as a double.  Binary16: 10 fraction bits, exponent range of
 * normals [-14, 15], subnormal spacing 2^-24, largest finite 65504.
 * ------------------------------------------------------------------------- */
static double to_half(double y) {
    if (y == 0.0 || !isfinite(y)) return y;
    double a = fabs(y);
    int e;
    frexp(a, &e);              /* a = f * 2^e, f in [0.5, 1) -> exponent e-1 */
    int ex = e - 1;
    if (ex < -14) ex = -14;    /* subnormal range keeps spacing 2^-24 */
    double quantum = ldexp(1.0, ex - 10);
    double r = nearbyint(a / quantum) * quantum;
    if (r > 65504.0) {
        /* values at or above 65520 round to infinity; below it to 65504 */
        r = (a >= 65520.0) ? INFINITY : 65504.0;
    }
    return y < 0 ? -r : r;
}

int orc_round_fp16(const double *x, int64_t count, double scale, double *y) {
    if (count < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < count; ++i) y[i] = to_half(x[i] * scale);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Tile-baseline view of the packed input-level triangle (Sec. 2.7 orders the
 * output by baseline, channel and polarisation product; the exact figure is
 * not in the text, so this is the reading taken):
 *   baseline index bl = a (a+1)/2 + b for tiles a >= b,
 *   products in the order XX, XY, YX, YY with p1 the pol of tile a and p2 of b:
 *     V_bl[p1 p2] = V[2a+p1, 2b+p2];
 *   for a == b the XY product lies above the diagonal and is conj(V[2a+1, 2a]).
 * vis_in: [L][P][2] (n_in = 2 n_tiles);  vis_out: [B][L][4][2], B = nt(nt+1)/2.
 * ------------------------------------------------------------------------- */
int orc_pack_tilebl(const double *vis_in, int L, int n_tiles, double *vis_out) {
    if (L < 1 || n_tiles < 1) return ORC_EINVAL;
    const int64_t n = 2 * (int64_t)n_tiles;
    const int64_t P = n * (n + 1) / 2;
    for (int64_t a = 0; a < n_tiles; ++a)
        for (int64_t b = 0; b <= a; ++b) {
            int64_t bl = a * (a + 1) / 2 + b;
            for (int c = 0; c < L; ++c)
                for (int p1 = 0; p1 < 2; ++p1)
                    for (int p2 = 0; p2 < 2; ++p2) {
                        int64_t r = 2 * a + p1, s = 2 * b + p2;
                        double re, im;
                        if (r >= s) {
                            const double *v = vis_in + ((int64_t)c * P + r * (r + 1) / 2 + s) * 2;
                            re = v[0]; im = v[1];
                        } else {
                            const double *v = vis_in + ((int64_t)c * P + s * (s + 1) / 2 + r) * 2;
                            re = v[0]; im = -v[1];
                        }
                        double *o = vis_out + ((bl * L + c) * 4 + p1 * 2 + p2) * 2;
                        o[0] = re; o[1] = im;
                    }
        }
    return ORC_OK;
}

/* -------------------------------------------------------------------------
 * Visibility weights (Sec. 4.1; the capture stage's zeroing flags, Sec. 2.4;
 * one weight per baseline/polarisation for all fine channels, Sec. 2.7).
 * flags: [n][n_ints * subs] bytes, nonzero = that input's 50 ms sub-block was
 * zeroed.  The weight of pair (n1, n2) in integration j is the fraction of
 * j's sub-blocks in which neither input was zeroed.  w: [n_ints][P].
 * ------------------------------------------------------------------------- */
int orc_vis_weights(const uint8_t *flags, int n, int subs, int n_ints, double *w) {
    if (n < 1 || subs < 1 || n_ints < 0) return ORC_EINVAL;
    const int64_t row = (int64_t)n_ints * subs;
    const int64_t P = (int64_t)n * (n + 1) / 2;
    for (int j = 0; j < n_ints; ++j)
        for (int64_t n1 = 0; n1 < n; ++n1)
            for (int64_t n2 = 0; n2 <= n1; ++n2) {
                int64_t both = 0;
                for (int b = 0; b < subs; ++b) {
                    const int64_t k = (int64_t)j * subs + b;
                    if (flags[n1 * row + k] == 0 && flags[n2 * row + k] == 0) ++both;
                }
                w[(int64_t)j * P + n1 * (n1 + 1) / 2 + n2] = (double)both / (double)subs;
            }
    return ORC_OK;
}

/* Normalisation by the weights (Sec. 4.1): V_j[c][p] / w_j[p] where w > 0;
 * a pair with w == 0 had a zeroed factor in every product, so its V is 0 and
 * stays as it is.  vis: [n_ints][L][P][2] in place. */
int orc_apply_weights(double *vis, const double *w, int n, int L, int n_ints) {
    if (n < 1 || L < 1 || n_ints < 0) return ORC_EINVAL;
    const int64_t P = (int64_t)n * (n + 1) / 2;
    for (int j = 0; j < n_ints; ++j)
        for (int c = 0; c < L; ++c)
            for (int64_t p = 0; p < P; ++p) {
                const double wt = w[(int64_t)j * P + p];
                if (wt > 0.0) {
                    double *v = vis + (((int64_t)j * L + c) * P + p) * 2;
                    v[0] = v[0] / wt;
                    v[1] = v[1] / wt;
                }
            }
    return ORC_OK;
}

/* -------------------------------------------------------------------------
 * Channel averaging (Sec. 2.6).  L fine channels (DC at c = L/2) are averaged
 * by F into N = L / F output channels arranged centre-symmetrically: output
 * channel o is centred (o - N/2) * F channels from DC (N/2 rounded down).
 *   F odd : the F channels at offsets d = -(F-1)/2 .. (F-1)/2, weight 1;
 *   F even: the F + 1 channels at d = -F/2 .. F/2, the two outermost weighted
 *           0.5, so that a channel boundary falls on a channel centre shared
 *           half and half by the two neighbours.
 * The centre output channel leaves out the DC channel and is divided by the
 * remaining weight (F - 1); every other channel by F.  With N even the
 * outermost output channel is the half channel at the coarse-channel edges
 * (its channels wrap round +-f_s/2).  F = 1 returns the input unchanged.
 * vis: [n_ints][L][P][2];  out: [n_ints][L/F][P][2].
 * ------------------------------------------------------------------------- */
int orc_fscrunch(const double *vis, int n, int L, int n_ints, int F, double *out) {
    if (n < 1 || L < 1 || n_ints < 0 || F < 1 || L % F) return ORC_EINVAL;
    const int64_t P = (int64_t)n * (n + 1) / 2;
    const int N = L / F, oc = N / 2;
    for (int j = 0; j < n_ints; ++j)
        for (int o = 0; o < N; ++o)
            for (int64_t p = 0; p < P; ++p) {
                double re = 0.0, im = 0.0, wsum = 0.0;
                const int half = F / 2;
                for (int d = -half; d <= half; ++d) {
                    if (F == 1) {
                        /* a single channel, no exclusion */
                    } else if (o == oc && d == 0) {
                        continue;                        /* DC left out of the centre channel */
                    }
                    double w = 1.0;
                    if (F % 2 == 0 && (d == -half || d == half)) w = 0.5;
                    const int c = ((L / 2 + (o - oc) * F + d) % L + L) % L;
                    const double *v = vis + (((int64_t)j * L + c) * P + p) * 2;
                    re += w * v[0];
                    im += w * v[1];
                    wsum += w;
                }
                double *y = out + (((int64_t)j * N + o) * P + p) * 2;
                y[0] = re / wsum;
                y[1] = im / wsum;
            }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Fractional delay and phase correction (Sec. 2.5.1, delay paragraph; Sec.
 * 4.3).  The capture stage shifts each signal path by whole samples (Sec.
 * 2.4.1); the residual fractional delay d (in samples, the delay to be applied,
 * updated every step of step_samples samples: 5 ms in the paper) is applied in
 * the frequency domain.  Delaying a signal by tau = d / f_s multiplies its
 * spectrum at sky frequency nu_c + f by exp(-2 pi i (nu_c + f) tau); for the
 * fftshifted channel c, f = (c - L/2) f_s / L, so every sample of the frame is
 * multiplied by
 *   g = exp(-2 pi i (c - L/2) d / L) * exp(-2 pi i (nu_c / f_s) d),
 * a phase gradient across the channels (its slope set by d alone) times a
 * phase offset set by the coarse channel's sky frequency nu_c.
 *   spec   : [M][L][n][2] doubles, corrected in place; spectrum m is the frame
 *            at stream samples (m0 + m) L .. (m0 + m + 1) L - 1
 *   delay  : [n][n_steps] samples; step s covers stream samples
 *            [s step_samples, (s + 1) step_samples) (a whole number of frames)
 *   nu_over_fs : nu_c / f_s
 * The phase is reduced to [-1/2, 1/2] revolutions in FP64 before cos/sin.
 * ------------------------------------------------------------------------- */
int orc_delay_correct(double *spec, int64_t M, int L, int n, int64_t m0, const double *delay, int64_t n_steps,
                      int64_t step_samples, double nu_over_fs) {
    if (M < 0 || L < 1 || n < 1 || m0 < 0 || step_samples < L || step_samples % L) return ORC_EINVAL;
    for (int64_t m = 0; m < M; ++m) {
        const int64_t s = (m0 + m) * L / step_samples;
        if (s >= n_steps) return ORC_EINVAL;
        for (int c = 0; c < L; ++c)
            for (int k = 0; k < n; ++k) {
                const double d = delay[(int64_t)k * n_steps + s];
                double ph = ((double)(c - L / 2) / (double)L + nu_over_fs) * d;   /* revolutions */
                ph -= nearbyint(ph);
                const double gr = cos(2.0 * M_PI * ph), gi = -sin(2.0 * M_PI * ph);
                double *x = spec + ((m * L + c) * (int64_t)n + k) * 2;
                const double xr = x[0], xi = x[1];
                x[0] = xr * gr - xi * gi;
                x[1] = xr * gi + xi * gr;
            }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Tied-array beamforming (Sec. 4.4) from the channelised voltages.
 * Coherent beams: the signal paths, each weighted by a complex gain that
 * aligns it for the beam's pointing, are summed coherently per channel and
 * spectrum:
 *   beams[m][c][b] = sum_n w[c][b][n] spec[m][c][n]
 *   spec : [M][L][n][2], w : [L][nb][n][2], beams : [M][L][nb][2].
 * Incoherent beam: the detected power of every signal path of each
 * polarisation p (input n = 2 tile + p) is summed over the inputs, t_avg
 * consecutive spectra and f_avg consecutive channels:
 *   out[j][o][p] = sum_{m = j t_avg}^{(j+1) t_avg - 1} sum_{c = o f_avg}^{(o+1) f_avg - 1}
 *                  sum_{n : n mod 2 = p} |spec[m][c][n]|^2
 *   out : [M / t_avg][L / f_avg][2] (t_avg divides M, f_avg divides L).
 * ------------------------------------------------------------------------- */
int orc_beamform(const double *spec, int64_t M, int L, int n, const double *w, int nb, double *beams) {
    if (M < 0 || L < 1 || n < 1 || nb < 1) return ORC_EINVAL;
    for (int64_t m = 0; m < M; ++m)
        for (int c = 0; c < L; ++c)
            for (int b = 0; b < nb; ++b) {
                double re = 0.0, im = 0.0;
                for (int k = 0; k < n; ++k) {
                    const double *x = spec + ((m * L + c) * (int64_t)n + k) * 2;
                    const double *g = w + (((int64_t)c * nb + b) * n + k) * 2;
                    re += g[0] * x[0] - g[1] * x[1];
                    im += g[0] * x[1] + g[1] * x[0];
                }
                double *y = beams + ((m * L + c) * (int64_t)nb + b) * 2;
                y[0] = re;
                y[1] = im;
            }
    return ORC_OK;
}

int orc_incoherent(const double *spec, int64_t M, int L, int n, int t_avg, int f_avg, double *out) {
    if (M < 0 || L < 1 || n < 1 || t_avg < 1 || f_avg < 1 || M % t_avg || L % f_avg) return ORC_EINVAL;
    const int64_t J = M / t_avg;
    const int O = L / f_avg;
    for (int64_t j = 0; j < J; ++j)
        for (int o = 0; o < O; ++o)
            for (int p = 0; p < 2; ++p) {
                double acc = 0.0;
                for (int64_t m = j * t_avg; m < (j + 1) * t_avg; ++m)
                    for (int c = o * f_avg; c < (o + 1) * f_avg; ++c)
                        for (int k = p; k < n; k += 2) {
                            const double *x = spec + ((m * L + c) * (int64_t)n + k) * 2;
                            acc += x[0] * x[0] + x[1] * x[1];
                        }
                out[(j * O + o) * 2 + p] = acc;
            }
    return ORC_OK;
}
