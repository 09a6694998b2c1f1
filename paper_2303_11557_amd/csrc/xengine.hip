// X-engine of the FX correlator (Morrison et al. 2023, Sec. 2.5.2): for each
// fine channel c and every input pair n1 >= n2 (autos included),
//   V[c][n1,n2] += sum_m X_n1[m,c] conj(X_n2[m,c]),
// accumulated into per-integration device integrators (Sec. 2.5.2, time
// integration) in the packed lower-triangle order p = n1(n1+1)/2 + n2.
//
// The complex Hermitian rank-k update is run as two real GEMMs over the
// channel-major rows of each input (real and imaginary parts of G frames):
//   Re V[n1,n2] = sum (re1 re2 + im1 im2) = A_n1 . A_n2,   A = the row
//   Im V[n1,n2] = sum (im1 re2 - re1 im2) = A_n1 . B_n2,   B = the row with
//                 each frame's (re, im) replaced by (-im, re)
// so every complex multiply-accumulate is four real ones and nothing is
// wasted on the real expansion.  Each 16-byte half of a row holds the real
// parts of 8 (FP16: 4) frames followed by their imaginary parts, so B is made
// from A in registers by swapping the two 8-byte quarters of a half and
// negating one of them.  Work is split into 128 x 128 tiles of the lower
// triangle.
//
//   INT8: v_mfma_i32_32x32x32_i8, int32 partials flushed to int64 integrators
//         at most every 65536 spectra (|partial| < 518160 * 4096 < 2^31).
//   FP16: v_mfma_f32_32x32x16_f16, FP32 partials flushed to FP64 integrators.
//   FP32: vector ALUs, 4 x 8 complex outputs per thread, two-level FP32
//         partials (see xengine_f32) flushed to FP64 integrators every 2048
//         spectra.
#include <type_traits>

#include "mwax_internal.h"

namespace mwax {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kTile = kXTile;       // tile edge in inputs (single-plan launches; a batch
                                    // instance may take kTileSmall, see xengine_batch)
constexpr int kTileSmall = kXTileSmall;
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
    using acc_t = v16i;                          // 16 spectra per row group
    // a row group adds at most (127 * 128 + 127^2) * 16 = 518160 to a partial
    // (the Im operand holds one's complements, see below), so 4096 groups
    // (65536 spectra) stay below 2^31
    static constexpr int kFlushGroups = 4096;
    __device__ static acc_t mma(uint4 a, uint4 b, acc_t c) {
        v4i av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, c, 0, 0, 0);
    }
};
template <>
struct MfmaT<MWAX_X_FP16> {
    using acc_t = v16f;                           // 8 spectra per row group
    static constexpr int kFlushGroups = 8192;     // 65536 spectra per FP32 partial
    __device__ static acc_t mma(uint4 a, uint4 b, acc_t c) {
        v8h av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, c, 0, 0, 0);
    }
};

// One workgroup = one channel x one 128 x 128 tile of the lower triangle.
// Four waves in a 2 x 2 layout, 64 x 64 outputs (2 x 2 blocks of 32 x 32) each,
// real and imaginary accumulators for every block (128 accumulator registers).
// Two workgroups share a CU (two waves per SIMD), so one workgroup's barrier
// latency is covered by the other's matrix work.
//
// The K loop runs over stages of kXG row groups.  Stages are copied from global
// memory straight into LDS (16 bytes per lane, no register staging and no LDS
// store instructions) into a ring of kNBuf stage buffers, kDist stages
// ahead of the matrix work, with one barrier per stage.  Each wave copies 32
// whole rows (1 KB of global memory) of each panel into one LDS block laid out
// [16-byte half][row], the layout the fragment reads want.  The ring buffers are separate LDS
// objects, so the compiler can tell a read of one buffer from the copies still
// landing in the others and does not wait for those.
//
// The Im operand B2 is formed in registers from the B fragment: its two 8-byte
// quarters (real parts, imaginary parts of the same frames) are swapped and the
// imaginary one is flipped -- FP16 by its sign bits, INT8 by its one's
// complement ~x = -x - 1.  The INT8 integrators therefore hold Im V[n1,n2] -
// sum_m re_n1[m], and the autos (whose imaginary parts are zero) hold exactly
// -sum_m re_n1[m]: the pack step subtracts an entry's auto from it, which makes
// the result exact without any extra work in this loop.  With ~im in
// [-128, 126] a row group adds at most 127 * 128 * 16 + 127^2 * 16 to a partial,
// and 65536 spectra stay below 2^31.
constexpr int kXG = 2;                      // row groups per stage
constexpr int kNBuf = 4;                    // stage buffers
constexpr int kDist = 2;                    // stages copied ahead of the matrix work (< kNBuf)
constexpr int kBlock = 32 * kRowBytes;      // LDS bytes of 32 rows: [half][row][16 B]
static_assert((kNBuf == 2 || kNBuf == 4) && kDist >= 1 && kDist < kNBuf, "ring of 2 or 4 stage buffers");

// Stage geometry of a TE x TE tile (TE = 128 or 64).  A 128-edge tile gives each
// of the four waves 64 x 64 outputs (2 x 2 blocks of 32 x 32) and each wave
// copies 32 rows of both panels; a 64-edge tile gives each wave one 32 x 32
// block and each wave copies 32 rows of one panel.
template <int TE, int DIST = kDist>
struct TileGeo {
    static_assert(TE == 128 || TE == 64, "tile edge");
    static_assert(DIST >= 1 && DIST < kNBuf, "copies run at most kNBuf - 1 stages ahead");
    static constexpr int MB = TE / 64;                   // 32 x 32 blocks per wave and dimension
    static constexpr int kGroupPitch = TE / 32 * kBlock;
    static constexpr int kPanel = kXG * kGroupPitch;     // one panel (A or B) of a stage
    static constexpr int kStage = 2 * kPanel;
    static constexpr int kCopiesPerStage = (TE == 128 ? 2 : 1) * kXG;   // copies per wave per stage
    // s_waitcnt immediate: vmcnt(copies of the DIST - 1 later stages), lgkmcnt(0)
    static constexpr int kWaitCopies = kCopiesPerStage * (DIST - 1);
    static_assert(kWaitCopies < 16, "vmcnt immediate");
    static constexpr int kStageWait = kWaitCopies | (7 << 4);
};
constexpr int kStage = TileGeo<kTile>::kStage;          // stage buffers are sized for the larger tile

struct XLds {
    uint8_t *buf[4];   // the first kNBuf are used
};
constexpr int kStage23 = kNBuf > 2 ? kStage : 16;

// Source of the row groups past the end of a segment (they must read as zero).
__device__ __align__(16) const uint8_t kZeroGroup[kTile * kRowBytes] = {};

// End of a stage: this wave's copies of the next stage have landed (the
// kDist - 1 later stages stay in flight) and its LDS reads have returned; then the
// workgroup barrier.  The barrier carries no memory fence of its own (a fence
// would wait for every copy in flight); the wait provides the ordering, and the
// memory clobber keeps the compiler from moving LDS accesses across it.
template <int TE, int DIST = kDist>
__device__ __forceinline__ void stage_barrier() {
    __builtin_amdgcn_s_waitcnt(TileGeo<TE, DIST>::kStageWait);
    asm volatile("s_barrier" ::: "memory");
}

// ATOMIC: flush with int64 atomic adds (another workgroup may be flushing other
// row groups of the same tile at the same time).
template <int XP, int TE, bool ACTIVE, bool ATOMIC = false>
__device__ __forceinline__ void xengine_tile_loop(const XArgs &a, const XLds &lds, int c, int rowA0, int rowB0,
                                                  int wr, int wc) {
    static_assert(!ATOMIC || XP == MWAX_X_INT8, "atomic flushes are exact for integer partials only");
    using GEO = TileGeo<TE>;
    constexpr int MB = GEO::MB, kGroupPitch = GEO::kGroupPitch, kPanel = GEO::kPanel;
    using T = MfmaT<XP>;
    using acc_t = typename T::acc_t;
    constexpr bool INT8 = XP == MWAX_X_INT8;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5, l32 = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);

    // Copies: wave w moves rows w * 32 .. w * 32 + 31 of both panels (TE = 128),
    // or rows (w % 2) * 32 .. + 31 of panel w / 2 (TE = 64); lane l takes half
    // l / 32 of its row and lands at byte l * 16 of the row's block.
    // Rows past the last input are read from a clamped (valid) address and not
    // cleared: row i of A and column j of B reach only output (i, j), and outputs
    // past the last input are never flushed.
    const int cblk = TE == 128 ? wave : (wave & 1);          // block within the panel
    const int cpanel = TE == 128 ? 0 : (wave >> 1) * kPanel;  // TE = 64: the panel this wave copies
    const int chalf = lane >> 5, crow = cblk * 32 + (lane & 31);
    const uint32_t offA = (uint32_t)min(rowA0 + crow, a.n_in - 1) * kRowBytes + chalf * 16;
    const uint32_t offB = (uint32_t)min(rowB0 + crow, a.n_in - 1) * kRowBytes + chalf * 16;
    const uint32_t offZ = (uint32_t)crow * kRowBytes + chalf * 16;
    const int64_t gstride = (int64_t)a.n_in * kRowBytes;   // bytes between row groups
    const uint8_t *base = a.chan + ((int64_t)c * a.NG + a.grp0) * gstride;
    const int ldst = cpanel + cblk * kBlock;
    const int nstages = (a.ngrp + kXG - 1) / kXG;

    // CHECK: the stage may reach past the segment end (its last stage)
    auto copy_stage = [&](int s, uint8_t *buf, auto check_c) {
        constexpr bool CHECK = decltype(check_c)::value;
#pragma unroll
        for (int k = 0; k < kXG; ++k) {
            const int g = s * kXG + k;
            const bool in = !CHECK || g < a.ngrp;
            const uint8_t *gb = in ? base + (int64_t)g * gstride : kZeroGroup;
            if constexpr (TE == 128) {
                __builtin_amdgcn_global_load_lds(gb + (in ? offA : offZ), buf + k * kGroupPitch + ldst, 16, 0, 0);
                __builtin_amdgcn_global_load_lds(gb + (in ? offB : offZ), buf + kPanel + k * kGroupPitch + ldst, 16,
                                                 0, 0);
            } else {
                // waves 0, 1 copy the A panel, waves 2, 3 the B panel
                const uint32_t off = in ? (wave < 2 ? offA : offB) : offZ;
                __builtin_amdgcn_global_load_lds(gb + off, buf + k * kGroupPitch + ldst, 16, 0, 0);
            }
        }
    };

    acc_t re[MB][MB], im[MB][MB];
    // fragment m of a wave's 32 MB rows is block MB * w + m; lane (half, l32)
    // reads half `half` of its row l32
    const int fa_off = wr * MB * kBlock + half * 512 + l32 * 16;
    const int fb_off = kPanel + wc * MB * kBlock + half * 512 + l32 * 16;
    constexpr uint32_t kFlip = INT8 ? 0xffffffffu : 0x80008000u;

    // One stage of matrix-core work from one buffer; the fragments of row group
    // k+1 are read while the MFMAs of group k run.
    auto compute = [&](const uint8_t *st) {
        uint4 fa[2][MB], fb[2][MB];
        auto read = [&](int k, int slot) {
            const int ko = k * kGroupPitch;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                fa[slot][m] = *reinterpret_cast<const uint4 *>(st + ko + fa_off + m * kBlock);
                fb[slot][m] = *reinterpret_cast<const uint4 *>(st + ko + fb_off + m * kBlock);
            }
        };
        read(0, 0);
#pragma unroll
        for (int k = 0; k < kXG; ++k) {
            if (k + 1 < kXG) read(k + 1, (k + 1) & 1);
            const int sl = k & 1;
            uint4 fb2[MB];
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const uint4 v = fb[sl][m];
                fb2[m] = make_uint4(v.z ^ kFlip, v.w ^ kFlip, v.x, v.y);
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb2 = 0; nb2 < MB; ++nb2) {
                    re[mb][nb2] = T::mma(fa[sl][mb], fb[sl][nb2], re[mb][nb2]);
                    im[mb][nb2] = T::mma(fa[sl][mb], fb2[nb2], im[mb][nb2]);
                }
        }
        // 2 MB reads and 2 MB^2 MFMAs per row group: the reads of group k+1 are
        // interleaved with the first MFMAs of group k
        constexpr int kReads = 2 * MB, kMfma = 2 * MB * MB;
        __builtin_amdgcn_sched_group_barrier(0x100, kReads, 0);    // reads, group 0
#pragma unroll
        for (int k = 0; k + 1 < kXG; ++k) {
#pragma unroll
            for (int q = 0; q < kReads; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one read of group k+1
            }
            if constexpr (kMfma > kReads) __builtin_amdgcn_sched_group_barrier(0x008, kMfma - kReads, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, kMfma, 0);     // MFMAs, last group
    };

    // Iteration on stage s held in buffer B: copy stage s + kDist into a buffer
    // last read by an earlier iteration, matrix work on stage s, wait for
    // stage s + 1, barrier.  Every iteration copies a stage (past the segment end
    // from the zero page), so exactly kCopiesPerStage copies per stage are in
    // flight and no copy sits behind a branch: for a copy behind a branch the
    // compiler would wait for every copy in flight before the next LDS read.
    // CHECK: tail iterations, which may reach past the segment end and skip the
    // matrix work of stages at or past s1.
    using Yes = std::true_type;
    using No = std::false_type;
    auto iteration = [&](int s, int s1, auto b_c, auto check_c) {
        constexpr int B = decltype(b_c)::value;
        constexpr bool CHECK = decltype(check_c)::value;
        copy_stage(s + kDist, lds.buf[(B + kDist) % kNBuf], check_c);
        if constexpr (ACTIVE) {
            if (!CHECK || s < s1) compute(lds.buf[B]);
        }
        stage_barrier<TE>();
    };
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    using B2 = std::integral_constant<int, 2>;
    using B3 = std::integral_constant<int, 3>;

#pragma unroll
    for (int b = 0; b < kDist; ++b) copy_stage(b, lds.buf[b], Yes{});
    stage_barrier<TE>();

    constexpr int kChunkStages = T::kFlushGroups / kXG;
    static_assert(kChunkStages % kNBuf == 0, "flush chunks must start on buffer 0");
    for (int s0 = 0; s0 < nstages; s0 += kChunkStages) {
        // s1 is a multiple of kNBuf or the segment end
        const int s1 = min(nstages, s0 + kChunkStages);
        if constexpr (ACTIVE) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb2 = 0; nb2 < MB; ++nb2) {
                    re[mb][nb2] = acc_t{};
                    im[mb][nb2] = acc_t{};
                }
        }
        // steady state: every stage copied is whole and before the last one
        const int sfull = min(s1, nstages - kDist - 1);
        int s = s0;
        for (; s + kNBuf <= sfull; s += kNBuf) {
            iteration(s, s1, B0{}, No{});
            iteration(s + 1, s1, B1{}, No{});
            if constexpr (kNBuf > 2) {
                iteration(s + 2, s1, B2{}, No{});
                iteration(s + 3, s1, B3{}, No{});
            }
        }
        for (; s < s1; s += kNBuf) {
            iteration(s, s1, B0{}, Yes{});
            iteration(s + 1, s1, B1{}, Yes{});
            if constexpr (kNBuf > 2) {
                iteration(s + 2, s1, B2{}, Yes{});
                iteration(s + 3, s1, B3{}, Yes{});
            }
        }
        if constexpr (ACTIVE) {
            // flush this chunk's partial sums into the integrators.  The base is made
            // opaque here so the compiler cannot hoist 64 integrator addresses out of
            // the K loop (they would occupy half the register file).
            uint8_t *ibase = reinterpret_cast<uint8_t *>(a.integ);
            int fr0 = rowA0, fc0 = rowB0;
            asm volatile("" : "+s"(ibase), "+s"(fr0), "+s"(fc0));
            // the first flush of a segment that starts its integration writes the
            // integrators instead of adding to them (no read)
            const bool store = a.first && s0 == 0;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int RB = wr * MB + mb;
#pragma unroll
                for (int nb2 = 0; nb2 < MB; ++nb2) {
                    const int CB = wc * MB + nb2;
                    const int n2 = fc0 + CB * 32 + l32;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int n1 = fr0 + RB * 32 + (r >> 2) * 8 + half * 4 + (r & 3);
                        if (n1 < a.n_in && n2 <= n1) {
                            const int64_t p = (int64_t)n1 * (n1 + 1) / 2 + n2;
                            if constexpr (ATOMIC) {
                                if (a.i32) {
                                    int *dst = reinterpret_cast<int *>(ibase) + 2 * ((int64_t)c * a.P + p);
                                    atomicAdd(dst, (int)re[mb][nb2][r]);
                                    atomicAdd(dst + 1, (int)im[mb][nb2][r]);
                                } else {
                                    unsigned long long *dst =
                                        reinterpret_cast<unsigned long long *>(ibase) + 2 * ((int64_t)c * a.P + p);
                                    atomicAdd(dst, (unsigned long long)(long long)re[mb][nb2][r]);
                                    atomicAdd(dst + 1, (unsigned long long)(long long)im[mb][nb2][r]);
                                }
                            } else if constexpr (INT8) {
                                if (a.i32) {
                                    int2 *dst = reinterpret_cast<int2 *>(ibase) + (int64_t)c * a.P + p;
                                    int2 v = make_int2(re[mb][nb2][r], im[mb][nb2][r]);
                                    if (!store) {
                                        const int2 o = *dst;
                                        v.x += o.x;
                                        v.y += o.y;
                                    }
                                    *dst = v;
                                } else {
                                    longlong2 *dst = reinterpret_cast<longlong2 *>(ibase) + (int64_t)c * a.P + p;
                                    longlong2 v = make_longlong2(re[mb][nb2][r], im[mb][nb2][r]);
                                    if (!store) {
                                        const longlong2 o = *dst;
                                        v.x += o.x;
                                        v.y += o.y;
                                    }
                                    *dst = v;
                                }
                            } else {
                                double2 *dst = reinterpret_cast<double2 *>(ibase) + (int64_t)c * a.P + p;
                                double2 v = make_double2((double)re[mb][nb2][r], (double)im[mb][nb2][r]);
                                if (!store) {
                                    const double2 o = *dst;
                                    v.x += o.x;
                                    v.y += o.y;
                                }
                                *dst = v;
                            }
                        }
                    }
                }
            }
        }
    }
    // the copies past the segment end must land before the LDS is reused (next
    // work item) or released (workgroup end)
    __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0)
}

// Workgroup -> (chunk, channel, tile): the tiles of one channel are consecutive,
// so they land on one XCD and share its L2; the chunks of a tile read disjoint
// row groups and run one after another (measured: 25 % less HBM traffic than
// interleaving them).
template <int XP>
__global__ __launch_bounds__(kThreads, 2) void xengine_mfma(XArgs a) {
    __shared__ __align__(16) uint8_t lds0[kStage], lds1[kStage], lds2[kStage23], lds3[kStage23];
    const XLds lds{{lds0, lds1, lds2, lds3}};
    const int nb = gridDim.x;
    const int lin = xcd_logical(blockIdx.x, nb);
    const int per_k = a.ntiles * a.L;
    const int ks = lin / per_k;
    const int rem = lin - ks * per_k;
    const int c = rem / a.ntiles, t = rem - c * a.ntiles;
    int I, J;
    tile_ij(t, I, J);
    const int rowA0 = I * kTile, rowB0 = J * kTile;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    XArgs b = a;
    b.grp0 = a.grp0 + (int64_t)ks * a.kchunk;
    b.ngrp = min(a.kchunk, a.ngrp - ks * a.kchunk);
    // A wave is idle on a diagonal tile above the diagonal, or when all its rows or
    // columns lie past the last input; it still stages data and meets the barriers.
    const bool idle = (I == J && wr < wc) || rowA0 + wr * 64 >= a.n_in || rowB0 + wc * 64 >= a.n_in;
    if constexpr (XP == MWAX_X_INT8) {
        if (a.nks > 1) {
            if (idle) xengine_tile_loop<XP, kTile, false, true>(b, lds, c, rowA0, rowB0, wr, wc);
            else xengine_tile_loop<XP, kTile, true, true>(b, lds, c, rowA0, rowB0, wr, wc);
            return;
        }
    }
    if (idle) xengine_tile_loop<XP, kTile, false>(b, lds, c, rowA0, rowB0, wr, wc);
    else xengine_tile_loop<XP, kTile, true>(b, lds, c, rowA0, rowB0, wr, wc);
}

// One work item of the batched kernel: tile (I, J) of edge TE.  A wave is idle
// on a diagonal tile above the diagonal, or when all its rows or columns lie past
// the last input; it still stages data and meets the barriers.
template <int XP, int TE>
__device__ __forceinline__ void batch_tile(const XArgs &a, const XLds &lds, int c, int I, int J, int wr, int wc,
                                           bool atomic) {
    const int rowA0 = I * TE, rowB0 = J * TE;
    const bool idle = (I == J && wr < wc) || rowA0 + wr * (TE / 2) >= a.n_in || rowB0 + wc * (TE / 2) >= a.n_in;
    if constexpr (XP == MWAX_X_INT8) {
        if (atomic) {
            if (idle) xengine_tile_loop<XP, TE, false, true>(a, lds, c, rowA0, rowB0, wr, wc);
            else xengine_tile_loop<XP, TE, true, true>(a, lds, c, rowA0, rowB0, wr, wc);
            return;
        }
    }
    if (idle) xengine_tile_loop<XP, TE, false>(a, lds, c, rowA0, rowB0, wr, wc);
    else xengine_tile_loop<XP, TE, true>(a, lds, c, rowA0, rowB0, wr, wc);
}

// Persistent batched form (see XBatchArgs): each workgroup takes items from the
// queue of its XCD until it is empty, then from the other queues in turn, and
// exits when all are empty.  Every item is one tile of one channel over one chunk
// of row groups, run by the same loop as the single-plan kernel.
template <int XP>
__global__ __launch_bounds__(kThreads, 2) void xengine_batch(XBatchArgs b) {
    __shared__ __align__(16) uint8_t lds0[kStage], lds1[kStage], lds2[kStage23], lds3[kStage23];
    __shared__ int s_item;
    const XLds lds{{lds0, lds1, lds2, lds3}};
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int home = blockIdx.x & (kXQueues - 1);
    for (int v = 0; v < kXQueues; ++v) {
        const int q = (home + v) & (kXQueues - 1);
        const int q0 = load_uniform(b.qbeg + q), qn = load_uniform(b.qbeg + q + 1) - q0;
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(&b.counters[q * kXCounterStride], 1);
            __syncthreads();
            const int k = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            if (k >= qn) break;
            const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)b.items[q0 + k]);
            const int d = (int)(it >> 24), c = (int)((it >> 14) & 1023), t = (int)((it >> 6) & 255);
            const int ks = (int)(it & 63);
            const XDesc xd = load_uniform(b.desc + d);
            XArgs a{};
            a.chan = xd.chan;
            a.NG = xd.NG;
            a.grp0 = xd.grp0 + (int64_t)ks * xd.kchunk;
            a.ngrp = min(xd.kchunk, xd.ngrp - ks * xd.kchunk);
            a.n_in = xd.n_in;
            a.integ = xd.integ;
            a.P = xd.P;
            a.first = xd.first;
            a.i32 = xd.i32;
            int I, J;
            tile_ij(t, I, J);
            if (xd.te == kTileSmall) {
                batch_tile<XP, kTileSmall>(a, lds, c, I, J, wr, wc, xd.ksplit > 1);
            } else {
                batch_tile<XP, kTile>(a, lds, c, I, J, wr, wc, xd.ksplit > 1);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Averaging X-engine (Sec. 2.6 applied inside the correlation): one workgroup =
// one output channel o of N = L / F x one 64 x 64 tile.  It correlates the fine
// channels of o one after another -- offsets |d| <= F / 2 around o's centre
// (the rule of average.hip: the outermost pair at weight 1/2 for even F, DC left
// out of the centre channel) -- with the MFMA K loop running over the
// channel-major rows of (channel, row group), stages never straddling two
// channels.  When a channel's last stage is done its partial sums are scaled
// (INT8: s_c^2) and weighted into FP32 sums held in registers, which are
// divided by the weight total and added (or, for the first segment of an
// integration, stored) once into FP64 integrators [N][P].  The fine-channel
// integrators are never written: per 250 ms integration at 256 tiles and
// L = 6400 that is 6.7 GB of flushes and 6.7 GB of pack reads avoided.
// The INT8 Im operand is the exact negation (-im, re), not the one's
// complement of the per-channel kernel, so each channel's partials are its
// exact sums before scaling.
// ---------------------------------------------------------------------------
// Copies run three stages ahead here (two in the per-channel kernel): a work
// item's stages are short (4 MFMAs per wave at 250 ms integrations) and every
// workgroup of a launch is resident at once, so the copies in flight are what
// hides the L2 latency.
constexpr int kAvgDist = 3;

template <int XP>
__global__ __launch_bounds__(kThreads, 4) void xengine_avg(XAvgArgs a) {
    constexpr int TE = kTileSmall;
    using GEO = TileGeo<TE, kAvgDist>;
    constexpr int kGroupPitch = GEO::kGroupPitch, kPanel = GEO::kPanel;
    using T = MfmaT<XP>;
    using acc_t = typename T::acc_t;
    constexpr bool INT8 = XP == MWAX_X_INT8;
    __shared__ __align__(16) uint8_t lds0[GEO::kStage], lds1[GEO::kStage], lds2[GEO::kStage], lds3[GEO::kStage];
    uint8_t *const bufs[4] = {lds0, lds1, lds2, lds3};
    static_assert(kNBuf == 4, "four stage buffers");

    const int nb = gridDim.x;
    const int lin = xcd_logical(blockIdx.x, nb);
    const int o = lin / a.ntiles;
    int I, J;
    tile_ij(lin - o * a.ntiles, I, J);
    const int rowA0 = I * TE, rowB0 = J * TE;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5, l32 = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const bool active = !((I == J && wr < wc) || rowA0 + wr * 32 >= a.n_in || rowB0 + wc * 32 >= a.n_in);

    // the fine channels of o: offsets d = -h .. h (DC skipped in the centre one),
    // channel (L/2 + (o - N/2) F + d) mod L.  They are walked with cursors: no
    // division or remainder in the loop, whose scalar work per stage is what
    // bounds a stage of four MFMAs per wave.
    const int h = a.F / 2, oc = a.N / 2;
    const bool even = (a.F & 1) == 0, centre = a.F > 1 && o == oc;
    const int nch = 2 * h + 1 - (centre ? 1 : 0);
    const float inv_wsum = 1.0f / (centre ? (float)(a.F - 1) : (float)a.F);
    const int c_first = ((a.L / 2 + (o - oc) * a.F - h) % a.L + a.L) % a.L;
    // next channel after c at offset d (skipping DC in the centre channel)
    auto next_channel = [&](int c, int d) {
        int n = c + ((centre && d == -1) ? 2 : 1);
        return n >= a.L ? n - a.L : n;
    };

    // copies: waves 0, 1 move 32 rows each of the A panel, waves 2, 3 of the B panel
    const int cblk = wave & 1, cpanel = (wave >> 1) * kPanel;
    const int chalf = lane >> 5, crow = cblk * 32 + (lane & 31);
    const int rowC0 = wave < 2 ? rowA0 : rowB0;
    const uint32_t offR = (uint32_t)min(rowC0 + crow, a.n_in - 1) * kRowBytes + chalf * 16;
    const uint32_t offZ = (uint32_t)crow * kRowBytes + chalf * 16;
    const int64_t gstride = (int64_t)a.n_in * kRowBytes;
    const int64_t cstride = a.NG * gstride;       // bytes between channels
    const int ldst = cpanel + cblk * kBlock;
    const int spc = (a.ngrp + kXG - 1) / kXG;     // stages per channel
    const int nst = nch * spc;

    // copy cursor: channel index, its channel and offset, stage within it, and the
    // address of the stage's first row group
    int cp_ci = 0, cp_c = c_first, cp_d = -h, cp_g = 0;
    if (centre && cp_d == 0) cp_d = 1;            // (h = 0 only when F = 1: no centre rule)
    const uint8_t *cp_base = a.chan + ((int64_t)cp_c * a.NG + a.grp0) * gstride;
    const uint8_t *cp_src = cp_base;
    const int64_t stage_bytes = (int64_t)kXG * gstride;
    auto copy_next = [&](uint8_t *buf) {
        const bool live = cp_ci < nch;
#pragma unroll
        for (int k = 0; k < kXG; ++k) {
            const bool in = live && cp_g + k < a.ngrp;
            const uint8_t *src = in ? cp_src + k * gstride + offR : kZeroGroup + offZ;
            __builtin_amdgcn_global_load_lds(src, buf + k * kGroupPitch + ldst, 16, 0, 0);
        }
        cp_g += kXG;
        cp_src += stage_bytes;
        if (cp_g >= a.ngrp) {
            cp_g = 0;
            ++cp_ci;
            const int nc = next_channel(cp_c, cp_d);
            cp_base += (int64_t)(nc - cp_c) * cstride;
            cp_src = cp_base;
            cp_c = nc;
            cp_d += (centre && cp_d == -1) ? 2 : 1;
        }
    };

    acc_t re{}, im{};
    float sr[16], si[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) sr[r] = si[r] = 0.0f;
    const int fa_off = wr * kBlock + half * 512 + l32 * 16;
    const int fb_off = kPanel + wc * kBlock + half * 512 + l32 * 16;

    auto compute = [&](const uint8_t *st) {
        uint4 fa[2], fb[2];
        fa[0] = *reinterpret_cast<const uint4 *>(st + fa_off);
        fb[0] = *reinterpret_cast<const uint4 *>(st + fb_off);
#pragma unroll
        for (int k = 0; k < kXG; ++k) {
            if (k + 1 < kXG) {
                fa[(k + 1) & 1] = *reinterpret_cast<const uint4 *>(st + (k + 1) * kGroupPitch + fa_off);
                fb[(k + 1) & 1] = *reinterpret_cast<const uint4 *>(st + (k + 1) * kGroupPitch + fb_off);
            }
            const uint4 v = fb[k & 1];
            uint4 fb2;
            if constexpr (INT8) fb2 = make_uint4(neg_i8x4(v.z), neg_i8x4(v.w), v.x, v.y);
            else fb2 = make_uint4(v.z ^ 0x80008000u, v.w ^ 0x80008000u, v.x, v.y);
            re = T::mma(fa[k & 1], v, re);
            im = T::mma(fa[k & 1], fb2, im);
        }
    };
    // Weight of every channel index ci (weight / weight total, times s_c^2): a
    // table held across the lanes, lane l holding ci = w0 + 64 t + l (t < 4) of
    // the window of 256 indices from w0, read with v_readlane when a channel is
    // done -- no memory access in the loop, whose vector-memory counter belongs
    // to the copies in flight.
    float ctab[4];
    auto load_window = [&](int w0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ci = w0 + 64 * t + lane;
            const int d = -h + ci + (centre && ci >= h ? 1 : 0);
            const int c = (((a.L / 2 + (o - oc) * a.F + d) % a.L) + a.L) % a.L;
            float coef = (even && (d == -h || d == h) ? 0.5f : 1.0f) * inv_wsum;
            if (a.scales && ci < nch) {
                const float sc = a.scales[c];
                coef *= sc * sc;
            }
            ctab[t] = coef;
        }
    };
    load_window(0);
    // compute cursor: channel index and the stage within the channel
    int cm_ci = 0, cm_ls = 0;
    auto iteration = [&](int s, auto b_c) {
        constexpr int B = decltype(b_c)::value;
        copy_next(bufs[(B + kAvgDist) % kNBuf]);
        if (s < nst) {
            if (active) compute(bufs[B]);
            if (++cm_ls == spc) {
                // the channel's partials, scaled and weighted, into the sums
                if (active) {
                    const int t = (cm_ci >> 6) & 3;
                    const float tv = t == 0 ? ctab[0] : (t == 1 ? ctab[1] : (t == 2 ? ctab[2] : ctab[3]));
                    const float coef = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tv), cm_ci & 63));
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        sr[r] = fmaf(coef, (float)re[r], sr[r]);
                        si[r] = fmaf(coef, (float)im[r], si[r]);
                    }
                    re = acc_t{};
                    im = acc_t{};
                }
                cm_ls = 0;
                if ((++cm_ci & 255) == 0 && cm_ci < nch) load_window(cm_ci);
            }
        }
        stage_barrier<TE, kAvgDist>();
    };

#pragma unroll
    for (int b = 0; b < kAvgDist; ++b) copy_next(bufs[b]);
    stage_barrier<TE, kAvgDist>();
    for (int s = 0; s < nst; s += kNBuf) {
        iteration(s, std::integral_constant<int, 0>{});
        iteration(s + 1, std::integral_constant<int, 1>{});
        iteration(s + 2, std::integral_constant<int, 2>{});
        iteration(s + 3, std::integral_constant<int, 3>{});
    }
    __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0): copies past the end have landed

    if (active) {
        double2 *dst0 = reinterpret_cast<double2 *>(a.integ) + (int64_t)o * a.P;
        const int n2 = rowB0 + wc * 32 + l32;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n1 = rowA0 + wr * 32 + (r >> 2) * 8 + half * 4 + (r & 3);
            if (n1 < a.n_in && n2 <= n1) {
                double2 *dst = dst0 + (int64_t)n1 * (n1 + 1) / 2 + n2;
                double2 v = make_double2((double)sr[r], (double)si[r]);
                if (!a.first) {
                    const double2 old = *dst;
                    v.x += old.x;
                    v.y += old.y;
                }
                *dst = v;
            }
        }
    }
}

__global__ void zero_i32_kernel(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
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
int xengine_tile_count(int n_in, int te) {
    const int t = (n_in + te - 1) / te;
    return t * (t + 1) / 2;
}

namespace {
// Resident workgroups of the single-plan MFMA kernel on the current device.
int resident_slots() {
    static int slots = 0;
    if (slots == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(&xengine_mfma<MWAX_X_INT8>), kThreads, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        slots = cus * per_cu;
    }
    return slots;
}

// Chunks per tile: the fewest that minimise the number of workgroup waves per
// unit of work, with at least kMinChunkGroups row groups per chunk.
constexpr int kMinChunkGroups = 64;
int pick_chunks(int64_t items, int ngrp, int slots) {
    int best = 1;
    double best_cost = 1e300;
    for (int k = 1; k <= 8; ++k) {
        if (k > 1 && (ngrp + k - 1) / k < kMinChunkGroups) break;
        const double waves = (double)((items * k + slots - 1) / slots);
        const double cost = waves / k;
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = k;
        }
    }
    return best;
}
}  // namespace

namespace {
// Chunks per tile of a single-plan launch (INT8 only; a.nks == 1 on entry asks
// for whole segments) and their size.
void set_chunks(int xprec, XArgs &a) {
    if (a.nks != 1) a.nks = xprec == MWAX_X_INT8 ? pick_chunks((int64_t)a.ntiles * a.L, a.ngrp, resident_slots()) : 1;
    a.kchunk = (a.ngrp + a.nks - 1) / a.nks;
    a.nks = (a.ngrp + a.kchunk - 1) / a.kchunk;   // no empty chunk
}
}  // namespace

bool xengine_accumulates(int xprec, const XArgs &args) {
    if (xprec == MWAX_X_FP32) return true;
    XArgs a = args;
    set_chunks(xprec, a);
    return a.nks > 1;
}

hipError_t launch_xengine(int xprec, const XArgs &args, hipStream_t s) {
    XArgs a = args;
    set_chunks(xprec, a);
    const int64_t blocks = (int64_t)a.ntiles * a.L * a.nks;
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

hipError_t launch_xengine_batch(int xprec, const XBatchArgs &b, int grid, hipStream_t s) {
    if (grid < 1) return hipSuccess;
    switch (xprec) {
        case MWAX_X_INT8:
            hipLaunchKernelGGL(xengine_batch<MWAX_X_INT8>, dim3((unsigned)grid), dim3(kThreads), 0, s, b);
            break;
        case MWAX_X_FP16:
            hipLaunchKernelGGL(xengine_batch<MWAX_X_FP16>, dim3((unsigned)grid), dim3(kThreads), 0, s, b);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xengine_avg(int xprec, const XAvgArgs &a, hipStream_t s) {
    const int64_t blocks = (int64_t)a.N * a.ntiles;
    if (blocks <= 0 || a.ngrp <= 0) return hipSuccess;
    switch (xprec) {
        case MWAX_X_INT8:
            hipLaunchKernelGGL(xengine_avg<MWAX_X_INT8>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
            break;
        case MWAX_X_FP16:
            hipLaunchKernelGGL(xengine_avg<MWAX_X_FP16>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *p, int n, hipStream_t s) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

int xengine_batch_max_grid(int xprec, int device) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        cus = 256;
    const void *fn = xprec == MWAX_X_INT8 ? reinterpret_cast<const void *>(&xengine_batch<MWAX_X_INT8>)
                                          : reinterpret_cast<const void *>(&xengine_batch<MWAX_X_FP16>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

}  // namespace mwax
