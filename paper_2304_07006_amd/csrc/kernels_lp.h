// Reduced-precision forms of the two bulk contractions.
//
// FORM 1 : FP32 MFMA (v_mfma_f32_16x16x4_f32).
// FORM 3 : split BF16, a = a0 + a1, products a0b0 + a0b1 + a1b0
//          (v_mfma_f32_16x16x32_bf16).
// FORM 6 : split BF16, a = a0 + a1 + a2, the six products of total order <= 2.
// a0 = bf16(a), a1 = bf16(a - a0), a2 = bf16(a - a0 - a1), all round-to-nearest;
// the residuals are exact in FP32.
//
// Accumulation is FP32 inside the MFMA over a segment of the summation index
// (grid points); each segment writes an FP32 partial and a second kernel sums
// the partials in FP64 in a fixed order (deterministic, no atomics).
//
// Operands live in a "k8-packed" layout [split][n/8][ld][8]: the 8 values of
// consecutive summation indices for one output column are contiguous, which is
// exactly one lane's operand of the BF16 MFMA (A[i][k], k = 8 (l/16) + e) and
// eight consecutive k-steps of the FP32 MFMA once the summation index inside a
// 32-step is permuted as k = 8 (l/16) + e (any permutation shared by A and B
// leaves the sum unchanged).
// Output layout of both MFMAs (decoded on gfx950): lane l holds rows
// 4 (l/16) + v, v = 0..3, of column l % 16.
#pragma once
#include "xtc_device.h"

#include <type_traits>

namespace xtc {

typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

template <int FORM> struct Lp;
template <> struct Lp<1> { static constexpr int NS = 1; typedef float T; };
template <> struct Lp<3> { static constexpr int NS = 2; typedef __bf16 T; };
template <> struct Lp<6> { static constexpr int NS = 3; typedef __bf16 T; };

constexpr int kLpK = 32;          // summation indices per k-step
constexpr int kLpRows = 32;       // K build: grid rows per workgroup
constexpr int kLpCols = 512;      // K build: pair columns per workgroup (ld multiple)
// LDS row pitch (elements) of the generated d tile.  BF16: 96 bytes, which
// makes the operand reads (ds_read_b128, lane -> row l%16, 16-byte chunk l/16)
// free of bank conflicts on gfx950 (measured; 80- and 64-byte pitches cost
// two cycles per 16 lanes).  FP32: 160 bytes.
template <int FORM> struct LpARow { static constexpr int v = FORM == 1 ? 40 : 48; };

template <int NS>
__device__ __forceinline__ void split_bf16(float x, __bf16 (&t)[NS]) {
    const __bf16 b0 = (__bf16)x;
    t[0] = b0;
    if constexpr (NS > 1) {
        const float r1 = x - (float)b0;
        const __bf16 b1 = (__bf16)r1;
        t[1] = b1;
        if constexpr (NS > 2) t[2] = (__bf16)(r1 - (float)b1);
    }
}

// split_bf16 for two values at once (packed round-to-nearest conversions).
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
template <int NS>
__device__ __forceinline__ void split_bf16_pair(f2 x, bf2 (&t)[NS]) {
    t[0] = __builtin_convertvector(x, bf2);
    if constexpr (NS > 1) {
        const f2 r1 = x - __builtin_convertvector(t[0], f2);
        t[1] = __builtin_convertvector(r1, bf2);
        if constexpr (NS > 2) t[2] = __builtin_convertvector(r1 - __builtin_convertvector(t[1], f2), bf2);
    }
}

// The split products of a form as (A-term, B-term) index pairs.  Callers loop
// over terms outermost, so consecutive MFMAs write different accumulators and
// never wait on each other's results.
template <int FORM> struct Terms;
template <> struct Terms<3> {
    static constexpr int n = 3;
    static constexpr int a[3] = {0, 0, 1};
    static constexpr int b[3] = {0, 1, 0};
};
template <> struct Terms<6> {
    static constexpr int n = 6;
    static constexpr int a[6] = {0, 0, 1, 0, 1, 2};
    static constexpr int b[6] = {0, 1, 0, 2, 1, 0};
};

__device__ __forceinline__ f4 mma_bf16(const bf8& a, const bf8& b, f4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// Tile of workgroup `id` in a flat grid of nstrip column strips x n_rt row
// tiles whose workgroups all read their strip's operand.  The dispatcher
// deals workgroup i to XCD i % 8, and each XCD has its own L2: the first
// 8 floor(nstrip/8) strips are therefore dealt whole, XCD x taking strips
// x, x+8, ... with each strip's row tiles in order, so that a strip is
// fetched into one L2 and shared there by the ~32 workgroups resident on
// that XCD; the remaining strips follow in plain order (row tile fastest).
// With plain order every XCD read every strip, and the strips that straddled
// a dispatch round twice (2.3x the L2 misses of the K build at N=128).
// Dealing pays only while the eight strips in flight fit the chip-wide
// last-level cache (256 MB), which then serves each XCD's rounds on its
// strip; with larger strips (deal = false) the plain order, in which all
// XCDs read the same strip and that cache serves seven of them, is faster
// (the one-component F build, 8 x 33.5 MB strips: 74.6 against 62.7 ms).
constexpr size_t kDealBytes = (size_t)192 << 20;   // eight strips at most
__device__ __forceinline__ void xcd_strip_tile(int id, int n_rt, int nstrip, bool deal, int& rt, int& strip) {
    const int q8 = deal ? nstrip / 8 : 0;
    if (id < 8 * q8 * n_rt) {
        const int li = id / 8;
        rt = li % n_rt;
        strip = id % 8 + 8 * (li / n_rt);
    } else {
        const int i2 = id - 8 * q8 * n_rt;
        rt = i2 % n_rt;
        strip = 8 * q8 + i2 / n_rt;
    }
}

// --------------------------------------------------------------------------
// Pack an FP64 row-major array src[nrows][ld_src] (columns < ncols valid) into
// the k8-packed operand format dst[s][n8][ld_dst][8]; rows >= nrows and
// columns >= ncols become 0.
template <int FORM>
__global__ __launch_bounds__(256) void k_pack_lp(const double* __restrict__ src, int nrows, int ld_src,
                                                 int ncols, int ld_dst, void* __restrict__ dst,
                                                 size_t split_stride) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    const int g8 = blockIdx.y;
    if (P >= ld_dst) return;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int g = 8 * g8 + e;
        v[e] = (g < nrows && P < ncols) ? (float)src[(size_t)g * ld_src + P] : 0.0f;
    }
    const size_t o = ((size_t)g8 * ld_dst + P) * 8;
    if constexpr (FORM == 1) {
        f4* d = (f4*)((float*)dst + o);
        d[0] = (f4){v[0], v[1], v[2], v[3]};
        d[1] = (f4){v[4], v[5], v[6], v[7]};
    } else {
        constexpr int NS = Lp<FORM>::NS;
        bf8 out[NS];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 t[NS];
            split_bf16<NS>(v[e], t);
#pragma unroll
            for (int s = 0; s < NS; ++s) out[s][e] = t[s];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) *(bf8*)((__bf16*)dst + s * split_stride + o) = out[s];
    }
}

// --------------------------------------------------------------------------
// u'(r)/r in FP32 for the reduced forms, from the hardware reciprocal and
// reciprocal square root (about 1 ulp each; the split-BF16 operands carry
// 2^-16 .. 2^-24 relative error, so IEEE division and square root would buy
// nothing).  Exactly 0 at r^2 == 0.
template <int KIND>
__device__ __forceinline__ float du_over_r_fast(float r2, const JasDev& J);

// The same without the r^2 == 0 branch, for d^x = (x - x') u'(r)/r: the caller
// passes r^2 + kR2Floor, so the value stays finite at coincident points, where
// the difference vector it multiplies is exactly zero (d^x = 0 exactly, as the
// branch gives).  kR2Floor is far below every r^2 the grid produces between
// distinct points (it moves a distance of 1e-6 bohr by 5e-19 relative).
constexpr float kR2Floor = 1e-30f;
template <int KIND>
__device__ __forceinline__ float du_over_r_nz(float r2, const JasDev& J) {
    const float rs = __builtin_amdgcn_rsqf(r2);      // 1/r
    const float r = r2 * rs;
    if constexpr (KIND == 0) {
        const float t = __builtin_amdgcn_rcpf(fmaf(J.fb, r, 1.0f));
        return 0.5f * rs * t * t;
    } else {
        const float q = __builtin_amdgcn_rcpf(1.0f + r);
        const float t = r * q;
        float p = J.fdcoef[15];
#pragma unroll
        for (int k = 14; k >= 0; --k) p = fmaf(p, t, J.fdcoef[k]);
        return p * q * q * rs;
    }
}

template <int KIND>
__device__ __forceinline__ float du_over_r_fast(float r2, const JasDev& J) {
    const float rs = __builtin_amdgcn_rsqf(r2);      // 1/r
    const float r = r2 * rs;
    float f;
    if constexpr (KIND == 0) {
        const float t = __builtin_amdgcn_rcpf(fmaf(J.fb, r, 1.0f));
        f = 0.5f * rs * t * t;
    } else {
        const float q = __builtin_amdgcn_rcpf(1.0f + r);
        const float t = r * q;
        float p = J.fdcoef[15];
#pragma unroll
        for (int k = 14; k >= 0; --k) p = fmaf(p, t, J.fdcoef[k]);
        f = p * q * q * rs;
    }
    return r2 > 0.0f ? f : 0.0f;
}

// S = u'' + 2 u'/r + u'^2 in FP32 (the scalar kernel of the two-body TC
// integrals), same reciprocal / reciprocal square root scheme; 0 at r^2 == 0.
template <int KIND>
__device__ __forceinline__ float scalar_S_fast(float r2, const JasDev& J) {
    const float rs = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rs;
    float up, upp;
    if constexpr (KIND == 0) {
        const float it = __builtin_amdgcn_rcpf(fmaf(J.fb, r, 1.0f));
        up = 0.5f * it * it;
        upp = -J.fb * it * it * it;
    } else {
        const float q = __builtin_amdgcn_rcpf(1.0f + r);
        const float t = r * q;
        float p1 = J.fdcoef[15], p2 = J.fd2coef[15];
#pragma unroll
        for (int k = 14; k >= 0; --k) {
            p1 = fmaf(p1, t, J.fdcoef[k]);
            p2 = fmaf(p2, t, J.fd2coef[k]);
        }
        const float q2 = q * q;
        up = p1 * q2;
        upp = q2 * (p2 * q2 - 2.0f * p1 * q);
    }
    const float s = upp + 2.0f * up * rs + up * up;
    return r2 > 0.0f ? s : 0.0f;
}

// K build, reduced precision, one segment [seg*seg_len, ...) of the sum over g'.
// Workgroup: 512 threads = 8 waves, tile 32 grid rows x 512 pair columns; each
// wave owns all 32 rows x 64 columns x 3 components (2 x 4 blocks x 3 = 24 FP32
// accumulator blocks), so every pair-density value is loaded by exactly one
// wave, two waves share each SIMD, and the whole next k-step of that operand is
// prefetched into registers while the current one is multiplied.
// The d^x tile (32 rows x 32 g' x 3 components, already split) is generated
// once per k-step by all 512 threads into LDS (double buffered) and shared by
// the eight waves: generation is amortised over 512 columns.
// NC = 1 builds F = S rho instead (the scalar kernel of the two-body TC
// integrals, one component), with the same tiling.
constexpr int kLpThreads = 512;
// Column blocks of 16 per wave and pair columns per workgroup.  The
// one-component build (F) generates as much per k-step as the three-component
// one but multiplies a third as much, so in the 3-product form each wave takes
// twice the columns (8 blocks), halving the generation per MFMA (Pade
// Jastrow: the power series' two polynomials leave no registers for it).
template <int KIND, int FORM, int NC> struct LpTile {
    static constexpr int NB = (NC == 1 && FORM == 3 && KIND == 0) ? 8 : 4;
    static constexpr int cols = (kLpThreads / 64) * 16 * NB;
};
static_assert(LpTile<0, 3, 3>::cols == kLpCols && LpTile<1, 3, 3>::cols == kLpCols,
              "the K build tiles ldL = a multiple of kLpCols");
template <int KIND, int FORM, int NC = 3>
__global__ __launch_bounds__(kLpThreads) void k_build_K_lp(const d4* __restrict__ pos,
                                                           const void* __restrict__ rho_lp, size_t split_stride,
                                                           int ldL, int ngp, int g0, int rows, int n_rt,
                                                           int seg_len, JasDev J, float* __restrict__ part,
                                                           int cap, int ncol, int n_ct, int nseg) {
    typedef typename Lp<FORM>::T T;
    constexpr int NS = Lp<FORM>::NS;
    constexpr int NB = LpTile<KIND, FORM, NC>::NB;       // 16-column blocks per wave
    constexpr int kWgCols = LpTile<KIND, FORM, NC>::cols;
    // two generation buffers as distinct arrays, so the compiler can prove the
    // writes of the next k-step do not alias the reads of the current one
    constexpr int kARow = LpARow<FORM>::v;
    typedef T ATile[NC][NS][kLpRows][kARow];
    __shared__ __attribute__((aligned(16))) ATile sA0;
    __shared__ __attribute__((aligned(16))) ATile sA1;
    // positions of the 32 g' of one k-step as x[], y[], z[], pad[] (double
    // buffered).  Each wave stages its own copy with one coalesced 16-byte load
    // per lane; a wave's LDS accesses execute in order, so no barrier is
    // involved, and the copy replaces 32-fold redundant global loads.  The
    // split-BF16 forms keep them in FP32 and form the differences in FP32:
    // rounding a position (|x| < 20 bohr) to FP32 moves it by at most 1e-6
    // bohr, a relative change of d below 1e-6 for r > 1 bohr and below the
    // 2^-16 of the split operands for r > 0.07 bohr; the FP32 form, whose
    // operands keep 2^-24, takes the differences in FP64 and rounds them once.
    typedef typename std::conditional<FORM == 1, double, float>::type PosT;
    typedef PosT PTile[4][kLpK];
    __shared__ __attribute__((aligned(16))) PTile sP0[kLpThreads / 64];
    __shared__ __attribute__((aligned(16))) PTile sP1[kLpThreads / 64];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // Flat grid over strips (column tile, segment of g') x row tiles, in the
    // XCD-aware order of xcd_strip_tile, so that the ~32 workgroups resident
    // on an XCD share one strip of the operand through its L2 while they
    // advance through g' together.  Column tiles with idle waves finish early
    // and would stagger every later workgroup (and break that sharing), so
    // they are dispatched last, after all full tiles of all segments.
    const int n_full = ((n_ct - 1) * kWgCols + 7 * 16 * NB < ncol) ? n_ct : n_ct - 1;
    int rt, ct, seg;
    {
        const int id = blockIdx.x, nf = n_rt * n_full * nseg;
        if (id < nf) {
            int strip;
            const bool deal = (size_t)8 * seg_len * kWgCols * NS * sizeof(T) <= kDealBytes;
            xcd_strip_tile(id, n_rt, n_full * nseg, deal, rt, strip);
            ct = strip % n_full;
            seg = strip / n_full;
        } else {
            rt = (id - nf) % n_rt;
            seg = (id - nf) / n_rt;
            ct = n_ct - 1;
        }
    }
    const int gs = seg * seg_len;
    const int ge = min(ngp, gs + seg_len);
    // generation role: one row, two consecutive g' per k-step.  Wave w covers
    // rows 4w..4w+3, each half-wave two rows 2 apart (16 lanes per row), so
    // that the 32 lanes of a half-wave store to 32 distinct LDS banks.
    const int grow = 4 * (threadIdx.x >> 6) + 2 * ((threadIdx.x >> 4) & 1) + ((threadIdx.x >> 5) & 1);
    const int gk = 2 * (threadIdx.x & 15);
    const d4 pr = pos[g0 + min(rt * kLpRows + grow, rows - 1)];
    const PosT prx = (PosT)pr.x, pry = (PosT)pr.y, prz = (PosT)pr.z;
    // MFMA role
    const int l16 = lane & 15, lk = lane >> 4;
    const int col0 = ct * kWgCols + wave * 16 * NB + l16;
    // waves whose columns all lie at or beyond ncol (never read) only help
    // to generate the shared tiles: no operand loads, MFMAs or stores
    const bool active = ct * kWgCols + wave * 16 * NB < ncol;

    f4 acc[NC][2][NB];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[c][h][b] = (f4){0.f, 0.f, 0.f, 0.f};

    // position staging: lane l holds half (x,y or z,pad) of position l/2 of a
    // k-step, loaded one k-step before it is stored to LDS (no branches, so the
    // wait for it does not also wait for the operand prefetch)
    // (addresses: a uniform base per k-step plus a fixed 32-bit lane offset,
    // so the address arithmetic stays scalar)
    const int sq = lane >> 1, shalf = lane & 1;
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    typedef PosT pos2 __attribute__((ext_vector_type(2)));
    const uint32_t s_off = (uint32_t)((4 * sq + 2 * shalf) * sizeof(double));
    dbl2 pstage;
    auto loadS = [&](int kk) {
        const char* ub = (const char*)pos + (size_t)kk * 4 * sizeof(double);
        pstage = *(const dbl2*)(ub + s_off);
    };
    auto storeS = [&](PTile& P, const dbl2 v) {
        P[2 * shalf][sq] = (PosT)v.x;
        P[2 * shalf + 1][sq] = (PosT)v.y;
    };
    auto gen = [&](const PTile& P, ATile& W) {
        const pos2 px = *(const pos2*)&P[0][gk], py = *(const pos2*)&P[1][gk], pz = *(const pos2*)&P[2][gk];
        float a[NC][2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float dx = (float)(prx - px[j]), dy = (float)(pry - py[j]), dz = (float)(prz - pz[j]);
            if constexpr (NC == 3) {
                const float f = du_over_r_nz<KIND>(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, kR2Floor))), J);
                a[0][j] = dx * f;
                a[1][j] = dy * f;
                a[2][j] = dz * f;
            } else {
                a[0][j] = scalar_S_fast<KIND>(fmaf(dx, dx, fmaf(dy, dy, dz * dz)), J);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (FORM == 1) {
                W[c][0][grow][gk] = a[c][0];
                W[c][0][grow][gk + 1] = a[c][1];
            } else {
                // the two g' of the lane split together: one packed conversion
                // per piece, and each piece stored as one 32-bit word
                bf2 t[NS];
                split_bf16_pair<NS>((f2){a[c][0], a[c][1]}, t);
#pragma unroll
                for (int s = 0; s < NS; ++s) *(bf2*)&W[c][s][grow][gk] = t[s];
            }
        }
    };

    // pair-density operand of the wave's 4 column blocks for one k-step
    typedef typename std::conditional<FORM == 1, f4[NB][2], bf8[NB][NS]>::type BOp;
    const uint32_t b_off = (uint32_t)(((size_t)lk * ldL + col0) * 8 * sizeof(T));   // lane offset, bytes
    auto loadB = [&](int kk, BOp& out) {
        const char* ub = (const char*)rho_lp + (size_t)(kk / 8) * ldL * 8 * sizeof(T);   // uniform
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if constexpr (FORM == 1) {
                const f4* p = (const f4*)(ub + b_off + 128 * b * sizeof(T));
                out[b][0] = p[0];
                out[b][1] = p[1];
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    out[b][s] = *(const bf8*)(ub + s * split_stride * sizeof(T) + b_off + 128 * b * sizeof(T));
            }
        }
    };

    BOp bnext;
    // one k-step: multiply the tile in R (and the operand prefetched in bnext)
    // while generating the next tile into W from the positions in PR,
    // prefetching the next operand, storing the positions two k-steps ahead
    // into PW and loading those three k-steps ahead
    auto step = [&](auto act, int kk, const ATile& R, ATile& W, const PTile& PR, PTile& PW) {
        constexpr bool ACT = decltype(act)::value;
        // next k-steps (near the end of the segment these re-read the last one
        // into idle buffers that are never consumed: no branch in the loop body)
        const int kn = min(kk + kLpK, ge - kLpK);
        const int kn3 = min(kk + 3 * kLpK, ge - kLpK);
        const dbl2 pst = pstage;   // positions two k-steps ahead (loaded last step)
        // the global loads for later k-steps are issued before anything else
        // of this step, so they have a whole k-step to arrive (without the
        // scheduling fence the compiler sinks them to the end of the step)
        loadS(kn3);
        if constexpr (!ACT) {
            gen(PR, W);
            storeS(PW, pst);
            return;
        }
        BOp bv;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int s = 0; s < (FORM == 1 ? 2 : NS); ++s) bv[b][s] = bnext[b][s];
        loadB(kn, bnext);
        // (the six-product form has no registers to spare for the longer live ranges)
        if constexpr (FORM != 6) __builtin_amdgcn_sched_barrier(0);
        if constexpr (FORM == 1) {
            gen(PR, W);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float av[NC][8];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const f4 x0 = *(const f4*)&R[c][0][16 * h + l16][8 * lk];
                    const f4 x1 = *(const f4*)&R[c][0][16 * h + l16][8 * lk + 4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) { av[c][e] = x0[e]; av[c][4 + e] = x1[e]; }
                }
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float be = e < 4 ? bv[b][0][e] : bv[b][1][e - 4];
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            acc[c][h][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c][e], be, acc[c][h][b], 0, 0, 0);
                    }
            }
        } else {
            gen(PR, W);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                bf8 av[NC][NS];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int s = 0; s < NS; ++s) av[c][s] = *(const bf8*)&R[c][s][16 * h + l16][8 * lk];
#pragma unroll
                for (int t = 0; t < Terms<FORM>::n; ++t)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            acc[c][h][b] = mma_bf16(av[c][Terms<FORM>::a[t]], bv[b][Terms<FORM>::b[t]], acc[c][h][b]);
            }
        }
        // the positions loaded one step ago go to LDS last, so the wait for
        // them never waits for this step's operand prefetch
        storeS(PW, pst);
        // instruction order: operand reads (and the three position reads of the
        // generation) first, then every MFMA paired with generation VALU work
        // for the next k-step
        constexpr int kMfmaHalf = (FORM == 1 ? 8 : (FORM == 3 ? 3 : 6)) * NC * NB;
        constexpr int kValuPer = FORM == 1 ? 1 : 2;
        __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __builtin_amdgcn_sched_group_barrier(0x100, NC * NS * (FORM == 1 ? 2 : 1), 0);
#pragma unroll
            for (int i = 0; i < kMfmaHalf; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, kValuPer, 0);
            }
        }
    };

    // prologue: positions of k-steps 0 and 1 to LDS, of k-step 2 to registers,
    // tile 0 generated
    loadB(gs, bnext);
    loadS(gs);
    storeS(sP0[wave], pstage);
    loadS(min(gs + kLpK, ge - kLpK));
    storeS(sP1[wave], pstage);
    loadS(min(gs + 2 * kLpK, ge - kLpK));
    gen(sP0[wave], sA0);
    __syncthreads();
    // (ge - gs) is a multiple of 2 k-steps: segments and the padded grid are
    // multiples of 64 points.  Step kk reads tile kk, generates tile kk+1 from
    // the positions stored one step earlier, and overwrites the position
    // buffer that the previous step's generation read.
    // (active is uniform per wave; both loops pass the same barriers)
    if (active) {
        for (int kk = gs; kk < ge; kk += 2 * kLpK) {
            step(std::true_type{}, kk, sA0, sA1, sP1[wave], sP0[wave]);
            __syncthreads();
            step(std::true_type{}, kk + kLpK, sA1, sA0, sP0[wave], sP1[wave]);
            __syncthreads();
        }
    } else {
        for (int kk = gs; kk < ge; kk += 2 * kLpK) {
            step(std::false_type{}, kk, sA0, sA1, sP1[wave], sP0[wave]);
            __syncthreads();
            step(std::false_type{}, kk + kLpK, sA1, sA0, sP0[wave], sP1[wave]);
            __syncthreads();
        }
        return;
    }

    const size_t cstride = (size_t)cap * ldL;
    float* out = part + (size_t)seg * NC * cstride;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rt * kLpRows + 16 * h + 4 * lk + v;
            if (r < rows) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        out[c * cstride + (size_t)r * ldL + col0 + 16 * b] = acc[c][h][b][v];
            }
        }
}

// K[c][r][P] = sum_s part[s][c][r][P] in FP64 (fixed order), for c < nc, r < rows, P < ldP;
// K's components are krows rows apart (a piece of a longer chunk).
__global__ void k_reduce_K(const float* __restrict__ part, int nseg, int cap, int ldL, int rows, int ldP,
                           double* __restrict__ K, int krows, int nc) {
    // four consecutive pairs per thread (ldP, ldL and the component strides are
    // multiples of 4): 16-byte partial loads, 32-byte stores, same summation order
    const size_t n4 = (size_t)nc * rows * (ldP / 4);
    const size_t cstride = (size_t)cap * ldL;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        const int P = (int)(i % (ldP / 4)) * 4;
        const size_t cr = i / (ldP / 4);
        const int r = (int)(cr % rows), c = (int)(cr / rows);
        const size_t o = c * cstride + (size_t)r * ldL + P;
        d4 s = (d4){0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < nseg; ++q) {
            const f4 v = *(const f4*)(part + (size_t)q * nc * cstride + o);
            s += (d4){(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
        }
        *(d4*)(K + ((size_t)c * krows + r) * ldP + P) = s;
    }
}

// --------------------------------------------------------------------------
// Transposed product over grid rows in reduced precision (the two-body
// assembly and the TC integral contractions), FP32 partials per row segment:
//   part[y][P][R] = sum_{c in group} sum_{g in segment} C_c[g][P] D_c[g][R]
// with y = group * nseg_r + segment, group = cpw consecutive components.
// Clp: [comps][NS][n8][ldC][8], one split c_split elements apart;
// Dlp: [comps][NS][n8][ldD][8], d_split apart; part[y] is ldC x ldD.
// Workgroup tile 128 (P) x 256 (R), waves 2 x 2 of 64 x 128 (4 x 8 MFMA
// blocks); n_pt = ldC / 128 tiles along P, ldD / 256 along R.  Only P < pmax,
// R < rmax are read by the reduction: tiles entirely beyond do nothing.
template <int FORM>
__global__ __launch_bounds__(256) void k_gemm_tn_lp(const void* __restrict__ Clp, int ldC, size_t c_split,
                                                    const void* __restrict__ Dlp, int ldD, size_t d_split,
                                                    int rows32, int n_pt, int pmax, int rmax, int cpw,
                                                    int seg_len, int nseg_r, float* __restrict__ part) {
    constexpr int NS = Lp<FORM>::NS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pt = blockIdx.x % n_pt, rt = blockIdx.x / n_pt;
    if (pt * 128 >= pmax || rt * 256 >= rmax) return;
    const int c0 = (blockIdx.y / nseg_r) * cpw, sg = blockIdx.y % nseg_r;
    const int gs = sg * seg_len, ge = min(rows32, gs + seg_len);
    const int l16 = lane & 15, lk = lane >> 4;
    const int P0 = pt * 128 + 64 * (wave & 1) + l16;
    const int R0 = rt * 256 + 128 * (wave >> 1) + l16;
    f4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
    for (int comp = c0; comp < c0 + cpw; ++comp)
    for (int kk = gs; kk < ge; kk += kLpK) {
        const size_t crow = (size_t)(kk / 8 + lk) * ldC;
        const size_t drow = (size_t)(kk / 8 + lk) * ldD;
        if constexpr (FORM == 1) {
            const float* Cb = (const float*)Clp + comp * NS * c_split;
            const float* Db = (const float*)Dlp + comp * NS * d_split;
            float av[4][8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const f4* p = (const f4*)(Cb + (crow + P0 + 16 * i) * 8);
                const f4 x0 = p[0], x1 = p[1];
                av[i][0] = x0[0]; av[i][1] = x0[1]; av[i][2] = x0[2]; av[i][3] = x0[3];
                av[i][4] = x1[0]; av[i][5] = x1[1]; av[i][6] = x1[2]; av[i][7] = x1[3];
            }
#pragma unroll
            for (int jh = 0; jh < 8; jh += 4) {
                float bv[4][8];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const f4* p = (const f4*)(Db + (drow + R0 + 16 * (jh + j)) * 8);
                    const f4 y0 = p[0], y1 = p[1];
#pragma unroll
                    for (int e = 0; e < 4; ++e) { bv[j][e] = y0[e]; bv[j][4 + e] = y1[e]; }
                }
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            acc[i][jh + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][e], bv[j][e], acc[i][jh + j], 0, 0, 0);
            }
        } else {
            const __bf16* Cb = (const __bf16*)Clp + comp * NS * c_split;
            const __bf16* Db = (const __bf16*)Dlp + comp * NS * d_split;
            bf8 av[4][NS];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int s = 0; s < NS; ++s) av[i][s] = *(const bf8*)(Cb + s * c_split + (crow + P0 + 16 * i) * 8);
#pragma unroll
            for (int jh = 0; jh < 8; jh += 4) {
                bf8 bv[4][NS];
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        bv[j][s] = *(const bf8*)(Db + s * d_split + (drow + R0 + 16 * (jh + j)) * 8);
#pragma unroll
                for (int t = 0; t < Terms<FORM>::n; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            acc[i][jh + j] = mma_bf16(av[i][Terms<FORM>::a[t]], bv[j][Terms<FORM>::b[t]], acc[i][jh + j]);
            }
        }
    }
    float* out = part + (size_t)blockIdx.y * ldC * ldD;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int P = P0 - l16 + 16 * i + 4 * lk + v;
#pragma unroll
            for (int j = 0; j < 8; ++j) out[(size_t)P * ldD + R0 + 16 * j] = acc[i][j][v];
        }
}

// The same product in split BF16 with both operands staged in LDS.
// Workgroup 512 threads = 8 waves as 4 (P) x 2 (R), tile 256 (P) x 256 (R),
// wave tile 64 x 128 (4 x 8 MFMA blocks, as in k_gemm_tn_lp).  Per k-step (32
// grid rows) the k8-packed tiles of C and D (256 columns each, all splits)
// are copied into LDS by direct 16-byte global-to-LDS loads (no registers
// involved), issued one k-step ahead, and read by the 2 (C) and 4 (D) waves
// that share them, instead of every wave fetching its own.  An LDS row (one
// 8-row group of one split, 256 columns x 16 bytes, 4 KB contiguous in
// global memory) is padded by 128 bytes, so each 16-lane phase of a b128
// read covers all 64 banks.  The two k-step buffers are separate objects,
// each named statically where it is filled or read (the k-step loop runs
// two k-steps per iteration): the compiler then knows that the reads of one
// need not wait for the loads into the other.
// Tiles are dealt to the XCDs (workgroup x runs on XCD x % 8) in contiguous
// ranges of a banded order (bands of kTnBand P tiles, R fastest within a
// band), so the ~32 workgroups resident on an XCD cover about 4 P x 8 R
// tiles and share 12 operand strips through its L2.
// ldC and ldD are multiples of 256; (component, grid row) k-steps of a
// workgroup's group and segment run as one sequence.
constexpr int kTnThreads = 512;
constexpr int kTnBand = 4;
template <int FORM>
__global__ __launch_bounds__(kTnThreads) void k_gemm_tn_lds(const void* __restrict__ Clp, int ldC, size_t c_split,
                                                            const void* __restrict__ Dlp, int ldD, size_t d_split,
                                                            int rows32, int n_pt, int n_rt, int per_xcd, int pmax,
                                                            int rmax, int cpw, int seg_len, int nseg_r,
                                                            float* __restrict__ part) {
    static_assert(FORM == 3 || FORM == 6, "split-BF16 forms only");
    typedef __attribute__((address_space(3))) void* lds_ptr;
    constexpr int NS = Lp<FORM>::NS;
    constexpr int kRowB = 256 * 16 + 128;           // bytes of one (split, 8-row group) LDS row
    constexpr int kTileB = NS * 4 * kRowB;          // one operand's tile of one k-step
    constexpr int kChunks = 2 * NS * 4 * 4;         // 1 KB direct-load chunks per k-step (both operands)
    constexpr int kPerW = kChunks / 8;              // per wave
    __shared__ __attribute__((aligned(1024))) char sm0[2 * kTileB];   // C, then D, of even k-steps
    __shared__ __attribute__((aligned(1024))) char sm1[2 * kTileB];   // odd k-steps
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int pt, rt;
    {
        const int loc = blockIdx.x >> 3, t = (blockIdx.x & 7) * per_xcd + loc;
        if (loc >= per_xcd || t >= n_pt * n_rt) return;
        const int band = min(t / (kTnBand * n_rt), (n_pt - 1) / kTnBand);
        const int r = t - band * kTnBand * n_rt;
        const int gw = min(kTnBand, n_pt - band * kTnBand);
        pt = band * kTnBand + r % gw;
        rt = r / gw;
    }
    if (pt * 256 >= pmax || rt * 256 >= rmax) return;
    const int c0 = (blockIdx.y / nseg_r) * cpw, sg = blockIdx.y % nseg_r;
    const int gs = sg * seg_len, ge = min(rows32, gs + seg_len);
    const int nk = (ge - gs) / kLpK;                // k-steps per component
    const int nq = nk * cpw;
    const int l16 = lane & 15, lk = lane >> 4;
    const int wp = wave & 3, wr = wave >> 2;
    const uint32_t loff = 16 * lane;

    // chunk j = wave + 8 i (i < kPerW / 2) of each operand's tile: LDS row
    // (split, 8-row group) j / 4 = wave / 4 + 2 i, its 1 KB piece wave % 4
    const uint32_t lpiece = 1024 * (wave & 3) + loff;
    const char* cbase = (const char*)Clp + (size_t)pt * 256 * 16;
    const char* dbase = (const char*)Dlp + (size_t)rt * 256 * 16;
    auto issue = [&](int q, char* buf) {
        const int comp = c0 + q / nk, g8 = (gs + kLpK * (q % nk)) / 8;
#pragma unroll
        for (int i = 0; i < kPerW / 2; ++i) {
            const int row = (wave >> 2) + 2 * i, sp = row >> 2, gg = row & 3;
            const char* cs = cbase + ((size_t)comp * NS + sp) * c_split * 2 + (size_t)(g8 + gg) * ldC * 16;
            const char* ds = dbase + ((size_t)comp * NS + sp) * d_split * 2 + (size_t)(g8 + gg) * ldD * 16;
            char* dst = buf + row * kRowB + 1024 * (wave & 3);
            __builtin_amdgcn_global_load_lds((const void*)(cs + lpiece), (lds_ptr)dst, 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(ds + lpiece), (lds_ptr)(dst + kTileB), 16, 0, 0);
        }
    };

    f4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
    auto multiply = [&](const char* buf) {
        bf8 av[4][NS];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int s = 0; s < NS; ++s)
                av[i][s] = *(const bf8*)&buf[(s * 4 + lk) * kRowB + (64 * wp + 16 * i + l16) * 16];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            bf8 bv[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s)
                bv[s] = *(const bf8*)&buf[kTileB + (s * 4 + lk) * kRowB + (128 * wr + 16 * j + l16) * 16];
#pragma unroll
            for (int t = 0; t < Terms<FORM>::n; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = mma_bf16(av[i][Terms<FORM>::a[t]], bv[Terms<FORM>::b[t]], acc[i][j]);
        }
        __builtin_amdgcn_s_waitcnt(0);              // this wave's loads of the next k-step
        __syncthreads();                            // everyone's, and this k-step read by all
    };
    if (nq > 0) {
        issue(0, sm0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    // even k-steps from sm0, odd ones from sm1, each k-step's successor
    // loaded into the other buffer while it is multiplied; an odd last k-step
    // (in sm0) after the loop
    int q = 0;
    for (; q + 1 < nq; q += 2) {
        issue(q + 1, sm1);
        multiply(sm0);
        if (q + 2 < nq) issue(q + 2, sm0);
        multiply(sm1);
    }
    if (q < nq) multiply(sm0);
    float* out = part + (size_t)blockIdx.y * ldC * ldD;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int P = pt * 256 + 64 * wp + 16 * i + 4 * lk + v;
#pragma unroll
            for (int j = 0; j < 8; ++j) out[(size_t)P * ldD + rt * 256 + 128 * wr + 16 * j + l16] = acc[i][j][v];
        }
}

// M[P][R] (+)= sum_s part[s][P][R] in FP64 (fixed order), P < pmax, R < rmax;
// part[s] has leading dimension ldpart and starts sstride floats after part[s-1].
__global__ void k_reduce_M(const float* __restrict__ part, int nseg, size_t sstride, int ldpart, int pmax, int rmax,
                           double* __restrict__ M, int ldM, int accumulate) {
    // four consecutive R per thread (rmax, ldpart, ldM and sstride are multiples
    // of 4): 16-byte partial loads, 32-byte accumulator accesses
    const size_t n4 = (size_t)pmax * (rmax / 4);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        const size_t P = i / (rmax / 4), R = (i % (rmax / 4)) * 4;
        const size_t o = P * ldpart + R;
        d4* m = (d4*)(M + P * ldM + R);
        d4 s = accumulate ? *m : (d4){0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < nseg; ++q) {
            const f4 v = *(const f4*)(part + q * sstride + o);
            s += (d4){(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
        }
        *m = s;
    }
}

// --------------------------------------------------------------------------
// Occupied-occupied pairs: colmap[j] = pair(occ[a], occ[b]) for a <= b (j in
// row-major order of (a, b)); rho_occ = rho[g][colmap[j]] in column tiles of
// tw pairs, tile-major ([ldO / tw][ngp][tw]), zero padded.
__global__ void k_occ_pairs(OccList occ, int N, int* __restrict__ colmap, int ldO) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ldO) return;
    const int n = occ.n;
    const int npair = n * (n + 1) / 2;
    if (j >= npair) { colmap[j] = -1; return; }
    int a = 0, rem = j;
    while (rem >= n - a) { rem -= n - a; ++a; }
    const int b = a + rem;
    colmap[j] = pair_sym(occ.k[a], occ.k[b], N);
}

// K[x][r][colmap[j]] = sum_s part[s][x][r][j] (FP64, fixed order), j < nmap.
__global__ void k_reduce_occ(const double* __restrict__ part, int nseg, int rows, int ldO, const int* __restrict__ colmap,
                             int nmap, int ldP, double* __restrict__ K) {
    const size_t n = (size_t)3 * rows * nmap;
    const size_t sstride = (size_t)3 * rows * ldO;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % nmap);
        const size_t xr = i / nmap;                  // x * rows + r
        double s = 0.0;
        for (int q = 0; q < nseg; ++q) s += part[q * sstride + xr * ldO + j];
        const int x = (int)(xr / rows), r = (int)(xr % rows);
        K[((size_t)x * rows + r) * ldP + colmap[j]] = s;
    }
}

__global__ void k_gather_occ(const double* __restrict__ rho, int ldP, int ngp, const int* __restrict__ colmap,
                             int ldO, int tw, double* __restrict__ rho_occ) {
    // column tiles of tw pairs, each [ngp][tw] contiguous: rho_occ[(j / tw) ngp tw + g tw + j % tw]
    const size_t n = (size_t)ngp * ldO;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % ldO);
        const size_t g = i / ldO;
        const int P = colmap[j];
        rho_occ[((size_t)(j / tw) * ngp + g) * tw + j % tw] = P >= 0 ? rho[g * ldP + P] : 0.0;
    }
}

}  // namespace xtc

namespace xtc {

// --------------------------------------------------------------------------
// Row-major split copy: dst[s][r][c] = term s of src[r][c] (r < rows, c < ld),
// used for the operands of the reduced-precision Pi contraction, whose
// summation index (the pair) is the contiguous one.
template <int FORM>
__global__ void k_split_rows(const double* __restrict__ src, size_t n, void* __restrict__ dst, size_t split_stride) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float v = (float)src[i];
        if constexpr (FORM == 1) {
            ((float*)dst)[i] = v;
        } else {
            constexpr int NS = Lp<FORM>::NS;
            __bf16 t[NS];
            split_bf16<NS>(v, t);
#pragma unroll
            for (int s = 0; s < NS; ++s) ((__bf16*)dst)[s * split_stride + i] = t[s];
        }
    }
}

// Split an FP64 row-major array src[nrows][ld] (ld a multiple of 8) into the
// k-packed operand format of k_nt_bf16, dst[s][ld/8][nrows][8]: element
// (j, k) goes to dst[s][k/8][j][k%8], so that the 8 consecutive k a lane
// multiplies are one 16-byte vector and 16 consecutive rows of one 8-k group
// are 256 contiguous bytes (row-major splits put them 2 ld bytes apart).
template <int FORM>
__global__ __launch_bounds__(256) void k_pack_kmajor(const double* __restrict__ src, int nrows, int ld,
                                                     __bf16* __restrict__ dst, size_t split_stride) {
    static_assert(FORM == 3 || FORM == 6, "split-BF16 forms only");
    constexpr int NS = Lp<FORM>::NS;
    const size_t n = (size_t)nrows * (ld / 8);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t j = i % nrows, k8 = i / nrows;      // consecutive threads: consecutive rows (16-byte stores)
        const d4* p = (const d4*)(src + j * ld + 8 * k8);
        const d4 x0 = p[0], x1 = p[1];
        bf8 out[NS];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 t[NS];
            split_bf16<NS>((float)(e < 4 ? x0[e] : x1[e - 4]), t);
#pragma unroll
            for (int q = 0; q < NS; ++q) out[q][e] = t[q];
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) *(bf8*)(dst + q * split_stride + (k8 * nrows + j) * 8) = out[q];
    }
}

// Gradient epilogue of one Pi value: dL/dc_j gains j t^(j-1) q^2 / r times
// (r_g - r_g') . Pi(g,g') (power Jastrow, u' = sum_j j c_j t^(j-1) q^2 with
// t = r q, q = 1/(1+r)); FP64, coincident points skipped.
__device__ __forceinline__ void pi_grad_point(const d4& pi, const d4& pj, float px, float py, float pz,
                                              double (&gsum)[16]) {
    const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (!(r2 > 0.0)) return;
    const double r = sqrt(r2);
    const double q = 1.0 / (1.0 + r);
    const double t = r * q;
    double tp = (dx * (double)px + dy * (double)py + dz * (double)pz) * q * q / r;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        gsum[j] = fma((double)(j + 1), tp, gsum[j]);
        tp *= t;
    }
}

// FP32 Pi tiles with the gradient epilogue (see k_pi_grad):
// Pi^x(g,g') = sum_P Kbar^x[g][P] rho[g'][P] with FP32 accumulation over all
// pairs; workgroup 4 waves as 2 (g) x 2 (g'), wave tile 16 g x 128 g' x 3.
// Kb: [3][rows][ldP], rr: [ngp][ldP] (row-major).  The split-BF16 forms use
// k_nt_bf16.
template <int FORM>
__global__ __launch_bounds__(256) void k_pi_grad_lp(const void* __restrict__ Kb, size_t kb_comp, size_t kb_split,
                                                    int rows, const void* __restrict__ rr, size_t rr_split,
                                                    int ldP, const d4* __restrict__ pos, int g0, int ngp, int n_jt,
                                                    int ncoef, double* __restrict__ part) {
    static_assert(FORM == 1, "FP32 form only");
    constexpr int NB = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int it = blockIdx.x / n_jt, jt = blockIdx.x % n_jt;
    const int i0 = it * 32 + 16 * (wave & 1), j0 = jt * 256 + 128 * (wave >> 1);
    const int l16 = lane & 15, kq = 8 * (lane >> 4);
    f4 acc[3][NB];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[x][b] = (f4){0.f, 0.f, 0.f, 0.f};
    const size_t irow = (size_t)min(i0 + l16, rows - 1);
    size_t jrow[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) jrow[b] = (size_t)min(j0 + 16 * b + l16, ngp - 1);
    for (int k = 0; k < ldP; k += kLpK) {
        const float* A = (const float*)Kb;
        const float* B = (const float*)rr;
        float av[3][8];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const f4* p = (const f4*)(A + x * kb_comp + irow * ldP + k + kq);
            const f4 y0 = p[0], y1 = p[1];
#pragma unroll
            for (int e = 0; e < 4; ++e) { av[x][e] = y0[e]; av[x][4 + e] = y1[e]; }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const f4* p = (const f4*)(B + jrow[b] * ldP + k + kq);
            const f4 y0 = p[0], y1 = p[1];
            const float bv[8] = {y0[0], y0[1], y0[2], y0[3], y1[0], y1[1], y1[2], y1[3]};
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int x = 0; x < 3; ++x)
                    acc[x][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x][e], bv[e], acc[x][b], 0, 0, 0);
        }
    }
    double gsum[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) gsum[j] = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * (lane >> 4) + v;          // FP32/BF16 MFMA output rows: 4 (l/16) + v
        if (i >= rows) continue;
        const d4 pi = pos[g0 + i];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int jg = j0 + 16 * b + l16;
            if (jg >= ngp) continue;
            pi_grad_point(pi, pos[jg], acc[0][b][v], acc[1][b][v], acc[2][b][v], gsum);
        }
    }
    __shared__ double red[4][16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        double v = gsum[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < 16 && threadIdx.x < ncoef)
        part[(size_t)blockIdx.x * 16 + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}


// Split-BF16 NT product out_c[i][j] = sum_k A_c[i][k] B[j][k] over NC
// components sharing B, staged like the K build: workgroup 512 threads = 8
// waves, tile 32 rows (i) x 512 columns (j), k-steps of 32.  Each k-step's
// split A tile (NC components x NS x 32 rows x 32 k) is loaded once by the
// whole workgroup into LDS (double buffered, the 96-byte row pitch of the K
// build) and shared by the eight waves; each wave loads B for its own 64
// columns (16 bytes per lane) one k-step ahead and owns 32 x 64 x NC FP32
// accumulators, so every operand value is fetched once per workgroup.  FP32
// accumulation over the whole k range.
// A: [NC][NS][ldk/8][rows][8] (component stride a_comp, split stride a_split),
// B: [NS][ldk/8][nB][8] (split stride b_split), both k-packed (k_pack_kmajor):
// each 16-byte operand vector and each 16-row block of one 8-k group is
// contiguous.  ldk is a multiple of 64.  Grid: n_rt x ceil(nB / 512) in the
// XCD-aware order of xcd_strip_tile, so the workgroups resident on an XCD
// share one B strip through its L2.
// Epilogues:
//  GRAD (NC = 3, the Pi contraction Pi^x(g,g') = sum_P Kbar^x[g][P] rho[g'][P]
//   with i = g - g0, j = g'): the gradient terms of every (g, g'), summed per
//   workgroup into part[blockIdx.x][16];
//  otherwise: out[c][i][j] = FP64 value (added to out with accumulate),
//   i < rows, j < nB (out + c * out_comp, leading dimension ldo).
constexpr int kPiThreads = 512;
template <int FORM, int NC, bool GRAD>
__global__ __launch_bounds__(kPiThreads) void k_nt_bf16(const __bf16* __restrict__ A, size_t a_comp, size_t a_split,
                                                        int rows, const __bf16* __restrict__ B, size_t b_split,
                                                        int nB, int ldk, int n_rt, const d4* __restrict__ pos,
                                                        int g0, int ncoef, double* __restrict__ out,
                                                        size_t out_comp, int ldo, int accumulate) {
    static_assert(FORM == 3 || FORM == 6, "split-BF16 forms only");
    static_assert(!GRAD || NC == 3, "the gradient epilogue takes the three components of Pi");
    constexpr int NS = Lp<FORM>::NS;
    constexpr int NB = 4;                              // 16-column blocks per wave
    constexpr int kARow = LpARow<FORM>::v;
    typedef __bf16 ATile[NC][NS][kLpRows][kARow];
    __shared__ __attribute__((aligned(16))) ATile sA0;
    __shared__ __attribute__((aligned(16))) ATile sA1;
    constexpr int kAVec = NC * NS * kLpRows * (kLpK / 8);         // 16-byte vectors of one tile
    constexpr int kAPer = (kAVec + kPiThreads - 1) / kPiThreads;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int rt, jt;
    const bool deal = (size_t)8 * ldk * 512 * NS * sizeof(__bf16) <= kDealBytes;
    xcd_strip_tile(blockIdx.x, n_rt, gridDim.x / n_rt, deal, rt, jt);   // strips: 512-column tiles of B
    const int l16 = lane & 15, lk = lane >> 4;

    // loader role: vector v = tid + 512 i is (component-split cs, 8-k chunk q,
    // row), rows fastest: the 32 rows of one chunk are 512 contiguous bytes
    const __bf16* asrc[kAPer];
    int adst[kAPer];
    bool aon[kAPer];
#pragma unroll
    for (int i = 0; i < kAPer; ++i) {
        const int v = threadIdx.x + kPiThreads * i;
        aon[i] = v < kAVec;
        const int row = v & (kLpRows - 1), q = (v >> 5) & 3, cs = aon[i] ? v >> 7 : 0;
        asrc[i] = A + (cs / NS) * a_comp + (cs % NS) * a_split +
                  ((size_t)q * rows + min(rt * kLpRows + row, rows - 1)) * 8;
        adst[i] = (cs * kLpRows + row) * kARow + 8 * q;
    }
    bf8 apre[kAPer];
    // the 8-k group k/8 starts k * rows elements in (k a multiple of 32)
    auto loadA = [&](int k) {
#pragma unroll
        for (int i = 0; i < kAPer; ++i)
            if (aon[i]) apre[i] = *(const bf8*)(asrc[i] + (size_t)k * rows);
    };
    auto storeA = [&](ATile& W) {
#pragma unroll
        for (int i = 0; i < kAPer; ++i)
            if (aon[i]) *(bf8*)(&W[0][0][0][0] + adst[i]) = apre[i];
    };
    // MFMA role: the wave's 64 columns (clamped; columns >= nB are never written)
    const int jbase = jt * (kPiThreads / 64) * 64 + wave * 64;
    const __bf16* bsrc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) bsrc[b] = B + ((size_t)lk * nB + min(jbase + 16 * b + l16, nB - 1)) * 8;
    bf8 bnext[NB][NS];
    auto loadB = [&](int k) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int s = 0; s < NS; ++s) bnext[b][s] = *(const bf8*)(bsrc[b] + s * b_split + (size_t)k * nB);
    };

    f4 acc[NC][2][NB];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[c][h][b] = (f4){0.f, 0.f, 0.f, 0.f};

    // per (row half, component): its split operand from LDS, then the split
    // products over the wave's 4 column blocks (consecutive MFMAs write
    // different accumulators)
    auto multiply = [&](const ATile& R, const bf8 (&bv)[NB][NS]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bf8 av[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) av[s] = *(const bf8*)&R[c][s][16 * h + l16][8 * lk];
#pragma unroll
                for (int t = 0; t < Terms<FORM>::n; ++t)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[c][h][b] = mma_bf16(av[Terms<FORM>::a[t]], bv[b][Terms<FORM>::b[t]], acc[c][h][b]);
            }
    };
    // one k-step: multiply tile R with the operand in bnext while loading the
    // next k-step (at the last step the last one again, into a buffer that is
    // never read: no branch in the loop body).  The six-product form has no
    // registers for two k-steps of its operand: it loads the next one after
    // the MFMAs are issued.
    auto step = [&](int k, const ATile& R, ATile& W) {
        const int kn = min(k + kLpK, ldk - kLpK);
        loadA(kn);
        if constexpr (FORM == 3) {
            bf8 bv[NB][NS];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int s = 0; s < NS; ++s) bv[b][s] = bnext[b][s];
            loadB(kn);
            multiply(R, bv);
        } else {
            multiply(R, bnext);
            loadB(kn);
        }
        storeA(W);
    };
    if constexpr (FORM == 3 && NC == 3) {
        // one barrier per two k-steps (four components have no registers for
        // the second B operand): a stage multiplies the two LDS tiles
        // of steps k and k + 1 while the tiles of k + 2 and k + 3 are written
        // to the other two buffers (four statically named buffers, two stages
        // per loop iteration); B of step k + 1 is loaded at the stage's start,
        // B of step k + 2 (the next stage's first) between its two halves
        __shared__ __attribute__((aligned(16))) ATile sA2;
        __shared__ __attribute__((aligned(16))) ATile sA3;
        bf8 aQ[kAPer], bQ[NB][NS];
        auto loadA_to = [&](int k, bf8 (&dst)[kAPer]) {
#pragma unroll
            for (int i = 0; i < kAPer; ++i)
                if (aon[i]) dst[i] = *(const bf8*)(asrc[i] + (size_t)min(k, ldk - kLpK) * rows);
        };
        auto storeA_from = [&](ATile& W, const bf8 (&src)[kAPer]) {
#pragma unroll
            for (int i = 0; i < kAPer; ++i)
                if (aon[i]) *(bf8*)(&W[0][0][0][0] + adst[i]) = src[i];
        };
        auto loadB_to = [&](int k, bf8 (&dst)[NB][NS]) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    dst[b][s] = *(const bf8*)(bsrc[b] + s * b_split + (size_t)min(k, ldk - kLpK) * nB);
        };
        // stage over steps k, k + 1 from tiles R0, R1; tiles of k + 2, k + 3
        // into W0, W1; bnext holds B of step k on entry and of step k + 2 on exit
        auto stage2 = [&](int k, const ATile& R0, const ATile& R1, ATile& W0, ATile& W1) {
            loadA_to(k + 2 * kLpK, apre);
            loadA_to(k + 3 * kLpK, aQ);
            bf8 bv[NB][NS];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int s = 0; s < NS; ++s) bv[b][s] = bnext[b][s];
            loadB_to(k + kLpK, bQ);
            multiply(R0, bv);
            loadB_to(k + 2 * kLpK, bnext);
            multiply(R1, bQ);
            storeA_from(W0, apre);
            storeA_from(W1, aQ);
        };
        loadA_to(0, apre);
        loadA_to(kLpK, aQ);
        loadB_to(0, bnext);
        storeA_from(sA0, apre);
        storeA_from(sA1, aQ);
        __syncthreads();
        int k = 0;
        for (; k + 4 * kLpK <= ldk; k += 4 * kLpK) {
            stage2(k, sA0, sA1, sA2, sA3);
            __syncthreads();
            stage2(k + 2 * kLpK, sA2, sA3, sA0, sA1);
            __syncthreads();
        }
        if (k < ldk) stage2(k, sA0, sA1, sA2, sA3);   // ldk = 64 mod 128: one more stage
    } else {
        loadA(0);
        loadB(0);
        storeA(sA0);
        __syncthreads();
        for (int k = 0; k < ldk; k += 2 * kLpK) {
            step(k, sA0, sA1);
            __syncthreads();
            step(k + kLpK, sA1, sA0);
            __syncthreads();
        }
    }

    if constexpr (!GRAD) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = rt * kLpRows + 16 * h + 4 * lk + v;    // MFMA output rows: 4 (l/16) + v
                if (i >= rows) continue;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int j = jbase + 16 * b + l16;
                    if (j >= nB) continue;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        double* o = out + c * out_comp + (size_t)i * ldo + j;
                        *o = (accumulate ? *o : 0.0) + (double)acc[c][h][b][v];
                    }
                }
            }
        return;
    } else {
        double gsum[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) gsum[j] = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = rt * kLpRows + 16 * h + 4 * lk + v;
                if (i >= rows) continue;
                const d4 pi = pos[g0 + i];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int jg = jbase + 16 * b + l16;
                    if (jg >= nB) continue;
                    pi_grad_point(pi, pos[jg], acc[0][h][b][v], acc[1][h][b][v], acc[2][h][b][v], gsum);
                }
            }
        __shared__ double red[kPiThreads / 64][16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            double v = gsum[j];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
            if (lane == 0) red[wave][j] = v;
        }
        __syncthreads();
        if (threadIdx.x < 16 && (int)threadIdx.x < ncoef) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < kPiThreads / 64; ++w) v += red[w][threadIdx.x];
            out[(size_t)blockIdx.x * 16 + threadIdx.x] = v;
        }
    }
}

}  // namespace xtc
