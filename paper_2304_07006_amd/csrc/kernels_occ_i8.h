// Occupied-occupied block of K from exact integer products, for the
// reduced-precision forms:
//   K^x_P(g) = sum_g' d^x(g,g') rho_P(g')      (Theory, definition of V)
// over the occupied pairs P, to the accuracy of an FP64 evaluation, on the
// int8 matrix cores (v_mfma_i32_16x16x64_i8) instead of the FP64 ones.
//
// Both operands become fixed-point numbers of six balanced base-128 digits
// relative to a power-of-two scale: S_d bounds 2|d^x| for the Jastrow at
// hand (|d^x| <= |u'(r)|), and S_P is the power of two above twice the
// largest |rho_P(g')| of pair P.  With v = d / S_d (or rho / S_P) in
// [-1/2, 1/2]:
//   v = sum_{i=1..6} a_i 2^(-7 i) + e,   |e| <= 2^-43,
// a_1 and a_4 in [-64, 64], the others in [-64, 63] (digits centred on zero,
// so that rounding and dropped terms carry no sign bias).  The digit products
// a_i b_j with i + j <= 7 (21 of the 36) are summed exactly in int32, one
// accumulator per order i + j; each dropped product is at most 2^-44 S_d S_P
// and all of them together below 2.87e-13 S_d S_P.
// The orders are combined in FP64 per segment of at most kI8SegMax grid
// points (|an accumulator| <= 6 x 64 x 64 per point, < 2^31 over a segment),
// and the segments are summed in FP64 afterwards.
//
// Digit tiles are laid out as the MFMA consumes them: one 16-byte operand
// per lane, lane l standing for pair (or row) l % 16 and grid points
// 16 (l / 16) + e, e = 0..15, of a 64-point k-step (both operands use the
// same assignment, so the sum over the 64 points does not depend on the
// order the hardware gives the bytes).  The int32 result of lane l holds
// rows 4 (l / 16) + v, v = 0..3, of column l % 16.
#pragma once
#include "xtc_device.h"

namespace xtc {

typedef int i4 __attribute__((ext_vector_type(4)));

constexpr int kI8Digits = 6;          // digits per operand
constexpr int kI8Orders = 6;          // accumulated orders i + j = 2..7
constexpr int kI8Kb = 64;             // grid points per MFMA k-step
constexpr int kI8TileB = 64 * 16;     // bytes of one digit tile (64 lanes x 16 bytes)
constexpr int kI8SegMax = 65536;      // grid points per int32 segment
constexpr int kI8MaxCT = 9;           // 16-pair column tiles per wave
constexpr int kI8Waves = 4;

// Power of two S > 2 m (1 for m = 0), so that |x| <= m gives |x| / S < 1/2.
__host__ __device__ inline double i8_scale(double m) {
    if (!(m > 0.0)) return 1.0;
    int e = 0;
    (void)frexp(m, &e);   // m < 2^e
    return ldexp(1.0, e + 1);
}

// Signed 7-bit field at bit `off` of x, sign-extended.
__device__ __forceinline__ int sfield7(int x, int off) { return (x << (25 - off)) >> 25; }

// The six digits of v from h = v 2^21 (|h| <= 2^20 plus rounding):
// h = H + L 2^-21 + e with integers |H|, |L| <= 2^20 (+1) and |e| <= 2^-22,
// then each of H, L = t 2^14 + m 2^7 + l with m, l in [-64, 63] and
// t in [-64, 64].  Adding 8256 = 64 (2^7 + 1) turns m and l into the fields
// (bits 7..13 and 0..6) with their top bit flipped; the FP64 roundings go
// through the 1.5 2^52 shifter, whose low word is the rounded integer.
__device__ __forceinline__ void i8_digits(double h, int d[kI8Digits]) {
    const double kShift = 6755399441055744.0;   // 1.5 * 2^52
    const double th = h + kShift;
    const double hr = th - kShift;
    const double tl = fma(h - hr, 2097152.0, kShift);
    const int H = (int)__builtin_bit_cast(unsigned long long, th);
    const int L = (int)__builtin_bit_cast(unsigned long long, tl);
    const int uh = H + 8256, ul = L + 8256;
    const int xh = uh ^ 0x2040, xl = ul ^ 0x2040;
    d[0] = uh >> 14;
    d[1] = sfield7(xh, 7);
    d[2] = sfield7(xh, 0);
    d[3] = ul >> 14;
    d[4] = sfield7(xl, 7);
    d[5] = sfield7(xl, 0);
}

__device__ __forceinline__ int i8_pack(int a, int b, int c, int d) {
    return (a & 255) | ((b & 255) << 8) | ((c & 255) << 16) | (d << 24);
}

// Per-pair largest |rho_P(g')| of the gathered occupied pairs
// (rho_occ[(P / tw) ngp tw + g' tw + P % tw]), as the bit pattern of a
// non-negative double (ordered like the value), max-combined into amax[P]
// (zero before the first launch).  Grid: (column tiles of 16 pairs, row
// chunks); 256 threads: 16 pairs x 16 rows at a time.
__global__ __launch_bounds__(256) void k_occ_absmax(const double* __restrict__ rho_occ, int ngp, int tw, int nOP,
                                                    int rows_per_block, unsigned long long* __restrict__ amax) {
    __shared__ double red[256];
    const int j = threadIdx.x & 15, rs = threadIdx.x >> 4;
    const int P = blockIdx.x * 16 + j;
    const int r0 = blockIdx.y * rows_per_block, r1 = min(ngp, r0 + rows_per_block);
    double m = 0.0;
    if (P < nOP) {
        const double* col = rho_occ + (size_t)(P / tw) * ngp * tw + P % tw;
        for (int g = r0 + rs; g < r1; g += 16) m = fmax(m, fabs(col[(size_t)g * tw]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    if (rs == 0 && P < nOP) {
        for (int i = 1; i < 16; ++i) m = fmax(m, red[16 * i + j]);
        atomicMax(amax + P, __builtin_bit_cast(unsigned long long, m));
    }
}

// Stage blocks of the main kernel, one per k-step kb and column group:
// the digit tiles of rho for the group's CT column tiles, [ct][s][lane]
// (16 bytes each; pairs >= nOP are zero), then the positions (x, y, z, 0)
// of the 64 points of k-step kb + 1 (zero past the grid), padded to whole
// 4 KB (one 1 KB chunk per wave and round; the padding is loaded, never
// read), so that each stage is one contiguous block of kBlockB bytes.
template <int CT> struct OccI8Stage {
    static constexpr int kDigitB = CT * kI8Digits * kI8TileB;
    static constexpr int kUsedB = kDigitB + kI8Kb * 32;
    static constexpr int kBlockB = (kUsedB + 4095) / 4096 * 4096;
    static constexpr int kPerWave = kBlockB / 1024 / kI8Waves;               // 1 KB direct-load chunks
};

// Digits: one thread per (kb, column tile ct8 of nct8 = groups x CT, lane).
template <int CT>
__global__ __launch_bounds__(256) void k_occ_slice(const double* __restrict__ rho_occ, int ngp, int tw, int nOP,
                                                   int groups, const unsigned long long* __restrict__ amax,
                                                   char* __restrict__ stages) {
    typedef OccI8Stage<CT> S;
    const int nct8 = groups * CT;
    const size_t n = (size_t)(ngp / kI8Kb) * nct8 * 64;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int lane = (int)(idx & 63);
        const size_t rest = idx >> 6;
        const int ct8 = (int)(rest % nct8);
        const size_t kb = rest / nct8;
        const int P = ct8 * 16 + (lane & 15);
        const int gq = (int)kb * kI8Kb + 16 * (lane >> 4);
        const bool on = P < nOP;
        const double hs = on ? 2097152.0 / i8_scale(__builtin_bit_cast(double, amax[P])) : 0.0;
        const double* col = rho_occ + (on ? (size_t)(P / tw) * ngp * tw + P % tw : 0);
        int w[kI8Digits][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int dg[4][kI8Digits];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double v = on ? col[(size_t)(gq + 4 * k + b) * tw] : 0.0;
                i8_digits(v * hs, dg[b]);
            }
#pragma unroll
            for (int s = 0; s < kI8Digits; ++s) w[s][k] = i8_pack(dg[0][s], dg[1][s], dg[2][s], dg[3][s]);
        }
        char* blk = stages + (kb * groups + ct8 / CT) * S::kBlockB + (size_t)(ct8 % CT) * kI8Digits * kI8TileB;
#pragma unroll
        for (int s = 0; s < kI8Digits; ++s)
            *(i4*)(blk + (s * 64 + lane) * 16) = (i4){w[s][0], w[s][1], w[s][2], w[s][3]};
    }
}

// Positions: one thread per (kb, group, point).
template <int CT>
__global__ __launch_bounds__(256) void k_occ_stage_pos(const d4* __restrict__ pos, int ngp, int groups,
                                                       char* __restrict__ stages) {
    typedef OccI8Stage<CT> S;
    const size_t n = (size_t)(ngp / kI8Kb) * groups * kI8Kb;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(idx % kI8Kb);
        const size_t kg = idx / kI8Kb;   // kb * groups + group
        const size_t g = (kg / groups + 1) * kI8Kb + p;
        *(d4*)(stages + kg * S::kBlockB + S::kDigitB + 32 * p) = g < (size_t)ngp ? pos[g] : (d4){0.0, 0.0, 0.0, 0.0};
    }
}

// Word 3 of a raw (untyped, unswizzled) buffer descriptor on gfx9-family GPUs.
constexpr int kI8RawBufferWord3 = 0x00020000;

// The block for rows [g0, g0 + rows).  Each wave owns one task: 16 rows
// (row block rb) and one component x of d, for the CT column tiles of column
// group blockIdx.z, so its accumulators are CT x 6 orders x 4 registers; task
// 4 blockIdx.x + wave is row block task / 3, component task % 3 (waves past
// the last task only help load).  blockIdx.y is the segment of seg_kb k-steps.
// Per k-step a wave generates its 16 rows' d^x for the next 64 points (FP64,
// then digits; 16 values per lane), while its MFMAs consume the current
// digits against the staged rho tiles: 21 CT MFMAs per k-step.  Each stage
// block (stages[kb][group], OccI8Stage) is copied by direct 16-byte
// buffer-to-LDS loads one k-step ahead into the other of two statically named
// buffers, as in k_build_K_occ.  part[seg][x][r][ldK] = the FP64 value of the
// segment's sum, for pair columns 16 (blockIdx.z CT + ct) + l % 16.
template <int KIND, int CT>
__global__ __launch_bounds__(256, 1) void k_build_K_occ_i8(const d4* __restrict__ pos, const char* __restrict__ stages,
                                                           int groups, int ngp, int g0, int rows, int n_rb, JasDev J,
                                                           double sd, const unsigned long long* __restrict__ amax,
                                                           double* __restrict__ part, int ldK, int seg_kb) {
    typedef OccI8Stage<CT> S;
    typedef __attribute__((address_space(3))) void* lds_ptr;
    __shared__ __attribute__((aligned(1024))) char sm0[S::kBlockB];
    __shared__ __attribute__((aligned(1024))) char sm1[S::kBlockB];
    __shared__ __attribute__((aligned(1024))) char smp[kI8Kb * 32];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int task = kI8Waves * blockIdx.x + wave;
    const int live = __builtin_amdgcn_readfirstlane(task < 3 * n_rb ? 1 : 0);
    const int rb = live ? task / 3 : 0;
    const int comp = live ? task % 3 : 0;
    const int cg = blockIdx.z;
    const int nkb = ngp / kI8Kb;
    const int kb0 = blockIdx.y * seg_kb;
    const int nst = min(seg_kb, nkb - kb0);
    const int q = lane >> 4;
    const int my = min(rb * 16 + (lane & 15), rows - 1);
    const d4 pg = pos[g0 + my];
    const double pc = comp == 0 ? pg.x : comp == 1 ? pg.y : pg.z;
    const double hs = 2097152.0 / sd;   // digits of d / sd from d 2^21 / sd
    const uint32_t loff = 16 * lane;

    // stage t: the block of k-step kb0 + t
    auto issue = [&](int t, char* buf) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(stages + ((size_t)(kb0 + t) * groups + cg) * S::kBlockB), (short)0, S::kBlockB,
            kI8RawBufferWord3);
#pragma unroll
        for (int i = 0; i < S::kPerWave; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(buf + 1024 * (wave + kI8Waves * i)), 16, loff,
                                                     1024 * (wave + kI8Waves * i), 0, 0);
    };

    // digits of d^comp for this lane's row and points 16 q + e of the k-step
    // whose positions are at p64 (LDS)
    auto gen = [&](const char* p64, i4 A[kI8Digits]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int dg[4][kI8Digits];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double* cq = (const double*)(p64 + 32 * (16 * q + 4 * k + b));
                const double cx = cq[0], cy = cq[1], cz = cq[2], cc = cq[comp];
                const double dx = pg.x - cx, dy = pg.y - cy, dz = pg.z - cz;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const double f = du_over_r<KIND>(r2, J);
                i8_digits((pc - cc) * (f * hs), dg[b]);
            }
#pragma unroll
            for (int s = 0; s < kI8Digits; ++s) A[s][k] = i8_pack(dg[0][s], dg[1][s], dg[2][s], dg[3][s]);
        }
    };

    i4 acc[CT][kI8Orders];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int o = 0; o < kI8Orders; ++o) acc[c][o] = (i4){0, 0, 0, 0};
    i4 A[kI8Digits];

    // one k-step from `buf`: the next k-step's digits, the products of this
    // one, then the wait for this wave's loads of the next stage and the
    // barrier that publishes everyone's (and ends all reads of this one)
    auto stage = [&](const char* buf) {
        if (live) {
            i4 An[kI8Digits];
            gen(buf + S::kDigitB, An);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                i4 b[kI8Digits];
#pragma unroll
                for (int s = 0; s < kI8Digits; ++s)
                    b[s] = *(const i4*)(buf + ((c * kI8Digits + s) * 64 + lane) * 16);
#pragma unroll
                for (int o = 0; o < kI8Orders; ++o)
#pragma unroll
                    for (int i = 0; i <= o; ++i)
                        acc[c][o] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[i], b[o - i], acc[c][o], 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < kI8Digits; ++s) A[s] = An[s];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    if (nst > 0) {
        // positions of the first k-step (inside the grid), then its stage
        const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(pos + (size_t)kb0 * kI8Kb), (short)0, kI8Kb * 32, kI8RawBufferWord3);
        if (wave < 2)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rp, (lds_ptr)(smp + 1024 * wave), 16, loff, 1024 * wave, 0, 0);
        issue(0, sm0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (live) gen(smp, A);
    }
    int t = 0;
    for (; t + 1 < nst; t += 2) {
        issue(t + 1, sm1);
        stage(sm0);
        if (t + 2 < nst) issue(t + 2, sm0);
        stage(sm1);
    }
    if (t < nst) stage(sm0);

    if (!live) return;
    double* out = part + (size_t)blockIdx.y * 3 * rows * ldK;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int P = 16 * (cg * CT + c) + (lane & 15);
        const double sc = sd * i8_scale(__builtin_bit_cast(double, amax[P]));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb * 16 + 4 * q + v;
            if (r < rows) {
                double s = 0.0;
#pragma unroll
                for (int o = kI8Orders - 1; o >= 0; --o) s += (double)acc[c][o][v] * ldexp(1.0, -7 * (o + 2));
                out[((size_t)comp * rows + r) * ldK + P] = s * sc;
            }
        }
    }
}

}  // namespace xtc
