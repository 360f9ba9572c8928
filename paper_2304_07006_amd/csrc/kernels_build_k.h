// Grid intermediate K^x_P(g) = sum_g' d^x(g,g') rho_P(g')  (FP64 MFMA).
//
// The sum over g' is a GEMM whose left operand d^x(g,g') is generated on chip
// from the grid positions (never stored: Ng^2 values) and whose right operand
// is the prepared weighted pair density rho[g'][P].  One MFMA
// v_mfma_f64_16x16x4_f64 consumes a 16(g) x 4(g') slab of d^x and a
// 4(g') x 16(P) slab of rho.
//
// Operand layouts of v_mfma_f64_16x16x4_f64 (64 lanes, lane l):
//   A[i][k]: i = l % 16, k = l / 16      B[k][j]: k = l / 16, j = l % 16
//   D[i][j]: lane l holds rows i = l/16 + 4 v, v = 0..3, column j = l % 16
//   (decoded on gfx950; it differs from the FP32 form's 4 (l/16) + v).
// Column block c of a wave's 128-column strip maps logical column j to
// P = col0 + 64 (c/4) + 4 j + (c%4): each lane then loads its B values as two
// 32-byte vectors and stores its outputs as 32-byte vectors.
#pragma once
#include "xtc_device.h"

namespace xtc {

constexpr int kKRowsPerWave = 16;
constexpr int kKWaves = 4;
constexpr int kKRows = kKRowsPerWave * kKWaves;   // 64 grid rows per workgroup

// Workgroup tile: 64 rows (g) x 128 pair columns; each wave owns 16 rows and
// the 3 vector components of all 128 columns (24 accumulator blocks).
// Tiles are numbered row-tile fastest, so workgroups resident at the same
// time share one 128-column strip of rho (read through L2), whatever XCD
// they land on.
template <int KIND>
__global__ __launch_bounds__(256) void k_build_K_f64(const d4* __restrict__ pos,
                                                     const double* __restrict__ rho, int ldP,
                                                     int ngp, int g0, int rows, int n_rt, JasDev J,
                                                     double* __restrict__ K) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rt = blockIdx.x % n_rt;
    const int ct = blockIdx.x / n_rt;
    const int rloc0 = rt * kKRows + wave * kKRowsPerWave;   // first local row of this wave
    const int my = min(rloc0 + (lane & 15), rows - 1);      // row whose d^x this lane generates
    const d4 pg = pos[g0 + my];
    const int kq = lane >> 4;
    const int col = ct * 128 + 4 * (lane & 15);

    d4 acc[3][8];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[x][c] = (d4){0.0, 0.0, 0.0, 0.0};

    const double* bp = rho + (size_t)kq * ldP + col;
    const d4* pp = pos + kq;
    d4 b0 = *(const d4*)bp;
    d4 b1 = *(const d4*)(bp + 64);
    d4 pc = *pp;
    for (int kk = 0; kk < ngp; kk += 4) {
        const d4 cb0 = b0, cb1 = b1, cp = pc;
        if (kk + 4 < ngp) {              // prefetch the next 4 grid columns
            bp += (size_t)4 * ldP;
            pp += 4;
            b0 = *(const d4*)bp;
            b1 = *(const d4*)(bp + 64);
            pc = *pp;
        }
        const double dx = pg.x - cp.x, dy = pg.y - cp.y, dz = pg.z - cp.z;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double f = du_over_r<KIND>(r2, J);
        const double ax = dx * f, ay = dy * f, az = dz * f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            acc[0][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, cb0[c], acc[0][c], 0, 0, 0);
            acc[1][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, cb0[c], acc[1][c], 0, 0, 0);
            acc[2][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(az, cb0[c], acc[2][c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            acc[0][4 + c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, cb1[c], acc[0][4 + c], 0, 0, 0);
            acc[1][4 + c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, cb1[c], acc[1][4 + c], 0, 0, 0);
            acc[2][4 + c] = __builtin_amdgcn_mfma_f64_16x16x4f64(az, cb1[c], acc[2][4 + c], 0, 0, 0);
        }
    }
    const size_t kstride = (size_t)rows * ldP;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = rloc0 + (lane >> 4) + 4 * v;
        if (r < rows) {
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                double* out = K + x * kstride + (size_t)r * ldP + col;
                *(d4*)out = (d4){acc[x][0][v], acc[x][1][v], acc[x][2][v], acc[x][3][v]};
                *(d4*)(out + 64) = (d4){acc[x][4][v], acc[x][5][v], acc[x][6][v], acc[x][7][v]};
            }
        }
    }
}

// Occupied-occupied block of K in FP64, for the reduced-precision forms: the
// same contraction as k_build_K_f64 over the gathered pair densities of the
// occupied pairs (column tiles of 16 NBLK pairs, tile-major:
// rho_occ[ct][ngp][16 NBLK]), one segment [blockIdx.y * seg_len, ...) of the
// sum over g' per grid.y (seg_len a multiple of 32), written to
// part[seg][x][r][ldO].  Workgroup: 64 rows x 16 NBLK columns; each wave owns
// 16 rows and NBLK 16-column blocks of all 3 components, so each FP64 d^x
// value a lane generates feeds 3 NBLK MFMAs (the host picks NBLK).  Each
// 32-point stage of the tile (32 x 16 NBLK doubles, contiguous) and its 32
// positions are copied by direct 16-byte global-to-LDS loads (no registers
// involved), issued one stage ahead into the other of two buffers and shared
// by the four waves, which read their operands from LDS; one barrier per
// stage.  (Operand loads from global memory issued by each wave were consumed
// in the k-step that issued them, the compiler rematerialising any prefetch,
// so the waves waited on them.)  The compiler still waits for the direct
// loads before a stage's first LDS read, as it cannot tell the buffers apart
// (naming them statically needs the stage loop unrolled twice, which spills
// the accumulators); two workgroups per CU cover that wait for each other.
template <int NBLK> struct OccLds {
    static constexpr int kSG = 32;                                    // grid points per stage
    static constexpr int kRowB = 128 * NBLK;                          // bytes of one tile row
    static constexpr int kChunks = kSG * kRowB / 1024;                // 1 KB direct-load chunks per stage
    static constexpr int kStageB = kChunks * 1024 + 1024;             // + 32 positions of 32 bytes
    static_assert(kChunks % 4 == 0, "chunks are dealt to 4 waves");
};

template <int KIND, int NBLK>
__global__ __launch_bounds__(256, 2) void k_build_K_occ(const d4* __restrict__ pos,
                                                            const double* __restrict__ rho_occ, int ldO, int ngp,
                                                            int g0, int rows, int n_rt, JasDev J,
                                                            double* __restrict__ part, int seg_len) {
    typedef OccLds<NBLK> C;
    typedef __attribute__((address_space(3))) void* lds_ptr;
    __shared__ __attribute__((aligned(1024))) char sm[2][C::kStageB];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rt = blockIdx.x % n_rt;
    const int ct = blockIdx.x / n_rt;
    const int gs = blockIdx.y * seg_len, ge = min(ngp, gs + seg_len);
    const int nst = (ge - gs) / C::kSG;
    const int rloc0 = rt * kKRows + wave * kKRowsPerWave;   // first local row of this wave
    const int my = min(rloc0 + (lane & 15), rows - 1);      // row whose d^x this lane generates
    const d4 pg = pos[g0 + my];
    const int kq = lane >> 4, l16 = lane & 15;
    const int col = ct * 16 * NBLK + l16;

    // direct loads: chunk wave + 4 i of a stage is its bytes [1024 chunk, +1024),
    // lane l the 16 of them at 1024 chunk + 16 l, in global memory and in LDS
    // (uniform base addresses plus one 32-bit lane offset)
    constexpr int kPer = C::kChunks / 4;
    const char* tile0 = (const char*)(rho_occ + (size_t)ct * ngp * 16 * NBLK);
    const uint32_t loff = 16 * lane;
    auto issue = [&](int st, int buf) {
        const char* ub = tile0 + (size_t)(gs + C::kSG * st) * C::kRowB + 1024 * wave;
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            __builtin_amdgcn_global_load_lds((const void*)(ub + 4096 * i + loff),
                                             (lds_ptr)(&sm[buf][1024 * (wave + 4 * i)]), 16, 0, 0);
        if (wave == 0)
            __builtin_amdgcn_global_load_lds((const void*)((const char*)(pos + gs + C::kSG * st) + loff),
                                             (lds_ptr)(&sm[buf][1024 * C::kChunks]), 16, 0, 0);
    };

    d4 acc[3][NBLK];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int c = 0; c < NBLK; ++c) acc[x][c] = (d4){0.0, 0.0, 0.0, 0.0};

    if (nst > 0) {
        issue(0, 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) issue(st + 1, buf ^ 1);
        const char* tile = sm[buf];
        const d4* sp = (const d4*)(tile + 1024 * C::kChunks);
#pragma unroll 1
        for (int t = 0; t < C::kSG / 4; ++t) {
            const int k = 4 * t + kq;                      // this lane's point of the k-step
            const d4 cp = sp[k];
            const double* brow = (const double*)(tile + k * C::kRowB) + l16;
            double cb[NBLK];
#pragma unroll
            for (int c = 0; c < NBLK; ++c) cb[c] = brow[16 * c];
            const double dx = pg.x - cp.x, dy = pg.y - cp.y, dz = pg.z - cp.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double f = du_over_r<KIND>(r2, J);
            const double ax = dx * f, ay = dy * f, az = dz * f;
#pragma unroll
            for (int c = 0; c < NBLK; ++c) {
                acc[0][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, cb[c], acc[0][c], 0, 0, 0);
                acc[1][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, cb[c], acc[1][c], 0, 0, 0);
                acc[2][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(az, cb[c], acc[2][c], 0, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);                     // this wave's loads of the next stage
        __syncthreads();                                   // everyone's, and this stage read by all
    }
    double* out = part + (size_t)blockIdx.y * 3 * rows * ldO;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = rloc0 + (lane >> 4) + 4 * v;
        if (r < rows) {
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
                for (int c = 0; c < NBLK; ++c) out[((size_t)x * rows + r) * ldO + col + 16 * c] = acc[x][c][v];
        }
    }
}

}  // namespace xtc
