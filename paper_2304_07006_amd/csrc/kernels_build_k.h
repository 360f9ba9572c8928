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
// same contraction as k_build_K_f64 over the gathered pair densities
// rho_occ[g'][ldO] of the occupied pairs, one segment [blockIdx.y * seg_len,
// ...) of the sum over g' per grid.y, written to part[seg][x][r][ldO].
// Workgroup: 64 rows x 16 NBLK columns; each wave owns 16 rows and NBLK
// 16-column blocks of all 3 components, so each FP64 d^x value a lane
// generates feeds 3 NBLK MFMAs.  From 8 blocks on the 24 NBLK accumulator
// registers per block column leave room for two waves per SIMD only (the
// second wave hides the operand loads of the first).  The host picks NBLK.
template <int KIND, int NBLK>
__global__ __launch_bounds__(256, NBLK >= 8 ? 2 : 1) void k_build_K_occ(const d4* __restrict__ pos, const double* __restrict__ rho_occ,
                                                     int ldO, int ngp, int g0, int rows, int n_rt, JasDev J,
                                                     double* __restrict__ part, int seg_len) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rt = blockIdx.x % n_rt;
    const int ct = blockIdx.x / n_rt;
    const int gs = blockIdx.y * seg_len, ge = min(ngp, gs + seg_len);
    const int rloc0 = rt * kKRows + wave * kKRowsPerWave;   // first local row of this wave
    const int my = min(rloc0 + (lane & 15), rows - 1);      // row whose d^x this lane generates
    const d4 pg = pos[g0 + my];
    const int kq = lane >> 4;
    const int col = ct * 16 * NBLK + (lane & 15);

    d4 acc[3][NBLK];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int c = 0; c < NBLK; ++c) acc[x][c] = (d4){0.0, 0.0, 0.0, 0.0};

    // operands of the next two k-steps in flight (a k-step's MFMAs are too short
    // to cover the load latency of the one after it); near the end of the
    // segment the last k-step is re-read into the slot that is never consumed
    const double* bp = rho_occ + (size_t)(gs + kq) * ldO + col;
    const d4* pp = pos + gs + kq;
    const int kl = ge - 4;                // last k-step of the segment
    double b0[NBLK], b1[NBLK];
    d4 p0, p1;
#pragma unroll
    for (int c = 0; c < NBLK; ++c) b0[c] = bp[16 * c];
    p0 = *pp;
    {
        const size_t o = (size_t)(min(gs + 4, kl) - gs);
#pragma unroll
        for (int c = 0; c < NBLK; ++c) b1[c] = bp[o * ldO + 16 * c];
        p1 = pp[o];
    }
    for (int kk = gs; kk < ge; kk += 4) {
        double cb[NBLK];
#pragma unroll
        for (int c = 0; c < NBLK; ++c) {
            cb[c] = b0[c];
            b0[c] = b1[c];
        }
        const d4 cp = p0;
        p0 = p1;
        {
            const size_t o = (size_t)(min(kk + 8, kl) - gs);
#pragma unroll
            for (int c = 0; c < NBLK; ++c) b1[c] = bp[o * ldO + 16 * c];
            p1 = pp[o];
        }
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
