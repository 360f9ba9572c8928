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
// positions are copied by direct 16-byte buffer-to-LDS loads (no registers
// involved; a buffer descriptor per stage in scalar registers, one 32-bit
// lane offset), issued one stage ahead into the other of two buffers and
// shared by the four waves, which read their operands from LDS; one barrier
// per stage.  The two buffers are separate objects named statically where
// they are filled or read (the stage loop runs two stages per iteration, with
// no exit in between), and the positions are read from LDS as scalars: the
// compiler then knows that a stage's reads need not wait for the loads still
// filling the other buffer.  (Operand loads from global memory issued by each
// wave were consumed in the k-step that issued them, the compiler
// rematerialising any prefetch, so the waves waited on them; with one buffer
// indexed by stage parity, 64-bit load addresses in vector registers or
// vector-typed position reads, the compiler waited for the next stage's loads
// before the first LDS read of each stage.)
template <int NBLK> struct OccLds {
    static constexpr int kSG = 32;                                    // grid points per stage
    static constexpr int kRowB = 128 * NBLK;                          // bytes of one tile row
    static constexpr int kChunks = kSG * kRowB / 1024;                // 1 KB direct-load chunks per stage
    static constexpr int kStageB = kChunks * 1024 + 1024;             // + 32 positions of 32 bytes
    static_assert(kChunks % 4 == 0, "chunks are dealt to 4 waves");
};
// Word 3 of a raw (untyped, unswizzled) buffer descriptor on gfx9-family GPUs.
constexpr int kRawBufferWord3 = 0x00020000;

template <int KIND, int NBLK>
__global__ __launch_bounds__(256, 2) void k_build_K_occ(const d4* __restrict__ pos,
                                                            const double* __restrict__ rho_occ, int ldO, int ngp,
                                                            int g0, int rows, int n_rt, JasDev J,
                                                            double* __restrict__ part, int seg_len) {
    typedef OccLds<NBLK> C;
    typedef __attribute__((address_space(3))) void* lds_ptr;
    __shared__ __attribute__((aligned(1024))) char sm0[C::kStageB];
    __shared__ __attribute__((aligned(1024))) char sm1[C::kStageB];
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
    constexpr int kPer = C::kChunks / 4;
    const char* seg0 = (const char*)(rho_occ + (size_t)ct * ngp * 16 * NBLK) + (size_t)gs * C::kRowB;
    const uint32_t loff = 16 * lane;
    auto issue = [&](int st, char* buf) {
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(seg0 + (size_t)st * C::kSG * C::kRowB), (short)0, C::kSG * C::kRowB, kRawBufferWord3);
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)(buf + 1024 * (wave + 4 * i)), 16, loff,
                                                     1024 * (wave + 4 * i), 0, 0);
        if (wave == 0) {
            const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(pos + gs + C::kSG * st), (short)0, C::kSG * (int)sizeof(d4), kRawBufferWord3);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rp, (lds_ptr)(buf + 1024 * C::kChunks), 16, loff, 0, 0, 0);
        }
    };

    d4 acc[3][NBLK];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int c = 0; c < NBLK; ++c) acc[x][c] = (d4){0.0, 0.0, 0.0, 0.0};

    // the 8 k-steps of the stage in `tile`, then the wait for this wave's
    // loads of the next stage and the barrier that publishes everyone's (and
    // ends every wave's reads of this one)
    auto stage = [&](const char* tile) {
#pragma unroll 1
        for (int t = 0; t < C::kSG / 4; ++t) {
            const int k = 4 * t + kq;                      // this lane's point of the k-step
            const double* cq = (const double*)(tile + 1024 * C::kChunks) + 4 * k;
            const double cx = cq[0], cy = cq[1], cz = cq[2];
            const double* brow = (const double*)(tile + k * C::kRowB) + l16;
            double cb[NBLK];
#pragma unroll
            for (int c = 0; c < NBLK; ++c) cb[c] = brow[16 * c];
            const double dx = pg.x - cx, dy = pg.y - cy, dz = pg.z - cz;
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
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    if (nst > 0) {
        issue(0, sm0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    // even stages from sm0, odd ones from sm1, each stage's successor loaded
    // into the other buffer while it is consumed; an odd last stage (in sm0)
    // after the loop
    int st = 0;
    for (; st + 1 < nst; st += 2) {
        issue(st + 1, sm1);
        stage(sm0);
        if (st + 2 < nst) issue(st + 2, sm0);
        stage(sm1);
    }
    if (st < nst) stage(sm0);
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
