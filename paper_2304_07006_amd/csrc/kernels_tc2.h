// Two-body transcorrelated integrals on the grid (Theory, definition of K):
//   K_pr^qs = 1/2 <pr| P^1_2 (lap_1 u + (grad_1 u)^2 + 2 grad_1 u . grad_1) |qs>.
// With rho_pq = w phi_p phi_q, S(g,g') = lap_1 u + |grad_1 u|^2 (symmetric; 0 at
// coincident points), F_R(g) = sum_g' S(g,g') rho_R(g'), the grid intermediate
// K_R(g) of the xTC path and rhog_pq(g) = w phi_p grad phi_q (ordered pairs):
//   K2[pq][rs] = A[P][R] + B[pq][R] + B[rs][P],
//   A = sum_g rho^T F (packed pairs),  B = sum_g sum_x rhog_x^T K_x.
#pragma once
#include "kernels_build_k.h"
#include "xtc_device.h"

namespace xtc {

// S = u'' + 2 u'/r + u'^2 from r^2 in FP64 (1/r and the reciprocals from the
// Newton-refined hardware approximations); exactly 0 at r^2 == 0.
template <int KIND>
__device__ __forceinline__ double scalar_S(double r2, const JasDev& J) {
    const double s = rsq_f64(r2);                 // 1/r (not finite at r2 == 0: selected away)
    const double r = r2 * s;
    double up, upp;
    if constexpr (KIND == 0) {
        const double it = rcp_f64(fma(J.b, r, 1.0));
        up = 0.5 * it * it;
        upp = -J.b * it * it * it;
    } else {
        const double q = rcp_f64(1.0 + r);
        const double t = r * q;
        double p1 = J.dcoef[15], p2 = J.d2coef[15];
#pragma unroll
        for (int k = 14; k >= 0; --k) {
            p1 = fma(p1, t, J.dcoef[k]);
            p2 = fma(p2, t, J.d2coef[k]);
        }
        const double q2 = q * q;
        up = p1 * q2;
        upp = q2 * (p2 * q2 - 2.0 * p1 * q);
    }
    const double v = upp + 2.0 * up * s + up * up;
    return r2 > 0.0 ? v : 0.0;
}

// F[g - g0][P] = sum_{g'} S(g, g') rho[g'][P] for the rows of the chunk
// (FP64 MFMA).  Workgroup 64 rows x 16 NBLK columns; each wave owns 16 rows
// and NBLK 16-column blocks; S generated per lane (row l%16, g' = kk + l/16).
template <int KIND, int NBLK>
__global__ __launch_bounds__(256) void k_build_F_f64(const d4* __restrict__ pos, const double* __restrict__ rho,
                                                     int ldP, int ngp, int g0, int rows, int n_rt, JasDev J,
                                                     double* __restrict__ F) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rt = blockIdx.x % n_rt;
    const int ct = blockIdx.x / n_rt;
    const int rloc0 = rt * kKRows + wave * kKRowsPerWave;
    const int my = min(rloc0 + (lane & 15), rows - 1);
    const d4 pg = pos[g0 + my];
    const int kq = lane >> 4;
    const int col = ct * 16 * NBLK + (lane & 15);
    d4 acc[NBLK];
#pragma unroll
    for (int c = 0; c < NBLK; ++c) acc[c] = (d4){0.0, 0.0, 0.0, 0.0};
    const double* bp = rho + (size_t)kq * ldP + col;
    const d4* pp = pos + kq;
    double b[NBLK];
#pragma unroll
    for (int c = 0; c < NBLK; ++c) b[c] = bp[16 * c];
    d4 pc = *pp;
    for (int kk = 0; kk < ngp; kk += 4) {
        double cb[NBLK];
#pragma unroll
        for (int c = 0; c < NBLK; ++c) cb[c] = b[c];
        const d4 cp = pc;
        if (kk + 4 < ngp) {
            bp += (size_t)4 * ldP;
            pp += 4;
#pragma unroll
            for (int c = 0; c < NBLK; ++c) b[c] = bp[16 * c];
            pc = *pp;
        }
        const double dx = pg.x - cp.x, dy = pg.y - cp.y, dz = pg.z - cp.z;
        const double s = scalar_S<KIND>(fma(dx, dx, fma(dy, dy, dz * dz)), J);
#pragma unroll
        for (int c = 0; c < NBLK; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(s, cb[c], acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = rloc0 + (lane >> 4) + 4 * v;
        if (r < rows) {
#pragma unroll
            for (int c = 0; c < NBLK; ++c) F[(size_t)r * ldP + col + 16 * c] = acc[c][v];
        }
    }
}

// rhog[x][g][p * N + q] = w_g phi_p(g) d_x phi_q(g) for the chunk rows
// (columns [N^2, ldN) zero).  phi, dphi: [N][Ng], [3][N][Ng].
__global__ void k_rhog(const double* __restrict__ w, const double* __restrict__ phi,
                       const double* __restrict__ dphi, int N, int Ng, int g0, int rows, int ldN,
                       size_t xstride, double* __restrict__ rhog) {
    const size_t n = (size_t)rows * ldN;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % ldN);
        const int g = g0 + (int)(i / ldN);
        double v[3] = {0.0, 0.0, 0.0};
        if (j < N * N) {
            const int p = j / N, q = j % N;
            const double a = w[g] * phi[(size_t)p * Ng + g];
#pragma unroll
            for (int x = 0; x < 3; ++x) v[x] = a * dphi[((size_t)x * N + q) * Ng + g];
        }
#pragma unroll
        for (int x = 0; x < 3; ++x) rhog[x * xstride + i] = v[x];
    }
}

// M[i][j] (+)= sum_c sum_{g<rows} A_c[g][i] B_c[g][j] on FP64 MFMA, i < 128 n_it,
// j < 128 n_jt.  Workgroup tile 128 x 128, four waves as 2 x 2 of 64 x 64;
// row block b of a wave maps logical row i to I0 + 4 i + b (and likewise for
// columns), so every lane loads one 32-byte vector of each operand per k-step.
__global__ __launch_bounds__(256) void k_gemm_tn_f64(const double* __restrict__ A, size_t a_cstride, int lda,
                                                     const double* __restrict__ B, size_t b_cstride, int ldb,
                                                     int ncomp, int rows, int n_it, double* __restrict__ M,
                                                     int ldm, int accumulate) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int it = blockIdx.x % n_it, jt = blockIdx.x / n_it;
    const int I0 = it * 128 + 64 * (wave & 1);
    const int J0 = jt * 128 + 64 * (wave >> 1);
    const int kq = lane >> 4;
    const int l16 = lane & 15;
    d4 acc[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[b][c] = (d4){0.0, 0.0, 0.0, 0.0};
    const d4 zero = {0.0, 0.0, 0.0, 0.0};
    for (int comp = 0; comp < ncomp; ++comp) {
        const double* Ap = A + comp * a_cstride + I0 + 4 * l16;
        const double* Bp = B + comp * b_cstride + J0 + 4 * l16;
        int g = kq;
        d4 a = g < rows ? *(const d4*)(Ap + (size_t)g * lda) : zero;
        d4 b = g < rows ? *(const d4*)(Bp + (size_t)g * ldb) : zero;
        for (int kk = 0; kk < rows; kk += 4) {
            const d4 ca = a, cb = b;
            g += 4;
            a = g < rows ? *(const d4*)(Ap + (size_t)g * lda) : zero;
            b = g < rows ? *(const d4*)(Bp + (size_t)g * ldb) : zero;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[i], cb[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int I = I0 + 4 * (lane >> 4) + 16 * v + i;
            d4* out = (d4*)(M + (size_t)I * ldm + J0 + 4 * l16);
            d4 val = {acc[i][0][v], acc[i][1][v], acc[i][2][v], acc[i][3][v]};
            if (accumulate) val += *out;
            *out = val;
        }
}

// K2[p][q][r][s] = A[P][R] + B[p N + q][R] + B[r N + s][P], P = pair(p,q), R = pair(r,s),
// with A taken as (A[P][R] + A[R][P]) / 2 (A is symmetric up to summation order)
// and the two B terms added as one commutative pair, so that
// K2[p][q][r][s] == K2[r][s][p][q] bitwise.
__global__ __launch_bounds__(256) void k_finalize_K2(const double* __restrict__ A, int ldP,
                                                     const double* __restrict__ B, int N,
                                                     double* __restrict__ K2) {
    const int p = blockIdx.y, q = blockIdx.z;
    const int pq = p * N + q;
    const int P = pair_sym(p, q, N);
    const int NN = N * N;
    for (int rs = blockIdx.x * blockDim.x + threadIdx.x; rs < NN; rs += gridDim.x * blockDim.x) {
        const int r = rs / N, s = rs % N;
        const int R = pair_sym(r, s, N);
        const double a = 0.5 * (A[(size_t)P * ldP + R] + A[(size_t)R * ldP + P]);
        K2[(size_t)pq * NN + rs] = a + (B[(size_t)pq * ldP + R] + B[(size_t)rs * ldP + P]);
    }
}

}  // namespace xtc
