// Adjoint of the xTC folding with respect to the power-Jastrow coefficients.
//
// Loss L = gE0 E0 + sum gh1 . h1 + sum gV2 . V2 (seeds given by the caller).
// h1 and E0 are linear in V2 (Appendix B), so L = sum_{abcd} Gt[abcd] V2[abcd]
// with the effective seed (gamma = diag(n) on the orbitals of the density)
//   Gt = gV2 + G1,  G1[a,b,c,c] -= n_c D'[a][b],  G1[a,c,c,d] += n_c D'[a][d] / 2,
//   D' = gh1 - (2/3) gE0 gamma.
// With V2[ab,cd] = -(M[P,R] + M[R,P]) (eq. tcmf:2el) the adjoint of the packed
// accumulator is symmetric:
//   Gbar[P][R] = -sum_{(a,b) in P, (c,d) in R} (Gt[abcd] + Gt[cdab])
// (sum over the ordered index pairs of each packed pair).  M = sum_g C^T D gives
//   Cbar_c = D_c Gbar,  Dbar_c = C_c Gbar     (row-major [rows][ldP], Gbar symmetric)
// and the local adjoint of eq. tcmf:inter gives Kbar.  Finally, K is linear in
// the coefficients, K^x_P(g) = sum_j c_j sum_g' (r_g - r_g')_x (gj'(r)/r) rho_P(g'),
//   dL/dc_j = sum_{g,g'} (gj'(r)/r) sum_x (r_g - r_g')_x Pi^x(g,g'),
//   Pi^x(g,g') = sum_P Kbar^x_P(g) rho_P(g'),  gj(r) = t^j,  gj'(r) = j t^(j-1)/(1+r)^2.
// Pi is never stored: each tile is reduced into 16 FP64 sums in the epilogue.
//
// Restricted open shell (Appendix A): blocks V2^ab[pq,rs] = -(M^b[P,R] + M^a[R,P])
// for ab in (aa, ab, bb), h1^s = -1/2 (sum_t V2^st . gamma^t - V2^ss[p,k,k,q] n^s_k)
// (V2^ba[pq,rs] = V2^ab[rs,pq]) and E0 = -1/3 sum_s h1^s . gamma^s give the
// effective seeds Gt^aa, Gt^ab, Gt^bb (seed_eff_open) and
//   Gbar^a[P][R] = -sum (Gt^aa[abcd] + Gt^aa[cdab] + Gt^ab[cdab]),
//   Gbar^b[P][R] = -sum (Gt^bb[abcd] + Gt^bb[cdab] + Gt^ab[abcd]),
// which are not symmetric.  M^t = sum_g C^T D^t then gives
//   Cbar_c = sum_t D^t_c Gbar^t^T,  Dbar^t_c = C_c Gbar^t,
// and the local adjoint sums the two spin channels: W, W~ come from the
// total density, Z~^t, Z^t from gamma^t (k_adj_T once per spin).
#pragma once
#include "kernels_contract.h"
#include "xtc_device.h"

namespace xtc {

// occupied orbitals whose T columns one thread of k_adj_T keeps in registers
// at a time (larger sets are taken in groups of this many)
constexpr int kAdjOccGroup = 24;

// ---------------------------------------------------------------- seeds --
// Effective seed Gt[a,b,c,d] (see the header comment); occw[p] = n_p, 0 for
// orbitals outside the density.
__device__ __forceinline__ double seed_eff(const double* __restrict__ gV2, const double* __restrict__ gh1,
                                           double gE0, const double* __restrict__ occw, int N, int a,
                                           int b, int c, int d) {
    const size_t NN = (size_t)N * N;
    double v = gV2 ? gV2[((size_t)a * N + b) * NN + (size_t)c * N + d] : 0.0;
    if (c == d && occw[c] != 0.0) {
        double dp = gh1 ? gh1[(size_t)a * N + b] : 0.0;
        if (a == b) dp -= (2.0 / 3.0) * gE0 * occw[a];
        v -= occw[c] * dp;
    }
    if (b == c && occw[b] != 0.0) {
        double dp = gh1 ? gh1[(size_t)a * N + d] : 0.0;
        if (a == d) dp -= (2.0 / 3.0) * gE0 * occw[a];
        v += 0.5 * occw[b] * dp;
    }
    return v;
}

// Effective seed of block `blk` (0: aa, 1: ab, 2: bb) of the open-shell loss
// (see the header comment): gV2 [3][N^4], gh1 [2][N^2] (either may be NULL),
// occw [3][N] = (n^a, n^b, n^a + n^b), 0 outside the density.
__device__ __forceinline__ double seed_eff_open(const double* __restrict__ gV2, const double* __restrict__ gh1,
                                                double gE0, const double* __restrict__ occw, int N, int blk, int a,
                                                int b, int c, int d) {
    const size_t NN = (size_t)N * N;
    // D'^s[p][q] = gh1^s[p][q] - (1/3) gE0 n^s_p [p == q]
    auto dprime = [&](int sp, int p, int q) {
        double v = gh1 ? gh1[sp * NN + (size_t)p * N + q] : 0.0;
        if (p == q) v -= (1.0 / 3.0) * gE0 * occw[sp * N + p];
        return v;
    };
    double v = gV2 ? gV2[blk * NN * NN + ((size_t)a * N + b) * NN + (size_t)c * N + d] : 0.0;
    if (blk != 1) {   // aa or bb: Coulomb-like and exchange terms of h1^s, s = the block's spin
        const int sp = blk / 2;
        if (c == d && occw[sp * N + c] != 0.0) v -= 0.5 * occw[sp * N + c] * dprime(sp, a, b);
        if (b == c && occw[sp * N + b] != 0.0) v += 0.5 * occw[sp * N + b] * dprime(sp, a, d);
    } else {          // ab: h1^a with t = b, and h1^b with t = a through V2^ba[pq,kk] = V2^ab[kk,pq]
        if (c == d && occw[N + c] != 0.0) v -= 0.5 * occw[N + c] * dprime(0, a, b);
        if (a == b && occw[a] != 0.0) v -= 0.5 * occw[a] * dprime(1, c, d);
    }
    return v;
}

// occw [3][N] = (n_p of the list's spin, total minus that, total) with 0
// outside the density (closed shell: n_p, n_p, 2 n_p; open shell with the
// alpha list: n^a, n^b, n^a + n^b); kidx[p] = position of p in occ or -1.
__global__ void k_occ_flags(OccList occ, int N, double* __restrict__ occw, int* __restrict__ kidx) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    int idx = -1;
    for (int i = 0; i < occ.n; ++i)
        if (occ.k[i] == p) idx = i;
    const double w = idx >= 0 ? occ.w[idx] : 0.0, wt = idx >= 0 ? occ.wt[idx] : 0.0;
    occw[p] = w;
    occw[N + p] = wt - w;
    occw[2 * N + p] = wt;
    kidx[p] = idx;
}

// Gbar[P][R] for P, R < Npair; zero in the padding.
__global__ __launch_bounds__(256) void k_make_gbar(const double* __restrict__ gV2, const double* __restrict__ gh1,
                                                   double gE0, const double* __restrict__ occw, int N,
                                                   int ldP, double* __restrict__ G) {
    const int R = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = blockIdx.y;
    if (R >= ldP) return;
    const int Npair = N * (N + 1) / 2;
    double acc = 0.0;
    if (P < Npair && R < Npair) {
        int p = 0, rem = P;
        while (rem >= N - p) { rem -= N - p; ++p; }
        const int q = p + rem;
        int r = 0;
        rem = R;
        while (rem >= N - r) { rem -= N - r; ++r; }
        const int s = r + rem;
        const int ab[2][2] = {{p, q}, {q, p}};
        const int cd[2][2] = {{r, s}, {s, r}};
        const int nab = p == q ? 1 : 2, ncd = r == s ? 1 : 2;
        for (int i = 0; i < nab; ++i)
            for (int j = 0; j < ncd; ++j) {
                const int a = ab[i][0], b = ab[i][1], c = cd[j][0], d = cd[j][1];
                acc += seed_eff(gV2, gh1, gE0, occw, N, a, b, c, d) + seed_eff(gV2, gh1, gE0, occw, N, c, d, a, b);
            }
    }
    G[(size_t)P * ldP + R] = -acc;
}

// Open shell: Gbar^a, Gbar^b [ldP][ldP] and their transposes GaT, GbT (see the
// header comment); zero in the padding.
__global__ __launch_bounds__(256) void k_make_gbar_open(const double* __restrict__ gV2, const double* __restrict__ gh1,
                                                        double gE0, const double* __restrict__ occw, int N, int ldP,
                                                        double* __restrict__ Ga, double* __restrict__ Gb,
                                                        double* __restrict__ GaT, double* __restrict__ GbT) {
    const int R = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = blockIdx.y;
    if (R >= ldP) return;
    const int Npair = N * (N + 1) / 2;
    double acc_a = 0.0, acc_b = 0.0;
    if (P < Npair && R < Npair) {
        int p = 0, rem = P;
        while (rem >= N - p) { rem -= N - p; ++p; }
        const int q = p + rem;
        int r = 0;
        rem = R;
        while (rem >= N - r) { rem -= N - r; ++r; }
        const int s = r + rem;
        const int ab[2][2] = {{p, q}, {q, p}};
        const int cd[2][2] = {{r, s}, {s, r}};
        const int nab = p == q ? 1 : 2, ncd = r == s ? 1 : 2;
        for (int i = 0; i < nab; ++i)
            for (int j = 0; j < ncd; ++j) {
                const int a = ab[i][0], b = ab[i][1], c = cd[j][0], d = cd[j][1];
                acc_a += seed_eff_open(gV2, gh1, gE0, occw, N, 0, a, b, c, d) +
                         seed_eff_open(gV2, gh1, gE0, occw, N, 0, c, d, a, b) +
                         seed_eff_open(gV2, gh1, gE0, occw, N, 1, c, d, a, b);
                acc_b += seed_eff_open(gV2, gh1, gE0, occw, N, 2, a, b, c, d) +
                         seed_eff_open(gV2, gh1, gE0, occw, N, 2, c, d, a, b) +
                         seed_eff_open(gV2, gh1, gE0, occw, N, 1, a, b, c, d);
            }
    }
    Ga[(size_t)P * ldP + R] = -acc_a;
    Gb[(size_t)P * ldP + R] = -acc_b;
    GaT[(size_t)R * ldP + P] = -acc_a;
    GbT[(size_t)R * ldP + P] = -acc_b;
}

// ------------------------------------------------------- NT GEMM (FP64) --
// Y[i][j] (+)= sum_k X[i][k] Gm[j][k] for i < rows, j < ldP, k < ldP, i.e.
// X Gm^T (closed shell: Gm = Gbar, symmetric).  Workgroup 4 waves as 2 x 2, wave tile 32 (i) x 64 (j).
// Each lane loads 4 consecutive k of one row per operand block (32-byte
// vectors); MFMA e of a 16-k step uses element e, i.e. the k index inside the
// step is permuted as 4 (l/16) + e identically for both operands.
__global__ __launch_bounds__(256) void k_gemm_xg_f64(const double* __restrict__ X, size_t ldx, int rows,
                                                     const double* __restrict__ Gm, int ldP, int n_jt,
                                                     double* __restrict__ Y, size_t ldy, int accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int it = blockIdx.x / n_jt, jt = blockIdx.x % n_jt;
    const int i0 = it * 64 + 32 * (wave & 1), j0 = jt * 128 + 64 * (wave >> 1);
    const int l16 = lane & 15, kq = 4 * (lane >> 4);
    d4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (d4){0.0, 0.0, 0.0, 0.0};
    const double* xr[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) xr[a] = X + (size_t)min(i0 + 16 * a + l16, rows - 1) * ldx + kq;
    const double* gr[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) gr[b] = Gm + (size_t)(j0 + 16 * b + l16) * ldP + kq;
    for (int k = 0; k < ldP; k += 16) {
        d4 xa[2], gb[4];
#pragma unroll
        for (int a = 0; a < 2; ++a) xa[a] = *(const d4*)(xr[a] + k);
#pragma unroll
        for (int b = 0; b < 4; ++b) gb[b] = *(const d4*)(gr[b] + k);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a][e], gb[b][e], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + 16 * a + (lane >> 4) + 4 * v;
            if (i < rows) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    double* y = Y + (size_t)i * ldy + j0 + 16 * b + l16;
                    *y = accumulate ? *y + acc[a][b][v] : acc[a][b][v];
                }
            }
        }
}

// ---------------------------------------------------- local adjoint --
// Per grid point g (one workgroup at a time): with X^x = K^x[:, occ],
// rho_o = rho[:, occ] and the half-weighted symmetric Abar', Bbar'^x
// (off-diagonal packed entries counted half in each full-matrix slot),
//   T^x[r][k] = -2 n_k sum_s (Abar'[r][s] X^x[s][k] + Bbar'^x[r][s] rho_o[s][k])
// and Wbar^x = sum_R Abar_R K^x_R.  T goes to scratch [rows][3][N][nocc].
// Open shell: one launch per spin channel (its Abar, Bbar slots and
// occupations), the second adding into T and Wbar (accumulate).
__global__ __launch_bounds__(256) void k_adj_T(const double* __restrict__ rho_rows, const double* __restrict__ K,
                                               const double* __restrict__ Y, size_t ystride, int rows, int ldP,
                                               int N, OccList occ, double* __restrict__ T,
                                               double* __restrict__ Wbar, int accumulate) {
    extern __shared__ d4 locc[];                    // [nocc][N] of (rho, Kx, Ky, Kz)
    __shared__ double red[3][4];
    const int n = occ.n;
    const size_t kstride = (size_t)rows * ldP;
    const double* Abar = Y + 3 * ystride;           // Y slots: 0..2 Kbar direct, 3 Abar, 4..6 Bbar
    for (int g = blockIdx.x; g < rows; g += gridDim.x) {
        const double* rg = rho_rows + (size_t)g * ldP;
        const double* kg = K + (size_t)g * ldP;
        for (int idx = threadIdx.x; idx < n * N; idx += blockDim.x) {
            const int kk = idx / N, r = idx % N;
            const int P = pair_sym(r, occ.k[kk], N);
            locc[idx] = (d4){rg[P], kg[P], kg[kstride + P], kg[2 * kstride + P]};
        }
        // Wbar^x = sum_R Abar_R K^x_R
        const int Npair = N * (N + 1) / 2;
        double w0 = 0, w1 = 0, w2 = 0;
        const double* ag = Abar + (size_t)g * ldP;
        for (int R = threadIdx.x; R < Npair; R += blockDim.x) {
            const double a = ag[R];
            w0 = fma(a, kg[R], w0);
            w1 = fma(a, kg[kstride + R], w1);
            w2 = fma(a, kg[2 * kstride + R], w2);
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            w0 += __shfl_xor(w0, m);
            w1 += __shfl_xor(w1, m);
            w2 += __shfl_xor(w2, m);
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0) { red[0][wave] = w0; red[1][wave] = w1; red[2][wave] = w2; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int x = 0; x < 3; ++x) {
                const double v = red[x][0] + red[x][1] + red[x][2] + red[x][3];
                Wbar[(size_t)g * 3 + x] = accumulate ? Wbar[(size_t)g * 3 + x] + v : v;
            }
        }
        // T rows: one thread per (r, group of kAdjOccGroup occupied columns),
        // the group's columns in registers
        const int ngrp = (n + kAdjOccGroup - 1) / kAdjOccGroup;
        for (int rq = threadIdx.x; rq < N * ngrp; rq += blockDim.x) {
            const int r = rq % N, k0 = (rq / N) * kAdjOccGroup;
            double t0[kAdjOccGroup], t1[kAdjOccGroup], t2[kAdjOccGroup];
#pragma unroll
            for (int kk = 0; kk < kAdjOccGroup; ++kk) t0[kk] = t1[kk] = t2[kk] = 0.0;
            const double* bx = Y + 4 * ystride + (size_t)g * ldP;
            const double* by = Y + 5 * ystride + (size_t)g * ldP;
            const double* bz = Y + 6 * ystride + (size_t)g * ldP;
            for (int s = 0; s < N; ++s) {
                const int R = pair_sym(r, s, N);
                const double h = r == s ? 1.0 : 0.5;
                const double a = h * ag[R], b0 = h * bx[R], b1 = h * by[R], b2 = h * bz[R];
#pragma unroll
                for (int kk = 0; kk < kAdjOccGroup; ++kk) {
                    if (k0 + kk < n) {
                        const d4 e = locc[(k0 + kk) * N + s];      // (rho_sk, K_sk)
                        t0[kk] = fma(a, e.y, fma(b0, e.x, t0[kk]));
                        t1[kk] = fma(a, e.z, fma(b1, e.x, t1[kk]));
                        t2[kk] = fma(a, e.w, fma(b2, e.x, t2[kk]));
                    }
                }
            }
            double* tg = T + (size_t)g * 3 * N * n;
#pragma unroll
            for (int kk = 0; kk < kAdjOccGroup; ++kk) {
                if (k0 + kk < n) {
                    const double m2n = -2.0 * occ.w[k0 + kk];
                    double* t = tg + r * n + k0 + kk;
                    t[(size_t)0 * N * n] = (accumulate ? t[(size_t)0 * N * n] : 0.0) + m2n * t0[kk];
                    t[(size_t)1 * N * n] = (accumulate ? t[(size_t)1 * N * n] : 0.0) + m2n * t1[kk];
                    t[(size_t)2 * N * n] = (accumulate ? t[(size_t)2 * N * n] : 0.0) + m2n * t2[kk];
                }
            }
        }
        __syncthreads();
    }
}

// Kbar^x_R = Cbar^x_R + Abar_R W^x + (Wt/2) Bbar^x_R + [a = b in occ] nt_a Wbar^x
//            + [b in occ] T^x[a][b] + [a in occ, a != b] T^x[b][a],   R = pair(a <= b)
// with nt the total occupations (closed shell 2 n) and, for the open shell,
// Abar and Bbar summed over the two spin channels (Y slots 3..6 and 7..10)
// (W, Wt from the per-point scalars S of the intermediates: S[0] = Wt/2,
// S[1..3] = W/2, the same in both channels).
// Written into Y slots 0..2 in place (Cbar there already).
__global__ void k_adj_assemble(double* __restrict__ Y, size_t ystride, const double* __restrict__ S,
                               const double* __restrict__ T, const double* __restrict__ Wbar,
                               const int* __restrict__ kidx, const double* __restrict__ occw, int rows, int ldP,
                               int N, int nocc, int nspin) {
    const int Npair = N * (N + 1) / 2;
    const size_t n = (size_t)rows * Npair;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(i / Npair), R = (int)(i % Npair);
        int a = 0, rem = R;
        while (rem >= N - a) { rem -= N - a; ++a; }
        const int b = a + rem;
        const double* s = S + (size_t)g * 8;
        const double hWt = s[0], W[3] = {2.0 * s[1], 2.0 * s[2], 2.0 * s[3]};
        const size_t o = (size_t)g * ldP + R;
        const double ab = Y[3 * ystride + o] + (nspin == 2 ? Y[7 * ystride + o] : 0.0);
        const int ka = kidx[a], kb = kidx[b];
        const double* tg = T + (size_t)g * 3 * N * nocc;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const double bb = Y[(4 + x) * ystride + o] + (nspin == 2 ? Y[(8 + x) * ystride + o] : 0.0);
            double v = Y[x * ystride + o] + ab * W[x] + hWt * bb;
            if (a == b && ka >= 0) v += occw[2 * N + a] * Wbar[(size_t)g * 3 + x];
            if (kb >= 0) v += tg[(size_t)x * N * nocc + a * nocc + kb];
            if (ka >= 0 && a != b) v += tg[(size_t)x * N * nocc + b * nocc + ka];
            Y[x * ystride + o] = v;
        }
    }
}

// ------------------------------------------- Pi tiles and the gradient --
// Pi^x(g,g') = sum_P Kbar^x[g][P] rho[g'][P]; workgroup 4 waves as 2 (g) x 2 (g'),
// wave tile 16 g x 64 g' x 3 components.  Epilogue: for every (g, g') the
// lane owns, s = sum_x (r_g - r_g')_x Pi^x / (r (1+r)^2) and
// part[wg][j-1] += j t^(j-1) s for j = 1..ncoef; then a fixed-order
// reduction over the workgroup.  r == 0 contributes 0.
constexpr int kGradMax = 16;
__global__ __launch_bounds__(256) void k_pi_grad(const double* __restrict__ Kbar, size_t kbstride, int rows,
                                                 const double* __restrict__ rho, int ldP, int Npair_pad16,
                                                 const d4* __restrict__ pos, int g0, int ngp, int n_jt,
                                                 int ncoef, double* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int it = blockIdx.x / n_jt, jt = blockIdx.x % n_jt;
    const int i0 = it * 32 + 16 * (wave & 1), j0 = jt * 128 + 64 * (wave >> 1);
    const int l16 = lane & 15, kq = 4 * (lane >> 4);
    d4 acc[3][4];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[x][b] = (d4){0.0, 0.0, 0.0, 0.0};
    const size_t irow = (size_t)min(i0 + l16, rows - 1);
    const double* kr[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) kr[x] = Kbar + x * kbstride + irow * ldP + kq;
    const double* rr[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) rr[b] = rho + (size_t)(j0 + 16 * b + l16) * ldP + kq;
    for (int k = 0; k < Npair_pad16; k += 16) {
        d4 ka[3], rb[4];
#pragma unroll
        for (int x = 0; x < 3; ++x) ka[x] = *(const d4*)(kr[x] + k);
#pragma unroll
        for (int b = 0; b < 4; ++b) rb[b] = *(const d4*)(rr[b] + k);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int x = 0; x < 3; ++x)
                    acc[x][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ka[x][e], rb[b][e], acc[x][b], 0, 0, 0);
    }
    double gsum[kGradMax];
#pragma unroll
    for (int j = 0; j < kGradMax; ++j) gsum[j] = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + (lane >> 4) + 4 * v;
        if (i >= rows) continue;
        const d4 pi = pos[g0 + i];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int jg = j0 + 16 * b + l16;
            if (jg >= ngp) continue;
            const d4 pj = pos[jg];
            const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            if (!(r2 > 0.0)) continue;
            const double r = sqrt(r2);
            const double q = 1.0 / (1.0 + r);
            const double t = r * q;
            const double s = (dx * acc[0][b][v] + dy * acc[1][b][v] + dz * acc[2][b][v]) * q * q / r;
            double tp = s;
#pragma unroll
            for (int j = 0; j < kGradMax; ++j) {
                gsum[j] = fma((double)(j + 1), tp, gsum[j]);
                tp *= t;
            }
        }
    }
    __shared__ double red[4][kGradMax];
#pragma unroll
    for (int j = 0; j < kGradMax; ++j) {
        double v = gsum[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kGradMax && threadIdx.x < ncoef)
        part[(size_t)blockIdx.x * kGradMax + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// acc[j] (+)= sum_b part[b][j] for j = blockIdx.x < ncoef, in a fixed order:
// thread t sums b = t, t + 256, ... serially, then a fixed tree over the 256
// thread sums; with `out`, also write acc[j] to out[j].  Launch: ncoef x 256.
__global__ __launch_bounds__(256) void k_reduce_grad(const double* __restrict__ part, int nblk, int ncoef,
                                                     double* __restrict__ acc, int accumulate,
                                                     double* __restrict__ out) {
    const int j = blockIdx.x;
    if (j >= ncoef) return;
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[(size_t)b * kGradMax + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = (accumulate ? acc[j] : 0.0) + red[0];
        acc[j] = v;
        if (out) out[j] = v;
    }
}

}  // namespace xtc
