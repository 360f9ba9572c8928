// Closed-shell intermediates, two-body assembly and one-body reduction (FP64).
//
// Notation (Appendix B, eq. tcmf:inter), per grid point g, k and l over the
// occupied orbitals, x over the Cartesian components:
//   rho_rs = w phi_r phi_s      K_rs = V_r^s (3-vector)
//   W  = 2 sum_k K_kk           Wt = 2 sum_k rho_kk
//   Zt_rs = sum_k K_rk . K_ks   Z_rs = sum_k (rho_rk K_ks + K_rk rho_ks)
//   A_rs = W . K_rs - Zt_rs     B_rs = Wt/2 K_rs - Z_rs
// C = [rho; Kx; Ky; Kz] and D = [A; Bx; By; Bz] are [4][rows][ldP] arrays,
// and eq. tcmf:2el becomes M[P][R] = sum_g sum_c C_c[g][P] D_c[g][R].
#pragma once
#include "xtc_device.h"

namespace xtc {

// The orbitals of the reference density with the occupations of one spin
// channel, w[i] (gamma^s = sum_i w[i] |k[i]><k[i]|), and of both spins
// together, wt[i] (closed shell: wt = 2 w).  128 entries cover every problem
// the on-chip staging of the intermediates admits (nocc * N <= 5120).
constexpr int kMaxOcc = 128;
struct OccList {
    int32_t n;
    int32_t k[kMaxOcc];
    double w[kMaxOcc];
    double wt[kMaxOcc];
};

// --------------------------------------------------------------------------
// Intermediates.  One workgroup handles one grid point at a time (grid-stride
// over the rows of the chunk).  The occupied columns (rho_rk, K_rk) of that
// point are gathered into LDS as [nocc][N][4] (each thread's loads of up to
// kIGather entries issued together); each thread then owns 4x4
// output blocks (r-block <= s-block) of the upper triangle and accumulates
// Zt and Z over k with register blocking.
// One spin channel s per launch: Z~ and Z carry the occupations n_k of that
// spin, W and W~ those of the total density.  Per-point scalars
// S[g] = (W~/2, W/2 (3), sum_k n_k A_kk, sum_k n_k B_kk (3)) feed the one-body
// reduction.
constexpr int kIGather = 4;
// Staged entry e of the intermediates' LDS array: 32 bytes, and with PAD 16
// more bytes after every 4 entries, so that the 16 lanes of a b128 read phase
// that fetch entries 4 apart (consecutive 4x4 tiles) hit distinct banks.
// (Entries are then 16-byte aligned only: accessed as two 16-byte halves.)
typedef double dpair __attribute__((ext_vector_type(2)));
template <bool PAD> __device__ __forceinline__ dpair* staged(char* base, int e) {
    return (dpair*)(base + 32 * e + (PAD ? 16 * (e >> 2) : 0));
}
template <bool PAD> __device__ __forceinline__ d4 ld_staged(char* base, int e) {
    const dpair* p = staged<PAD>(base, e);
    const dpair lo = p[0], hi = p[1];
    return (d4){lo.x, lo.y, hi.x, hi.y};
}
template <bool PAD> __device__ __forceinline__ void st_staged(char* base, int e, const d4& v) {
    dpair* p = staged<PAD>(base, e);
    p[0] = (dpair){v.x, v.y};
    p[1] = (dpair){v.z, v.w};
}
template <bool PAD>
__global__ __launch_bounds__(256) void k_intermediates(const double* __restrict__ rho_rows,
                                                       const double* __restrict__ K, int rows,
                                                       int ldP, int N, OccList occ,
                                                       double* __restrict__ D, size_t dstride,
                                                       double* __restrict__ S) {
    extern __shared__ __attribute__((aligned(16))) char lraw[];   // [nocc][N] of (rho, Kx, Ky, Kz)
    __shared__ double sW[4];                       // Wx, Wy, Wz, Wt
    const int n = occ.n;
    const size_t kstride = (size_t)rows * ldP;
    const int nb = (N + 3) / 4;
    const int ntiles = nb * (nb + 1) / 2;
    for (int g = blockIdx.x; g < rows; g += gridDim.x) {
        const double* rg = rho_rows + (size_t)g * ldP;
        const double* kg = K + (size_t)g * ldP;
        // every thread issues the loads of up to kIGather entries before storing
        for (int base = threadIdx.x; base < n * N; base += kIGather * 256) {
            d4 e[kIGather];
#pragma unroll
            for (int u = 0; u < kIGather; ++u) {
                const int idx = base + 256 * u;
                if (idx < n * N) {
                    const int kk = idx / N, r = idx % N;
                    const int P = pair_sym(r, occ.k[kk], N);
                    e[u] = (d4){rg[P], kg[P], kg[kstride + P], kg[2 * kstride + P]};
                }
            }
#pragma unroll
            for (int u = 0; u < kIGather; ++u)
                if (base + 256 * u < n * N) st_staged<PAD>(lraw, base + 256 * u, e[u]);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            // wave 0: W, Wt and the per-point scalars of the one-body reduction,
            // lanes over occupied k, then a fixed-pattern butterfly sum.
            const int lane = threadIdx.x;
            // W = sum_k wt_k K_kk and W~ = sum_k wt_k rho_kk over the total
            // density (Appendix A; 2 gamma for the closed shell, Appendix B);
            // w0..w2 = W/2, wt = W~/2
            double w0 = 0, w1 = 0, w2 = 0, wt = 0;
            for (int kk = 0; kk < n; ++kk) {           // every lane, same order
                const d4 e = ld_staged<PAD>(lraw, kk * N + occ.k[kk]);
                const double nk = occ.wt[kk];
                wt = fma(nk, e.x, wt); w0 = fma(nk, e.y, w0); w1 = fma(nk, e.z, w1); w2 = fma(nk, e.w, w2);
            }
            wt *= 0.5; w0 *= 0.5; w1 *= 0.5; w2 *= 0.5;
            double a = 0, b0 = 0, b1 = 0, b2 = 0;
            for (int kk = lane; kk < n; kk += 64) {
                const int k = occ.k[kk];
                const d4 e = ld_staged<PAD>(lraw, kk * N + k);       // (rho_kk, K_kk)
                double zt = 0, z0 = 0, z1 = 0, z2 = 0;
                for (int ll = 0; ll < n; ++ll) {
                    const d4 f = ld_staged<PAD>(lraw, ll * N + k);   // (rho_kl, K_kl)
                    const double nl = occ.w[ll];
                    zt = fma(nl, f.y * f.y + f.z * f.z + f.w * f.w, zt);
                    z0 = fma(nl, 2.0 * f.x * f.y, z0); z1 = fma(nl, 2.0 * f.x * f.z, z1);
                    z2 = fma(nl, 2.0 * f.x * f.w, z2);
                }
                const double nk = occ.w[kk];
                a = fma(nk, 2.0 * (w0 * e.y + w1 * e.z + w2 * e.w) - zt, a);   // n_k A_kk
                b0 = fma(nk, wt * e.y - z0, b0); b1 = fma(nk, wt * e.z - z1, b1);
                b2 = fma(nk, wt * e.w - z2, b2);                               // n_k B_kk
            }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                a += __shfl_xor(a, m); b0 += __shfl_xor(b0, m);
                b1 += __shfl_xor(b1, m); b2 += __shfl_xor(b2, m);
            }
            if (lane == 0) {
                sW[0] = 2.0 * w0; sW[1] = 2.0 * w1; sW[2] = 2.0 * w2; sW[3] = 2.0 * wt;
                double* s = S + (size_t)g * 8;
                s[0] = wt; s[1] = w0; s[2] = w1; s[3] = w2;
                s[4] = a; s[5] = b0; s[6] = b1; s[7] = b2;
            }
        }
        __syncthreads();
        const double W0 = sW[0], W1 = sW[1], W2 = sW[2], hWt = 0.5 * sW[3];
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
            int bi = 0, rem = t;
            while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
            const int bj = bi + rem;
            double zt[4][4], z0[4][4], z1[4][4], z2[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) zt[i][j] = z0[i][j] = z1[i][j] = z2[i][j] = 0.0;
            int ri[4], sj[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ri[i] = min(4 * bi + i, N - 1);
                sj[i] = min(4 * bj + i, N - 1);
            }
            for (int kk = 0; kk < n; ++kk) {
                const int row = kk * N;
                const double nk = occ.w[kk];
                d4 a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = ld_staged<PAD>(lraw, row + ri[i]);
                    b[i] = nk * ld_staged<PAD>(lraw, row + sj[i]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        zt[i][j] = fma(a[i].y, b[j].y, fma(a[i].z, b[j].z, fma(a[i].w, b[j].w, zt[i][j])));
                        z0[i][j] = fma(a[i].x, b[j].y, fma(a[i].y, b[j].x, z0[i][j]));
                        z1[i][j] = fma(a[i].x, b[j].z, fma(a[i].z, b[j].x, z1[i][j]));
                        z2[i][j] = fma(a[i].x, b[j].w, fma(a[i].w, b[j].x, z2[i][j]));
                    }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = 4 * bi + i, s = 4 * bj + j;
                    if (r < N && s < N && r <= s) {
                        const int P = pair_index(r, s, N);
                        const double k0 = kg[P], k1 = kg[kstride + P], k2 = kg[2 * kstride + P];
                        double* dg = D + (size_t)g * ldP + P;
                        dg[0] = fma(W0, k0, fma(W1, k1, W2 * k2)) - zt[i][j];
                        dg[dstride] = hWt * k0 - z0[i][j];
                        dg[2 * dstride] = hWt * k1 - z1[i][j];
                        dg[3 * dstride] = hWt * k2 - z2[i][j];
                    }
                }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Two-body assembly M[P][R] (+)= sum_c sum_{g<rows} C_c[g][P] D_c[g][R]
// on FP64 MFMA.  Workgroup tile 128 x 128, four waves as 2 x 2, each wave
// 64 x 64 (4 x 4 MFMA blocks).  Row block b of a wave maps logical row i to
// P = P0 + 4 i + b (and likewise for columns), so every lane loads one
// 32-byte vector of each operand per k-step.
__global__ __launch_bounds__(256) void k_gemm2b_f64(const double* __restrict__ rho_rows,
                                                    const double* __restrict__ K,
                                                    const double* __restrict__ D, size_t dstride,
                                                    int rows, int ldP, int n_t,
                                                    double* __restrict__ M, int accumulate) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int pt = blockIdx.x % n_t, rt = blockIdx.x / n_t;
    const int P0 = pt * 128 + 64 * (wave & 1);
    const int R0 = rt * 128 + 64 * (wave >> 1);
    const int kq = lane >> 4;
    const int l16 = lane & 15;
    const size_t kstride = (size_t)rows * ldP;
    d4 acc[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[b][c] = (d4){0.0, 0.0, 0.0, 0.0};
    const d4 zero = {0.0, 0.0, 0.0, 0.0};
    for (int comp = 0; comp < 4; ++comp) {
        const double* A = (comp == 0 ? rho_rows : K + (size_t)(comp - 1) * kstride) + P0 + 4 * l16;
        const double* B = D + (size_t)comp * dstride + R0 + 4 * l16;
        int g = kq;
        d4 a = g < rows ? *(const d4*)(A + (size_t)g * ldP) : zero;
        d4 b = g < rows ? *(const d4*)(B + (size_t)g * ldP) : zero;
        for (int kk = 0; kk < rows; kk += 4) {
            const d4 ca = a, cb = b;
            g += 4;
            a = g < rows ? *(const d4*)(A + (size_t)g * ldP) : zero;
            b = g < rows ? *(const d4*)(B + (size_t)g * ldP) : zero;
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
            const int P = P0 + 4 * (lane >> 4) + 16 * v + i;   // logical row (l/16) + 4v
            d4* out = (d4*)(M + (size_t)P * ldP + R0 + 4 * l16);
            d4 val = {acc[i][0][v], acc[i][1][v], acc[i][2][v], acc[i][3][v]};
            if (accumulate) val += *out;
            *out = val;
        }
}

// V2[p][q][r][s] = -(M2[P][R] + M1[R][P]).  Closed shell: M1 = M2 = M, and all
// eight index symmetries hold bitwise because both terms are read for every
// ordering.  Open shell, spins (s, t) of (pq, rs): M2 = M^t, M1 = M^s
// (Appendix A, [Delta U]^{st}[pq, rs] = -(f^t(pq, rs) + f^s(rs, pq))).
__global__ __launch_bounds__(256) void k_finalize_V2(const double* __restrict__ M1, const double* __restrict__ M2,
                                                     int ldP, int N, double* __restrict__ V2) {
    const int p = blockIdx.y, q = blockIdx.z;
    const int pq = p * N + q;
    const int P = pair_sym(p, q, N);
    const int NN = N * N;
    for (int rs = blockIdx.x * blockDim.x + threadIdx.x; rs < NN; rs += gridDim.x * blockDim.x) {
        const int r = rs / N, s = rs % N;
        const int R = pair_sym(r, s, N);
        V2[(size_t)pq * NN + rs] = -(M2[(size_t)P * ldP + R] + M1[(size_t)R * ldP + P]);
    }
}

// --------------------------------------------------------------------------
// One-body reduction, term 1 (diagonal-sum terms), partial over grid splits:
//   T1[split][P] = sum_{g in split} rho_P a + K_P.b + rb A_P + kb.B_P
// with rb = W~/2, kb = W/2 and (a, b) = sum_k n_k (A_kk, B_kk) of this channel,
// or, when S2 (the other spin channel) is given, the mean over both channels
// (Appendix A: the sum over the spin tau of [Delta U]^{s tau} gamma^tau).
__global__ __launch_bounds__(256) void k_onebody_T1(const double* __restrict__ rho_rows,
                                                    const double* __restrict__ K,
                                                    const double* __restrict__ D, size_t dstride,
                                                    const double* __restrict__ S, const double* __restrict__ S2,
                                                    int rows, int ldP, int Npair, double* __restrict__ T1) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    const int split = blockIdx.y, nsplit = gridDim.y;
    if (P >= Npair) return;
    const size_t kstride = (size_t)rows * ldP;
    const int gb = (int)(((long)rows * split) / nsplit), ge = (int)(((long)rows * (split + 1)) / nsplit);
    double acc = 0.0;
    for (int g = gb; g < ge; ++g) {
        const double* s = S + (size_t)g * 8;
        double ab[4] = {s[4], s[5], s[6], s[7]};
        if (S2) {
            const double* s2 = S2 + (size_t)g * 8;
#pragma unroll
            for (int i = 0; i < 4; ++i) ab[i] = 0.5 * (ab[i] + s2[4 + i]);
        }
        const size_t o = (size_t)g * ldP + P;
        acc = fma(rho_rows[o], ab[0], acc);
        acc = fma(K[o], ab[1], fma(K[kstride + o], ab[2], fma(K[2 * kstride + o], ab[3], acc)));
        acc = fma(D[o], s[0], acc);
        acc = fma(D[dstride + o], s[1], fma(D[2 * dstride + o], s[2], fma(D[3 * dstride + o], s[3], acc)));
    }
    T1[(size_t)split * ldP + P] = acc;
}

// One-body reduction, exchange term, partial over grid splits:
//   E[split][p][q] = sum_{g in split} sum_k n_k sum_c C_c[g][pair(p,k)] D_c[g][pair(k,q)]
// Workgroup: a 64 x 64 block of (p,q), 4 x 4 per thread (strided by 16); the occupied columns
// of C and rows of D for that block are staged in LDS per grid point.
constexpr int kEBlk = 64;
__global__ __launch_bounds__(256) void k_onebody_E(const double* __restrict__ rho_rows,
                                                   const double* __restrict__ K,
                                                   const double* __restrict__ D, size_t dstride,
                                                   int rows, int ldP, int N, OccList occ,
                                                   double* __restrict__ E) {
    extern __shared__ double sh[];                 // cs[nocc][64], ds[nocc][64]
    const int n = occ.n;
    double* cs = sh;
    double* ds = sh + n * kEBlk;
    const int nbk = (N + kEBlk - 1) / kEBlk;
    const int pb = blockIdx.x % nbk, qb = blockIdx.x / nbk;
    const int split = blockIdx.y, nsplit = gridDim.y;
    const int gb = (int)(((long)rows * split) / nsplit), ge = (int)(((long)rows * (split + 1)) / nsplit);
    // 16 x 16 threads, 4 x 4 each: p = 64 pb + ti + 16 i, q = 64 qb + tj + 16 j
    // (the 16 lanes of a row read 16 consecutive staged values: no LDS bank
    // conflicts, where 4 consecutive values per thread conflicted)
    const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
    const size_t kstride = (size_t)rows * ldP;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int g = gb; g < ge; ++g) {
        for (int comp = 0; comp < 4; ++comp) {
            const double* Cg = (comp == 0 ? rho_rows : K + (size_t)(comp - 1) * kstride) + (size_t)g * ldP;
            const double* Dg = D + (size_t)comp * dstride + (size_t)g * ldP;
            __syncthreads();
            for (int idx = threadIdx.x; idx < n * kEBlk; idx += blockDim.x) {
                const int kk = idx / kEBlk, j = idx % kEBlk;
                const int k = occ.k[kk];
                const int p = pb * kEBlk + j, q = qb * kEBlk + j;
                cs[idx] = p < N ? Cg[pair_sym(p, k, N)] : 0.0;
                ds[idx] = q < N ? occ.w[kk] * Dg[pair_sym(k, q, N)] : 0.0;
            }
            __syncthreads();
            for (int kk = 0; kk < n; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = cs[kk * kEBlk + ti + 16 * i];
                    b[i] = ds[kk * kEBlk + tj + 16 * i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
            }
        }
    }
    const size_t NN = (size_t)N * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = pb * kEBlk + ti + 16 * i, q = qb * kEBlk + tj + 16 * j;
            if (p < N && q < N) E[split * NN + (size_t)p * N + q] = acc[i][j];
        }
}

// Fold the split partials of one chunk into the packed FP64 accumulator:
//   h1acc[pair(p,q)] (+)= sum_s T1[s][P] - 1/2 (sum_s E[s][p][q] + sum_s E[s][q][p])
__global__ void k_onebody_accumulate(const double* __restrict__ T1, int nsplit_t1,
                                     const double* __restrict__ E, int nsplit_e, int ldP, int N,
                                     double* __restrict__ h1acc, int accumulate) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    const int Npair = N * (N + 1) / 2;
    if (P >= Npair) return;
    int p = 0, rem = P;
    while (rem >= N - p) { rem -= N - p; ++p; }
    const int q = p + rem;
    double t = 0.0;
    for (int s = 0; s < nsplit_t1; ++s) t += T1[(size_t)s * ldP + P];
    const size_t NN = (size_t)N * N;
    double epq = 0.0, eqp = 0.0;
    for (int s = 0; s < nsplit_e; ++s) {
        epq += E[s * NN + (size_t)p * N + q];
        eqp += E[s * NN + (size_t)q * N + p];
    }
    const double v = t - 0.5 * (epq + eqp);
    h1acc[P] = accumulate ? h1acc[P] + v : v;
}

// h1[p][q] = h1acc[pair(p,q)] (symmetric bitwise) for one spin channel, or for
// both (h1acc2, h1 + N^2) in the open-shell form.  E0 = -(2/3) sum_k n_k h1[k][k]
// (Appendix B), or -(1/3) sum_s sum_k n^s_k h1^s[k][k] (Appendix A), summed in
// occ order by one thread.
__global__ void k_onebody_finalize(const double* __restrict__ h1acc, const double* __restrict__ h1acc2, int N,
                                   OccList occ, OccList occ2, double* __restrict__ h1, double* __restrict__ E0) {
    const int pq = blockIdx.x * blockDim.x + threadIdx.x;
    if (pq < N * N) {
        const int p = pq / N, q = pq % N;
        h1[pq] = h1acc[pair_sym(p, q, N)];
        if (h1acc2) h1[N * N + pq] = h1acc2[pair_sym(p, q, N)];
    }
    if (pq == 0) {
        double e = 0.0;
        for (int kk = 0; kk < occ.n; ++kk) e = fma(occ.w[kk], h1acc[pair_index(occ.k[kk], occ.k[kk], N)], e);
        if (h1acc2) {
            for (int kk = 0; kk < occ2.n; ++kk)
                e = fma(occ2.w[kk], h1acc2[pair_index(occ2.k[kk], occ2.k[kk], N)], e);
            *E0 = -(1.0 / 3.0) * e;
        } else {
            *E0 = -(2.0 / 3.0) * e;
        }
    }
}

}  // namespace xtc
