// Symmetric (Loewdin) orthonormalisation of tabulated functions under the
// grid weights, in FP64:  S = chi diag(w) chi^T,  phi = S^{-1/2} chi.
//
// S^{-1/2} comes from a cyclic Jacobi eigen-decomposition (parallel
// round-robin ordering), which keeps the small eigenvalues of an
// ill-conditioned positive definite S to high relative accuracy.
#pragma once
#include "xtc_device.h"

namespace xtc {

// S partials: part[seg][i][j] = sum_{g in seg} w_g chi_i(g) chi_j(g) for i, j < ldS.
// FP64 MFMA, workgroup 4 waves as 2 x 2, wave tile 32 x 32; each lane loads 4
// consecutive grid points of one row (k permuted as 4 (l/16) + e for both operands).
__global__ __launch_bounds__(256) void k_syrk_w_part(const double* __restrict__ chi, const double* __restrict__ w,
                                                     int N, int Ng, int ldS, int n_t, int seg_len,
                                                     double* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int it = blockIdx.x / n_t, jt = blockIdx.x % n_t;
    const int seg = blockIdx.y;
    const int i0 = it * 64 + 32 * (wave & 1), j0 = jt * 64 + 32 * (wave >> 1);
    const int l16 = lane & 15, kq = 4 * (lane >> 4);
    const int gs = seg * seg_len, ge = min(Ng, gs + seg_len);
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (d4){0.0, 0.0, 0.0, 0.0};
    int ri[2], rj[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        ri[a] = min(i0 + 16 * a + l16, N - 1);
        rj[a] = min(j0 + 16 * a + l16, N - 1);
    }
    for (int g = gs; g < ge; g += 16) {
        double wv[4];
        double xa[2][4], xb[2][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gg = g + kq + e;
            const bool ok = gg < ge;
            wv[e] = ok ? w[gg] : 0.0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                xa[a][e] = ok ? chi[(size_t)ri[a] * Ng + gg] * wv[e] : 0.0;
                xb[a][e] = ok ? chi[(size_t)rj[a] * Ng + gg] : 0.0;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a][e], xb[b][e], acc[a][b], 0, 0, 0);
    }
    double* out = part + (size_t)seg * ldS * ldS;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + 16 * a + (lane >> 4) + 4 * v;
#pragma unroll
            for (int b = 0; b < 2; ++b) out[(size_t)i * ldS + j0 + 16 * b + l16] = acc[a][b][v];
        }
}

// S[i][j] = S[j][i] = sum_seg part[seg][min][max] (fixed order, exactly symmetric); U = I.
__global__ void k_syrk_reduce(const double* __restrict__ part, int nseg, int N, int ldS, double* __restrict__ S,
                              double* __restrict__ U) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * N) return;
    const int i = idx / N, j = idx % N;
    const int a = min(i, j), b = max(i, j);
    double s = 0.0;
    for (int q = 0; q < nseg; ++q) s += part[(size_t)q * ldS * ldS + (size_t)a * ldS + b];
    S[idx] = s;
    U[idx] = i == j ? 1.0 : 0.0;
}

// Cyclic Jacobi on the symmetric N x N matrix S (global memory, one workgroup):
// each round applies N'/2 disjoint rotations (round-robin pairing, N' = N
// rounded up to even, the extra index is a dummy), rows first, then columns,
// and accumulates U <- U J.  Sweeps continue while the off-diagonal mass
// exceeds (1e-15)^2 of the diagonal mass, at most max_sweeps (every thread
// takes the same decision).  On exit diag(S) holds the eigenvalues and the
// columns of U the eigenvectors.
constexpr int kJacobiThreads = 1024;
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi(double* __restrict__ S, double* __restrict__ U, int N,
                                                           int max_sweeps, int* __restrict__ sweeps_out) {
    __shared__ double cs[256][2];
    __shared__ int pq[256][2];
    __shared__ double red[kJacobiThreads / 64][2];
    __shared__ int stop;
    const int Np = N + (N & 1);
    const int half = Np / 2;
    const int tid = threadIdx.x;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // convergence test on the current matrix
        double off = 0.0, dia = 0.0;
        for (int idx = tid; idx < N * N; idx += blockDim.x) {
            const int i = idx / N, j = idx % N;
            const double v = S[idx];
            if (i == j) dia += v * v; else off += v * v;
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            off += __shfl_xor(off, m);
            dia += __shfl_xor(dia, m);
        }
        if ((tid & 63) == 0) { red[tid >> 6][0] = off; red[tid >> 6][1] = dia; }
        __syncthreads();
        if (tid == 0) {
            double o = 0.0, d = 0.0;
            for (int k = 0; k < (int)(blockDim.x / 64); ++k) { o += red[k][0]; d += red[k][1]; }
            stop = !(o > 1e-30 * d);
        }
        __syncthreads();
        if (stop) break;
        for (int round = 0; round < Np - 1; ++round) {
            // pairing: index 0 fixed, the others rotate
            if (tid < half) {
                auto player = [&](int slot) { return slot == 0 ? 0 : 1 + (slot - 1 + round) % (Np - 1); };
                const int p = player(tid), q = player(Np - 1 - tid);
                const int a = min(p, q), b = max(p, q);
                double c = 1.0, s = 0.0;
                if (b < N) {
                    const double apq = S[(size_t)a * N + b];
                    if (apq != 0.0) {
                        const double app = S[(size_t)a * N + a], aqq = S[(size_t)b * N + b];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                cs[tid][0] = c; cs[tid][1] = s;
                pq[tid][0] = a; pq[tid][1] = b;
            }
            __syncthreads();
            // rows a, b of every pair: S <- J^T S
            for (int idx = tid; idx < half * N; idx += blockDim.x) {
                const int r = idx / N, k = idx % N;
                const int a = pq[r][0], b = pq[r][1];
                if (b >= N) continue;
                const double c = cs[r][0], s = cs[r][1];
                const double xa = S[(size_t)a * N + k], xb = S[(size_t)b * N + k];
                S[(size_t)a * N + k] = c * xa - s * xb;
                S[(size_t)b * N + k] = s * xa + c * xb;
            }
            __syncthreads();
            // columns a, b of every pair: S <- S J, U <- U J
            for (int idx = tid; idx < half * N; idx += blockDim.x) {
                const int r = idx / N, k = idx % N;
                const int a = pq[r][0], b = pq[r][1];
                if (b >= N) continue;
                const double c = cs[r][0], s = cs[r][1];
                const double xa = S[(size_t)k * N + a], xb = S[(size_t)k * N + b];
                S[(size_t)k * N + a] = c * xa - s * xb;
                S[(size_t)k * N + b] = s * xa + c * xb;
                const double ua = U[(size_t)k * N + a], ub = U[(size_t)k * N + b];
                U[(size_t)k * N + a] = c * ua - s * ub;
                U[(size_t)k * N + b] = s * ua + c * ub;
            }
            __syncthreads();
        }
    }
    if (tid == 0) *sweeps_out = sweep;
}

// X = U diag(lambda^-1/2) U^T with lambda = diag(S) after the Jacobi sweeps.
__global__ void k_inv_sqrt(const double* __restrict__ S, const double* __restrict__ U, int N, double* __restrict__ X) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * N) return;
    const int i = idx / N, j = idx % N;
    const int a = min(i, j), b = max(i, j);       // exact symmetry of X
    double s = 0.0;
    for (int k = 0; k < N; ++k) s += U[(size_t)a * N + k] * U[(size_t)b * N + k] / sqrt(S[(size_t)k * N + k]);
    X[idx] = s;
}

// phi[i][g] = sum_j X[i][j] chi[j][g]; X staged in LDS, one thread per (i, g).
__global__ __launch_bounds__(256) void k_apply_X(const double* __restrict__ X, const double* __restrict__ chi, int N,
                                                 int Ng, double* __restrict__ phi) {
    extern __shared__ double sx[];                 // [N][N]... only row block used
    const int i = blockIdx.y;
    for (int j = threadIdx.x; j < N; j += blockDim.x) sx[j] = X[(size_t)i * N + j];
    __syncthreads();
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Ng) return;
    double s = 0.0;
    for (int j = 0; j < N; ++j) s = fma(sx[j], chi[(size_t)j * Ng + g], s);
    phi[(size_t)i * Ng + g] = s;
}

// Convergence record of the Jacobi solve: out[0] = sweeps taken, out[1] = the
// smallest eigenvalue (NaN if any is NaN).
__global__ void k_lowdin_status(const double* __restrict__ S, int N, const int* __restrict__ sweeps,
                                double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m = S[0];
    for (int i = 1; i < N; ++i) {
        const double v = S[(size_t)i * N + i];
        m = (v < m || v != v) ? v : m;
    }
    out[0] = (double)*sweeps;
    out[1] = m;
}

__global__ void k_diag_copy(const double* __restrict__ S, int N, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) out[i] = S[(size_t)i * N + i];
}

}  // namespace xtc
