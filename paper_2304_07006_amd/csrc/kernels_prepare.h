// Operand preparation: padded positions, weighted pair densities, fills.
#pragma once
#include "xtc_device.h"

namespace xtc {

// pos[g] = (x, y, z, 0) for g < Ng; zero rows up to the padded grid length.
__global__ void k_prepare_pos(const double* __restrict__ xyz, int Ng, int ngp, d4* __restrict__ pos) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngp) return;
    d4 v = {0.0, 0.0, 0.0, 0.0};
    if (g < Ng) {
        v.x = xyz[3 * (size_t)g + 0];
        v.y = xyz[3 * (size_t)g + 1];
        v.z = xyz[3 * (size_t)g + 2];
    }
    pos[g] = v;
}

// rho[g][P] = w_g phi_p(g) phi_q(g) for g < Ng and P = pair(p,q) < Npair;
// zero in the padded rows and columns.  One workgroup per 32 grid rows: the
// orbital values of those rows are staged in LDS (phi is [N][Ng]).
constexpr int kPrepRows = 32;
__global__ __launch_bounds__(256) void k_prepare_rho(const double* __restrict__ phi,
                                                     const double* __restrict__ w, int N, int Ng,
                                                     int ngp, int ldP, double* __restrict__ rho) {
    extern __shared__ double sphi[];              // [N][kPrepRows]
    const int g0 = blockIdx.x * kPrepRows;
    for (int idx = threadIdx.x; idx < N * kPrepRows; idx += blockDim.x) {
        const int p = idx / kPrepRows, j = idx % kPrepRows;
        const int g = g0 + j;
        sphi[idx] = (g < Ng) ? phi[(size_t)p * Ng + g] : 0.0;
    }
    __syncthreads();
    const int Npair = N * (N + 1) / 2;
    for (int P = threadIdx.x; P < ldP; P += blockDim.x) {
        int p = 0, q = 0;
        if (P < Npair) {
            // invert pair(p,q) = p*N - p(p-1)/2 + (q-p)
            int rem = P;
            while (rem >= N - p) { rem -= N - p; ++p; }
            q = p + rem;
        }
        for (int j = 0; j < kPrepRows; ++j) {
            const int g = g0 + j;
            if (g >= ngp) break;
            double v = 0.0;
            if (P < Npair && g < Ng) v = w[g] * sphi[p * kPrepRows + j] * sphi[q * kPrepRows + j];
            rho[(size_t)g * ldP + P] = v;
        }
    }
}

__global__ void k_fill(double* __restrict__ p, size_t n, double v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace xtc
