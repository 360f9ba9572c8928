// Frozen-core folding of the folded operator (the xTC-FC scheme of the
// results section: corrections computed with all electrons, then the standard
// closed-shell frozen-core equations), with V2[p][q][r][s] = (pq|rs):
//   E  = E0 + 2 sum_c h1[c][c] + sum_{c,d} (2 (cc|dd) - (cd|dc))
//   h[i][j] = h1[a_i][a_j] + sum_c (2 (a_i a_j|cc) - (a_i c|c a_j))
//   V[i][j][k][l] = V2[a_i][a_j][a_k][a_l]
// Every output element is one thread's fixed-order sum (deterministic).
#pragma once
#include "xtc_device.h"

namespace xtc {

constexpr int kMaxFcList = 256;
struct IdxList {
    int32_t n;
    int32_t k[kMaxFcList];
};

__global__ void k_fc_onebody(const double* __restrict__ V2, const double* __restrict__ h1, int N, IdxList core,
                             IdxList act, double* __restrict__ h) {
    const int ij = blockIdx.x * blockDim.x + threadIdx.x;
    const int na = act.n;
    if (ij >= na * na) return;
    const int p = act.k[ij / na], q = act.k[ij % na];
    const size_t n = (size_t)N;
    double v = h1[p * n + q];
    for (int cc = 0; cc < core.n; ++cc) {
        const int c = core.k[cc];
        v += 2.0 * V2[((p * n + q) * n + c) * n + c] - V2[((p * n + c) * n + c) * n + q];
    }
    h[ij] = v;
}

__global__ void k_fc_energy(const double* __restrict__ V2, const double* __restrict__ h1,
                            const double* __restrict__ E0, int N, IdxList core, double* __restrict__ E) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const size_t n = (size_t)N;
    double e1 = 0.0, e2 = 0.0;
    for (int ci = 0; ci < core.n; ++ci) {
        const int c = core.k[ci];
        e1 += h1[c * n + c];
        for (int di = 0; di < core.n; ++di) {
            const int d = core.k[di];
            e2 += 2.0 * V2[((c * n + c) * n + d) * n + d] - V2[((c * n + d) * n + d) * n + c];
        }
    }
    *E = *E0 + 2.0 * e1 + e2;
}

__global__ void k_fc_gather(const double* __restrict__ V2, int N, IdxList act, double* __restrict__ V) {
    const int na = act.n;
    const size_t total = (size_t)na * na * na * na;
    const size_t n = (size_t)N;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int l = (int)(t % na), k = (int)((t / na) % na), j = (int)((t / ((size_t)na * na)) % na),
                  i = (int)(t / ((size_t)na * na * na));
        V[t] = V2[((act.k[i] * n + act.k[j]) * n + act.k[k]) * n + act.k[l]];
    }
}

}  // namespace xtc
