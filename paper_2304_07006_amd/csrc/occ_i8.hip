// Launchers of the integer-sliced occupied-occupied block (occ_i8.h).
#include "occ_i8.h"

#include <algorithm>
#include <cmath>

#include "kernels_occ_i8.h"

namespace xtc {

OccI8Plan occ_i8_plan(int nOP) {
    const int nct = (nOP + 15) / 16;
    const int groups = (nct + kI8MaxCT - 1) / kI8MaxCT;
    const int ct = (nct + groups - 1) / groups;
    return {ct, groups, groups * ct};
}

long occ_i8_max_points(int max_seg) { return (long)max_seg * kI8SegMax; }

double occ_i8_dscale(const JasDev& J) {
    if (J.kind == 0) return 1.0;
    // u'(r) = g(t) = p(t) (1 - t)^2 with t = r/(1+r) in [0, 1) and
    // p(t) = sum_k dcoef[k] t^k.  |g| is bounded by its largest value on a
    // grid of spacing h = 1/4096 plus h/2 times a Lipschitz bound of g on
    // [0, 1]: |g'| = |p' (1-t)^2 - 2 p (1-t)| <= sum_k (k + 2) |dcoef[k]|.
    constexpr int kGrid = 4096;
    double lip = 0.0, gmax = 0.0;
    for (int k = 0; k < 16; ++k) lip += (k + 2) * std::fabs(J.dcoef[k]);
    for (int i = 0; i <= kGrid; ++i) {
        const double t = (double)i / kGrid;
        double p = J.dcoef[15];
        for (int k = 14; k >= 0; --k) p = p * t + J.dcoef[k];
        gmax = std::max(gmax, std::fabs(p) * (1.0 - t) * (1.0 - t));
    }
    const double u = (gmax + 0.5 * lip / kGrid) * (1.0 + 1e-12);   // + the rounding of this evaluation
    if (!(u < 1e300)) return 0.0;   // no usable bound (coefficients near the FP64 range)
    if (!(u > 0.0)) return 1.0;
    int e = 0;
    const double f = std::frexp(2.0 * u, &e);   // 2u = f 2^e, f in [0.5, 1)
    return f == 0.5 ? 2.0 * u : std::ldexp(1.0, e);
}

int balanced_segments(long tiles, long slots, int lo, int hi) {
    slots = std::max(slots, 1L);
    int best = lo;
    double best_eff = 0.0;
    for (int ns = lo; ns <= hi; ++ns) {
        const long t = tiles * ns;
        const double eff = (double)t / (double)(((t + slots - 1) / slots) * slots);
        if (eff >= 0.9) return ns;
        if (eff > best_eff) {
            best_eff = eff;
            best = ns;
        }
    }
    return best;
}

size_t occ_i8_stage_bytes(const OccI8Plan& plan, int ngp) {
    const size_t used = (size_t)plan.ct * kI8Digits * kI8TileB + kI8Kb * 32;
    return (size_t)(ngp / kI8Kb) * plan.groups * ((used + 4095) / 4096 * 4096);   // OccI8Stage<ct>::kBlockB
}

namespace {

template <int CT>
hipError_t prepare_ct(const double* rho_occ, const d4* pos, int ngp, int tw, int nOP, int groups,
                      const unsigned long long* amax, char* stages, hipStream_t st) {
    const size_t nd = (size_t)(ngp / kI8Kb) * groups * CT * 64;
    hipLaunchKernelGGL(k_occ_slice<CT>, dim3((unsigned)std::min<size_t>((nd + 255) / 256, 16384)), dim3(256), 0, st,
                       rho_occ, ngp, tw, nOP, groups, amax, stages);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t np = (size_t)(ngp / kI8Kb) * groups * kI8Kb;
    hipLaunchKernelGGL(k_occ_stage_pos<CT>, dim3((unsigned)std::min<size_t>((np + 255) / 256, 16384)), dim3(256), 0,
                       st, pos, ngp, groups, stages);
    return hipGetLastError();
}

}  // namespace

hipError_t occ_i8_prepare(const double* rho_occ, const d4* pos, int ngp, int tw, int nOP, const OccI8Plan& plan,
                          unsigned long long* amax, void* stages, hipStream_t st) {
    const int chunks = std::max(1, std::min(64, ngp / 2048));
    const int per = (ngp + chunks - 1) / chunks;
    hipLaunchKernelGGL(k_occ_absmax, dim3((unsigned)((nOP + 15) / 16), (unsigned)chunks), dim3(256), 0, st, rho_occ,
                       ngp, tw, nOP, per, amax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    char* sb = (char*)stages;
    switch (plan.ct) {
        case 1: return prepare_ct<1>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 2: return prepare_ct<2>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 3: return prepare_ct<3>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 4: return prepare_ct<4>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 5: return prepare_ct<5>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 6: return prepare_ct<6>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 7: return prepare_ct<7>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 8: return prepare_ct<8>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        case 9: return prepare_ct<9>(rho_occ, pos, ngp, tw, nOP, plan.groups, amax, sb, st);
        default: return hipErrorInvalidValue;
    }
}

namespace {

template <int KIND, int CT>
int build_ct(const d4* pos, const void* stages, const OccI8Plan& plan, int ngp, int g0, int rows, const JasDev& J,
             const unsigned long long* amax, double* part, int ldK, int max_seg, hipStream_t st) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_build_K_occ_i8<KIND, CT>, 256, 0) !=
            hipSuccess)
        return 0;
    const int nkb = ngp / kI8Kb;
    const int kb_max = kI8SegMax / kI8Kb;
    const int lo = std::max(4, (nkb + kb_max - 1) / kb_max);
    if (lo > max_seg) return 0;
    const int n_rb = (rows + 15) / 16;
    const int n_wg = (3 * n_rb + kI8Waves - 1) / kI8Waves;
    const long tiles = (long)n_wg * plan.groups;
    const int want = balanced_segments(tiles, (long)cus * std::max(per_cu, 1), lo, max_seg);
    const int seg_kb = (nkb + want - 1) / want;
    const int nseg = (nkb + seg_kb - 1) / seg_kb;   // every segment starts inside the grid
    hipLaunchKernelGGL((k_build_K_occ_i8<KIND, CT>), dim3((unsigned)n_wg, (unsigned)nseg, (unsigned)plan.groups),
                       dim3(256), 0, st, pos, (const char*)stages, plan.groups, ngp, g0, rows, n_rb, J,
                       occ_i8_dscale(J), amax, part, ldK, seg_kb);
    return hipGetLastError() == hipSuccess ? nseg : 0;
}

template <int KIND>
int build_kind(const d4* pos, const void* stages, const OccI8Plan& plan, int ngp, int g0, int rows, const JasDev& J,
               const unsigned long long* amax, double* part, int ldK, int max_seg, hipStream_t st) {
#define XTC_OCC_I8_CASE(ct)                                                                                         \
    case ct:                                                                                                        \
        return build_ct<KIND, ct>(pos, stages, plan, ngp, g0, rows, J, amax, part, ldK, max_seg, st);
    switch (plan.ct) {
        XTC_OCC_I8_CASE(1)
        XTC_OCC_I8_CASE(2)
        XTC_OCC_I8_CASE(3)
        XTC_OCC_I8_CASE(4)
        XTC_OCC_I8_CASE(5)
        XTC_OCC_I8_CASE(6)
        XTC_OCC_I8_CASE(7)
        XTC_OCC_I8_CASE(8)
        XTC_OCC_I8_CASE(9)
        default: return 0;
    }
#undef XTC_OCC_I8_CASE
}

}  // namespace

int occ_i8_build(const d4* pos, const void* stages, const OccI8Plan& plan, int ngp, int g0, int rows, const JasDev& J,
                 const unsigned long long* amax, double* part, int ldK, int max_seg, hipStream_t st) {
    if (ldK < 16 * plan.nct8 || rows < 1 || ngp % kI8Kb) return 0;
    return J.kind == 0 ? build_kind<0>(pos, stages, plan, ngp, g0, rows, J, amax, part, ldK, max_seg, st)
                       : build_kind<1>(pos, stages, plan, ngp, g0, rows, J, amax, part, ldK, max_seg, st);
}

}  // namespace xtc
