// Host interface of the integer-sliced occupied-occupied block of K
// (kernels_occ_i8.h; built in its own translation unit, occ_i8.hip, so that
// its MFMA accumulators may live in the accumulation registers).
#pragma once
#include <hip/hip_runtime.h>

#include "xtc_device.h"

namespace xtc {

// Column tiling of nOP occupied pairs: groups of ct 16-pair tiles (ct <= 9,
// the accumulators one wave holds), nct8 = groups x ct tiles in all.  The
// library uses the block for one group only (more regenerate d's digits
// once per group and measured slower than the FP64 block).
struct OccI8Plan {
    int ct, groups, nct8;
};
OccI8Plan occ_i8_plan(int nOP);

// Largest grid (padded points) the block handles with at most `max_seg`
// int32 segments.
long occ_i8_max_points(int max_seg);

// Power-of-two scale S_d >= 2 max|d^x| for the Jastrow (|d^x| <= |u'(r)|):
// 1 for Pade (u' = 1/(2 (1 + b r)^2) <= 1/2), else the power of two at or
// above twice a bound of |u'| = |p(t)| (1-t)^2 over t = r/(1+r) in [0, 1)
// (its largest value on a fine grid plus a Lipschitz margin); 0 when that
// bound is not finite (the FP64 block then serves).
double occ_i8_dscale(const JasDev& J);

// The fewest segments in [lo, hi] whose last round of `tiles` equal-work
// workgroups per segment keeps at least 90% of `slots` resident workgroups
// busy, else the most balanced one found.
int balanced_segments(long tiles, long slots, int lo, int hi);

// Bytes of the stage blocks (occ_i8_prepare) for ngp padded points.
size_t occ_i8_stage_bytes(const OccI8Plan& plan, int ngp);

// Stage blocks of the occupied pairs' rho (nct8 x 16 pair columns, ngp
// points) from rho_occ (column tiles of tw pairs, [ngp][tw] each) and the
// positions pos [ngp].  amax (16 nct8 entries) must hold zeros; it receives
// the per-pair largest |rho|.  Returns the launch status.
hipError_t occ_i8_prepare(const double* rho_occ, const d4* pos, int ngp, int tw, int nOP, const OccI8Plan& plan,
                          unsigned long long* amax, void* stages, hipStream_t st);

// The block for rows [g0, g0 + rows): FP64 segment partials
// part[seg][x][r][ldK] (ldK >= 16 nct8) for pair columns < 16 nct8.
// Returns the number of segments (at most max_seg), 0 if the grid needs
// more or a HIP call failed.
int occ_i8_build(const d4* pos, const void* stages, const OccI8Plan& plan, int ngp, int g0, int rows, const JasDev& J,
                 const unsigned long long* amax, double* part, int ldK, int max_seg, hipStream_t st);

}  // namespace xtc
