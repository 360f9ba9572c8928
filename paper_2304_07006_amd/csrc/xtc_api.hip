// libxtc: C ABI (include/xtc.h) over the gfx950 kernels.
//
// Host side only validates, lays out the caller's workspace and launches.
// Workspace layout (all offsets 256-byte aligned), for ldP = xtc_pair_ld(N)
// and ngp = Ng rounded up to 128:
//   pos    [ngp] x 4 doubles          grid positions (x, y, z, 0)
//   rho    [ngp][ldP] doubles         weighted pair densities, zero padded
//   rho_lp [NS][ngp/8][ldL][8]        reduced-precision rho (k8-packed), prec != FP64
//   rho_occ[ldO/tw][ngp][tw], colmap[ldO]  FP64 rho of the occupied-occupied pairs
//                                     (column tiles of tw = 16 occNB pairs)
//   stg, amax                         digit stage blocks and per-pair largest |rho|
//                                     of the integer occupied block (occ_i8.h)
//   M      [ldP][ldP] doubles         FP64 accumulator of the two-body term
//   h1acc  [ldP] doubles              FP64 accumulator of the one-body term
//   T1     [kT1Split][ldP] doubles    per-split partials (one-body, term 1)
//   E      [kESplit][N][N] doubles    per-split partials (one-body, exchange)
//   S      [cap][8] doubles           per-point scalars of the current chunk
//   D      [4][cap][ldP] doubles      A, Bx, By, Bz of the current chunk
//   Kpart  [nsegK][3][kcap][ldL] f32  K-build segment partials of kcap rows (prec != FP64)
//   CDlp   [8][NS][cap/8][ldL][8]     C and D of the chunk, k8-packed (prec != FP64)
//   Mpart  [kMSegGroup][4][ldL][ldL] f32  two-body partials of a group of row segments
// and with XTC_WITH_BACKWARD in prec (the adjoint reuses M for Gbar):
//   Kc [3][cap][ldP], Y [7][cap][ldP], T [cap][3][N][nocc], Wbar [cap][3],
//   gpart [ceil(cap/32) * ngp/128][16], gacc [16], occw [N] f64, kidx [N],
//   reduced forms: rhoR (split rho: FP32 row-major [1][ngp][ldP], split BF16
//   k-packed [NS][ldP/8][ngp][8]), KbL [7][NS][cap * ldP] (split operands of
//   the chunk, same two layouts), split-BF16 3-product form: GsL (k-packed
//   split Gbar, [2][ldP/8][ldP][8])
// and with XTC_WITH_TC2 (two-body TC integrals; ldN = N^2 rounded up to 128):
//   Atc [ldP][ldP], Btc [ldN][ldP] FP64 accumulators, Ftc [cap][ldP],
//   Rg [3][cap][ldN] (w phi grad phi of the chunk)
// ldL = ldP rounded up to 512.  The chunk capacity `cap` is the largest
// multiple of 32 rows that fits in the bytes the caller passes, so every call
// with the same ws_bytes agrees on it.  The segment partials of the reduced
// forms are bounded: the K build runs over a chunk in equal row pieces of at
// most kcap rows (kcap = min(cap, the multiple of 1024 rows whose partials
// fit kKpartBudget bytes, at least 1024)), and the two-body GEMM over groups of
// kMSegGroup row segments, each piece reduced into its FP64 result before the
// next one reuses the partial buffer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/xtc.h"
#include "kernels_build_k.h"
#include "kernels_contract.h"
#include "kernels_fc.h"
#include "kernels_tc2.h"
#include "kernels_lp.h"
#include "kernels_bwd.h"
#include "kernels_lowdin.h"
#include "kernels_prepare.h"
#include "occ_i8.h"

using namespace xtc;

namespace {

thread_local std::string g_err;

xtc_status fail(xtc_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
xtc_status fail(xtc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

constexpr int kT1Split = 64;
constexpr int kESplitMax = 256;
constexpr size_t kAlign = 256;
constexpr int kMaxN = 256;
// Grid points: kernels index the padded grid with 32-bit integers; 2^28 points
// of even one orbital pair already take 275 GB for rho alone.
constexpr int kMaxNg = 1 << 28;
constexpr size_t kLdsMax = 160 * 1024;
// The kernels that stage the occupied columns in dynamic LDS (nocc N of
// (rho, Kx, Ky, Kz)) also keep a few static reduction slots (at most 96 B);
// a workgroup's static plus dynamic LDS must fit kLdsMax.
constexpr size_t kLdsStaticReserve = 1024;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int pair_ld(int N) {
    const long npair = (long)N * (N + 1) / 2;
    return (int)((npair + kPairTile - 1) / kPairTile * kPairTile);
}

// FP32 accumulation segments of the reduced-precision forms (the partials are
// summed in FP64): g' per segment of the K build, grid rows per segment of the
// two-body GEMM.  The split-BF16 forms' error is their dropped products, so
// long segments cost nothing there; the FP32 form's error grows with the
// segment (one rounding per 4 products in v_mfma_f32_16x16x4_f32) and at
// N=128, Ng=150 000 needs 8x and 4x shorter ones to meet the 1e-6 Eh bars.
constexpr int kSegK = 8192, kSegKF32 = 1024;
constexpr int kSegM = 2048, kSegMF32 = 512;
constexpr int kRowQuant = 32;
constexpr int kOccSegMax = 32;  // most segments of the FP64 occupied-block sum over g'
constexpr size_t kKpartBudget = (size_t)16 << 30;  // bytes of K-build segment partials
constexpr int kKpartQuant = 1024;                  // rows: 32 row tiles, one XCD's resident set
constexpr int kMSegGroup = 2;                      // row segments per two-body GEMM launch

struct Layout {
    int N, Ng, nocc, ldP, ngp, Npair, prec;
    int form, ns, es, ldL, ldO, nOP, occNB, nsegK, nspin, ldN, segK, segM;
    int nY;              // adjoint Y slots: Cbar (3), then Abar, Bbar (4) per spin channel
    OccI8Plan i8;        // column tiling of the integer occupied block
    bool i8ok;           // one column group and the grid fits its int32 segments (else the FP64 block serves)
    int ldK8;            // row stride of its segment partials (16 i8.nct8)
    bool tc2;
    bool bwd;
    size_t pos, rho, rho_lp, rho_occ, colmap, stg, amax, M, h1acc, T1, E, gacc, occw, kidx, rhoR, GsL, Atc, Btc, GT;
    size_t fixed;        // bytes of everything that does not scale with the chunk rows (plus reserves)
    size_t chunk0;       // offset of the first chunk buffer (S)
    size_t per_row;      // bytes per chunk row (without the K-build partials)
    size_t kpart_row;    // bytes per row of the K-build partials
    int kcap_max;        // most rows of one K-build piece
    int cap;             // chunk rows that fit (multiple of kRowQuant)
    int kcap;            // rows of the K-build partial buffer: min(cap, kcap_max)
    size_t mslab;        // bytes of the two-body partials of one segM-row segment
    size_t cdw;          // packed operand elements per row and split (CDlp)
    size_t S, D, Kpart, CDlp, Mpart, Kocc, Kc, Y, T, Wbar, gpart, KbL, Ftc, Rg, end;
};

int form_of(int prec) {
    prec &= 0xF;
    return prec == XTC_FP32 ? 1 : prec == XTC_BF16X3 ? 3 : prec == XTC_BF16X6 ? 6 : 0;
}


// 16-column blocks per wave of the FP64 occupied-block kernel, in [1, 9]:
// the count minimising padded columns x (1 + 1/(2 nb)), i.e. the MFMA work
// plus the FP64 generation of the d tile, which each wave repeats for its
// nb blocks.
int occ_blocks(int nOP) {
    int best = 1;
    double best_cost = 1e300;
    for (int nb = 1; nb <= 9; ++nb) {
        const double cost = (double)align_up((size_t)nOP, (size_t)16 * nb) * (1.0 + 0.5 / nb);
        if (cost < best_cost) {
            best = nb;
            best_cost = cost;
        }
    }
    return best;
}

Layout make_layout(const xtc_problem* pb, int prec) {
    Layout L{};
    L.N = pb->N;
    L.Ng = pb->Ng;
    L.nocc = pb->nocc;
    L.nspin = pb->occ_n_beta ? 2 : 1;
    L.prec = prec;
    L.ldP = pair_ld(pb->N);
    L.Npair = pb->N * (pb->N + 1) / 2;
    L.ngp = (int)align_up((size_t)pb->Ng, kGridPad);
    L.form = form_of(prec);
    L.ns = L.form == 1 ? 1 : L.form == 3 ? 2 : L.form == 6 ? 3 : 0;
    L.es = L.form == 1 ? 4 : 2;
    L.ldL = (int)align_up((size_t)L.ldP, kLpCols);
    L.nOP = pb->nocc * (pb->nocc + 1) / 2;
    L.occNB = occ_blocks(L.nOP);
    L.ldO = (int)align_up((size_t)L.nOP, (size_t)16 * L.occNB);
    L.i8 = occ_i8_plan(L.nOP);
    // the integer block serves one column group (at most 144 occupied pairs):
    // with two, each of them regenerates d's digits, and at N=160 with 20
    // occupied orbitals it measured slower than the FP64 block
    L.i8ok = L.ngp <= occ_i8_max_points(kOccSegMax) && L.i8.groups == 1;
    L.ldK8 = 16 * L.i8.nct8;
    L.segK = L.form == 1 ? kSegKF32 : kSegK;
    L.segM = L.form == 1 ? kSegMF32 : kSegM;
    L.nsegK = (L.ngp + L.segK - 1) / L.segK;
    L.bwd = (prec & XTC_WITH_BACKWARD) != 0;
    L.tc2 = (prec & XTC_WITH_TC2) != 0;
    L.nY = 3 + 4 * L.nspin;
    L.ldN = (int)align_up((size_t)pb->N * pb->N, 128);
    const bool lp = L.form != 0;
    size_t off = 0;
    L.pos = off;     off = align_up(off + (size_t)L.ngp * 4 * sizeof(double), kAlign);
    L.rho = off;     off = align_up(off + (size_t)L.ngp * L.ldP * sizeof(double), kAlign);
    L.rho_lp = off;  off = align_up(off + (lp ? (size_t)L.ns * L.ngp * L.ldL * L.es : 0), kAlign);
    L.rho_occ = off; off = align_up(off + (lp ? (size_t)L.ngp * L.ldO * sizeof(double) : 0), kAlign);
    L.colmap = off;  off = align_up(off + (lp ? (size_t)L.ldO * sizeof(int) : 0), kAlign);
    const bool i8 = lp && L.i8ok;
    L.stg = off;     off = align_up(off + (i8 ? occ_i8_stage_bytes(L.i8, L.ngp) : 0), kAlign);
    L.amax = off;    off = align_up(off + (i8 ? (size_t)L.ldK8 * sizeof(double) : 0), kAlign);
    L.M = off;       off = align_up(off + (size_t)L.nspin * L.ldP * L.ldP * sizeof(double), kAlign);
    L.h1acc = off;   off = align_up(off + (size_t)L.nspin * L.ldP * sizeof(double), kAlign);
    L.T1 = off;      off = align_up(off + (size_t)kT1Split * L.ldP * sizeof(double), kAlign);
    L.E = off;       off = align_up(off + (size_t)kESplitMax * L.N * L.N * sizeof(double), kAlign);
    L.gacc = off;    off = align_up(off + (L.bwd ? kGradMax * sizeof(double) : 0), kAlign);
    L.occw = off;    off = align_up(off + (L.bwd ? (size_t)3 * L.N * sizeof(double) : 0), kAlign);
    L.kidx = off;    off = align_up(off + (L.bwd ? (size_t)L.N * sizeof(int) : 0), kAlign);
    L.rhoR = off;    off = align_up(off + (L.bwd && lp ? (size_t)L.ns * L.ngp * L.ldP * L.es : 0), kAlign);
    const bool bsplit = L.bwd && L.form == 3;   // split-BF16 X Gbar products (3-product form)
    // open shell: Gbar^a, Gbar^b in M, their transposes in GT; split copies
    // (k-packed) of Gbar (closed) or of Gbar^a, Gbar^b, Gbar^aT, Gbar^bT
    L.GT = off;      off = align_up(off + (L.bwd && L.nspin == 2 ? (size_t)2 * L.ldP * L.ldP * sizeof(double) : 0),
                                    kAlign);
    L.GsL = off;     off = align_up(off + (bsplit ? (size_t)(L.nspin == 2 ? 4 : 1) * L.ns * L.ldP * L.ldP * L.es : 0),
                                    kAlign);
    L.Atc = off;     off = align_up(off + (L.tc2 ? (size_t)L.ldP * L.ldP * sizeof(double) : 0), kAlign);
    L.Btc = off;     off = align_up(off + (L.tc2 ? (size_t)L.ldN * L.ldP * sizeof(double) : 0), kAlign);
    const size_t gslab = (size_t)(L.ngp / 128) * kGradMax * sizeof(double);   // one 32-row tile of partials
    // partials of one row segment: the four components of the two-body GEMM, or
    // the TC integrals' B (three components summed in one partial)
    L.mslab = lp ? std::max((size_t)4 * L.ldL * L.ldL, L.tc2 ? (size_t)L.ldN * L.ldL : 0) * sizeof(float) : 0;
    // packed operands: C and D of the two-body GEMM (8 components of ldL), or
    // w phi grad phi (3 of ldN) and K (3 of ldL) of the TC integrals
    L.cdw = std::max((size_t)8 * L.ldL, L.tc2 ? (size_t)3 * L.ldN + (size_t)3 * L.ldL : 0);
    const size_t mslab = L.mslab;
    L.chunk0 = off;
    L.fixed = off + (size_t)kMSegGroup * mslab + (L.bwd ? gslab : 0) + 16 * kAlign;
    L.per_row = (size_t)L.nspin * (8 * sizeof(double) + (size_t)4 * L.ldP * sizeof(double));
    if (lp) L.per_row += (size_t)kOccSegMax * 3 * std::max(L.ldO, L.ldK8) * sizeof(double);
    if (lp) L.per_row += L.cdw * L.ns * L.es;
    L.kpart_row = lp ? (size_t)L.nsegK * 3 * L.ldL * sizeof(float) : 0;
    L.kcap_max = lp ? (int)std::max<size_t>(kKpartQuant, kKpartBudget / L.kpart_row / kKpartQuant * kKpartQuant) : 0;
    if (L.tc2) L.per_row += (size_t)L.ldP * sizeof(double) + (size_t)3 * L.ldN * sizeof(double);
    if (L.bwd)
        L.per_row += (size_t)(3 + L.nY) * L.ldP * sizeof(double) + (size_t)3 * L.N * L.nocc * sizeof(double) +
                     3 * sizeof(double) + (gslab + 31) / 32 + (lp ? (size_t)7 * L.ns * L.ldP * L.es : 0);
    L.cap = 0;
    return L;
}

// Bytes of a workspace for chunks of `rows` rows (a multiple of kRowQuant).
size_t layout_bytes(const Layout& L, size_t rows) {
    return L.fixed + rows * L.per_row + std::min(rows, (size_t)L.kcap_max) * L.kpart_row;
}

// Chunk capacity that `bytes` allows (the inverse of layout_bytes), and the
// offsets of the chunk buffers for it.
void place_chunk(Layout& L, size_t bytes) {
    long cap = 0;
    if (bytes > L.fixed) {
        const size_t b = bytes - L.fixed;
        const size_t c1 = b / (L.per_row + L.kpart_row);   // rows, if the partials cover all of them
        if (c1 <= (size_t)L.kcap_max) cap = (long)c1;
        else cap = (long)((b - (size_t)L.kcap_max * L.kpart_row) / L.per_row);
    }
    cap = cap / kRowQuant * kRowQuant;
    const long most = (long)align_up((size_t)L.Ng, kRowQuant);
    if (cap > most) cap = most;
    L.cap = (int)cap;
    L.kcap = std::min(L.cap, L.kcap_max);
    const bool lp = L.form != 0;
    const size_t gslab = (size_t)(L.ngp / 128) * kGradMax * sizeof(double);
    size_t off = L.chunk0;
    L.S = off;       off = align_up(off + (size_t)L.nspin * cap * 8 * sizeof(double), kAlign);
    L.D = off;       off = align_up(off + (size_t)L.nspin * 4 * cap * L.ldP * sizeof(double), kAlign);
    L.Kpart = off;   off = align_up(off + (lp ? (size_t)L.kcap * L.kpart_row : 0), kAlign);
    L.CDlp = off;    off = align_up(off + (lp ? L.cdw * L.ns * cap * L.es : 0), kAlign);
    L.Mpart = off;   off = align_up(off + (size_t)kMSegGroup * L.mslab, kAlign);
    L.Kocc = off;    off = align_up(off + (lp ? (size_t)kOccSegMax * 3 * cap * std::max(L.ldO, L.ldK8) * sizeof(double) : 0),
                                    kAlign);
    const bool b = L.bwd;
    L.Kc = off;      off = align_up(off + (b ? (size_t)3 * cap * L.ldP * sizeof(double) : 0), kAlign);
    L.Y = off;       off = align_up(off + (b ? (size_t)L.nY * cap * L.ldP * sizeof(double) : 0), kAlign);
    L.T = off;       off = align_up(off + (b ? (size_t)cap * 3 * L.N * L.nocc * sizeof(double) : 0), kAlign);
    L.Wbar = off;    off = align_up(off + (b ? (size_t)cap * 3 * sizeof(double) : 0), kAlign);
    L.gpart = off;   off = align_up(off + (b ? (size_t)((cap + 31) / 32) * gslab : 0), kAlign);
    L.KbL = off;     off = align_up(off + (b && lp ? (size_t)7 * L.ns * cap * L.ldP * L.es : 0), kAlign);
    L.Ftc = off;     off = align_up(off + (L.tc2 ? (size_t)cap * L.ldP * sizeof(double) : 0), kAlign);
    L.Rg = off;      off = align_up(off + (L.tc2 ? (size_t)3 * cap * L.ldN * sizeof(double) : 0), kAlign);
    L.end = off;
    if (L.end > bytes) L.cap = 0;   // cannot happen by construction; refuse rather than overrun
}

// LDS of k_intermediates: the padded layout (16 bytes after every 4 entries)
// when it fits, else the plain one (check_problem admits sizes up to the
// plain layout's limit)
bool intermediates_padded(const Layout& L) {
    const size_t e = (size_t)L.nocc * L.N;
    return e * 32 + ((e + 3) / 4) * 16 <= kLdsMax - kLdsStaticReserve;
}
size_t lds_intermediates(const Layout& L) {
    const size_t e = (size_t)L.nocc * L.N;
    return e * 32 + (intermediates_padded(L) ? ((e + 3) / 4) * 16 : 0);
}

xtc_status check_problem(const xtc_problem* pb) {
    if (!pb) return fail(XTC_E_ARG, "problem is NULL");
    if (pb->reserved != 0) return fail(XTC_E_ARG, "problem.reserved must be 0");
    if (pb->N < 1 || pb->N > kMaxN) return fail(XTC_E_ARG, "N=%d outside [1,%d]", pb->N, kMaxN);
    if (pb->Ng < 1) return fail(XTC_E_ARG, "Ng=%d < 1", pb->Ng);
    if (pb->Ng > kMaxNg) return fail(XTC_E_UNSUPPORTED, "Ng=%d above %d", pb->Ng, kMaxNg);
    if (pb->nocc < 1 || pb->nocc > pb->N || pb->nocc > kMaxOcc)
        return fail(XTC_E_ARG, "nocc=%d outside [1,min(N,%d)]", pb->nocc, kMaxOcc);
    if (!pb->xyz || !pb->w || !pb->phi || !pb->occ) return fail(XTC_E_ARG, "NULL array in problem");
    std::vector<char> seen(pb->N, 0);
    for (int i = 0; i < pb->nocc; ++i) {
        const int k = pb->occ[i];
        if (k < 0 || k >= pb->N) return fail(XTC_E_ARG, "occ[%d]=%d outside [0,N)", i, k);
        if (seen[k]) return fail(XTC_E_ARG, "occ[%d]=%d repeated", i, k);
        seen[k] = 1;
        if (pb->occ_n && !std::isfinite(pb->occ_n[i])) return fail(XTC_E_ARG, "occ_n[%d] not finite", i);
        if (pb->occ_n_beta && !std::isfinite(pb->occ_n_beta[i]))
            return fail(XTC_E_ARG, "occ_n_beta[%d] not finite", i);
    }
    if ((size_t)pb->nocc * pb->N * 4 * sizeof(double) > kLdsMax - kLdsStaticReserve)
        return fail(XTC_E_UNSUPPORTED, "nocc*N=%d exceeds the on-chip staging of the intermediates",
                    pb->nocc * pb->N);
    return XTC_OK;
}

xtc_status check_prec(int prec) {
    const int base = prec & 0xF;
    if ((prec & ~(0xF | XTC_WITH_BACKWARD | XTC_WITH_TC2)) ||
        (base != XTC_FP64 && base != XTC_FP32 && base != XTC_BF16X3 && base != XTC_BF16X6))
        return fail(XTC_E_ARG, "prec=%d unknown", prec);
    return XTC_OK;
}

xtc_status check_jastrow(const xtc_jastrow* j, JasDev* out) {
    if (!j) return fail(XTC_E_ARG, "jastrow is NULL");
    JasDev d{};
    d.kind = j->kind;
    if (j->kind == 0) {
        if (!(std::isfinite(j->b) && j->b >= 0.0)) return fail(XTC_E_ARG, "Pade b=%g must be finite and >= 0", j->b);
        d.b = j->b;
        d.ncoef = 0;
    } else if (j->kind == 1) {
        if (j->ncoef < 1 || j->ncoef > 16) return fail(XTC_E_ARG, "ncoef=%d outside [1,16]", j->ncoef);
        for (int k = 0; k < j->ncoef; ++k) {
            if (!std::isfinite(j->coef[k])) return fail(XTC_E_ARG, "coef[%d] not finite", k);
            d.dcoef[k] = (k + 1) * j->coef[k];
            if (k >= 1) d.d2coef[k - 1] = (k + 1) * k * j->coef[k];
        }
        d.ncoef = j->ncoef;
    } else {
        return fail(XTC_E_ARG, "jastrow kind=%d unknown", j->kind);
    }
    d.fb = (float)d.b;
    for (int k = 0; k < 16; ++k) {
        d.fdcoef[k] = (float)d.dcoef[k];
        d.fd2coef[k] = (float)d.d2coef[k];
    }
    *out = d;
    return XTC_OK;
}

xtc_status check_ws(const Layout& L, void* ws, size_t bytes) {
    if (!ws) return fail(XTC_E_WORKSPACE, "workspace is NULL");
    if ((uintptr_t)ws % kAlign) return fail(XTC_E_WORKSPACE, "workspace not 256-byte aligned");
    if (L.cap < kRowQuant)
        return fail(XTC_E_WORKSPACE, "workspace of %zu bytes holds no chunk (need >= %zu)", bytes,
                    layout_bytes(L, kRowQuant));
    return XTC_OK;
}

xtc_status check_range(const Layout& L, int g0, int g1) {
    if (!(0 <= g0 && g0 < g1 && g1 <= L.Ng)) return fail(XTC_E_ARG, "rows [%d,%d) not inside [0,%d)", g0, g1, L.Ng);
    if (g1 - g0 > L.cap)
        return fail(XTC_E_WORKSPACE, "chunk of %d rows exceeds the workspace capacity of %d rows", g1 - g0, L.cap);
    return XTC_OK;
}

xtc_status check_align(const void* p, const char* name) {
    if ((uintptr_t)p % 32) return fail(XTC_E_ARG, "%s must be 32-byte aligned", name);
    return XTC_OK;
}

// Occupations of spin channel `spin` (0 alpha, 1 beta) and of the total
// density.  Closed shell (occ_n_beta NULL): one channel, total = 2 n.
OccList make_occ(const xtc_problem* pb, int spin = 0) {
    OccList o{};
    o.n = pb->nocc;
    for (int i = 0; i < pb->nocc; ++i) {
        const double na = pb->occ_n ? pb->occ_n[i] : 1.0;
        o.k[i] = pb->occ[i];
        if (pb->occ_n_beta) {
            const double nb = pb->occ_n_beta[i];
            o.w[i] = spin == 0 ? na : nb;
            o.wt[i] = na + nb;
        } else {
            o.w[i] = na;
            o.wt[i] = 2.0 * na;
        }
    }
    return o;
}

xtc_status launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(XTC_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return XTC_OK;
}

template <typename T>
T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

xtc_status fill(double* p, size_t n, hipStream_t st) {
    if (n == 0) return XTC_OK;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, n, 0.0);
    return launched("fill");
}

// Intermediates of rows [g0, g1) into D and S of the workspace.
xtc_status run_intermediates(const Layout& L, const xtc_problem* pb, const double* K, int g0, int g1,
                             void* ws, hipStream_t st) {
    const int rows = g1 - g0;
    const double* rho_rows = at<double>(ws, L.rho) + (size_t)g0 * L.ldP;
    const size_t dstride = (size_t)L.cap * L.ldP;
    const int blocks = std::min(rows, 4096);
    const size_t lds = lds_intermediates(L);
    const bool pad = intermediates_padded(L);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(pad ? (const void*)k_intermediates<true> : (const void*)k_intermediates<false>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError();   // do not leave the error for the caller's next HIP call
            return fail(XTC_E_HIP, "intermediates LDS attribute: %s", hipGetErrorString(e));
        }
    }
    for (int sp = 0; sp < L.nspin; ++sp) {
        if (pad)
            hipLaunchKernelGGL(k_intermediates<true>, dim3(blocks), dim3(256), lds, st, rho_rows, K, rows, L.ldP, L.N,
                               make_occ(pb, sp), at<double>(ws, L.D) + (size_t)sp * 4 * dstride, dstride,
                               at<double>(ws, L.S) + (size_t)sp * L.cap * 8);
        else
            hipLaunchKernelGGL(k_intermediates<false>, dim3(blocks), dim3(256), lds, st, rho_rows, K, rows, L.ldP,
                               L.N, make_occ(pb, sp), at<double>(ws, L.D) + (size_t)sp * 4 * dstride, dstride,
                               at<double>(ws, L.S) + (size_t)sp * L.cap * 8);
        xtc_status s;
        if ((s = launched("intermediates")) != XTC_OK) return s;
    }
    return XTC_OK;
}

// ---------------------------------------------------------------- reduced precision
template <int FORM>
xtc_status pack_lp(const double* src, int nrows, int ld_src, int ncols, int n8, int ld_dst, void* dst,
                   size_t split_stride, hipStream_t st) {
    hipLaunchKernelGGL((k_pack_lp<FORM>), dim3((ld_dst + 255) / 256, n8), dim3(256), 0, st, src, nrows, ld_src, ncols,
                       ld_dst, dst, split_stride);
    return launched("pack_lp");
}

xtc_status pack_any(int form, const double* src, int nrows, int ld_src, int ncols, int n8, int ld_dst, void* dst,
                    size_t split_stride, hipStream_t st) {
    switch (form) {
        case 1: return pack_lp<1>(src, nrows, ld_src, ncols, n8, ld_dst, dst, split_stride, st);
        case 3: return pack_lp<3>(src, nrows, ld_src, ncols, n8, ld_dst, dst, split_stride, st);
        default: return pack_lp<6>(src, nrows, ld_src, ncols, n8, ld_dst, dst, split_stride, st);
    }
}

template <int KIND, int FORM, int NC = 3>
void launch_build_lp(const Layout& L, int g0, int rows, const JasDev& J, void* ws, hipStream_t st) {
    const int n_rt = (rows + kLpRows - 1) / kLpRows;
    // ldL is a multiple of 512; a 1024-column tile past it has only inactive waves there
    constexpr int cols = LpTile<KIND, FORM, NC>::cols;
    const int n_ct = (L.ldL + cols - 1) / cols;
    hipLaunchKernelGGL((k_build_K_lp<KIND, FORM, NC>), dim3(n_rt * n_ct * L.nsegK), dim3(kLpThreads), 0, st,
                       at<d4>(ws, L.pos), at<void>(ws, L.rho_lp), (size_t)L.ngp * L.ldL, L.ldL, L.ngp, g0, rows, n_rt,
                       L.segK, J, at<float>(ws, L.Kpart), L.kcap, L.ldP, n_ct, L.nsegK);
}

// Segments of the g' sum of the FP64 occupied block for a grid of `tiles`
// workgroups per segment: the fewest, from 4, whose last round of workgroups
// keeps at least 90% of the `slots` resident workgroups busy (equal-work
// workgroups finish in rounds, and a short last round idles the rest of the
// chip), else the best found.
int occ_segments(long tiles, long slots) { return balanced_segments(tiles, slots, 4, kOccSegMax); }

// Launch the FP64 occupied block with the segment count from the kernel's
// occupancy on the current device; returns that count (0 on a HIP error).
template <int KIND, int NB>
int launch_build_occ_nb(const Layout& L, int g0, int rows, int n_rt, const JasDev& J, void* ws, hipStream_t st) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_build_K_occ<KIND, NB>, 256, 0) !=
            hipSuccess)
        return 0;
    const long tiles = (long)n_rt * (L.ldO / (16 * NB));
    const int want = occ_segments(tiles, (long)std::max(cus, 1) * std::max(per_cu, 1));
    const int seg_len = (int)align_up((size_t)((L.ngp + want - 1) / want), 32);   // whole 32-point stages
    const int nseg = (L.ngp + seg_len - 1) / seg_len;   // every segment starts inside the grid
    const dim3 grid((unsigned)tiles, nseg);
    hipLaunchKernelGGL((k_build_K_occ<KIND, NB>), grid, dim3(256), 0, st, at<d4>(ws, L.pos), at<double>(ws, L.rho_occ),
                       L.ldO, L.ngp, g0, rows, n_rt, J, at<double>(ws, L.Kocc), seg_len);
    return nseg;
}

template <int KIND>
int launch_build_occ(const Layout& L, int g0, int rows, int n_rt, const JasDev& J, void* ws, hipStream_t st) {
    switch (L.occNB) {
        case 1: return launch_build_occ_nb<KIND, 1>(L, g0, rows, n_rt, J, ws, st);
        case 2: return launch_build_occ_nb<KIND, 2>(L, g0, rows, n_rt, J, ws, st);
        case 3: return launch_build_occ_nb<KIND, 3>(L, g0, rows, n_rt, J, ws, st);
        case 4: return launch_build_occ_nb<KIND, 4>(L, g0, rows, n_rt, J, ws, st);
        case 5: return launch_build_occ_nb<KIND, 5>(L, g0, rows, n_rt, J, ws, st);
        case 6: return launch_build_occ_nb<KIND, 6>(L, g0, rows, n_rt, J, ws, st);
        case 7: return launch_build_occ_nb<KIND, 7>(L, g0, rows, n_rt, J, ws, st);
        case 8: return launch_build_occ_nb<KIND, 8>(L, g0, rows, n_rt, J, ws, st);
        default: return launch_build_occ_nb<KIND, 9>(L, g0, rows, n_rt, J, ws, st);
    }
}

// The split K build of rows [g0, g0 + rows) (nc = 3: K, or nc = 1: F of the
// TC integrals) in equal pieces (multiples of 32 rows) of at most kcap rows:
// segment partials, then their FP64 sum into out[c][r][P] (component stride
// `rows` rows).  Each piece costs about a millisecond of launch ramp and tail
// at N=160, so the pieces are as few as the partial buffer allows.
template <int NC>
xtc_status build_lp_pieces(const Layout& L, int g0, int rows, const JasDev& J, double* out, void* ws, hipStream_t st) {
    xtc_status s;
    const int npiece = (rows + L.kcap - 1) / L.kcap;
    const int piece = std::min(L.kcap, (int)align_up((size_t)((rows + npiece - 1) / npiece), kRowQuant));
    for (int r0 = 0; r0 < rows; r0 += piece) {
        const int nr = std::min(piece, rows - r0);
        if (J.kind == 0) {
            if (L.form == 1) launch_build_lp<0, 1, NC>(L, g0 + r0, nr, J, ws, st);
            else if (L.form == 3) launch_build_lp<0, 3, NC>(L, g0 + r0, nr, J, ws, st);
            else launch_build_lp<0, 6, NC>(L, g0 + r0, nr, J, ws, st);
        } else {
            if (L.form == 1) launch_build_lp<1, 1, NC>(L, g0 + r0, nr, J, ws, st);
            else if (L.form == 3) launch_build_lp<1, 3, NC>(L, g0 + r0, nr, J, ws, st);
            else launch_build_lp<1, 6, NC>(L, g0 + r0, nr, J, ws, st);
        }
        if ((s = launched(NC == 3 ? "build_K_lp" : "build_F_lp")) != XTC_OK) return s;
        const size_t n4 = (size_t)NC * nr * L.ldP / 4;   // k_reduce_K: four pairs per thread
        const unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 16384);
        hipLaunchKernelGGL(k_reduce_K, dim3(blocks), dim3(256), 0, st, at<float>(ws, L.Kpart), L.nsegK, L.kcap,
                           L.ldL, nr, L.ldP, out + (size_t)r0 * L.ldP, rows, NC);
        if ((s = launched("reduce_K")) != XTC_OK) return s;
    }
    return XTC_OK;
}

// How the occupied-occupied pairs of K are computed in the reduced forms.
enum OccMode {
    kOccReduced = 0,   // left in the reduced arithmetic (XTC_K_REDUCED_OCC)
    kOccExact = 1,     // integer-sliced block if the grid fits it, else FP64 MFMA
    kOccFP64 = 2       // FP64 MFMA block (XTC_K_OCC_FP64)
};

xtc_status build_K_lp(const Layout& L, int g0, int rows, const JasDev& J, double* K, int occ, void* ws,
                      hipStream_t st) {
    xtc_status s;
    if ((s = build_lp_pieces<3>(L, g0, rows, J, K, ws, st)) != XTC_OK) return s;
    if (occ == kOccReduced) return XTC_OK;
    // occupied-occupied pairs, written over the reduced-precision values:
    // segments of the sum over g' (enough, and evenly enough, to fill the chip),
    // FP64 partials, then a fixed-order reduction scattered into K
    double* part = at<double>(ws, L.Kocc);
    int nseg = 0, ldK = L.ldO;
    if (occ == kOccExact && L.i8ok && occ_i8_dscale(J) > 0.0) {
        ldK = L.ldK8;
        nseg = occ_i8_build(at<d4>(ws, L.pos), at<void>(ws, L.stg), L.i8, L.ngp, g0, rows, J,
                            at<unsigned long long>(ws, L.amax), part, ldK, kOccSegMax, st);
        if (nseg == 0) {
            const hipError_t e = hipGetLastError();   // 0 segments without a HIP error: a layout check failed
            return e != hipSuccess ? fail(XTC_E_HIP, "integer occupied block: %s", hipGetErrorString(e))
                                   : fail(XTC_E_UNSUPPORTED, "integer occupied block: grid or rows outside its range");
        }
        if ((s = launched("build_K_occ_i8")) != XTC_OK) return s;
    } else {
        const int n_rt = (rows + kKRows - 1) / kKRows;
        nseg = J.kind == 0 ? launch_build_occ<0>(L, g0, rows, n_rt, J, ws, st)
                           : launch_build_occ<1>(L, g0, rows, n_rt, J, ws, st);
        if (nseg == 0) return fail(XTC_E_HIP, "occupancy query of the occupied-block kernel failed");
        if ((s = launched("build_K_occ_f64")) != XTC_OK) return s;
    }
    const size_t nel = (size_t)3 * rows * L.nOP;
    hipLaunchKernelGGL(k_reduce_occ, dim3((unsigned)std::min<size_t>((nel + 255) / 256, 8192)), dim3(256), 0, st, part,
                       nseg, rows, ldK, at<int>(ws, L.colmap), L.nOP, L.ldP, K);
    return launched("reduce_occ");
}

// part[y] = C^T D over one row segment of seg_len rows and a group of cpw of the
// ncomp components, y = group * nseg_r + segment (k_gemm_tn_lp); returns the
// number of partials written through *nparts.
xtc_status gemm_tn_lp(int form, const void* C, int ldC, size_t c_split, const void* D, int ldD, size_t d_split,
                      int rows32, int pmax, int rmax, int ncomp, int cpw, int seg_len, float* part, int* nparts,
                      hipStream_t st) {
    const int nseg_r = (rows32 + seg_len - 1) / seg_len;
    if (form == 3 && ldC % 256 == 0 && ldD % 256 == 0) {
        // both operands staged in LDS (256 x 256 tiles over [0, pmax) x [0, rmax)),
        // dealt to the 8 XCDs in ranges of per_xcd tiles
        const int n_pt = (pmax + 255) / 256, n_rt = (rmax + 255) / 256;
        const int per_xcd = (n_pt * n_rt + 7) / 8;
        const dim3 grid(8 * per_xcd, (ncomp / cpw) * nseg_r);
        hipLaunchKernelGGL((k_gemm_tn_lds<3>), grid, dim3(kTnThreads), 0, st, C, ldC, c_split, D, ldD, d_split, rows32,
                           n_pt, n_rt, per_xcd, pmax, rmax, cpw, seg_len, nseg_r, part);
        *nparts = (int)grid.y;
        return launched("gemm_tn_lds");
    }
    const int n_pt = ldC / 128, n_rt = ldD / 256;
    const dim3 grid(n_pt * n_rt, (ncomp / cpw) * nseg_r);
    if (form == 1)
        hipLaunchKernelGGL((k_gemm_tn_lp<1>), grid, dim3(256), 0, st, C, ldC, c_split, D, ldD, d_split, rows32, n_pt,
                           pmax, rmax, cpw, seg_len, nseg_r, part);
    else if (form == 3)
        hipLaunchKernelGGL((k_gemm_tn_lp<3>), grid, dim3(256), 0, st, C, ldC, c_split, D, ldD, d_split, rows32, n_pt,
                           pmax, rmax, cpw, seg_len, nseg_r, part);
    else
        hipLaunchKernelGGL((k_gemm_tn_lp<6>), grid, dim3(256), 0, st, C, ldC, c_split, D, ldD, d_split, rows32, n_pt,
                           pmax, rmax, cpw, seg_len, nseg_r, part);
    *nparts = (int)grid.y;
    return launched("gemm_tn_lp");
}

// M[P][R] (+)= sum of nparts partials of ldC x ldD floats, P < pmax, R < rmax.
xtc_status reduce_parts(const float* part, int nparts, int ldC, int ldD, int pmax, int rmax, double* M, int ldM,
                        int accumulate, hipStream_t st) {
    const size_t n4 = (size_t)pmax * rmax / 4;   // k_reduce_M: four R per thread
    const unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 16384);
    hipLaunchKernelGGL(k_reduce_M, dim3(blocks), dim3(256), 0, st, part, nparts, (size_t)ldC * ldD, ldD, pmax, rmax, M,
                       ldM, accumulate);
    return launched("reduce_M");
}

// M (+)= C^T D over rows32 packed operand rows (reduced forms), launched in
// groups of kMSegGroup row segments of segM rows: each group's FP32 partials
// are summed in FP64 into M before the next group reuses the partial buffer.
xtc_status gemm_tn_grouped(const Layout& L, const char* C, int ldC, size_t c_split, const char* D, int ldD,
                           size_t d_split, int rows32, int pmax, int rmax, int ncomp, int cpw, double* M, int ldM,
                           int accumulate, void* ws, hipStream_t st) {
    xtc_status s;
    float* part = at<float>(ws, L.Mpart);
    const int group = kMSegGroup * L.segM;
    for (int q0 = 0; q0 < rows32; q0 += group) {
        const int nr = std::min(group, rows32 - q0);
        const size_t shift = (size_t)(q0 / 8) * 8 * L.es;   // bytes per packed row group and column
        int np = 0;
        if ((s = gemm_tn_lp(L.form, C + shift * ldC, ldC, c_split, D + shift * ldD, ldD, d_split, nr, pmax, rmax,
                            ncomp, cpw, L.segM, part, &np, st)) != XTC_OK)
            return s;
        if ((s = reduce_parts(part, np, ldC, ldD, pmax, rmax, M, ldM, q0 == 0 ? accumulate : 1, st)) != XTC_OK)
            return s;
    }
    return XTC_OK;
}

xtc_status gemm2b_lp(const Layout& L, const double* K, int g0, int rows, int accumulate, void* ws, hipStream_t st) {
    xtc_status s;
    const int rows32 = (int)align_up((size_t)rows, kRowQuant);
    const int n8 = rows32 / 8;
    const size_t split_stride = (size_t)L.cap * L.ldL;                 // elements of one split of one component
    const size_t comp_bytes = (size_t)L.ns * split_stride * L.es;
    char* cd = at<char>(ws, L.CDlp);
    const double* rho_rows = at<double>(ws, L.rho) + (size_t)g0 * L.ldP;
    for (int c = 0; c < 4; ++c) {
        const double* src = c == 0 ? rho_rows : K + (size_t)(c - 1) * rows * L.ldP;
        if ((s = pack_any(L.form, src, rows, L.ldP, L.ldP, n8, L.ldL, cd + c * comp_bytes, split_stride, st)) != XTC_OK)
            return s;
    }
    // one spin channel at a time: its D into the operand buffer, GEMM, reduction into M^s
    for (int sp = 0; sp < L.nspin; ++sp) {
        const double* D = at<double>(ws, L.D) + (size_t)sp * 4 * L.cap * L.ldP;
        for (int c = 0; c < 4; ++c) {
            if ((s = pack_any(L.form, D + (size_t)c * L.cap * L.ldP, rows, L.ldP, L.ldP, n8, L.ldL,
                              cd + (4 + c) * comp_bytes, split_stride, st)) != XTC_OK)
                return s;
        }
        if ((s = gemm_tn_grouped(L, cd, L.ldL, split_stride, cd + 4 * comp_bytes, L.ldL, split_stride, rows32, L.ldP,
                                 L.ldP, 4, 1, at<double>(ws, L.M) + (size_t)sp * L.ldP * L.ldP, L.ldP, accumulate,
                                 ws, st)) != XTC_OK)
            return s;
    }
    return XTC_OK;
}

xtc_status split_rows_any(int form, const double* src, size_t n, void* dst, size_t split_stride, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
    if (form == 1) hipLaunchKernelGGL(k_split_rows<1>, dim3(blocks), dim3(256), 0, st, src, n, dst, split_stride);
    else if (form == 3) hipLaunchKernelGGL(k_split_rows<3>, dim3(blocks), dim3(256), 0, st, src, n, dst, split_stride);
    else hipLaunchKernelGGL(k_split_rows<6>, dim3(blocks), dim3(256), 0, st, src, n, dst, split_stride);
    return launched("split_rows");
}

// Split an FP64 row-major [nrows][ld] array into the k-packed operand format
// of k_nt_bf16 (split-BF16 forms).
xtc_status pack_kmajor_any(int form, const double* src, int nrows, int ld, void* dst, size_t split_stride,
                           hipStream_t st) {
    const size_t n = (size_t)nrows * (ld / 8);
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
    if (form == 3)
        hipLaunchKernelGGL(k_pack_kmajor<3>, dim3(blocks), dim3(256), 0, st, src, nrows, ld, (__bf16*)dst,
                           split_stride);
    else
        hipLaunchKernelGGL(k_pack_kmajor<6>, dim3(blocks), dim3(256), 0, st, src, nrows, ld, (__bf16*)dst,
                           split_stride);
    return launched("pack_kmajor");
}

// The adjoint's X Gbar products in the split-BF16 3-product form (k_nt_bf16,
// FP32 accumulation over all pairs): Y_c (+)= X_c Gm^T for NC consecutive
// components sharing one right operand (X k-packed splits [NC][2][ldP/8][rows][8]
// with component stride a_comp, Gm k-packed splits [2][ldP/8][ldP][8], Y FP64
// [NC][cap][ldP] with component stride ystride).  The seven operands of a spin
// channel form two groups: D_{1..3} with Gbar, and rho, K^{x,y,z} with Gbar^T.
template <int NC>
xtc_status xg_group(const __bf16* X, size_t a_comp, size_t a_split, int rows, const __bf16* Gs, int ldP,
                    double* Y, size_t ystride, int accumulate, hipStream_t st) {
    const int n_rt = (rows + kLpRows - 1) / kLpRows, n_jt = (ldP + kPiThreads - 1) / kPiThreads;
    hipLaunchKernelGGL((k_nt_bf16<3, NC, false>), dim3(n_rt * n_jt), dim3(kPiThreads), 0, st, X, a_comp, a_split,
                       rows, Gs, (size_t)ldP * ldP, ldP, ldP, n_rt, (const d4*)nullptr, 0, 0, Y, ystride, ldP,
                       accumulate);
    return launched("gemm_xg_bf16");
}

xtc_status build_K_any(const Layout& L, const JasDev& J, int g0, int rows, double* K, int occ, void* ws,
                       hipStream_t st) {
    if (L.form != 0) return build_K_lp(L, g0, rows, J, K, occ, ws, st);
    const int n_rt = (rows + kKRows - 1) / kKRows;
    const int n_ct = L.ldP / 128;
    const dim3 grid(n_rt * n_ct);
    if (J.kind == 0)
        hipLaunchKernelGGL(k_build_K_f64<0>, grid, dim3(256), 0, st, at<d4>(ws, L.pos), at<double>(ws, L.rho),
                           L.ldP, L.ngp, g0, rows, n_rt, J, K);
    else
        hipLaunchKernelGGL(k_build_K_f64<1>, grid, dim3(256), 0, st, at<d4>(ws, L.pos), at<double>(ws, L.rho),
                           L.ldP, L.ngp, g0, rows, n_rt, J, K);
    return launched("build_K");
}

}  // namespace

extern "C" {

int32_t xtc_pair_ld(int32_t N) { return N >= 1 ? pair_ld(N) : 0; }

const char* xtc_last_error(void) { return g_err.c_str(); }

size_t xtc_workspace_size(const xtc_problem* pb, int32_t prec, int32_t chunk_rows) {
    if (check_problem(pb) != XTC_OK) return 0;
    if (check_prec(prec) != XTC_OK) return 0;
    if (chunk_rows < 1 || chunk_rows > pb->Ng) {
        fail(XTC_E_ARG, "chunk_rows=%d outside [1,Ng]", chunk_rows);
        return 0;
    }
    Layout L = make_layout(pb, prec);
    return layout_bytes(L, align_up((size_t)chunk_rows, kRowQuant));
}

xtc_status xtc_prepare(const xtc_problem* pb, int32_t prec, int32_t chunk_rows, void* ws, size_t ws_bytes,
                       void* stream) {
    xtc_status s;
    if ((s = check_problem(pb)) != XTC_OK) return s;
    if ((s = check_prec(prec)) != XTC_OK) return s;
    Layout L = make_layout(pb, prec);
    place_chunk(L, ws_bytes);
    if ((s = check_ws(L, ws, ws_bytes)) != XTC_OK) return s;
    if (chunk_rows < 1 || chunk_rows > L.cap)
        return fail(XTC_E_WORKSPACE, "chunk_rows=%d exceeds the workspace capacity of %d rows", chunk_rows, L.cap);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_prepare_pos, dim3((L.ngp + 255) / 256), dim3(256), 0, st, pb->xyz, L.Ng, L.ngp,
                       at<d4>(ws, L.pos));
    if ((s = launched("prepare_pos")) != XTC_OK) return s;
    const size_t lds = (size_t)L.N * kPrepRows * sizeof(double);
    hipLaunchKernelGGL(k_prepare_rho, dim3(L.ngp / kPrepRows), dim3(256), lds, st, pb->phi, pb->w, L.N, L.Ng,
                       L.ngp, L.ldP, at<double>(ws, L.rho));
    if ((s = launched("prepare_rho")) != XTC_OK) return s;
    if (L.form != 0) {
        if ((s = pack_any(L.form, at<double>(ws, L.rho), L.ngp, L.ldP, L.ldP, L.ngp / 8, L.ldL, at<void>(ws, L.rho_lp),
                          (size_t)L.ngp * L.ldL, st)) != XTC_OK)
            return s;
        hipLaunchKernelGGL(k_occ_pairs, dim3((L.ldO + 255) / 256), dim3(256), 0, st, make_occ(pb), L.N,
                           at<int>(ws, L.colmap), L.ldO);
        if ((s = launched("occ_pairs")) != XTC_OK) return s;
        hipLaunchKernelGGL(k_gather_occ, dim3(4096), dim3(256), 0, st, at<double>(ws, L.rho), L.ldP, L.ngp,
                           at<int>(ws, L.colmap), L.ldO, 16 * L.occNB, at<double>(ws, L.rho_occ));
        if ((s = launched("gather_occ")) != XTC_OK) return s;
        if (L.i8ok) {
            if ((s = fill(at<double>(ws, L.amax), (size_t)L.ldK8, st)) != XTC_OK) return s;
            if (occ_i8_prepare(at<double>(ws, L.rho_occ), at<d4>(ws, L.pos), L.ngp, 16 * L.occNB, L.nOP, L.i8,
                               at<unsigned long long>(ws, L.amax), at<void>(ws, L.stg), st) != hipSuccess)
                return fail(XTC_E_HIP, "occ_i8_prepare: %s", hipGetErrorString(hipGetLastError()));
        }
        // the adjoint's Pi operand: k-packed splits of rho (FP32: row-major)
        if (L.bwd && L.form == 1 &&
            (s = split_rows_any(L.form, at<double>(ws, L.rho), (size_t)L.ngp * L.ldP, at<void>(ws, L.rhoR),
                                (size_t)L.ngp * L.ldP, st)) != XTC_OK)
            return s;
        if (L.bwd && L.form != 1 &&
            (s = pack_kmajor_any(L.form, at<double>(ws, L.rho), L.ngp, L.ldP, at<void>(ws, L.rhoR),
                                 (size_t)L.ngp * L.ldP, st)) != XTC_OK)
            return s;
    }
    // zero the accumulators of every spin channel and the chunk buffers of the
    // intermediates (their padding columns are never written afterwards and
    // must read as 0: the adjoint sums over all ldP columns of D)
    if ((s = fill(at<double>(ws, L.M), (size_t)L.nspin * L.ldP * L.ldP, st)) != XTC_OK) return s;
    if ((s = fill(at<double>(ws, L.h1acc), (size_t)L.nspin * L.ldP, st)) != XTC_OK) return s;
    if ((s = fill(at<double>(ws, L.D), (size_t)L.nspin * 4 * L.cap * L.ldP, st)) != XTC_OK) return s;
    if (L.tc2) {
        if ((s = fill(at<double>(ws, L.Atc), (size_t)L.ldP * L.ldP, st)) != XTC_OK) return s;
        if ((s = fill(at<double>(ws, L.Btc), (size_t)L.ldN * L.ldP, st)) != XTC_OK) return s;
    }
    return XTC_OK;
}

xtc_status xtc_build_K(const xtc_problem* pb, const xtc_jastrow* jas, int32_t g0, int32_t g1, int32_t prec,
                       double* K, void* ws, size_t ws_bytes, void* stream) {
    xtc_status s;
    JasDev J;
    if ((prec & XTC_K_REDUCED_OCC) && (prec & XTC_K_OCC_FP64))
        return fail(XTC_E_ARG, "prec: XTC_K_REDUCED_OCC and XTC_K_OCC_FP64 together");
    const int occ = (prec & XTC_K_REDUCED_OCC) ? kOccReduced : (prec & XTC_K_OCC_FP64) ? kOccFP64 : kOccExact;
    prec &= ~(XTC_K_REDUCED_OCC | XTC_K_OCC_FP64);
    if ((s = check_problem(pb)) != XTC_OK) return s;
    if ((s = check_prec(prec)) != XTC_OK) return s;
    if ((s = check_jastrow(jas, &J)) != XTC_OK) return s;
    if (!K) return fail(XTC_E_ARG, "K is NULL");
    if ((s = check_align(K, "K")) != XTC_OK) return s;
    Layout L = make_layout(pb, prec);
    place_chunk(L, ws_bytes);
    if ((s = check_ws(L, ws, ws_bytes)) != XTC_OK) return s;
    if ((s = check_range(L, g0, g1)) != XTC_OK) return s;
    return build_K_any(L, J, g0, g1 - g0, K, occ, ws, (hipStream_t)stream);
}

xtc_status xtc_contract_2body(const xtc_problem* pb, const double* K, int32_t g0, int32_t g1, int32_t prec,
                              int32_t flags, double* V2, void* ws, size_t ws_bytes, void* stream) {
    xtc_status s;
    if ((s = check_problem(pb)) != XTC_OK) return s;
    if ((s = check_prec(prec)) != XTC_OK) return s;
    if (!K) return fail(XTC_E_ARG, "K is NULL");
    if ((s = check_align(K, "K")) != XTC_OK) return s;
    if (flags & ~(XTC_RESET | XTC_FINALIZE)) return fail(XTC_E_ARG, "flags=%d unknown bits", flags);
    if ((flags & XTC_FINALIZE) && !V2) return fail(XTC_E_ARG, "V2 is NULL with XTC_FINALIZE");
    Layout L = make_layout(pb, prec);
    place_chunk(L, ws_bytes);
    if ((s = check_ws(L, ws, ws_bytes)) != XTC_OK) return s;
    if ((s = check_range(L, g0, g1)) != XTC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = run_intermediates(L, pb, K, g0, g1, ws, st)) != XTC_OK) return s;
    const int rows = g1 - g0;
    if (L.form != 0) {
        if ((s = gemm2b_lp(L, K, g0, rows, (flags & XTC_RESET) ? 0 : 1, ws, st)) != XTC_OK) return s;
    } else {
        const int n_t = L.ldP / 128;
        const double* rho_rows = at<double>(ws, L.rho) + (size_t)g0 * L.ldP;
        const size_t dstride = (size_t)L.cap * L.ldP;
        for (int sp = 0; sp < L.nspin; ++sp) {
            hipLaunchKernelGGL(k_gemm2b_f64, dim3(n_t * n_t), dim3(256), 0, st, rho_rows, K,
                               at<double>(ws, L.D) + (size_t)sp * 4 * dstride, dstride, rows, L.ldP, n_t,
                               at<double>(ws, L.M) + (size_t)sp * L.ldP * L.ldP, (flags & XTC_RESET) ? 0 : 1);
            if ((s = launched("gemm_2body")) != XTC_OK) return s;
        }
    }
    if (flags & XTC_FINALIZE) {
        const int NN = L.N * L.N;
        const size_t N4 = (size_t)NN * NN;
        const double* Ma = at<double>(ws, L.M);
        const double* Mb = Ma + (size_t)L.ldP * L.ldP;
        const dim3 grid((NN + 255) / 256, L.N, L.N);
        // closed shell: V2 = block (a, a); open shell: blocks (a, a), (a, b), (b, b)
        hipLaunchKernelGGL(k_finalize_V2, grid, dim3(256), 0, st, Ma, Ma, L.ldP, L.N, V2);
        if ((s = launched("finalize_V2")) != XTC_OK) return s;
        if (L.nspin == 2) {
            hipLaunchKernelGGL(k_finalize_V2, grid, dim3(256), 0, st, Ma, Mb, L.ldP, L.N, V2 + N4);
            if ((s = launched("finalize_V2")) != XTC_OK) return s;
            hipLaunchKernelGGL(k_finalize_V2, grid, dim3(256), 0, st, Mb, Mb, L.ldP, L.N, V2 + 2 * N4);
            if ((s = launched("finalize_V2")) != XTC_OK) return s;
        }
    }
    return XTC_OK;
}

xtc_status xtc_contract_1body_0body(const xtc_problem* pb, const double* K, int32_t g0, int32_t g1,
                                    int32_t prec, int32_t flags, double* h1, double* E0, void* ws,
                                    size_t ws_bytes, void* stream) {
    xtc_status s;
    if ((s = check_problem(pb)) != XTC_OK) return s;
    if ((s = check_prec(prec)) != XTC_OK) return s;
    if (!K) return fail(XTC_E_ARG, "K is NULL");
    if ((s = check_align(K, "K")) != XTC_OK) return s;
    if (flags & ~(XTC_RESET | XTC_FINALIZE | XTC_REUSE_INTERMEDIATES))
        return fail(XTC_E_ARG, "flags=%d unknown bits", flags);
    if ((flags & XTC_FINALIZE) && (!h1 || !E0)) return fail(XTC_E_ARG, "h1/E0 NULL with XTC_FINALIZE");
    Layout L = make_layout(pb, prec);
    place_chunk(L, ws_bytes);
    if ((s = check_ws(L, ws, ws_bytes)) != XTC_OK) return s;
    if ((s = check_range(L, g0, g1)) != XTC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    // the intermediates of this chunk (D = [A; B] and the per-row scalars S)
    // are in the workspace already when the two-body call has just made them
    if (!(flags & XTC_REUSE_INTERMEDIATES) && (s = run_intermediates(L, pb, K, g0, g1, ws, st)) != XTC_OK) return s;
    const int rows = g1 - g0;
    const double* rho_rows = at<double>(ws, L.rho) + (size_t)g0 * L.ldP;
    const size_t dstride = (size_t)L.cap * L.ldP;
    const int nsplit_t1 = std::min(kT1Split, rows);
    const int nbk = (L.N + kEBlk - 1) / kEBlk;
    int nsplit_e = std::max(1, std::min(kESplitMax, 1024 / (nbk * nbk)));
    nsplit_e = std::min(nsplit_e, rows);
    const size_t lds = (size_t)2 * L.nocc * kEBlk * sizeof(double);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_onebody_E,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(XTC_E_HIP, "onebody_E LDS attribute: %s", hipGetErrorString(e));
        }
    }
    const double* S = at<double>(ws, L.S);
    const size_t sstride = (size_t)L.cap * 8;
    // per spin channel (T1 and E are scratch of one channel at a time)
    for (int sp = 0; sp < L.nspin; ++sp) {
        const double* Ds = at<double>(ws, L.D) + (size_t)sp * 4 * dstride;
        hipLaunchKernelGGL(k_onebody_T1, dim3((L.Npair + 255) / 256, nsplit_t1), dim3(256), 0, st, rho_rows, K, Ds,
                           dstride, S + sp * sstride, L.nspin == 2 ? S + (1 - sp) * sstride : nullptr, rows, L.ldP,
                           L.Npair, at<double>(ws, L.T1));
        if ((s = launched("onebody_T1")) != XTC_OK) return s;
        hipLaunchKernelGGL(k_onebody_E, dim3(nbk * nbk, nsplit_e), dim3(256), lds, st, rho_rows, K, Ds, dstride,
                           rows, L.ldP, L.N, make_occ(pb, sp), at<double>(ws, L.E));
        if ((s = launched("onebody_E")) != XTC_OK) return s;
        hipLaunchKernelGGL(k_onebody_accumulate, dim3((L.Npair + 255) / 256), dim3(256), 0, st,
                           at<double>(ws, L.T1), nsplit_t1, at<double>(ws, L.E), nsplit_e, L.ldP, L.N,
                           at<double>(ws, L.h1acc) + (size_t)sp * L.ldP, (flags & XTC_RESET) ? 0 : 1);
        if ((s = launched("onebody_accumulate")) != XTC_OK) return s;
    }
    if (flags & XTC_FINALIZE) {
        const int NN = L.N * L.N;
        const double* ha = at<double>(ws, L.h1acc);
        hipLaunchKernelGGL(k_onebody_finalize, dim3((NN + 255) / 256), dim3(256), 0, st, ha,
                           L.nspin == 2 ? ha + L.ldP : nullptr, L.N, make_occ(pb, 0), make_occ(pb, 1), h1, E0);
        if ((s = launched("onebody_finalize")) != XTC_OK) return s;
    }
    return XTC_OK;
}

xtc_status xtc_backward(const xtc_problem* pb, const xtc_jastrow* jas, int32_t prec, const double* gV2,
                        const double* gh1, double gE0, double* gcoef, void* ws, size_t ws_bytes, void* stream) {
    xtc_status s;
    JasDev J;
    if ((s = check_problem(pb)) != XTC_OK) return s;
    if ((s = check_prec(prec)) != XTC_OK) return s;
    if ((s = check_jastrow(jas, &J)) != XTC_OK) return s;
    if (J.kind != 1) return fail(XTC_E_UNSUPPORTED, "the adjoint is taken with respect to power-form coefficients");
    if (!(prec & XTC_WITH_BACKWARD)) return fail(XTC_E_ARG, "prec must carry XTC_WITH_BACKWARD");
    if (!gcoef) return fail(XTC_E_ARG, "gcoef is NULL");
    if (!std::isfinite(gE0)) return fail(XTC_E_ARG, "gE0 not finite");
    Layout L = make_layout(pb, prec);
    place_chunk(L, ws_bytes);
    if ((s = check_ws(L, ws, ws_bytes)) != XTC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const bool open = L.nspin == 2;
    const OccList occ = make_occ(pb, 0);
    hipLaunchKernelGGL(k_occ_flags, dim3((L.N + 255) / 256), dim3(256), 0, st, occ, L.N, at<double>(ws, L.occw),
                       at<int>(ws, L.kidx));
    if ((s = launched("occ_flags")) != XTC_OK) return s;
    // adjoint of the packed accumulator(s): Gm[t] is the right operand of the
    // Cbar products (Gbar^t) and Gm[2 + t] that of the Abar, Bbar products
    // (Gbar^t transposed); closed shell: one symmetric Gbar for both
    const size_t gsz = (size_t)L.ldP * L.ldP;
    double* G = at<double>(ws, L.M);
    const double* Gm[4] = {G, G, G, G};
    if (!open) {
        hipLaunchKernelGGL(k_make_gbar, dim3((L.ldP + 255) / 256, L.ldP), dim3(256), 0, st, gV2, gh1, gE0,
                           at<double>(ws, L.occw), L.N, L.ldP, G);
    } else {
        double* GT = at<double>(ws, L.GT);
        hipLaunchKernelGGL(k_make_gbar_open, dim3((L.ldP + 255) / 256, L.ldP), dim3(256), 0, st, gV2, gh1, gE0,
                           at<double>(ws, L.occw), L.N, L.ldP, G, G + gsz, GT, GT + gsz);
        Gm[1] = G + gsz;
        Gm[2] = GT;
        Gm[3] = GT + gsz;
    }
    if ((s = launched("make_gbar")) != XTC_OK) return s;
    // the X Gbar products in split BF16 only in the 3-product form: the MFMA's
    // FP32 accumulation rounds with a small negative bias, which the six-product
    // form (twice the accumulations per k-step, and a smaller random error to
    // hide it) carries coherently into the gradient; it keeps them in FP64
    const bool bsplit = L.form == 3;
    const __bf16* Gs[4];
    for (int i = 0; i < 4; ++i) {
        const int slot = open ? i : 0;
        Gs[i] = at<__bf16>(ws, L.GsL) + (size_t)slot * L.ns * gsz;
        if (bsplit && (open || i == 0) &&
            (s = pack_kmajor_any(L.form, Gm[i], L.ldP, L.ldP, (void*)Gs[i], gsz, st)) != XTC_OK)
            return s;
    }
    const size_t ystride = (size_t)L.cap * L.ldP;
    double* Kc = at<double>(ws, L.Kc);
    double* Y = at<double>(ws, L.Y);
    const int n_jt_pi = L.ngp / 128;
    bool first = true;
    for (int g0 = 0; g0 < L.Ng; g0 += L.cap) {
        const int rows = std::min(L.cap, L.Ng - g0);
        const bool last = g0 + rows >= L.Ng;
        if ((s = build_K_any(L, J, g0, rows, Kc, kOccExact, ws, st)) != XTC_OK) return s;
        if ((s = run_intermediates(L, pb, Kc, g0, g0 + rows, ws, st)) != XTC_OK) return s;
        const double* rho_rows = at<double>(ws, L.rho) + (size_t)g0 * L.ldP;
        const size_t kstride = (size_t)rows * L.ldP;
        // Y slots: 0..2 Cbar_{1..3} = sum_t D^t_{1..3} Gbar^t^T, then per spin
        // channel t: 3 + 4t Abar^t = rho Gbar^t, 4 + 4t .. 6 + 4t Bbar^t = K Gbar^t
        const double* rk[4] = {rho_rows, Kc, Kc + kstride, Kc + 2 * kstride};
        const size_t a_split = (size_t)rows * L.ldP, a_comp = (size_t)L.ns * a_split;
        char* xs = at<char>(ws, L.KbL);
        // split-BF16: rho and K to k-packed splits once (slots 3..6), D^t (slots 0..2) per channel
        if (bsplit)
            for (int y = 0; y < 4; ++y)
                if ((s = pack_kmajor_any(L.form, rk[y], rows, L.ldP, xs + (3 + y) * a_comp * L.es, a_split, st)) !=
                    XTC_OK)
                    return s;
        for (int t = 0; t < L.nspin; ++t) {
            const double* D = at<double>(ws, L.D) + (size_t)t * 4 * ystride;
            const double* dsrc[3] = {D + ystride, D + 2 * ystride, D + 3 * ystride};
            double* Yab = Y + (size_t)(3 + 4 * t) * ystride;
            if (bsplit) {
                for (int y = 0; y < 3; ++y)
                    if ((s = pack_kmajor_any(L.form, dsrc[y], rows, L.ldP, xs + y * a_comp * L.es, a_split, st)) !=
                        XTC_OK)
                        return s;
                if ((s = xg_group<3>((const __bf16*)xs, a_comp, a_split, rows, Gs[t], L.ldP, Y, ystride, t, st)) !=
                    XTC_OK)
                    return s;
                if ((s = xg_group<4>((const __bf16*)(xs + 3 * a_comp * L.es), a_comp, a_split, rows, Gs[2 + t],
                                     L.ldP, Yab, ystride, 0, st)) != XTC_OK)
                    return s;
            } else {
                const int n_it = (rows + 63) / 64, n_jt = L.ldP / 128;
                for (int y = 0; y < 7; ++y) {
                    const double* X = y < 3 ? dsrc[y] : rk[y - 3];
                    double* Yy = y < 3 ? Y + (size_t)y * ystride : Yab + (size_t)(y - 3) * ystride;
                    hipLaunchKernelGGL(k_gemm_xg_f64, dim3(n_it * n_jt), dim3(256), 0, st, X, (size_t)L.ldP, rows,
                                       Gm[y < 3 ? t : 2 + t], L.ldP, n_jt, Yy, (size_t)L.ldP, y < 3 ? t : 0);
                    if ((s = launched("gemm_xg")) != XTC_OK) return s;
                }
            }
        }
        const size_t lds = (size_t)L.nocc * L.N * 4 * sizeof(double);
        if (lds > 64 * 1024) {
            const hipError_t e = hipFuncSetAttribute((const void*)k_adj_T, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)lds);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(XTC_E_HIP, "adj_T LDS attribute: %s", hipGetErrorString(e));
            }
        }
        for (int t = 0; t < L.nspin; ++t) {
            hipLaunchKernelGGL(k_adj_T, dim3(std::min(rows, 4096)), dim3(256), lds, st, rho_rows, Kc,
                               Y + (size_t)4 * t * ystride, ystride, rows, L.ldP, L.N, make_occ(pb, t),
                               at<double>(ws, L.T), at<double>(ws, L.Wbar), t);
            if ((s = launched("adj_T")) != XTC_OK) return s;
        }
        const size_t nel = (size_t)rows * L.Npair;
        hipLaunchKernelGGL(k_adj_assemble, dim3((unsigned)std::min<size_t>((nel + 255) / 256, 16384)), dim3(256), 0, st,
                           Y, ystride, at<double>(ws, L.S), at<double>(ws, L.T), at<double>(ws, L.Wbar),
                           at<int>(ws, L.kidx), at<double>(ws, L.occw), rows, L.ldP, L.N, L.nocc, L.nspin);
        if ((s = launched("adj_assemble")) != XTC_OK) return s;
        const int n_it_pi = (rows + 31) / 32;
        int nblk_pi;
        if (L.form == 0) {
            nblk_pi = n_it_pi * n_jt_pi;
            hipLaunchKernelGGL(k_pi_grad, dim3(nblk_pi), dim3(256), 0, st, Y, ystride, rows, at<double>(ws, L.rho),
                               L.ldP, L.ldP, at<d4>(ws, L.pos), g0, L.ngp, n_jt_pi, J.ncoef, at<double>(ws, L.gpart));
            if ((s = launched("pi_grad")) != XTC_OK) return s;
        } else {
            // Kbar of the chunk to split operands (FP32: row-major; split BF16:
            // k-packed), then the reduced Pi tiles
            const size_t kb_split = (size_t)rows * L.ldP, kb_comp = (size_t)L.ns * kb_split;
            char* kb = at<char>(ws, L.KbL);
            for (int x = 0; x < 3; ++x) {
                s = L.form == 1 ? split_rows_any(L.form, Y + x * ystride, (size_t)rows * L.ldP,
                                                 kb + x * kb_comp * L.es, kb_split, st)
                                : pack_kmajor_any(L.form, Y + x * ystride, rows, L.ldP, kb + x * kb_comp * L.es,
                                                  kb_split, st);
                if (s != XTC_OK) return s;
            }
            const size_t rr_split = (size_t)L.ngp * L.ldP;
            if (L.form == 1) {
                const int n_jt_lp = (L.ngp + 255) / 256;
                nblk_pi = n_it_pi * n_jt_lp;
                hipLaunchKernelGGL(k_pi_grad_lp<1>, dim3(nblk_pi), dim3(256), 0, st, (const void*)kb, kb_comp, kb_split,
                                   rows, at<void>(ws, L.rhoR), rr_split, L.ldP, at<d4>(ws, L.pos), g0, L.ngp, n_jt_lp,
                                   J.ncoef, at<double>(ws, L.gpart));
            } else {
                const int n_rt = (rows + kLpRows - 1) / kLpRows;
                const int n_jt = (L.ngp + kPiThreads - 1) / kPiThreads;
                nblk_pi = n_rt * n_jt;
                const __bf16* kbb = (const __bf16*)kb;
                const __bf16* rrb = at<__bf16>(ws, L.rhoR);
                if (L.form == 3)
                    hipLaunchKernelGGL((k_nt_bf16<3, 3, true>), dim3(nblk_pi), dim3(kPiThreads), 0, st, kbb, kb_comp,
                                       kb_split, rows, rrb, rr_split, L.ngp, L.ldP, n_rt, at<d4>(ws, L.pos), g0,
                                       J.ncoef, at<double>(ws, L.gpart), (size_t)0, 0, 0);
                else
                    hipLaunchKernelGGL((k_nt_bf16<6, 3, true>), dim3(nblk_pi), dim3(kPiThreads), 0, st, kbb, kb_comp,
                                       kb_split, rows, rrb, rr_split, L.ngp, L.ldP, n_rt, at<d4>(ws, L.pos), g0,
                                       J.ncoef, at<double>(ws, L.gpart), (size_t)0, 0, 0);
            }
            if ((s = launched("pi_grad_lp")) != XTC_OK) return s;
        }
        hipLaunchKernelGGL(k_reduce_grad, dim3(J.ncoef), dim3(256), 0, st, at<double>(ws, L.gpart), nblk_pi, J.ncoef,
                           at<double>(ws, L.gacc), first ? 0 : 1, last ? gcoef : nullptr);
        if ((s = launched("reduce_grad")) != XTC_OK) return s;
        first = false;
    }
    return XTC_OK;
}

// ------------------------------------------------------------- Loewdin --
namespace {
constexpr int kLowdinSeg = 4096;
constexpr int kJacobiMaxSweeps = 40;
struct LowdinLayout {
    int ldS, nseg;
    size_t part, S, U, X, sweeps, status, total;
};
LowdinLayout lowdin_layout(int N, int Ng) {
    LowdinLayout L{};
    L.ldS = (int)align_up((size_t)N, 64);
    L.nseg = (Ng + kLowdinSeg - 1) / kLowdinSeg;
    size_t off = 0;
    L.part = off;   off = align_up(off + (size_t)L.nseg * L.ldS * L.ldS * sizeof(double), kAlign);
    L.S = off;      off = align_up(off + (size_t)N * N * sizeof(double), kAlign);
    L.U = off;      off = align_up(off + (size_t)N * N * sizeof(double), kAlign);
    L.X = off;      off = align_up(off + (size_t)N * N * sizeof(double), kAlign);
    L.sweeps = off; off = align_up(off + sizeof(int), kAlign);
    L.status = off; off = align_up(off + 2 * sizeof(double), kAlign);
    L.total = off;
    return L;
}

xtc_status check_lowdin_args(int N, int Ng, const double* chi, const double* w, const double* phi) {
    if (N < 1 || N > kMaxN || Ng < 1) return fail(XTC_E_ARG, "N=%d or Ng=%d out of range", N, Ng);
    if (Ng > kMaxNg) return fail(XTC_E_UNSUPPORTED, "Ng=%d above %d", Ng, kMaxNg);
    if (!chi || !w || !phi) return fail(XTC_E_ARG, "NULL array");
    return XTC_OK;
}

xtc_status run_lowdin(const LowdinLayout& L, int N, int Ng, const double* chi, const double* w, double* phi,
                      double* lambda, void* ws, hipStream_t st);

// Scratch of xtc_lowdin_noalloc: a file-scope device array, one copy per
// device the library runs on (held until the process ends).  In host code
// `scratch` names the symbol only; its device address on each device comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kNoAllocBytes = XTC_LOWDIN_NOALLOC_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[XTC_LOWDIN_NOALLOC_BYTES];

namespace {
xtc_status scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(XTC_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(XTC_E_UNSUPPORTED, "device %d above %d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(XTC_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return XTC_OK;
}
}  // namespace

xtc_status xtc_tc_2body(const xtc_problem* pb, const xtc_jastrow* jas, const double* dphi, const double* K,
                        int32_t g0, int32_t g1, int32_t prec, int32_t flags, double* K2, void* ws, size_t ws_bytes,
                        void* stream) {
    xtc_status s;
    JasDev J;
    if ((s = check_problem(pb)) != XTC_OK) return s;
    if ((s = check_prec(prec)) != XTC_OK) return s;
    if ((s = check_jastrow(jas, &J)) != XTC_OK) return s;
    if (!(prec & XTC_WITH_TC2)) return fail(XTC_E_ARG, "prec must carry XTC_WITH_TC2");
    if (!dphi || !K) return fail(XTC_E_ARG, "dphi or K is NULL");
    if ((s = check_align(K, "K")) != XTC_OK) return s;
    if (flags & ~(XTC_RESET | XTC_FINALIZE)) return fail(XTC_E_ARG, "flags=%d unknown bits", flags);
    if ((flags & XTC_FINALIZE) && !K2) return fail(XTC_E_ARG, "K2 is NULL with XTC_FINALIZE");
    Layout L = make_layout(pb, prec);
    place_chunk(L, ws_bytes);
    if ((s = check_ws(L, ws, ws_bytes)) != XTC_OK) return s;
    if ((s = check_range(L, g0, g1)) != XTC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int rows = g1 - g0;
    // F for the chunk rows: scalar kernel S against all g', in the arithmetic of
    // prec (reduced forms: the K-build kernel with one component, segment
    // partials in the K-build partial buffer, FP64 reduction)
    double* F = at<double>(ws, L.Ftc);
    if (L.form == 0) {
        const int n_rt = (rows + kKRows - 1) / kKRows;
        const dim3 gF(n_rt * (L.ldP / 128));
        if (J.kind == 0)
            hipLaunchKernelGGL((k_build_F_f64<0, 8>), gF, dim3(256), 0, st, at<d4>(ws, L.pos), at<double>(ws, L.rho),
                               L.ldP, L.ngp, g0, rows, n_rt, J, F);
        else
            hipLaunchKernelGGL((k_build_F_f64<1, 8>), gF, dim3(256), 0, st, at<d4>(ws, L.pos), at<double>(ws, L.rho),
                               L.ldP, L.ngp, g0, rows, n_rt, J, F);
    } else if ((s = build_lp_pieces<1>(L, g0, rows, J, F, ws, st)) != XTC_OK) {
        return s;
    }
    if ((s = launched("build_F")) != XTC_OK) return s;
    double* Rg = at<double>(ws, L.Rg);
    const size_t xs = (size_t)L.cap * L.ldN;
    const size_t nrg = (size_t)rows * L.ldN;
    hipLaunchKernelGGL(k_rhog, dim3((unsigned)std::min<size_t>((nrg + 255) / 256, 16384)), dim3(256), 0, st, pb->w,
                       pb->phi, dphi, L.N, L.Ng, g0, rows, L.ldN, xs, Rg);
    if ((s = launched("rhog")) != XTC_OK) return s;
    const int acc = (flags & XTC_RESET) ? 0 : 1;
    const double* rho_rows = at<double>(ws, L.rho) + (size_t)g0 * L.ldP;
    double* Atc = at<double>(ws, L.Atc);
    double* Btc = at<double>(ws, L.Btc);
    if (L.form == 0) {
        const int nP = L.ldP / 128, nN = L.ldN / 128;
        hipLaunchKernelGGL(k_gemm_tn_f64, dim3(nP * nP), dim3(256), 0, st, rho_rows, (size_t)0, L.ldP, F, (size_t)0,
                           L.ldP, 1, rows, nP, Atc, L.ldP, acc);
        if ((s = launched("gemm_tc_A")) != XTC_OK) return s;
        hipLaunchKernelGGL(k_gemm_tn_f64, dim3(nN * nP), dim3(256), 0, st, Rg, xs, L.ldN, K, (size_t)rows * L.ldP,
                           L.ldP, 3, rows, nN, Btc, L.ldP, acc);
        if ((s = launched("gemm_tc_B")) != XTC_OK) return s;
    } else {
        // reduced forms: both contractions as split products over the chunk rows,
        // FP32 partials per segM rows, FP64 reduction into the accumulators
        const int rows32 = (int)align_up((size_t)rows, kRowQuant);
        const int n8 = rows32 / 8;
        char* cd = at<char>(ws, L.CDlp);
        const size_t sL = (size_t)L.cap * L.ldL, sN = (size_t)L.cap * L.ldN;   // elements of one split
        const size_t cL = (size_t)L.ns * sL * L.es, cN = (size_t)L.ns * sN * L.es;   // bytes of one component
        if ((s = pack_any(L.form, rho_rows, rows, L.ldP, L.ldP, n8, L.ldL, cd, sL, st)) != XTC_OK) return s;
        if ((s = pack_any(L.form, F, rows, L.ldP, L.ldP, n8, L.ldL, cd + cL, sL, st)) != XTC_OK) return s;
        if ((s = gemm_tn_grouped(L, cd, L.ldL, sL, cd + cL, L.ldL, sL, rows32, L.ldP, L.ldP, 1, 1, Atc, L.ldP, acc, ws,
                                 st)) != XTC_OK)
            return s;
        char* kd = cd + 3 * cN;
        for (int x = 0; x < 3; ++x) {
            if ((s = pack_any(L.form, Rg + x * xs, rows, L.ldN, L.ldN, n8, L.ldN, cd + x * cN, sN, st)) != XTC_OK)
                return s;
            if ((s = pack_any(L.form, K + (size_t)x * rows * L.ldP, rows, L.ldP, L.ldP, n8, L.ldL, kd + x * cL, sL,
                              st)) != XTC_OK)
                return s;
        }
        // the three components of rhog_pq . K_R summed inside each workgroup
        if ((s = gemm_tn_grouped(L, cd, L.ldN, sN, kd, L.ldL, sL, rows32, L.N * L.N, L.ldP, 3, 3, Btc, L.ldP, acc, ws,
                                 st)) != XTC_OK)
            return s;
    }
    if (flags & XTC_FINALIZE) {
        const int NN = L.N * L.N;
        hipLaunchKernelGGL(k_finalize_K2, dim3((NN + 255) / 256, L.N, L.N), dim3(256), 0, st, Atc, L.ldP, Btc, L.N,
                           K2);
        if ((s = launched("finalize_K2")) != XTC_OK) return s;
    }
    return XTC_OK;
}

xtc_status xtc_frozen_core(int32_t N, const double* V2, const double* h1, const double* E0, int32_t ncore,
                           const int32_t* core, int32_t nact, const int32_t* act, double* V2_act, double* h1_act,
                           double* E_fc, void* stream) {
    if (N < 1 || N > kMaxN) return fail(XTC_E_ARG, "N=%d outside [1,%d]", N, kMaxN);
    if (ncore < 0 || ncore > kMaxFcList || nact < 1 || nact > kMaxFcList || ncore + nact > N)
        return fail(XTC_E_ARG, "ncore=%d, nact=%d invalid for N=%d", ncore, nact, N);
    if (!V2 || !h1 || !E0 || !act || (ncore > 0 && !core) || !V2_act || !h1_act || !E_fc)
        return fail(XTC_E_ARG, "NULL argument");
    std::vector<char> seen(N, 0);
    IdxList c{}, a{};
    c.n = ncore;
    a.n = nact;
    for (int i = 0; i < ncore + nact; ++i) {
        const int k = i < ncore ? core[i] : act[i - ncore];
        if (k < 0 || k >= N) return fail(XTC_E_ARG, "orbital %d outside [0,N)", k);
        if (seen[k]) return fail(XTC_E_ARG, "orbital %d listed twice (core and active must be disjoint)", k);
        seen[k] = 1;
        if (i < ncore) c.k[i] = k;
        else a.k[i - ncore] = k;
    }
    hipStream_t st = (hipStream_t)stream;
    xtc_status s;
    hipLaunchKernelGGL(k_fc_onebody, dim3((nact * nact + 255) / 256), dim3(256), 0, st, V2, h1, N, c, a, h1_act);
    if ((s = launched("fc_onebody")) != XTC_OK) return s;
    hipLaunchKernelGGL(k_fc_energy, dim3(1), dim3(64), 0, st, V2, h1, E0, N, c, E_fc);
    if ((s = launched("fc_energy")) != XTC_OK) return s;
    const size_t total = (size_t)nact * nact * nact * nact;
    hipLaunchKernelGGL(k_fc_gather, dim3((unsigned)std::min<size_t>((total + 255) / 256, 65536)), dim3(256), 0, st, V2,
                       N, a, V2_act);
    return launched("fc_gather");
}

size_t xtc_lowdin_workspace_size(int32_t N, int32_t Ng) {
    if (N < 1 || N > kMaxN || Ng < 1 || Ng > kMaxNg) {
        fail(Ng > kMaxNg ? XTC_E_UNSUPPORTED : XTC_E_ARG, "N=%d or Ng=%d out of range", N, Ng);
        return 0;
    }
    return lowdin_layout(N, Ng).total;
}

xtc_status xtc_lowdin(int32_t N, int32_t Ng, const double* chi, const double* w, double* phi, double* lambda,
                      void* ws, size_t ws_bytes, void* stream) {
    xtc_status s;
    if ((s = check_lowdin_args(N, Ng, chi, w, phi)) != XTC_OK) return s;
    if (!ws) return fail(XTC_E_WORKSPACE, "workspace is NULL");
    if ((uintptr_t)ws % kAlign) return fail(XTC_E_WORKSPACE, "workspace not 256-byte aligned");
    const LowdinLayout L = lowdin_layout(N, Ng);
    if (ws_bytes < L.total) return fail(XTC_E_WORKSPACE, "workspace of %zu bytes < %zu", ws_bytes, L.total);
    return run_lowdin(L, N, Ng, chi, w, phi, lambda, ws, (hipStream_t)stream);
}

xtc_status xtc_lowdin_noalloc(int32_t N, int32_t Ng, const double* chi, const double* w, double* phi,
                              double* lambda, void* stream) {
    xtc_status s;
    if ((s = check_lowdin_args(N, Ng, chi, w, phi)) != XTC_OK) return s;
    const LowdinLayout L = lowdin_layout(N, Ng);
    if (L.total > kNoAllocBytes)
        return fail(XTC_E_UNSUPPORTED, "N=%d, Ng=%d needs %zu bytes of scratch, above the %zu of the static array", N,
                    Ng, L.total, kNoAllocBytes);
    void* ws = nullptr;
    if ((s = scratch_of_current_device(&ws)) != XTC_OK) return s;
    return run_lowdin(L, N, Ng, chi, w, phi, lambda, ws, (hipStream_t)stream);
}
}  // extern "C"

namespace {
xtc_status run_lowdin(const LowdinLayout& L, int N, int Ng, const double* chi, const double* w, double* phi,
                      double* lambda, void* ws, hipStream_t st) {
    xtc_status s;
    const int n_t = L.ldS / 64;
    hipLaunchKernelGGL(k_syrk_w_part, dim3(n_t * n_t, L.nseg), dim3(256), 0, st, chi, w, N, Ng, L.ldS, n_t,
                       kLowdinSeg, at<double>(ws, L.part));
    if ((s = launched("syrk_w")) != XTC_OK) return s;
    const int NN = N * N;
    hipLaunchKernelGGL(k_syrk_reduce, dim3((NN + 255) / 256), dim3(256), 0, st, at<double>(ws, L.part), L.nseg, N,
                       L.ldS, at<double>(ws, L.S), at<double>(ws, L.U));
    if ((s = launched("syrk_reduce")) != XTC_OK) return s;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJacobiThreads), 0, st, at<double>(ws, L.S), at<double>(ws, L.U), N,
                       kJacobiMaxSweeps, at<int>(ws, L.sweeps));
    if ((s = launched("jacobi")) != XTC_OK) return s;
    // convergence and positive definiteness are checked before anything is
    // written to phi or lambda (one synchronisation of the stream)
    hipLaunchKernelGGL(k_lowdin_status, dim3(1), dim3(64), 0, st, at<double>(ws, L.S), N, at<int>(ws, L.sweeps),
                       at<double>(ws, L.status));
    if ((s = launched("lowdin_status")) != XTC_OK) return s;
    double stat[2] = {0.0, 0.0};
    hipError_t e = hipMemcpyAsync(stat, at<double>(ws, L.status), sizeof stat, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(XTC_E_HIP, "lowdin status read-back: %s", hipGetErrorString(e));
    if (stat[0] >= kJacobiMaxSweeps)
        return fail(XTC_E_ARG, "Jacobi eigensolver of the grid overlap did not converge in %d sweeps",
                    kJacobiMaxSweeps);
    if (!(stat[1] > 0.0))
        return fail(XTC_E_ARG, "grid overlap matrix is not positive definite (smallest eigenvalue %g)", stat[1]);
    hipLaunchKernelGGL(k_inv_sqrt, dim3((NN + 255) / 256), dim3(256), 0, st, at<double>(ws, L.S), at<double>(ws, L.U),
                       N, at<double>(ws, L.X));
    if ((s = launched("inv_sqrt")) != XTC_OK) return s;
    hipLaunchKernelGGL(k_apply_X, dim3((Ng + 255) / 256, N), dim3(256), (size_t)N * sizeof(double), st,
                       at<double>(ws, L.X), chi, N, Ng, phi);
    if ((s = launched("apply_X")) != XTC_OK) return s;
    if (lambda) {
        hipLaunchKernelGGL(k_diag_copy, dim3((N + 255) / 256), dim3(256), 0, st, at<double>(ws, L.S), N, lambda);
        if ((s = launched("diag_copy")) != XTC_OK) return s;
    }
    return XTC_OK;
}
}  // namespace
