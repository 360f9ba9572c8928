/*
 * xtc.h -- C ABI of libxtc: the xTC folding of the transcorrelated three-body
 * operator into effective zero-, one- and two-body terms, on one MI355X.
 *
 * What is computed (Christlmaier et al., "xTC: An efficient treatment of
 * three-body interactions in transcorrelated methods"):
 *
 *   grid intermediate (Theory, definition under eq. Ldecomp)
 *     K^x_pq(g) = sum_g' w_g' d^x(g,g') phi_p(g') phi_q(g'),
 *     d^x(g,g') = (r_g - r_g')_x u'(|r_g - r_g'|) / |r_g - r_g'|  (0 at r_g == r_g')
 *   closed-shell intermediates and two-body correction (Appendix B, eq. tcmf:2el,
 *   eq. tcmf:inter)    V2[p][q][r][s] = Delta U_pr^qs
 *   one-body correction (Appendix B)  h1[p][q] = Delta h_p^q
 *   zero-body term (Appendix B)       E0 = <Psi0|L|Psi0> = -(2/3) sum_k n_k h1[k][k]
 *   (k over the orbitals of the reference density, n_k their per-spin occupations)
 *
 * Conventions shared by every entry point
 *   - Orbitals are real.  p,q,r,s in [0,N).  A pair index P = pair(p,q), p <= q,
 *     enumerates the upper triangle row by row:
 *       pair(p,q) = p*N - p*(p-1)/2 + (q-p),   Npair = N(N+1)/2.
 *     Pair-indexed device arrays have a padded leading dimension
 *     ldP = xtc_pair_ld(N) >= Npair (a multiple of 128); columns [Npair, ldP)
 *     are written as zero and otherwise ignored.
 *   - All array pointers are DEVICE pointers owned by the caller unless marked
 *     HOST.  The library never allocates, frees or retains caller memory.
 *   - Scratch memory is a caller-provided device workspace of at least
 *     xtc_workspace_size() bytes (256-byte aligned).  Between xtc_prepare and
 *     the last call of a pass it carries state (the prepared operands and the
 *     FP64 accumulators of the two- and one-body terms); do not share one
 *     workspace between passes that overlap in time.
 *   - Every call is asynchronous and stream-ordered on `stream` (a hipStream_t
 *     passed as void*, NULL = the default stream).  It returns after host-side
 *     validation and kernel launch; no call synchronises the host.
 *   - On any non-OK status nothing has been launched and no output or
 *     workspace byte has been written, except XTC_E_HIP which reports a failed
 *     launch (earlier kernels of the same call may have run).  The message of
 *     the last failure on the calling thread is returned by xtc_last_error().
 *   - NaN and Inf in the inputs are not checked; they propagate.
 */
#ifndef XTC_H
#define XTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XTC_OK = 0,
    XTC_E_ARG = -1,          /* invalid argument (see each call)                      */
    XTC_E_WORKSPACE = -2,    /* workspace NULL, misaligned or smaller than required   */
    XTC_E_HIP = -3,          /* a HIP runtime call or kernel launch failed            */
    XTC_E_UNSUPPORTED = -4   /* valid but unsupported combination                     */
} xtc_status;

/* Arithmetic of the two bulk contractions (K build and two-body assembly).
 * XTC_FP64   : FP64 MFMA throughout.
 * XTC_FP32   : FP32 MFMA products, FP32 accumulation within blocks of grid
 *              points, FP64 accumulation across blocks.
 * XTC_BF16X3 : operands split a = a0 + a1 (a0 = bf16(a), a1 = bf16(a - a0));
 *              products a0 b0 + a0 b1 + a1 b0 on BF16 MFMA, FP32 accumulation
 *              within blocks, FP64 across blocks.
 * XTC_BF16X6 : three-way split a = a0 + a1 + a2; the six products of total
 *              order <= 2 (a0b0, a0b1, a1b0, a0b2, a1b1, a2b0).
 * In every form the intermediates and the one- and zero-body reductions are
 * computed in FP64, and the occupied-occupied block of K to near-FP64
 * accuracy: by default from exact integer products of the operands written
 * as six base-128 digits against power-of-two scales (int8 MFMA, int32 sums;
 * each operand within 2^-43 of its scale, the digit products of order 8 and
 * up left out: about sqrt(Ng) 2^-44 of the scales' product per entry, with
 * random sign), or in FP64 arithmetic (XTC_K_OCC_FP64 on xtc_build_K, and
 * for more than 144 occupied pairs, i.e. more than 16 occupied orbitals, or
 * grids above 2^21 points). */
typedef enum { XTC_FP64 = 0, XTC_FP32 = 1, XTC_BF16X3 = 2, XTC_BF16X6 = 3 } xtc_prec;

/* OR-ed into prec: lay the workspace out for xtc_backward as well (extra
 * per-row buffers), and for xtc_tc_2body (its accumulators and chunk
 * buffers).  Every call on that workspace must pass the same value. */
enum { XTC_WITH_BACKWARD = 0x10, XTC_WITH_TC2 = 0x20 };

/* OR-ed into the prec of xtc_build_K only (other calls reject it): in the
 * reduced forms, keep the occupied-occupied pairs of K in the reduced
 * arithmetic instead of recomputing them in FP64.  For passes that need no
 * FP64 zero-body term, such as the TC integrals of xtc_tc_2body, whose
 * accuracy the reduced form sets anyway; an E0 computed from such K carries
 * the reduced form's error.  No effect in XTC_FP64. */
enum { XTC_K_REDUCED_OCC = 0x40 };

/* OR-ed into the prec of xtc_build_K only (other calls reject it; not
 * together with XTC_K_REDUCED_OCC): compute the occupied-occupied pairs of K
 * of the reduced forms with FP64 MFMA instead of the integer-sliced products,
 * e.g. to compare the two.  No effect in XTC_FP64. */
enum { XTC_K_OCC_FP64 = 0x80 };

/* flags of the contraction calls */
enum {
    XTC_RESET = 1,       /* zero the accumulator before adding this chunk           */
    XTC_FINALIZE = 2,    /* after adding this chunk, write the outputs              */
    /* xtc_contract_1body_0body only: the caller asserts that the workspace
     * still holds this chunk's intermediates, computed by an
     * xtc_contract_2body call on the same problem, workspace, K (contents
     * unchanged), g0, g1 and prec with no other call on that workspace in
     * between; they are then not recomputed.  Not checked: a false assertion
     * gives wrong h1 and E0. */
    XTC_REUSE_INTERMEDIATES = 4
};

/* Electron-electron Jastrow u(r12) (paper: Theory, Jastrow factorisation; the
 * build uses electron-electron forms only).  Passed by value; no lifetime.
 *   kind 0 (Pade) : u = r / (2 (1 + b r)),                 b >= 0, finite
 *   kind 1 (power): u = sum_{k=1..ncoef} coef[k-1] t^k,    t = r/(1+r), 1 <= ncoef <= 16 */
typedef struct {
    int32_t kind;
    int32_t ncoef;
    double b;
    double coef[16];
} xtc_jastrow;

/* The problem: orbitals on a weighted grid and the per-spin one-body density
 * gamma of the reference, diagonal in the orbital basis:
 *   gamma = sum_i occ_n[i] |occ[i]><occ[i]|   (per spin; the factor two of spin
 *   integration is in the equations, Appendix B).
 * occ_n == NULL means 1 for every listed orbital: the closed-shell determinant
 * (gamma = projector onto occ).  Other values give the uses of the closed-shell
 * equations with a non-idempotent density that the paper makes: the natural
 * orbitals and occupations of a correlated density (eq. tcmf:1el and
 * eq. tcmf:0el then hold approximately, higher cumulants neglected), and the
 * spin-averaged approximation for an open-shell determinant (1 for doubly and
 * 1/2 for singly occupied orbitals; Appendix B, closing remark; results
 * section on the SA approximation).  A non-diagonal gamma is used through its
 * natural orbitals (phi' = U^T phi, occ_n = eigenvalues); the outputs are
 * then in that basis.
 *   xyz [Ng][3] bohr, w [Ng], phi [N][Ng] (orthonormal under w: not checked),
 *   occ [nocc] HOST int32, distinct, in [0,N);
 *   occ_n [nocc] HOST double, finite, or NULL.
 * Limits: 1 <= N <= 256, 1 <= nocc <= min(N, 128), Ng >= 1 (XTC_E_ARG
 * otherwise); nocc * N * 32 bytes (the occupied columns of rho and K staged
 * on chip per grid point) at most 159 KB, i.e. nocc * N <= 5088, and
 * Ng <= 2^28 (XTC_E_UNSUPPORTED otherwise).
 *
 * Open shell (restricted open-shell working equations, Appendix A): with
 * occ_n_beta != NULL the alpha and beta densities differ,
 *   gamma^a = sum_i occ_n[i] |occ[i]><occ[i]|,  gamma^b = sum_i occ_n_beta[i] |occ[i]><occ[i]|
 * (same spatial orbitals and Jastrow for both spins; list every orbital that
 * either spin occupies, with 0 where one spin leaves it empty).  The outputs
 * are then spin-resolved:
 *   V2 [3][N][N][N][N]: blocks [Delta U]^{aa}, [Delta U]^{ab}, [Delta U]^{bb}
 *      (V2[1][p][q][r][s] = [Delta U_pr^qs]^{ab}: pq alpha, rs beta; the
 *      (b, a) block is V2[1][r][s][p][q]),
 *   h1 [2][N][N]: [Delta h]^a, [Delta h]^b,
 *   E0 = -1/3 sum_s [Delta h]^s . gamma^s.
 * Intermediates W and W~ use the total density, Z~ and Z that of each spin;
 * the two-body GEMM runs once per spin.  xtc_backward takes spin-blocked
 * seeds for such a problem (see there). */
typedef struct {
    int32_t N;
    int32_t Ng;
    int32_t nocc;
    int32_t reserved;        /* must be 0 */
    const double *xyz;
    const double *w;
    const double *phi;
    const int32_t *occ;      /* HOST */
    const double *occ_n;     /* HOST, or NULL (all 1) */
    const double *occ_n_beta;  /* HOST, or NULL (closed shell / spin-averaged) */
} xtc_problem;

/* Padded leading dimension of pair-indexed arrays: Npair rounded up to 128. */
int32_t xtc_pair_ld(int32_t N);

/* Bytes of workspace needed for problem `pb` with contraction arithmetic
 * `prec` and grid chunks of at most `chunk_rows` rows (1 <= chunk_rows <= Ng).
 * Returns 0 for invalid arguments (message in xtc_last_error()). */
size_t xtc_workspace_size(const xtc_problem *pb, int32_t prec, int32_t chunk_rows);

/* Prepare a pass: tabulate the weighted pair densities rho_pq(g) = w_g phi_p phi_q
 * (eq. tcmf:inter) and grid positions in the workspace, in FP64 and in the
 * operand format of `prec`, copy occ to the device and zero the accumulators.
 * Must precede the other calls of a pass; reads xyz, w, phi, occ. */
xtc_status xtc_prepare(const xtc_problem *pb, int32_t prec, int32_t chunk_rows,
                       void *ws, size_t ws_bytes, void *stream);

/* Build the grid intermediate (Theory, definition of V under eq. Ldecomp) for
 * output rows g in [g0, g1):
 *   K[x][g-g0][P] = sum_{g'=0}^{Ng-1} w_g' d^x(g,g') phi_p(g') phi_q(g'),  x = 0,1,2
 * K: device [3][g1-g0][ldP] FP64 (columns >= Npair written as 0).
 * The gradient is taken with respect to the first argument of u (the
 * electron sitting on grid point g).  In the reduced forms the occupied-
 * occupied pairs are recomputed to FP64 accuracy (unless prec has
 * XTC_K_REDUCED_OCC).
 * Errors: XTC_E_ARG for !(0 <= g0 < g1 <= Ng), g1-g0 > chunk_rows of the
 * workspace, bad Jastrow, NULL K. */
xtc_status xtc_build_K(const xtc_problem *pb, const xtc_jastrow *jas,
                       int32_t g0, int32_t g1, int32_t prec, double *K,
                       void *ws, size_t ws_bytes, void *stream);

/* Two-body correction (Appendix B / eq. tcmf:2el).  From K of rows [g0,g1)
 * (as written by xtc_build_K) form the closed-shell intermediates A, B
 * (eq. tcmf:inter) and add
 *   M[P][R] += sum_{g in [g0,g1)} rho_P(g) A_R(g) + K_P(g) . B_R(g)
 * into the FP64 accumulator in the workspace.  With XTC_FINALIZE, write
 *   V2[p][q][r][s] = Delta U_pr^qs = -(M[pair(p,q)][pair(r,s)] + M[pair(r,s)][pair(p,q)])
 * to V2 (device [N][N][N][N] FP64, chemist order (pq|rs)); the eight index
 * symmetries hold bitwise.  V2 may be NULL unless XTC_FINALIZE is set. */
xtc_status xtc_contract_2body(const xtc_problem *pb, const double *K,
                              int32_t g0, int32_t g1, int32_t prec, int32_t flags,
                              double *V2, void *ws, size_t ws_bytes, void *stream);

/* One- and zero-body corrections (Appendix B), as an FP64 grid reduction.
 * Substituting eq. tcmf:2el into the one-body equation of Appendix B gives,
 * per grid point, with k over occ and n_k = occ_n (1 if NULL), rb = sum_k n_k rho_kk,
 * kb = sum_k n_k K_kk, a = sum_k n_k A_kk, b = sum_k n_k B_kk:
 *   h1[p][q] += rho_pq a + K_pq.b + rb A_pq + kb.B_pq
 *              - 1/2 sum_k n_k (rho_pk A_kq + K_pk.B_kq + rho_qk A_kp + K_qk.B_kp)
 * With XTC_FINALIZE, write h1 (device [N][N] FP64, symmetric bitwise) and
 * E0 = -(2/3) sum_k n_k h1[k][k] (device, one FP64).  The reduction is always
 * FP64; `prec` names the arithmetic the workspace was prepared for.
 * The intermediates A, B are recomputed from K unless flags has
 * XTC_REUSE_INTERMEDIATES (directly after xtc_contract_2body on this chunk).
 * h1 and E0 may be NULL unless XTC_FINALIZE is set. */
xtc_status xtc_contract_1body_0body(const xtc_problem *pb, const double *K,
                                    int32_t g0, int32_t g1, int32_t prec, int32_t flags,
                                    double *h1, double *E0,
                                    void *ws, size_t ws_bytes, void *stream);

/* Adjoint of the loss
 *   L = gE0 * E0 + sum_pq gh1[p][q] h1[p][q] + sum_pqrs gV2[p][q][r][s] V2[p][q][r][s]
 * with respect to the power-Jastrow coefficients (kind 1 only):
 *   gcoef[k-1] = dL/dc_k,  k = 1..ncoef   (device, FP64, written at the end).
 * The effective seed of V2 folds gh1 and gE0 through the linear one- and
 * zero-body equations of Appendix B; the packed two-body accumulator's adjoint
 * is propagated through eq. tcmf:2el and eq. tcmf:inter to the grid
 * intermediate, and K is linear in the coefficients (Theory, definition of V),
 * so dL/dc_k = sum_{g,g'} d_k^x(g,g') Kbar^x(g) . rho(g').  K is recomputed
 * chunk by chunk (never stored); the contraction with the Jastrow basis runs
 * over all (g, g') in FP64 with a fixed-order reduction (deterministic).
 * Requires a workspace prepared (xtc_prepare) with prec | XTC_WITH_BACKWARD.
 * gV2: device [N]^4 or NULL (= 0); gh1: device [N][N] or NULL; gE0: host value.
 * Open shell (occ_n_beta set): the loss of the spin-resolved outputs,
 *   L = gE0 * E0 + sum_s gh1[s] . h1[s] + sum_b gV2[b] . V2[b],
 * gV2 device [3][N]^4 (blocks aa, ab, bb as xtc_contract_2body writes them),
 * gh1 device [2][N][N] (alpha, beta); the folding follows Appendix A and the
 * two accumulators M^a, M^b get separate, non-symmetric adjoints.
 * The K recompute follows prec (reduced forms keep the occupied block FP64);
 * the adjoint GEMMs and the coefficient contraction are FP64.
 * Errors: XTC_E_UNSUPPORTED for a Pade Jastrow.  The occupied set has the
 * forward's limits (nocc <= 128, nocc * N <= 5088). */
xtc_status xtc_backward(const xtc_problem *pb, const xtc_jastrow *jas, int32_t prec,
                        const double *gV2, const double *gh1, double gE0, double *gcoef,
                        void *ws, size_t ws_bytes, void *stream);

/* Symmetric (Loewdin) orthonormalisation under the grid weights, FP64.
 * The paper works with orthonormal orbitals (HF orbitals, Results section);
 * on a Monte-Carlo grid the functions are orthonormalised under the same
 * quadrature that the grid intermediates use:
 *   S[m][n] = sum_g w_g chi_m(g) chi_n(g),   phi = S^{-1/2} chi
 * with S^{-1/2} symmetric (cyclic Jacobi eigen-decomposition of S, which keeps
 * small eigenvalues to high relative accuracy; S must be positive definite).
 * chi, phi: device [N][Ng]; w: device [Ng]; lambda: device [N] (eigenvalues
 * of S, unordered) or NULL.  Workspace of xtc_lowdin_workspace_size(N, Ng)
 * bytes, 256-byte aligned; no state is kept in it after the call.
 * 1 <= N <= 256 and Ng >= 1 (XTC_E_ARG), Ng <= 2^28 (XTC_E_UNSUPPORTED).
 * Unlike the other calls it synchronises `stream` once, after the eigensolver,
 * to check it: XTC_E_ARG if the Jacobi sweeps did not converge or S is not
 * positive definite (smallest eigenvalue <= 0 or NaN); phi and lambda are not
 * written then. */
size_t xtc_lowdin_workspace_size(int32_t N, int32_t Ng);
xtc_status xtc_lowdin(int32_t N, int32_t Ng, const double *chi, const double *w, double *phi,
                      double *lambda, void *ws, size_t ws_bytes, void *stream);

/* xtc_lowdin for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the scratch taken from a file-scope device
 * array of XTC_LOWDIN_NOALLOC_BYTES instead of a caller workspace.  Each
 * device the library runs on holds its own copy of that array until the
 * process ends; the call allocates nothing.  The array's device address is
 * looked up on the first call on each device (with that device current).
 * Sizes whose workspace (xtc_lowdin_workspace_size) exceeds the array return
 * XTC_E_UNSUPPORTED before anything is launched; N = 128 fits up to
 * Ng ~ 2 x 10^6 grid points, N = 256 up to Ng ~ 5 x 10^5.
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (other streams or host threads) race and give undefined
 * results; calls on one stream are ordered.  Nothing in the array needs to
 * start at zero (every scratch word is written before it is read).
 * Like xtc_lowdin it synchronises `stream` once to check the eigensolver. */
#define XTC_LOWDIN_NOALLOC_BYTES ((size_t)64 << 20)
xtc_status xtc_lowdin_noalloc(int32_t N, int32_t Ng, const double *chi, const double *w, double *phi,
                              double *lambda, void *stream);

/* Two-body transcorrelated integrals on the grid (Theory, definition of K):
 *   K_pr^qs = 1/2 <pr| P^1_2 (lap_1 u + (grad_1 u)^2 + 2 grad_1 u . grad_1) |qs>
 * with both electrons on the grid, written as K2[p][q][r][s] = K_pr^qs
 * (p, q electron 1; the order of V2).  With rho_pq = w phi_p phi_q,
 * S(g,g') = lap_1 u + |grad_1 u|^2 (0 at coincident points),
 * F_R(g) = sum_g' S(g,g') rho_R(g'), the grid intermediate K of the same rows
 * (as written by xtc_build_K) and rhog_pq = w phi_p grad phi_q:
 *   K2[pq][rs] = A[P][R] + B[pq][R] + B[rs][P],
 *   A = sum_g rho_P F_R,  B[pq][R] = sum_g rhog_pq . K_R,
 * accumulated chunk by chunk like xtc_contract_2body (XTC_RESET, XTC_FINALIZE)
 * into FP64 accumulators in the workspace.  K2 satisfies
 * K2[p][q][r][s] = K2[r][s][p][q] but not the p <-> q symmetry (the integrals
 * are not hermitian).  F (the sum over g') and the contractions A and B (sums
 * over the chunk rows) follow prec like K: FP64, or the reduced form's products
 * with FP32 partials per segment of rows (of g' for F) and FP64 sums of the
 * partials; the accumulators across chunks are FP64.  The occupied-occupied
 * FP64 pass of xtc_build_K is not needed here (XTC_K_REDUCED_OCC).
 * Needs xtc_prepare with prec | XTC_WITH_TC2.
 * dphi: device [3][N][Ng], the gradients of the orbitals on the grid;
 * K: device [3][g1-g0][ldP]; K2: device [N]^4, may be NULL unless XTC_FINALIZE. */
xtc_status xtc_tc_2body(const xtc_problem *pb, const xtc_jastrow *jas, const double *dphi,
                        const double *K, int32_t g0, int32_t g1, int32_t prec, int32_t flags,
                        double *K2, void *ws, size_t ws_bytes, void *stream);

/* Frozen-core folding of the closed-shell outputs (xTC-FC, results section:
 * the corrections are computed with all electrons and the standard frozen-core
 * equations are applied afterwards).  With (pq|rs) = V2[p][q][r][s] and the
 * core orbitals c doubly occupied:
 *   E_fc      = E0 + 2 sum_c h1[c][c] + sum_{c,d} (2 (cc|dd) - (cd|dc))
 *   h1_act[i][j] = h1[a_i][a_j] + sum_c (2 (a_i a_j|cc) - (a_i c|c a_j))
 *   V2_act[i][j][k][l] = V2[a_i][a_j][a_k][a_l]
 * V2 [N]^4, h1 [N][N], E0 [1]: device, as written by the contraction calls;
 * core [ncore], act [nact]: HOST int32, disjoint, in [0,N), ncore >= 0,
 * nact >= 1, each at most 256; V2_act [nact]^4, h1_act [nact][nact],
 * E_fc [1]: device outputs.  Deterministic; no workspace. */
xtc_status xtc_frozen_core(int32_t N, const double *V2, const double *h1, const double *E0,
                           int32_t ncore, const int32_t *core, int32_t nact, const int32_t *act,
                           double *V2_act, double *h1_act, double *E_fc, void *stream);

/* Message for the last non-OK status returned on the calling thread. */
const char *xtc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* XTC_H */
