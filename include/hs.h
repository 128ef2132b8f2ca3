/*
 * hs.h -- C ABI of the MI355X (gfx950) implementation of the matrix-free Hermite
 * Galerkin method on hyperbolically reduced index sets (Brumm, arXiv 1403.3511).
 *
 * Conventions for every entry point
 *   - Every call returns an int32 status: HS_OK (0), an informational code (> 0) or an
 *     error (< 0).  No call aborts or throws across this boundary.  The text of the
 *     last error of the calling thread is available from hs_last_error().
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device" pointers are
 *     caller-owned GPU allocations (e.g. the data of a PyTorch CUDA/HIP tensor) that must
 *     stay alive and unmodified while work that uses them is in flight.  Device pointers
 *     must be 16-byte aligned (256 recommended).
 *   - Work is enqueued on the caller's hipStream_t (passed as void*; NULL means the
 *     default stream).  Nothing synchronises unless its name ends in _sync.
 *   - Handles (hs_index, hs_pot, hs_batch, hs_mlp) are host objects owned by the
 *     library; destroy them with the matching *_destroy call.  A handle may be used by
 *     one thread at a time.
 *   - Complex vectors are interleaved (re, im): complex128 = 2 x float64 (HS_C128) or
 *     complex64 = 2 x float32 (HS_C64).
 *
 * Notation.  N is the dimension, B the product bound of the index set
 *     K = { k in N_0^N : prod_l (1 + k_l) <= B }              (paper Sec. 1.2),
 * i.e. B = K_paper + 1.  H = D + W^pol(X_K) with D = diag(sum_l (k_l + 1/2)) and W the
 * potential minus |x|^2/2 (Sec. 1.2), W^pol(X_K) the formal insertion of the coordinate
 * matrices X_K^(l) (Sec. 3.1-3.2, eq. Horner), axis N applied first, axis 1 last.
 * Besides the hyperbolic cross, index sets may be boxes, total-degree sets, padded
 * crosses or any downward-closed set given as a list (HS_SET_*); the operator is
 * defined the same way on each.
 *
 * The paper's three interfaces: the fast algorithm (Fig. 3) is hs_apply_h, the direct
 * operation (Sec. 3.1) hs_apply_x, the time propagation (Fig. 4) hs_step / hs_propagate.
 */
#ifndef HS_H
#define HS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------- */
#define HS_OK 0
#define HS_INFO_BREAKDOWN 1   /* Lanczos stopped early; see m_eff                       */
#define HS_E_INVALID -1       /* bad argument (null handle/pointer, N/B out of range ...) */
#define HS_E_OVERFLOW -2      /* a size does not fit the index types                    */
#define HS_E_NOMEM -3         /* host allocation failed                                 */
#define HS_E_WORKSPACE -4     /* caller buffer smaller than the size query returned     */
#define HS_E_UNSUPPORTED -5   /* combination not implemented (e.g. basis/kernel class)  */
#define HS_E_HIP -6           /* a HIP runtime call failed; text in hs_last_error        */
#define HS_E_NONFINITE -7     /* non-finite coefficients                                */
#define HS_E_IO -8            /* a checkpoint file cannot be read or written, or is corrupt */

/* ---- dtypes, bases ------------------------------------------------------------ */
#define HS_C128 0 /* complex float64 */
#define HS_C64 1  /* complex float32 (float32 arithmetic in the matvec) */

#define HS_BASIS_MONO 0 /* p_a(x) = x^a                                              */
#define HS_BASIS_CHEB 1 /* p_a(x) = T_a(x / scale), Chebyshev 1st kind (Sec. 1.3)     */
#define HS_BASIS_HERM 2 /* p_a(x) = H_a(x / scale), physicists' Hermite polynomials   */

#define HS_NMAX 16

#define HS_SET_HYPERBOLIC 0   /* prod(1 + k_l) <= B (paper Sec. 1.2)                       */
#define HS_SET_BOX 1          /* {0..K}^N (K_full)                                          */
#define HS_SET_TOTAL_DEGREE 2 /* |k|_1 <= D                                                 */
#define HS_SET_LIST 3         /* an explicit downward-closed set                            */
#define HS_SET_PADDED 4       /* prod(1 + max(k_l - w, 0)) <= B: the cross widened by w     */

#define HS_FORM_PAPER 0 /* the fast operator F: factors applied axis N first (eq. Horner)   */
#define HS_FORM_SYM 1   /* its symmetric part D + (F + F_rev)/2 (see hs_pot_set_form)     */

typedef struct hs_index_s *hs_index;
typedef struct hs_pot_s *hs_pot;
typedef struct hs_batch_s *hs_batch;
typedef struct hs_mlp_s *hs_mlp;

/* Text of the last error on this thread (truncated to len-1 bytes, NUL-terminated). */
int32_t hs_last_error(char *buf, size_t len);
/* Library version string, e.g. "1.0 gfx950". */
const char *hs_version(void);

/* ---- index set (paper Sec. 1.2; neighbour maps k +- e_l for Sec. 3.1) ------------
 * hs_index_create enumerates K_N(B) on the host.  Layout: rows are grouped in tiles
 * that share the prefix (k_1..k_{N-d}); inside a tile the suffix (k_{N-d+1}..k_N) runs
 * over one global list of K_d(B) sorted by (prod(1+s), lex), so a tile with remaining
 * bound b holds exactly the first |K_d(b)| entries of that list.  tile_dim d in 1..N
 * (0 = library choice).  Requires 1 <= N <= HS_NMAX, 1 <= B <= 65536, |K| < 2^31.
 * (Sets given as a list have tile dimension 0: one row per tile.)                   */
int32_t hs_index_create(int32_t N, int64_t B, int32_t tile_dim, hs_index *out);
int32_t hs_index_destroy(hs_index idx);
/* |K_N(B)| without enumerating the set (the same bounds on N and B as hs_index_create;
 * counts saturate at 2^62).  Host only; for sizing batches and buffers beforehand.   */
int32_t hs_index_count(int32_t N, int64_t B, int64_t *n);
/* |K|, the number of rows of every vector over this set. */
int32_t hs_index_size(hs_index idx, int64_t *n);
/* tile_dim actually used, number of tiles, length of the global suffix list. */
int32_t hs_index_info(hs_index idx, int32_t *tile_dim, int64_t *ntiles, int64_t *nsuffix);
/* Multi-index of every row in library order: host_out has n*N uint16, row-major.     */
int32_t hs_index_multi_indices(hs_index idx, uint16_t *host_out);
/* Device metadata: query the size, then upload into a caller device buffer of at
 * least that many bytes (stream-ordered host->device copy from pinned staging held by
 * the handle).  Every compute call on this index takes the same device pointer.     */
int32_t hs_index_device_bytes(hs_index idx, int64_t *bytes);
int32_t hs_index_upload(hs_index idx, void *dev, int64_t bytes, void *stream);
/* Fibres of every axis for chained recurrence passes (an addition to paper Sec. 3.2,
 * eq. Horner, whose passes apply the basis's three-term recurrence along one axis at a
 * time): the generic program's chains of passes along one axis, and the split form's
 * combination with the chains that follow it, then run as single launches over that
 * axis's fibres (rows differing in k_l alone) instead of one launch per pass, with
 * results equal bit for bit.  The fibres serve only once the block carrying them is
 * uploaded; an index without them keeps one launch per pass.  Appends about 12 bytes per row and axis to the device
 * block: call it before hs_index_device_bytes and hs_index_upload (a block sized or
 * uploaded before must be sized and uploaded again).  Idempotent.  HS_E_OVERFLOW for
 * sets of 2^31 rows or more, fibres longer than 65535 rows, or lists beyond 16 GiB;
 * HS_E_NOMEM when host memory runs out (the handle is then unchanged).             */
int32_t hs_index_build_fibres(hs_index idx);

/* Box sets {0..Kmax}^N (the full index set K_full of paper Sec. 4.1-4.2), in the same
 * tiled layout (every tile holds the whole suffix list, in lexicographic order), for
 * the error diagnostics below; every H application and step accepts them in the
 * paper's operator form.  Kmax <= 65535, fewer than 2^31 rows.                       */
int32_t hs_index_create_box(int32_t N, int64_t Kmax, int32_t tile_dim, hs_index *out);
/* Total-degree sets {k : |k|_1 <= D}, another downward-closed family on which the
 * method applies unchanged (paper Sec. 1.2 requires only that k - e_l stays in the set),
 * in the same tiled layout (suffixes graded by |s|_1).  D <= 65535, fewer than 2^31
 * rows.  Every H application and step accepts them in the paper's operator form.    */
int32_t hs_index_create_total_degree(int32_t N, int64_t D, int32_t tile_dim, hs_index *out);
/* Any downward-closed set, given as n distinct multi-indices (host, n x N uint16, any
 * order; the library keeps them in lexicographic order, see hs_index_multi_indices).
 * The paper's method needs only that k - e_l lies in the set whenever k does and
 * k_l > 0 (Sec. 1.2); the call checks this and returns HS_E_INVALID otherwise (also
 * for repeated rows).  For N >= 3 (and N = 1) the tiles are the distinct prefixes of
 * the first N - 1 coordinates with the last coordinate as the suffix (tile dimension 1:
 * downward closure makes every fibre {0..L-1}), and the fused H kernels serve them; for
 * N = 2 every axis is a prefix axis (one row per tile, the generic row kernels).
 * Paper's operator form only.                                                        */
int32_t hs_index_create_from_list(int32_t N, int64_t n, const uint16_t *k_host, hs_index *out);
/* Padded crosses {k : prod(1 + max(k_l - w, 0)) <= B}: the hyperbolic cross K_N(B)
 * widened by w in every axis (it contains every k + d with k in K_N(B), |d_l| <= w), in
 * the tiled layout with suffixes graded by the same product.  With w at least the
 * largest per-axis degree of a potential, no intermediate index of the fast algorithm's
 * product between two rows of K_N(B) leaves it, so on those rows the fast algorithm on
 * the padded cross is the exact Galerkin product of K_N(B) (see hs_error_split).
 * 1 <= B, B + w <= 65536, w <= 16, fewer than 2^31 rows.  Paper's operator form.   */
int32_t hs_index_create_padded(int32_t N, int64_t B, int64_t w, int32_t tile_dim, hs_index *out);
/* map_host[r] = the row of box that holds row r's multi-index of sub (sub->size int32),
 * -1 when it lies outside.  box may be any set kind (a box or a padded cross for
 * hs_error_split; any target for moving vectors between sets).  Host only.          */
int32_t hs_index_embed(hs_index sub, hs_index box, int32_t *map_host);

/* ---- potential (paper Sec. 1.3; W = V - |x|^2/2, Sec. 1.2) ---------------------
 * Terms t = 0..nterms-1 with per-axis degrees degrees[t*N + l] in the given basis and
 * time-dependent coefficients  beta_t(t) = base_t + amp_t * sin(freq_t * t + phase_t).
 * subtract_harmonic != 0 (monomial basis only) turns V into W by lowering the x_l^2
 * coefficient by 1/2 for every axis.  The compiler classifies the potential:
 *   class HH (every monomial, after basis change, is x_l^a with a <= 3 or
 *   x_l^a x_{l+1} with a <= 2): served by the fused row kernel;
 *   otherwise: served by the generic recurrence-pass program.                       */
int32_t hs_pot_create(int32_t N, int32_t basis, double scale, int32_t nterms,
                      const uint16_t *degrees, const double *base, const double *amp,
                      const double *freq, const double *phase, int32_t subtract_harmonic,
                      hs_pot *out);
int32_t hs_pot_destroy(hs_pot pot);
/* 1 if the fused (class HH) kernel serves this potential, 0 for the generic program. */
int32_t hs_pot_is_fused(hs_pot pot, int32_t *fused);
/* Device parameter block of the potential: size query and stream-ordered upload.   */
int32_t hs_pot_device_bytes(hs_pot pot, int64_t *bytes);
int32_t hs_pot_upload(hs_pot pot, void *dev, int64_t bytes, void *stream);
/* Evaluate the term coefficients at time t on the device (paper Fig. 4 step (1)),
 * writing them into the device parameter block; graph-capturable (t is read from the
 * device scalar t_dev when t_dev != NULL, else the host value t is used).           */
int32_t hs_pot_set_time(hs_pot pot, void *pot_dev, double t, const double *t_dev, void *stream);
/* Operator form used by every later call with this potential.  HS_FORM_PAPER (the
 * default) is the fast operator F of the paper, factors applied axis N first.  On a
 * reduced set the truncated coordinate matrices do not commute (paper Sec. 4.2, after
 * Lemma 1), so F is not symmetric there; each X_K is symmetric, so F^T = F_rev (the
 * reversed factor order) and HS_FORM_SYM = D + (F + F_rev)/2 is the symmetric part of
 * the same discretisation.  HS_FORM_SYM is served for potentials of the fused class on
 * index sets with a specialised kernel that lists every row (else the H application
 * returns HS_E_UNSUPPORTED); batches accept HS_FORM_PAPER only.  A host-side setting:
 * no device block changes.  Returns HS_E_UNSUPPORTED for a potential outside the fused
 * class, HS_E_INVALID for an unknown form.                                            */
int32_t hs_pot_set_form(hs_pot pot, int32_t form);
/* Replace the time-dependent base coefficients by values already on the device
 * (nterms doubles, e.g. written by the surrogate or the quadrature kernels).          */
int32_t hs_pot_set_coeffs_device(hs_pot pot, void *pot_dev, const double *coef_dev, void *stream);

/* ---- H application (paper Sec. 3.2, eq. Horner; Fig. 4 step (2)) ----------------
 * y = (D + W^pol(X_K)) c for the coefficients currently in pot_dev.  c and y are
 * device vectors of |K| complex values in library row order, of the given dtype;
 * c != y.  ws is a device workspace of hs_workspace_bytes(..., m = 0) bytes (may be
 * NULL when that size is 0).                                                         */
int32_t hs_workspace_bytes(hs_index idx, hs_pot pot, int32_t dtype, int32_t m, int64_t *bytes);
int32_t hs_apply_h(hs_index idx, const void *idx_dev, hs_pot pot, const void *pot_dev,
                   int32_t dtype, const void *c, void *y, void *ws, void *stream);

/* ---- direct operation (paper Sec. 3.1, eq. DirectOperationWithX; Fig. 3) --------
 * y = X_K^(l) c, the Galerkin matrix of the coordinate x_l on the set, applied without
 * assembly: y_k = sqrt(k_l / 2) c_{k - e_l} + sqrt((k_l + 1) / 2) c_{k + e_l}, where a
 * neighbour outside K contributes nothing.  axis = l - 1 (0-based, as the columns of
 * the degree arrays).  c and y: device vectors of |K| complex values of the given dtype
 * in library row order, c != y.  Serves every set kind; no workspace.               */
int32_t hs_apply_x(hs_index idx, const void *idx_dev, int32_t axis, int32_t dtype, const void *c,
                   void *y, void *stream);

/* ---- time step (paper Sec. 2, eq. expMPR; Fig. 4) ----------------------------
 * One exponential-midpoint step of length h with an m-step Lanczos exponential:
 * coefficients at t + h/2, m applications of H, c <- V_m exp(-i h T_m) e_1 ||c||.
 * c is complex128 (state) whatever dtype is; dtype selects the precision of the
 * Krylov vectors and the matvec (HS_C64: complex64 vectors and float32 matvec,
 * float64 dot products, norms, T_m eigensolve and combination).  reorth != 0 adds one
 * classical Gram-Schmidt pass per Lanczos step.  m <= 32.  ws holds
 * hs_workspace_bytes(..., m) bytes.  t_dev (device double, may be NULL) supplies t
 * and is advanced by h on the device, so a captured graph can be replayed per step.
 * diag_dev (device, may be NULL) receives the (m_eff, alpha[0..m), beta[0..m))
 * record of the step as doubles: 1 + 2m values.                                     */
int32_t hs_step(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev, int32_t dtype,
                double t, double *t_dev, double h, int32_t m, int32_t reorth, void *c, void *ws,
                double *diag_dev, void *stream);

/* hs_step_static: hs_step without a workspace argument, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses that forbid
 * allocation).  The workspace is a fixed array of HS_STEP_STATIC_MAX_BYTES in the
 * library's code object, one per GPU, held until the process ends; the call allocates
 * nothing (no hipMalloc, no library allocator).  Arguments, results and the device
 * clock t_dev as for hs_step.  HS_E_WORKSPACE when hs_workspace_bytes(idx, pot, dtype, m)
 * exceeds the array (for complex128 and m = 10, sets up to about 190,000 rows).  All
 * calls on one GPU share its array: calls that overlap in time on one GPU (several
 * streams or threads) race and must be serialised by the caller.                  */
#define HS_STEP_STATIC_MAX_BYTES (32 << 20)
int32_t hs_step_static(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev, int32_t dtype,
                       double t, double *t_dev, double h, int32_t m, int32_t reorth, void *c,
                       double *diag_dev, void *stream);

/* Sets of at most `rows` rows (default 1024; the kernel holds one row per thread, at most
 * 1024, so larger values act as 1024) run hs_step / hs_propagate of the paper's operator
 * form with a fused-class potential as one launch of one workgroup: the whole
 * Lanczos step in one kernel, with the same recurrences, breakdown rule and workspace
 * layout as the general step, and its reductions in another fixed order (results agree
 * to rounding, and each path repeats bit for bit).  0 always takes the general step.
 * Process-wide; not meant to change while steps are in flight.                        */
int32_t hs_set_small_step_rows(int64_t rows);
int32_t hs_get_small_step_rows(int64_t *rows);

/* ---- time propagation (paper Sec. 2.2; Fig. 4 time_propagation) --------------------
 * nsteps consecutive hs_step calls on the same stream, with the same arguments: step n
 * starts at t0 + n h (or at the value in t_dev, which each step advances by h).  c is
 * overwritten with c(t0 + nsteps h); ws as for hs_step.  nsteps = 0 does nothing.  The
 * whole call can be captured into one HIP graph.  An error stops at the failing step
 * (earlier steps have been enqueued).                                                  */
int32_t hs_propagate(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev, int32_t dtype,
                     double t0, double *t_dev, double h, int32_t m, int32_t reorth, int64_t nsteps,
                     void *c, void *ws, void *stream);

/* ---- fourth-order step (paper Sec. 2.1, eq. 2stageMagnus) ------------------------
 * Two-stage Gauss-Legendre Magnus scheme: Omega = -i h M with
 *   M = (A_1 + A_2)/2 - i (sqrt(3) h / 12) (A_2 A_1 - A_1 A_2),  A_j = H(t + c_j h),
 *   c_{1,2} = 1/2 -+ sqrt(3)/6.
 * The two coefficient sets live in two device parameter blocks of the same potential
 * (pot_dev1, pot_dev2: distinct buffers of hs_pot_device_bytes bytes, both uploaded
 * with hs_pot_upload; the step overwrites their coefficients).  For fused-class
 * potentials on sets with a specialised kernel, M is applied by two fused passes with
 * Abar = (A_1 + A_2)/2, Delta = (A_2 - A_1)/2, A_2 A_1 - A_1 A_2 = 2 (Delta Abar - Abar
 * Delta) (the fast operator is linear in the coefficients); otherwise by four H
 * applications and one combination pass.
 * hs_magnus4_workspace_bytes(m = 0) sizes the workspace of hs_apply_magnus4, m >= 1
 * that of hs_step_magnus4 (three vectors more than hs_workspace_bytes).
 * hs_apply_magnus4: y = M c with the coefficients currently in the two blocks (c != y).
 * hs_step_magnus4: c <- V_m exp(-i h T_m) e_1 ||c|| with T_m from m Lanczos steps on M;
 * arguments, dtype, reorth, t_dev and diag_dev as for hs_step.                       */
int32_t hs_magnus4_workspace_bytes(hs_index idx, hs_pot pot, int32_t dtype, int32_t m, int64_t *bytes);
int32_t hs_apply_magnus4(hs_index idx, const void *idx_dev, hs_pot pot, const void *pot_dev1,
                         const void *pot_dev2, int32_t dtype, double h, const void *c, void *y,
                         void *ws, void *stream);
int32_t hs_step_magnus4(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev1, void *pot_dev2,
                        int32_t dtype, double t, double *t_dev, double h, int32_t m, int32_t reorth,
                        void *c, void *ws, double *diag_dev, void *stream);

/* ---- local error diagnostics (paper Sec. 5.1, eqs. ErrorQuadratureDef and
 * ErrorGridReductionDef; Sec. 6.1) ---------------------------------------------------
 * For a vector v on the set sub (complex128, library order):
 *   e_red  = W^pol(X_K) v - Omega(W^pol(X_full) Omega_+(v))   (index set reduction)
 *   e_quad = W_{K,pol} v - W^{GH(K)}_{K,pol} v                  (quadrature)
 * where box is K_full = {0..K}^N containing sub (by Lemma 1 the fast algorithm on it,
 * restricted to sub, is the Gauss-Hermite matrix W^{GH(K)}), and pad is a box padded by
 * at least half the potential's largest per-axis degree, on which the fast algorithm
 * restricted to sub is the exact Galerkin product W_{K,pol} v.  pad may be NULL (then
 * e_quad is not written).  box_map / pad_map: hs_index_embed(sub, box / pad), uploaded
 * (device int32, sub->size).  The paper's operator form only.  ws holds
 * hs_error_split_workspace_bytes bytes.
 * At scale, where no box fits: for a hyperbolic cross sub = K_N(B), box may be the
 * padded cross of the same B widened by w >= the largest per-axis degree, with pad
 * NULL.  Then e_red = W^pol(X_K) v - W_{K,pol} v, the whole gap between the fast
 * algorithm and the exact Galerkin product on K (= E^red - E^quad of the box form).    */
int32_t hs_error_split_workspace_bytes(hs_index sub, hs_index box, hs_index pad, hs_pot pot, int64_t *bytes);
int32_t hs_error_split(hs_index sub, const void *sub_dev, hs_index box, const void *box_dev,
                       const int32_t *box_map_dev, hs_index pad, const void *pad_dev,
                       const int32_t *pad_map_dev, hs_pot pot, const void *pot_dev, const void *v,
                       void *e_quad, void *e_red, void *ws, void *stream);

/* ---- the unperturbed Lanczos process (paper Sec. 6.2, eq.
 * ErrorPerturbedLanczosAnalysis) --------------------------------------------------------
 * The paper's perturbation analysis compares the Lanczos process on A = D_K + W_{K,pol},
 * the exact Galerkin matrix, with the process on the fast algorithm (hs_step).  These
 * calls apply that exact operator on the rows of sub, as the fast algorithm on pad
 * restricted to sub: pad is a box reaching ceil(a/2) beyond every coordinate of sub (a
 * the potential's largest per-axis degree; sub a hyperbolic cross, a box or a total-
 * degree set), or, for a hyperbolic cross, the padded cross of the same bound widened by
 * w >= a (hs_index_create_padded).  pad_map_dev: hs_index_embed(sub, pad), uploaded
 * (device int32, sub->size).  complex128 vectors of sub; the paper's operator form.
 * hs_exact_workspace_bytes(m = 0) sizes hs_apply_exact's workspace, m >= 1 that of
 * hs_step_exact.  hs_apply_exact: y = (D + W_{K,pol}) x (x != y).  hs_step_exact: one
 * exponential-midpoint step with m Lanczos steps on the exact operator; t, t_dev, h,
 * reorth, diag_dev as for hs_step.  The difference of hs_step and hs_step_exact from
 * one start vector is the perturbation error of the Lanczos process; hs_step_exact with
 * a large m approximates exp(-i h A) c for the unperturbed Lanczos error.
 * HS_E_INVALID for a pad that does not carry the exact operator, HS_E_UNSUPPORTED for
 * sub given as a list or the symmetrised form.                                       */
int32_t hs_exact_workspace_bytes(hs_index sub, hs_index pad, hs_pot pot, int32_t m, int64_t *bytes);
int32_t hs_apply_exact(hs_index sub, hs_index pad, const void *pad_dev, const int32_t *pad_map_dev, hs_pot pot,
                       const void *pot_dev, const void *x, void *y, void *ws, void *stream);
int32_t hs_step_exact(hs_index sub, hs_index pad, const void *pad_dev, const int32_t *pad_map_dev, hs_pot pot,
                      void *pot_dev, double t, double *t_dev, double h, int32_t m, int32_t reorth, void *c,
                      void *ws, double *diag_dev, void *stream);

/* ---- batched form: many (index, potential) instances in one persistent launch ----
 * Instances are described by handles plus their uploaded device blocks (which must stay
 * alive); vectors of all instances are packed back to back in one device buffer with
 * offsets given by hs_batch_offsets (complex elements, host int64[n+1]).  Supported:
 * fused-class potentials in the paper's operator form on hyperbolic index sets built
 * with the default tile dimension, N 2..8, fewer than 2^31 rows in total (else
 * HS_E_UNSUPPORTED / HS_E_OVERFLOW; a form changed after creation is refused by the
 * next call).                                                                        */
int32_t hs_batch_create(int32_t n, const hs_index *idx, const void *const *idx_dev,
                        const hs_pot *pot, void *const *pot_dev, hs_batch *out);
int32_t hs_batch_destroy(hs_batch b);
int32_t hs_batch_offsets(hs_batch b, int64_t *host_out);
int32_t hs_batch_device_bytes(hs_batch b, int64_t *bytes);
int32_t hs_batch_upload(hs_batch b, void *dev, int64_t bytes, void *stream);
int32_t hs_batch_workspace_bytes(hs_batch b, int32_t m, int64_t *bytes);
/* y = H_i c_i for every instance i, one persistent launch (complex128). */
int32_t hs_batch_apply_h(hs_batch b, const void *batch_dev, const void *c, void *y, void *ws,
                         void *stream);
/* One exponential-midpoint Lanczos step for every instance (complex128); the time is
 * read from t_dev when it is not NULL and then advanced by h on the device.  ws holds
 * hs_batch_workspace_bytes(b, m) bytes. */
int32_t hs_batch_step(hs_batch b, void *batch_dev, double t, double *t_dev, double h, int32_t m,
                      int32_t reorth, void *c, void *ws, void *stream);
/* The batched H application runs one persistent kernel per (N, prefix axes) class present
 * (N = 2..8 at the default tile dimension), one after the other on the stream, so each
 * class runs at the occupancy of its own register count.  Work items are 64 rows (a chunk
 * of a long tile, or 64 rows of the short-tile list); each class's items are split into
 * one contiguous range per XCD, and a workgroup takes `grab` consecutive items per atomic
 * increment of its range's counter.  Item order: 0 = largest instances first, 1 = the
 * instances of a class interleaved chunk by chunk.
 * hs_batch_set_launch sets the workgroup size wg (64, 128, 256) and the resident
 * workgroups per compute unit per_cu (1..64) of every class; 0 keeps the current value.
 * hs_batch_get_launch reports them for the class holding the most rows.
 * hs_batch_autotune_sync times, for each item order, every class over wg x per_cu x grab
 * (3 x 4 x 3 candidates, each class alone), then the whole application per order, and
 * keeps the fastest order with its per-class settings; it rewrites the item list in
 * batch_dev (and the host image that hs_batch_upload copies) and synchronises the
 * stream.  The first failure is returned.
 * Instances whose potential has no x_l^2 or x_l x_{l+1} monomials take their long tiles
 * by the single-instance path's multi-tile work items (a second kernel per class), so a
 * batched row equals the single-instance row bit for bit; the tuning covers both kinds.
 * hs_batch_tuning writes the item order and, for each of the 7 classes, 10 int32
 * (N, prefix axes, then for the row kernel and the multi-tile kernel: work items, wg,
 * per_cu, grab) into table (70 int32, host).                                          */
int32_t hs_batch_set_launch(hs_batch b, int32_t wg, int32_t per_cu);
int32_t hs_batch_get_launch(hs_batch b, int32_t *wg, int32_t *per_cu);
int32_t hs_batch_tuning(hs_batch b, int32_t *order, int32_t *table);
int32_t hs_batch_autotune_sync(hs_batch b, const void *batch_dev, const void *c, void *y,
                               void *ws, void *stream);

/* ---- learned coefficients: Gauss-Hermite projection and a BF16-MFMA MLP --------
 * Potential family W(x) = - sum_i a_i exp(-|x - c_i(t)|^2 / (2 sigma^2)) in N <= 4
 * dimensions with G <= 4 wells, c_i(t) = base_i + rho (cos(omega t + phi_i) u_i + sin(omega t + phi_i) w_i)
 * with geometry (base, u, w, phi) fixed per family; parameters per sample
 * p = (t, a_1..a_G, sigma, rho, omega).  Coefficients: Hermite polynomials
 * H_a(x) = prod_l H_{a_l}(x_l) (physicists') with |a| <= D in lexicographic order of a.
 *
 * hs_gh_project: alpha_a = <W, H_a> / <H_a, H_a> with weight exp(-|x|^2), by product
 * Gauss-Hermite quadrature with Q <= 32 nodes per axis (paper Sec. 4.1), D <= 8, for
 * nsamp parameter rows (device, nsamp x (4 + G) doubles) into coef (device, nsamp x
 * ncoef doubles, ncoef = C(N + D, N)).  geometry (host): base, u, w as G x N doubles
 * each, then phase (G doubles).  The nodes and weights are computed on the host (the
 * eigenvalues of the Hermite Jacobi matrix); one workgroup per sample; asynchronous on
 * the stream.  HS_E_INVALID for sizes out of range.                                  */
int32_t hs_gh_ncoef(int32_t N, int32_t D, int32_t *ncoef);
/* hs_gh_rule: the Q-point Gauss-Hermite rule for the weight exp(-x^2) that
 * hs_gh_project uses (paper Sec. 4.1; the nodes are the eigenvalues of the Jacobi matrix
 * X_full of Sec. 4.2, found by Sturm-sequence bisection and one Newton step), written to
 * the host arrays x (ascending) and w of Q doubles each.  Host only, no device call.
 * HS_E_INVALID for Q outside 1..32 or NULL outputs; HS_E_NONFINITE if the bisection does
 * not isolate Q distinct nodes.                                                      */
int32_t hs_gh_rule(int32_t Q, double *x_host, double *w_host);
int32_t hs_gh_project(int32_t N, int32_t G, int32_t D, int32_t Q, const double *geometry_host,
                      int32_t nsamp, const double *params_dev, double *coef_dev, void *stream);
/* hs_cheb_interp: Chebyshev interpolation of the same Gaussian-well W on the cube
 * [-L, L]^N (paper Sec. 1.3, step (1) of Fig. 4): the tensor interpolant on the
 * (R + 1)^N first-kind Chebyshev points L cos((2k + 1) pi / (2 (R + 1))),
 *   alpha_r = prod_l (2 - [r_l = 0]) / (R + 1) sum_k W(x_k) prod_l cos(r_l theta_{k_l}),
 * returned for the multi-indices r with every r_l <= R and |r| <= D, in lexicographic
 * order (hs_cheb_ncoef counts them; for D <= R this is C(N + D, N)), as coefficients of
 * T_r(x / L) = prod_l T_{r_l}(x_l / L): a potential created with HS_BASIS_CHEB, scale L
 * and these degrees takes them through hs_pot_set_coeffs_device.  N <= 4, G <= 4,
 * R <= 15, (R + 1)^N + (R + 1)^2 <= 8192 (HS_E_UNSUPPORTED above), at most 512
 * coefficients; params, coef and geometry as for hs_gh_project; one workgroup per
 * sample; asynchronous on the stream.                                                */
int32_t hs_cheb_ncoef(int32_t N, int32_t D, int32_t R, int32_t *ncoef);
int32_t hs_cheb_interp(int32_t N, int32_t G, int32_t D, int32_t R, double L, const double *geometry_host,
                       int32_t nsamp, const double *params_dev, double *coef_dev, void *stream);

/* MLP in -> hidden -> hidden -> out with SiLU; BF16 operands on MFMA, FP32 accumulate,
 * FP32 master weights and Adam.  in <= 32, hidden a multiple of 64 (<= 512), out <= 512.
 * The device block (hs_mlp_device_bytes) holds weights, Adam moments and the
 * input/output normalisation; hs_mlp_upload_params sets weights (host float32:
 * W1 (hid x in), b1, W2 (hid x hid), b2, W3 (out x hid), b3) and normalisation
 * (in_lo[in], in_hi[in], out_mean[out], out_std[out]).                              */
int32_t hs_mlp_create(int32_t in, int32_t hidden, int32_t out, hs_mlp *mlp);
int32_t hs_mlp_destroy(hs_mlp mlp);
int32_t hs_mlp_device_bytes(hs_mlp mlp, int32_t max_batch, int64_t *bytes);
int32_t hs_mlp_upload_params(hs_mlp mlp, void *dev, const float *weights_host,
                             const float *norm_host, void *stream);
int32_t hs_mlp_download_params(hs_mlp mlp, const void *dev, float *weights_host, void *stream);
/* Forward on raw parameters x (device, batch x in float64) -> coefficients (device,
 * batch x out float64), de-normalised. */
int32_t hs_mlp_predict(hs_mlp mlp, void *dev, int32_t batch, const double *x_dev,
                       double *coef_dev, void *stream);
/* Surrogate coefficients with the quadrature as fallback: the network predicts every
 * row, then rows with any input outside the network's training box (in_lo, in_hi of
 * the normalisation) are recomputed by the Gauss-Hermite projection (Q nodes).  The
 * network must have 4 + G inputs and C(N + D, N) outputs.  used_quad_dev (device,
 * nsamp int32, may be NULL) receives 1 for rows taken from the quadrature.  No host
 * synchronisation: the choice is made per row on the device.                        */
int32_t hs_sur_coeffs(hs_mlp mlp, void *dev, int32_t N, int32_t G, int32_t D, int32_t Q,
                      const double *geometry_host, int32_t nsamp, const double *params_dev,
                      double *coef_dev, int32_t *used_quad_dev, void *stream);
/* One training step on (x, target coefficients) (device float64), MSE on normalised
 * outputs, Adam(lr, 0.9, 0.999, 1e-8).  loss_dev (device float, may be NULL) receives
 * the loss.  grads_dev (device, may be NULL) receives the float32 gradients in the
 * weight layout above (before the update).                                          */
int32_t hs_mlp_train_step(hs_mlp mlp, void *dev, int32_t batch, const double *x_dev,
                          const double *target_dev, float lr, float *loss_dev,
                          float *grads_dev, void *stream);

/* ---- debug build: neighbour-index checks ---------------------------------------------
 * Built with -DHS_DEBUG_BOUNDS (libhs_debug.so, see the package's build), the H-application
 * kernels check every tile record, work item, suffix-stencil offset and neighbour index
 * they use against the sizes of the set and the vector; a failed check is counted in the
 * index's device block (and the unchecked access is skipped where the hardware would not
 * bound it), so the kernels never fault.  hs_debug_checks reports whether this library
 * has the checks (1) or not (0; the release build, where they compile to nothing).
 * hs_index_debug_read copies the index's two counters (number of failed checks, code of
 * the first: 1 record, 2 work item, 3 suffix offset, 4 neighbour index, 5 tile position,
 * 6 row) to counts_host (host uint32[2]) after the work already enqueued on stream, and
 * zeroes them when clear != 0; it synchronises the stream.  hs_index_upload zeroes them.  */
int32_t hs_debug_checks(int32_t *built);
int32_t hs_index_debug_read(hs_index idx, const void *idx_dev, uint32_t *counts_host, int32_t clear, void *stream);

/* ---- checkpoint and resume (an addition: the state of Fig. 4's time_propagation) ----
 * The state of a propagation is (c^n, t_n, n) plus the configuration that produced it.
 * hs_checkpoint_save writes bytes bytes of src (the coefficient vector, any dtype) and a
 * caller-written header text (JSON by convention: t_n, n, the index set, the potential,
 * seeds) to path.  The file is
 *   "HSCKPT01" | u64 header bytes | header | u64 data bytes | u64 FNV-1a 64 of the data | data
 * (little-endian), written to path + ".tmp" and renamed over path, so an interrupted save
 * leaves the previous file intact.  src is device memory when src_on_device != 0 (the
 * call waits for the work already enqueued on stream, then copies through a 64 MiB
 * pinned buffer: it synchronises the stream), host memory otherwise.
 * hs_checkpoint_info (host only) checks a file's framing and returns its header
 * (NUL-terminated, truncated to cap - 1 bytes; header_out may be NULL), the header's full
 * length and the data size.
 * hs_checkpoint_load reads the data into dst (device when dst_on_device != 0, after the
 * work already enqueued on stream; synchronises the stream) after verifying the checksum
 * over the whole file, so a corrupt file leaves dst untouched.
 * Errors: HS_E_INVALID for NULL arguments, a negative size, or a destination size that
 * differs from the file's; HS_E_IO for files that cannot be opened, written or renamed,
 * that are not checkpoint files, are truncated, or fail the checksum; HS_E_HIP for a
 * failed copy.  Resuming from a checkpoint reproduces the uninterrupted run bit for bit
 * (the step is deterministic).                                                          */
int32_t hs_checkpoint_save(const char *path, const char *header_json, const void *src, int64_t bytes,
                           int32_t src_on_device, void *stream);
int32_t hs_checkpoint_info(const char *path, char *header_out, int64_t cap, int64_t *header_len,
                           int64_t *data_bytes);
int32_t hs_checkpoint_load(const char *path, void *dst, int64_t bytes, int32_t dst_on_device, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HS_H */
