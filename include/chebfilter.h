/*
 * chebfilter.h - C ABI of the MI355X (gfx950) Chebyshev-filtered subspace
 * iteration for the enriched spectral finite-element Kohn-Sham problem
 * (Kanungo & Gavini, "Large-scale all-electron density functional theory
 * calculations using an enriched finite element basis").
 *
 * Discrete problem (Sec. IV.A, Eq. SEPEFEM, H2x2, M2x2):
 *   H^E = [[H^cc, H^ec^T], [H^ec, H^ee]],  M^E = [[M^cc, M^ec^T], [M^ec, M^ee]]
 * with the free classical DOFs first (n_h of them) and the enrichment DOFs
 * last (n_e).  M^cc is the GLL-lumped diagonal (Sec. III.B).  The library
 * works on the standard form H~ = (M^E)^-1 H^E (Sec. V) and never assembles
 * a global matrix: H^cc and H^ec/M^ec enter only as per-cell blocks
 * (Sec. V, matrix-free elemental products followed by assembly).
 *
 * Conventions for every entry point:
 *  - Return value is cf_status; CF_OK = 0.  Nothing aborts, throws or prints;
 *    chebfilter_last_error() returns a message for the last failure.
 *  - Block arguments (X, Y) are DEVICE pointers to FP64 matrices, row-major
 *    [n][ld] with n = n_h + n_e rows (classical rows first) and ld >= N
 *    columns; the caller owns them.  Y must not overlap X.  Any ld works; an
 *    ld that is a multiple of 16 (with 128-byte aligned blocks) puts every
 *    row segment the kernels gather on a cache-line boundary, which is faster.
 *  - Work is enqueued on the context's stream and is asynchronous unless an
 *    entry point says it synchronises.  Calls on one context must not
 *    overlap (the context is not thread-safe).
 *  - The library keeps no caller pointer after a call returns.
 */
#ifndef CHEBFILTER_H
#define CHEBFILTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cf_ctx cf_ctx;

typedef enum {
  CF_OK = 0,
  CF_EINVAL = 1,     /* invalid argument (sizes, indices, bounds, pointers)   */
  CF_ENOMEM = 2,     /* device allocation failed or N above max_cols          */
  CF_ENOTSPD = 3,    /* Schur complement / Gram / projected overlap not SPD   */
  CF_ENUMERIC = 4,   /* NaN/Inf detected                                      */
  CF_EDEVICE = 5,    /* HIP runtime or library error                          */
  CF_ENOTCONV = 6    /* eigensolver did not converge                          */
} cf_status;

typedef enum { CF_FP64 = 0, CF_FP32 = 1, CF_BF16 = 2 } cf_prec;

/* Discrete problem.  HOST pointers, read during chebfilter_init only.
 * npc = (p+1)^3 local nodes per cell, x fastest. */
typedef struct {
  int32_t p;                 /* element degree; the library supports 1 <= p <= 4     */
  int64_t n_cells;           /* E                                                      */
  int64_t n_h;               /* free classical DOFs                                    */
  int64_t n_e;               /* enrichment DOFs                                        */
  const int64_t *cell_dof;   /* [E*npc] free classical DOF of each local node, -1 marks
                                a Dirichlet node (Sec. III.A, homogeneous Dirichlet)  */
  const double *H_cc;        /* [E*npc*npc] elemental H^cc_e, row-major, symmetric
                                (Eq. Hcc)                                              */
  const double *M_cc_diag;   /* [n_h] assembled GLL-lumped M^cc, all > 0 (Sec. III.B) */
  const int64_t *enr_ptr;    /* [E+1] CSR over cells: enrichment functions whose support
                                meets the cell                                         */
  const int64_t *enr_idx;    /* [enr_ptr[E]] alpha in [0, n_e), distinct within a cell */
  const double *H_ec;        /* [enr_ptr[E]*npc] per-cell H^ec_e rows (row alpha,
                                column local node) (Eq. Hec)                           */
  const double *M_ec;        /* [enr_ptr[E]*npc] per-cell M^ec_e rows (Eq. Mec)        */
  const double *H_ee;        /* [n_e*n_e] assembled H^ee, symmetric (Eq. Hee)          */
  const double *M_ee;        /* [n_e*n_e] assembled M^ee, symmetric (Eq. Mee)          */
} cf_problem;

typedef struct {
  int32_t device;            /* HIP device ordinal                                     */
  void *stream;              /* hipStream_t to enqueue on (NULL = default stream)      */
  int64_t max_cols;          /* largest block width N any later call may pass          */
  int64_t col_chunk;         /* columns of the internal work blocks (0 or >= max_cols:
                                max_cols).  Wider blocks are processed in chunks of
                                col_chunk columns (the filter and the products are
                                column-independent; the projection works on column
                                slabs), so device workspace grows with col_chunk, not
                                with N.  The work blocks' leading dimension is
                                col_chunk rounded up to a multiple of 16.  Batches
                                ignore it.                                             */
  int32_t check_finite;      /* nonzero: filter/rayleigh_ritz check outputs for NaN/Inf */
} cf_options;

/* Build a context: validate the problem, upload element data, colour cells so
 * that cells of one colour share no DOF, form the Schur complement
 * S = M^ee - M^ec (M^cc)^-1 M^ec^T (Sec. IV.D) in FP64 on the device and
 * factor it.  Returns CF_ENOTSPD if S is not positive definite, CF_EINVAL for
 * malformed input, CF_ENOMEM if workspace for max_cols columns does not fit.
 * Synchronises.  On failure *out is NULL. */
cf_status chebfilter_init(const cf_problem *prob, const cf_options *opt, cf_ctx **out);

/* Release every device buffer of the context.  NULL is accepted. */
cf_status chebfilter_destroy(cf_ctx *ctx);

/* Message describing the last failure on ctx (or of the last failed init when
 * ctx is NULL).  Valid until the next call on the same context. */
const char *chebfilter_last_error(const cf_ctx *ctx);

/* Problem sizes as seen by the library (n = n_h + n_e). */
cf_status chebfilter_sizes(const cf_ctx *ctx, int64_t *n_h, int64_t *n_e, int64_t *max_cols);

/* Y = H^E X  (Eq. H2x2; elemental products + assembly, Sec. V).  0 <= N <= max_cols. */
cf_status chebfilter_apply_H(cf_ctx *ctx, const double *X, int64_t ldx, double *Y, int64_t ldy,
                             int64_t N);

/* Y = M^E X  (Eq. M2x2). */
cf_status chebfilter_apply_M(cf_ctx *ctx, const double *X, int64_t ldx, double *Y, int64_t ldy,
                             int64_t N);

/* Y = (M^E)^-1 X by the block-wise (Banachiewicz) inverse of Sec. IV.D:
 * u = D^-1 x_c, w = x_e - M^ec u, z = S^-1 w, y_e = z, y_c = u - D^-1 M^ec^T z,
 * with D = M^cc diagonal and S the Schur complement.  The S solve is FP64. */
cf_status chebfilter_apply_Sinv(cf_ctx *ctx, const double *X, int64_t ldx, double *Y,
                                int64_t ldy, int64_t N);

/* Y = T_m(t(H~)) X, t(x) = (2x - a - b)/(b - a), H~ = (M^E)^-1 H^E, by the
 * three-term Chebyshev recurrence (Sec. V).  m = 0 copies X.  Requires b > a,
 * both finite, m >= 0.  prec selects the arithmetic of the recurrence:
 *   CF_FP64  everything in FP64;
 *   CF_FP32  recurrence blocks, elemental and coupling products in FP32 (FP32
 *            MFMA); enrichment-row sums, the Schur-complement solve and its
 *            output in FP64; X is rounded to FP32 on entry, Y widened to FP64;
 *   CF_BF16  as CF_FP32, but the elemental products of the cells with no DOF
 *            in the enriched region take the cell matrices and the gathered
 *            vector tiles in BF16 (FP32 accumulation); cells touching that
 *            region stay FP32, because BF16 rounding there excites the
 *            near-null space of M^E, which (M^E)^-1 amplifies.
 * The reduced forms hold their iterates scaled by powers of two chosen on the
 * device from the growth of the last two iterates, and return the unscaled
 * T_m(t(H~)) X in FP64 (bit for bit the unscaled FP32 recurrence wherever that
 * one stays inside FP32's normal range).
 * The reduced forms keep FP32 copies of the operator (and BF16 cell matrices)
 * on the device from their first use until chebfilter_destroy, plus two FP32
 * blocks of n x max_cols.  Their results carry FP32 (or BF16) rounding: they
 * are meant for filter passes followed by an FP64 cleanup pass.  Other prec
 * values return CF_EINVAL. */
cf_status chebfilter_filter(cf_ctx *ctx, const double *X, int64_t ldx, double *Y, int64_t ldy,
                            int64_t N, int32_t m, double a, double b, int32_t prec);

/* Multi-pass low-degree filter (used for the gold nano-clusters of Sec. VI
 * against the loss of conditioning of one high-degree pass): `passes`
 * applications of T_m(t(H~)) with the block replaced by its Ritz vectors
 * (chebfilter_rayleigh_ritz) between passes:
 *   Y = T_m(t) Q_{p-1},  Q_i = RR(T_m(t) Q_{i-1}),  Q_0 = X.
 * The span equals that of T_m(t)^passes X.  The Ritz basis keeps every column
 * aligned with its own eigen-direction, so each pass amplifies the columns one
 * by one (a triangular Cholesky-QR basis would mix them).  passes = 1 is
 * chebfilter_filter.  Uses the context's work blocks; synchronises. */
cf_status chebfilter_filter_multipass(cf_ctx *ctx, const double *X, int64_t ldx, double *Y,
                                     int64_t ldy, int64_t N, int32_t m, int32_t passes, double a,
                                     double b, int32_t prec);

/* Tile shape of the reduced-precision cell product (a launch parameter, not
 * part of the method): nsb = 1 or 2 sixteen-column MFMA blocks per column
 * tile, for the FP32-input cells (prec = CF_FP32) or the BF16-input cells
 * (prec = CF_BF16) of the context.  Both shapes compute bit-identical
 * results; two blocks fill a 128-byte line per gathered row, one keeps the
 * registers (and so the occupancy) lower.  Defaults: FP32 1, BF16 2.
 * CF_EINVAL on another prec or nsb. */
cf_status chebfilter_set_cell_tile(cf_ctx *ctx, int32_t prec, int32_t nsb);

/* Autotuner of the reduced forms' tile shapes: runs chebfilter_filter(ctx, X,
 * ldx, Y, ldy, N, m, a, b, prec) once as a warm-up and `reps` times timed
 * (HIP events on the context's stream) for each candidate and keeps the
 * fastest for later calls.  First the cell product's column blocks per tile
 * (returned in *choice, may be null); then, for problems with enrichment,
 * the FP32 coupling partials' split of a workgroup's 8 waves between 16-row
 * output blocks and parts of the 128 local nodes (1 x 8, 2 x 4 or 4 x 2),
 * one choice per bucket of enriched cells by their number of 16-function row
 * blocks (1, 2, 3, >= 4; uneven enrichment counts per cell, Sec. IV.C),
 * bucket by bucket with the others fixed (chebfilter_tuning reads the map).
 * The choices change only the order of FP32 sums.  Y is overwritten; prec is
 * CF_FP32 or CF_BF16; m >= 1, reps >= 1.  Synchronises. */
cf_status chebfilter_autotune(cf_ctx *ctx, const double *X, int64_t ldx, double *Y, int64_t ldy,
                              int64_t N, int32_t m, double a, double b, int32_t prec, int32_t reps,
                              int32_t *choice);

/* In place: Y <- Q with Q^T Q = I and span(Q) = span(Y), by Cholesky-QR
 * applied twice after scaling columns to unit length (the orthonormalisation
 * step of Sec. V).  Falls back to a shifted first pass if the Gram matrix is
 * not numerically positive definite.  Synchronises; CF_ENOTSPD if even the
 * shifted pass fails (e.g. a zero column). */
cf_status chebfilter_cholqr(cf_ctx *ctx, double *Y, int64_t ldy, int64_t N);

/* In place Rayleigh-Ritz (Sec. V): orthonormalise Y (as chebfilter_cholqr),
 * project H^E and M^E onto it, solve the N x N generalized symmetric problem
 * Q^T H Q c = theta Q^T M Q c and rotate: Y <- Q C.  On return Y holds
 * M-orthonormal Ritz vectors and theta_host[0..N) the Ritz values in
 * ascending order (host memory).  Synchronises. */
cf_status chebfilter_rayleigh_ritz(cf_ctx *ctx, double *Y, int64_t ldy, int64_t N,
                                   double *theta_host);

/* k-step Lanczos on H~ in the M^E inner product (H~ is self-adjoint there,
 * so the "few Arnoldi iterations" of Sec. V reduce to Lanczos), started from
 * the device vector v0[n].  Returns on the host the smallest Ritz value of the
 * k x k tridiagonal (*lmin_est) and the upper bound theta_max + ||f_k||_M
 * (*b_upper).  1 <= k <= 64.  Synchronises. */
cf_status chebfilter_lanczos_bounds(cf_ctx *ctx, const double *v0, int32_t k, double *lmin_est,
                                    double *b_upper);

/* chebfilter_lanczos_bounds for callers that cannot allocate device memory
 * (tight self-consistent-step loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with every piece of work memory the run needs
 * (work rows, the four Lanczos vectors, coupling partials, the enriched-cell
 * buffer, w, z, coefficients, partial sums) taken from a fixed device array
 * of 64 MiB that the library holds on each GPU from its first use until the
 * process ends, instead of the context's work blocks.  It calls no
 * allocation routine.  The scratch needed is about
 *   8 bytes x (5 n + coupling rows + 128 x enriched cells + 2 n_e + 1160);
 * a larger problem returns CF_ENOMEM with the size it would need (the
 * context's chebfilter_lanczos_bounds still works for it).  All calls on one
 * GPU share that array: calls that overlap on one GPU (several host threads,
 * or several streams, without ordering) race and return wrong bounds.  The
 * run clears what must start at zero.  Synchronises. */
cf_status chebfilter_lanczos_bounds_noalloc(cf_ctx *ctx, const double *v0, int32_t k,
                                            double *lmin_est, double *b_upper);

/* Per-kernel timing with HIP events on the context's stream.  enable != 0
 * starts recording (and clears the totals); name selects a kernel family
 * ("cell_gemm": the MFMA cell products, N > 1; "cell_gemv": single-column
 * cell products; "cell_gemm_fp32", "cell_gemm_bf16", "enr_part",
 * "enr_reduce", "enr_q", "enr_gemm", "gram", "rotate", "epilogue",
 * "assemble").  The query returns the number of timed launches, their summed
 * duration and the algorithmic flops credited to them (cell products:
 * 2 npc^2 N per cell; 0 where not counted).  Synchronises on query. */
cf_status chebfilter_profile(cf_ctx *ctx, int32_t enable);
cf_status chebfilter_profile_query(cf_ctx *ctx, const char *name, int64_t *launches,
                                   double *total_ms, double *total_flops);

/* ---- Batches of independent problems ------------------------------------
 * Many discrete problems (Sec. IV) filtered together: each problem is the
 * method of Sec. V on its own, and the batch only changes how the work is
 * launched.  Entries that point to the same cf_problem share one device copy
 * of the operator; every entry has its own blocks, interval and workspace.
 * The options (device, stream, max_cols, check_finite) apply to every entry.
 * Array arguments are HOST arrays with one element per entry (device
 * pointers for blocks).  Calls on one batch must not overlap. */
typedef struct cf_batch cf_batch;

/* Build the contexts of count entries (probs[i] as for chebfilter_init).
 * On failure *out is null and chebfilter_batch_last_error(NULL) explains. */
cf_status chebfilter_init_batch(const cf_problem *const *probs, int32_t count,
                                const cf_options *opt, cf_batch **out);
cf_status chebfilter_batch_destroy(cf_batch *batch);
const char *chebfilter_batch_last_error(const cf_batch *batch);
/* Row counts of entry i (its blocks have n_h + n_e rows). */
cf_status chebfilter_batch_sizes(const cf_batch *batch, int32_t i, int64_t *n_h, int64_t *n_e);

/* Y[i] = T_m(t_i(H~_i)) X[i] for every entry, t_i(x) = (2x - a[i] - b[i])/(b[i] - a[i])
 * (Sec. V recurrence, per entry as chebfilter_filter).  1 <= N[i] <= max_cols.
 * CF_FP32 and CF_BF16 run every entry in the same launches: per step one
 * launch per cell colour (colour k of all entries together; BF16: two, cells
 * near the enriched region in FP32), one per coupling/Schur/epilogue kernel,
 * each work item addressing its entry through a device descriptor table; the
 * result of each entry is bit for bit that of chebfilter_filter with the same
 * prec.  With use_graph != 0 the launches of the whole filter are captured
 * once per (m, prec) into a HIP graph on an internal stream and replayed (the
 * descriptors, updated before each replay, carry the blocks and intervals).
 * The work is ordered after prior work on the options' stream, and later work
 * there waits for it.  CF_FP64 (and m = 0) runs chebfilter_filter entry by
 * entry.  The first reduced call allocates the FP32 workspace of every entry
 * (two n x max_cols FP32 blocks plus the per-call work blocks). */
cf_status chebfilter_filter_batch(cf_batch *batch, const double *const *X, const int64_t *ldx,
                                  double *const *Y, const int64_t *ldy, const int64_t *N,
                                  int32_t m, const double *a, const double *b, int32_t prec,
                                  int32_t use_graph);

/* The autotuner of chebfilter_autotune for the batched filter: times the
 * graph-replayed batched filter with one and with two column blocks per tile
 * of the batched reduced cell product (FP32-input cells for CF_FP32,
 * BF16-input cells for CF_BF16), keeps the fastest for the batch's later
 * calls (the captured graph is rebuilt when the shape changes) and returns
 * it in *choice.  Arguments as chebfilter_filter_batch; Y is overwritten.
 * Synchronises. */
cf_status chebfilter_batch_autotune(cf_batch *batch, const double *const *X, const int64_t *ldx,
                                    double *const *Y, const int64_t *ldy, const int64_t *N,
                                    int32_t m, const double *a, const double *b, int32_t prec,
                                    int32_t reps, int32_t *choice);

/* Tuning state of a context (chebfilter_tuning) or a batch
 * (chebfilter_batch_tuning): the column blocks per tile of the FP32-input and
 * BF16-input cell products and the coupling map (2 bits per row-block bucket
 * 1, 2, 3, >= 4, lowest bits first: 0 -> 1 row block x 8 k parts, 1 -> 2 x 4,
 * 2 -> 4 x 2).  set_map >= 0 sets the map first (CF_EINVAL for a code 3 or a
 * value above 255); output pointers may be null. */
cf_status chebfilter_tuning(cf_ctx *ctx, int32_t set_map, int32_t *nsb_fp32, int32_t *nsb_bf16,
                            int32_t *coupling_map);
cf_status chebfilter_batch_tuning(cf_batch *batch, int32_t set_map, int32_t *nsb_fp32,
                                  int32_t *nsb_bf16, int32_t *coupling_map);

/* chebfilter_rayleigh_ritz for every entry (Sec. V's projection), with one
 * host synchronisation for the whole batch: every entry is orthonormalised by
 * two unshifted Cholesky-QR passes and projected with no host wait, the
 * projected pencils of equal width go to one batched generalized eigensolve,
 * and a predicated rotation writes Y[i] only where every step succeeded.  An
 * entry whose orthonormalisation or eigensolve failed is then redone by
 * chebfilter_rayleigh_ritz (shifted Cholesky-QR, its own errors).  Results
 * equal the single-problem call to rounding.  theta_host[i] receives N[i]
 * values.  On an error (message names the entry) the blocks of other entries
 * may already hold their Ritz vectors; the failing entry's block is the
 * filtered block or, if the eigensolve failed, an orthonormal basis of it.
 * Workspace: per entry two max_cols^2 pencils, allocated on the first call. */
cf_status chebfilter_rayleigh_ritz_batch(cf_batch *batch, double *const *Y, const int64_t *ldy,
                                         const int64_t *N, double *const *theta_host);

/* chebfilter_lanczos_bounds for every entry (Sec. V's upper bound), one host
 * synchronisation: the k-step runs of entries that share a problem are the
 * columns of one block (up to max_cols runs), so each step applies the
 * operator once per problem; runs stay independent, and the bounds equal the
 * single-vector call's to rounding.  lmin_est[i], b_upper[i].  Workspace: four
 * blocks of (largest n) x (largest group) doubles, allocated on the first call. */
cf_status chebfilter_lanczos_bounds_batch(cf_batch *batch, const double *const *v0, int32_t k,
                                          double *lmin_est, double *b_upper);

/* ---- Operator updates and Ritz residuals ---------------------------------- */

/* Replace the elemental H^cc_e (same layout and checks as cf_problem.H_cc):
 * the update of a self-consistent step, where only the potential changes.
 * H^ec, H^ee, D, M^ec and the Schur complement are unchanged.  The reduced
 * copies are refreshed.  Synchronises. */
cf_status chebfilter_update_H_cc(cf_ctx *ctx, const double *H_cc);

/* ---- Element blocks of the plain cells on the device ----------------------- */

/* Reference tables for chebfilter_assemble_cells (Sec. III.B, Eq. HBlocks):
 * the classical block of a cell outside every enrichment support is
 * H^cc_e = K + B^T diag(w .* V_e) B, with K [npc][npc] the kinetic block
 * 1/2 int grad N_a . grad N_b (identical for the cells of the uniform mesh;
 * symmetric to 1e-10 relative, symmetrised), B [nq][npc] the shape-function
 * values at the cell's nq Gauss points (the same in every cell) and w [nq]
 * the quadrature weights times the cell Jacobian.  Host arrays, row-major,
 * copied; 1 <= nq <= 4096.  Synchronises.  CF_EINVAL on non-finite input. */
cf_status chebfilter_assembly_tables(cf_ctx *ctx, int32_t nq, const double *B, const double *w,
                                     const double *K);

/* Assemble H^cc_e on the device for the ncells cells listed in cells (host
 * int32, distinct, cells without enrichment functions: the blocks of cells
 * inside an enrichment support use the adaptive rule of Sec. IV.C and stay
 * host input) from V (device FP64, row i = the potential at the nq Gauss
 * points of cells[i], leading dimension ldv >= nq): the quadrature sum runs
 * as an FP64 MFMA contraction per cell and overwrites the context's block of
 * that cell (written exactly symmetric); the reduced-precision copies are
 * refreshed.  This is the per-step operator update of a self-consistent
 * iteration when the potential lives on the device.  Enqueued on the
 * context's stream (waits only when the cell list differs from the last
 * call's).  CF_EINVAL without tables, on a bad, repeated or enriched cell. */
cf_status chebfilter_assemble_cells(cf_ctx *ctx, const int32_t *cells, int64_t ncells, const double *V,
                                    int64_t ldv);

/* Copy the current H^cc_e of the listed cells (host int32) into out (host,
 * [ncells][npc][npc]).  Synchronises. */
cf_status chebfilter_get_H_cc(cf_ctx *ctx, const int32_t *cells, int64_t ncells, double *out);

/* ---- Element blocks of the cells with an adaptive rule, on the device ------- */

/* The adaptive quadrature grid of Sec. IV.C and the enrichment functions of
 * Sec. IV.A-B, for chebfilter_assemble_enriched.  The grid of a cell is the list
 * of boxes that the divide-and-conquer refinement accepted; each box carries
 * the tensor ng^3 Gauss rule (points box_lo + box_size (x_i, x_j, x_k), i
 * fastest; weights box_size^3 w_i w_j w_k).  The grid is fixed for a mesh; only
 * the potential at its points changes from one self-consistent step to the
 * next.  Enrichment function alpha = I * n_per_atom + m belongs to atom I:
 * a radial part R(r) = sum of c r^k exp(-zeta r) over the shell's terms, times
 * a real harmonic (l = 0: 1/sqrt(4 pi); l = 1: sqrt(3/(4 pi)) (y, z, x)/r, in
 * that order), times the smooth cutoff h of Eq. Moll1 with
 * r~ = 1 - t (r - r0) / r0.  n_per_atom = sum over shells of 2l + 1.  Every
 * cell's enrichment list (cf_problem.enr_idx) must consist of whole atoms,
 * ascending.  All arrays are host arrays, copied. */
typedef struct {
  int64_t ncells;             /* listed cells: every cell with enrichment functions, plus any
                               * plain cell whose block needs the adaptive rule             */
  const int32_t *cells;       /* [ncells] distinct cell indices                              */
  const double *cell_lo;      /* [ncells][3] lower corner of each listed cell                */
  double h;                   /* cell side                                                   */
  int32_t n_nodes;            /* 1D nodes per axis (p + 1), n_nodes^3 = nodes per cell, <= 8  */
  const double *nodes;        /* [n_nodes] increasing, on [0, 1]; local node a = i + n j + n^2 k */
  int32_t ng;                 /* Gauss points per axis in a box, 1..8                        */
  const double *gauss_x;      /* [ng] in (0, 1)                                              */
  const double *gauss_w;      /* [ng] summing to 1                                           */
  const int64_t *box_ptr;     /* [ncells + 1], box_ptr[0] = 0: boxes of cells[i]              */
  const double *box_lo;       /* [nbox][3] lower corners (inside the cell)                   */
  const double *box_size;     /* [nbox] sides                                                */
  int32_t n_atoms;            /* n_atoms * n_per_atom = n_e                                  */
  const double *centers;      /* [n_atoms][3]                                                */
  int32_t n_shells;           /* shells per atom, the same for every atom                    */
  const int32_t *shell_l;     /* [n_shells] 0 or 1                                           */
  const int32_t *shell_term_ptr; /* [n_shells + 1], [0] = 0: terms of each shell            */
  const double *term_c;       /* [nterm] coefficients                                        */
  const int32_t *term_k;      /* [nterm] powers of r, l <= k <= 16                           */
  const double *term_zeta;    /* [nterm] exponents >= 0                                      */
  double r0, t;               /* cutoff radius and transition width (Eq. Moll1), > 0         */
} cf_adaptive_grid;

/* Upload the grid and the enrichment description (validated; CF_EINVAL with a
 * message on any violation above, on a missing kinetic block: call
 * chebfilter_assembly_tables first, or when a cell with enrichment functions
 * is not listed).  The partial H^ee blocks of the assembly are summed in fixed
 * batches of cells (at most 512 MiB of partials each), decided here.
 * Synchronises. */
cf_status chebfilter_enriched_tables(cf_ctx *ctx, const cf_adaptive_grid *grid);

/* Number of points of the uploaded grid (sum over boxes of ng^3): the length
 * of the potential array of chebfilter_assemble_enriched. */
cf_status chebfilter_adaptive_points(const cf_ctx *ctx, int64_t *npoints);

/* Recompute, on the device, the Hamiltonian blocks that the potential enters
 * on the listed cells (Eq. HBlocks with the adaptive rule, Sec. IV.C):
 *   H^cc_e = K + sum_q w_q V_q N_a N_b                       (every listed cell)
 *   H^ec_e = sum_q w_q (V_q N_al N_a + 1/2 grad N_al . grad N_a)
 *   H^ee   = sum over cells of sum_q w_q (V_q N_al N_be + 1/2 grad N_al . grad N_be)
 * with K the kinetic block of chebfilter_assembly_tables and V (device FP64,
 * [npoints]) the potential at the grid's points, box by box.  The quadrature
 * sums run as FP64 MFMA contractions; H^cc_e and H^ee are written exactly
 * symmetric; H^ee sums the cells in a fixed order (no atomics).  Then the
 * enrichment block of the block-wise inverse's step, H^ee - M^ec D^-1 H^ec^T
 * (Sec. IV.D), is rebuilt from the new blocks and the reduced-precision copies
 * are refreshed.  M^ec, M^ee, D and the Schur complement do not depend on the
 * potential and are unchanged.  Enqueued on the context's stream; uses the
 * context's work blocks.  CF_EINVAL without a grid or with a null V. */
cf_status chebfilter_assemble_enriched(cf_ctx *ctx, const double *V);

/* Copy the current H^ec (host, [nnz][npc] in cf_problem.H_ec's layout) and
 * H^ee (host, [n_e][n_e]); either may be null.  Synchronises. */
cf_status chebfilter_get_coupling(cf_ctx *ctx, double *H_ec, double *H_ee);

/* ---- Self-consistent field quantities around the eigensolver --------------
 * Sec. II and Sec. V.  The density and the potentials live on the quadrature
 * points: the plain cells' Gauss points (the rule of chebfilter_assembly_tables,
 * cell by cell in cell order), then the adaptive grid's points (the grid of
 * chebfilter_enriched_tables, box by box).  In this layout the effective
 * potential is the input of both assembly entry points (chebfilter_scf_assemble).
 * The electrostatic enrichment set is empty: the Hartree potential is the
 * classical finite-element solution of Eq. Hartree_possion (discretised as
 * Eq. discretePoissonCFEM) with zero Dirichlet values, for the density less a
 * neutralising Gaussian of the same charge; the Gaussian's potential
 * Q erf(r/s)/r is added back at the points. */
typedef struct {
  const double *cell_lo;      /* [n_cells][3] lower corner of every cell                       */
  const double *plain_ref;    /* [nq][3] points of the plain rule on the unit cube, in the order
                               * of the assembly table's rows (x fastest)                        */
  double comp_center[3];      /* centre c of the neutralising Gaussian                         */
  double comp_width;          /* its width s > 0: rho_g = Q (s sqrt pi)^-3 exp(-|x-c|^2/s^2)   */
  int32_t cg_max_iter;        /* Poisson CG: iteration limit >= 1                              */
  double cg_tol;              /* and relative residual ||b - A phi|| / ||b|| > 0               */
  int32_t mix_depth;          /* Anderson stages kept, 1..8                                    */
  double mix_beta;            /* Anderson step beta > 0                                        */
} cf_scf_setup;

/* Points, weights, per-colour cell lists, the Poisson matrix block and its
 * Jacobi diagonal, and the work buffers.  Requires chebfilter_assembly_tables
 * and chebfilter_enriched_tables.  CF_EINVAL on bad settings.  Synchronises. */
cf_status chebfilter_scf_setup(cf_ctx *ctx, const cf_scf_setup *setup);

/* Number of points (the length of every field array), of which the first
 * nplain_points are the plain cells'. */
cf_status chebfilter_scf_sizes(const cf_ctx *ctx, int64_t *npoints, int64_t *nplain_points);

/* Coordinates [npoints][3] and weights [npoints] (Jacobian included) of the
 * points, host copies (either may be null).  Synchronises. */
cf_status chebfilter_scf_geometry(cf_ctx *ctx, double *xyz, double *w);

/* Occupations and Fermi level (Eq. FermiDirac, Eq. Mu): f_i = 1 / (1 +
 * exp((eps_i - mu) / kT)) with 2 sum_i f_i = n_electrons, mu by bisection
 * on [min eps - 40 kT, max eps + 40 kT].  Host arrays eps, f [N].  CF_EINVAL
 * unless 0 < n_electrons < 2 N, kT > 0 and eps finite.  No context. */
cf_status chebfilter_fermi_level(const double *eps, int64_t N, double n_electrons, double kT,
                                 double *f, double *mu);

/* Electron density at the points (Eq. Rho): rho(x) = 2 sum_j f_j psi_j(x)^2
 * with psi_j the basis expansion of column j of X (device, [n][ldx], the
 * layout of every block).  Per cell, the density matrix D_e = Y_e diag(2 f) Y_e^T
 * of the cell's rows (FP64 MFMA), then rho_q = Phi_q^T D_e Phi_q with the
 * basis values Phi_q at the cell's points (FP64 MFMA).  f_host [N] host.
 * rho device [npoints].  Synchronises. */
cf_status chebfilter_scf_density(cf_ctx *ctx, const double *X, int64_t ldx, int64_t N,
                                 const double *f_host, double *rho);

/* Effective potential at the points (Eq. veff): V_eff = v_ext + V_H + V_xc,
 * with V_xc the LDA of Sec. II (the Perdew-Zunger fit of Ceperley-Alder,
 * spin unpolarised) and V_H from the Poisson problem above, solved by
 * Jacobi-preconditioned conjugate gradients on the device (matrix products
 * cell by cell, colour by colour), started from the previous call's
 * solution.  Device arrays [npoints]: rho, v_ext (the external potential at
 * the points), v_eff (output).  terms (host [5]): int rho, E_xc = int rho
 * eps_xc, int rho V_xc, 1/2 int rho V_H, the final relative CG residual;
 * cg_iters (may be null).  CF_ENOTCONV if the CG limit is reached first.
 * Synchronises. */
cf_status chebfilter_scf_potential(cf_ctx *ctx, const double *rho, const double *v_ext,
                                   double *v_eff, double *terms, int32_t *cg_iters);

/* The Hamiltonian blocks for a new effective potential at the points:
 * chebfilter_assemble_cells on the plain cells and chebfilter_assemble_enriched
 * on the adaptive grid.  v_eff device [npoints]. */
cf_status chebfilter_scf_assemble(cf_ctx *ctx, const double *v_eff);

/* n-stage Anderson mixing of the density (Sec. V): the pair (rho_in, rho_out)
 * joins a history of the last mix_depth pairs; with residuals F_k = rho_out,k
 * - rho_in,k, the coefficients c (sum c_k = 1) minimise || sum c_k F_k ||_w in
 * the weighted point inner product, and rho_next = sum c_k (rho_in,k + beta
 * F_k).  Device arrays [npoints]; res_norm (host, may be null) receives
 * || rho_out - rho_in ||_w of the new pair, the SCF convergence measure.
 * CF_EINVAL on a singular history.  Synchronises. */
cf_status chebfilter_scf_mix(cf_ctx *ctx, const double *rho_in, const double *rho_out,
                             double *rho_next, double *res_norm);

/* Forget the mixing history. */
cf_status chebfilter_scf_mix_reset(cf_ctx *ctx);

/* res_host[j] = || H^E z_j - theta_j M^E z_j ||_{(M^E)^-1} for the columns z_j of
 * Z with theta_host[j] (the Ritz residual in the dual norm of Sec. V's
 * generalized problem).  Uses the context's work blocks; synchronises. */
cf_status chebfilter_residual_norms(cf_ctx *ctx, const double *Z, int64_t ldz, int64_t N,
                                    const double *theta_host, double *res_host);

/* ---- Learned filter bounds ---------------------------------------------------
 * A fully connected network (FP32; depth hidden layers of width units with
 * GELU, linear output) with hand-written forward, backward (mean squared
 * error) and Adam kernels.  Parameters are a flat FP32 array: for each layer l,
 * W_l [out_l][in_l] row-major then b_l [out_l]; the caller supplies the initial
 * values.  Device arrays: X [B][n_in], targets and outputs [B][n_out]. */
typedef struct cf_mlp cf_mlp;
cf_status chebfilter_mlp_create(int32_t device, void *stream, int32_t n_in, int32_t width,
                                int32_t depth, int32_t n_out, int32_t max_batch, cf_mlp **out);
cf_status chebfilter_mlp_destroy(cf_mlp *mlp);
const char *chebfilter_mlp_last_error(const cf_mlp *mlp);
cf_status chebfilter_mlp_sizes(const cf_mlp *mlp, int64_t *nparams);
/* host arrays of nparams floats; reset_adam zeroes the Adam moments and step count */
cf_status chebfilter_mlp_set_params(cf_mlp *mlp, const float *host, int32_t reset_adam);
cf_status chebfilter_mlp_get_params(cf_mlp *mlp, float *host);
/* Y = net(X), 1 <= B <= max_batch */
cf_status chebfilter_mlp_forward(cf_mlp *mlp, const float *X, int32_t B, float *Y);
/* loss = mean over the B x n_out entries of (net(X) - T)^2 and its gradient
 * (kept on the device for chebfilter_mlp_adam_step; copied to grad_host
 * [nparams] if non-null).  Synchronises. */
cf_status chebfilter_mlp_loss_grad(cf_mlp *mlp, const float *X, const float *T, int32_t B,
                                   float *loss_host, float *grad_host);
/* One Adam update (Kingma & Ba, bias-corrected) with the last gradient. */
cf_status chebfilter_mlp_adam_step(cf_mlp *mlp, float lr, float beta1, float beta2, float eps);
/* Affine normalisation used by chebfilter_bounds_predict: inputs (x - mean)/std,
 * outputs mean + std * y.  Host arrays of n_in, n_in, n_out, n_out. */
cf_status chebfilter_mlp_set_normalization(cf_mlp *mlp, const double *in_mean, const double *in_std,
                                           const double *out_mean, const double *out_std);

/* Scale-free network inputs from raw history: steps x 8 raw features, oldest
 * first (theta_1, theta_Nw, theta_N, b used, m used, largest and median
 * residual norm, largest change of the wanted Ritz values).  With theta_N and
 * w = b - theta_N of the last step: energies (the first four) become
 * (x - theta_N)/w, the degree m/100, the last three log10(x/w + 1e-30).
 * CF_EINVAL if w <= 0.  Host arrays of 8 * steps. */
cf_status chebfilter_bounds_features(const double *history, int32_t steps, double *out);

/* Filter interval and degree for the next step (the bound b of Sec. V and
 * the degree, whose choice the paper ties to the spectral width) from the
 * network, fed chebfilter_bounds_features(history) (n_in = 8 x steps).  Its
 * outputs, after the output normalisation, are (alpha, beta, m) with
 * a = theta_N + alpha w and b = theta_N + beta w (theta_N, w of the last step).
 * Guard: the prediction is used only if it is finite and beta lies within
 * [0.98, 2]; b then gets a 5 % margin above theta_N (an overestimated b only
 * damps less; an underestimated one would amplify the top of the spectrum),
 * a is kept if it lies in [theta_Nw, theta_N + (b - theta_N)/4] (else
 * theta_N), and m is rounded, capped at the degree where the filter amplifies
 * theta_1 1e12 times more than theta_Nw (the dynamic range the FP64
 * orthonormalisation resolves) and clamped to [m_min, m_max].  Otherwise the
 * Lanczos bound (chebfilter_lanczos_bounds with v0, lanczos_k) is used, with
 * a = theta_N and the last degree, and *fallback = 1.  Synchronises. */
cf_status chebfilter_bounds_predict(cf_ctx *ctx, cf_mlp *mlp, const double *history,
                                    const double *v0, int32_t lanczos_k, int32_t m_min,
                                    int32_t m_max, double *a, double *b, int32_t *m,
                                    int32_t *fallback);

/* Degree rule of the filter (Sec. V: the degree is chosen from the damped
 * interval and the wanted part of the spectrum): the smallest m with
 * T_m(|t(theta_w)|) >= rho, t(x) = (2x - a - b)/(b - a), capped where the
 * amplification of theta_1 over theta_w reaches 1e12 (the FP64 range of the
 * orthonormalisation), clamped to [m_min, m_max].  Host arithmetic only.
 * CF_EINVAL for b <= a, rho <= 1 or a bad range. */
cf_status chebfilter_degree_rule(double theta_1, double theta_w, double a, double b, double rho,
                                 int32_t m_min, int32_t m_max, int32_t *m);

/* The 8 raw features of one self-consistent step (host arrays): theta_1,
 * theta_wanted, theta_N, b used, m used, largest and median residual norm of
 * the wanted pairs, largest change of the wanted Ritz values from theta_prev.
 * Host arithmetic only. */
cf_status chebfilter_step_summary(const double *theta, const double *theta_prev, int32_t N,
                                  int32_t wanted, double b_used, int32_t m_used,
                                  const double *res, double *out);

/* One training sample for the bounds network on the context's current
 * operator: input[8 x steps] = chebfilter_bounds_features(history), target =
 * ((a* - theta_N)/w, (b* - theta_N)/w, m*) with a* = theta[N-1] (host Ritz
 * values of the current subspace), b* the upper bound of a k-step Lanczos run
 * from the device vector v0, m* = chebfilter_degree_rule(theta[0],
 * theta[wanted-1], a*, b*, 100, m_min, m_max), theta_N and w = b - theta_N of
 * the history's last step.  Synchronises. */
cf_status chebfilter_bounds_label(cf_ctx *ctx, const double *history, int32_t steps,
                                  const double *theta, int32_t N, int32_t wanted,
                                  const double *v0, int32_t k, int32_t m_min, int32_t m_max,
                                  double *input, double *target);

/* chebfilter_mlp_set_normalization with the per-column mean and standard
 * deviation of a corpus (inputs [count][n_in], targets [count][n_out], host,
 * row-major); a constant column gets standard deviation 1. */
cf_status chebfilter_mlp_fit_normalization(cf_mlp *mlp, const double *inputs,
                                           const double *targets, int64_t count);

/* The network's normalisation applied to host rows: which = 0 raw inputs
 * [count][n_in], which = 1 raw targets [count][n_out], into FP32 out (the
 * training data of chebfilter_mlp_loss_grad). */
cf_status chebfilter_mlp_normalize(cf_mlp *mlp, int32_t which, const double *x, int64_t count,
                                   float *out);

/* Raw outputs [count][n_out] of raw inputs [count][n_in] (host), through the
 * normalisation and the network.  Synchronises. */
cf_status chebfilter_mlp_predict(cf_mlp *mlp, const double *x_raw, int64_t count, double *y_raw);

#ifdef __cplusplus
}
#endif

#endif /* CHEBFILTER_H */
