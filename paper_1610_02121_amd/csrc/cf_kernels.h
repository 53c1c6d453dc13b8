// Device kernels of the Chebyshev-filter library (gfx950).  Host launch
// wrappers are declared here; every wrapper enqueues on the given stream and
// returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cf {

constexpr int NPAD = 128;     // local nodes per cell padded to a multiple of 16 (npc <= 128)
constexpr int CELL_NT = 16;   // column tile of the cell-product kernel
constexpr int GT = 64;        // output tile of the Gram / rotation kernels

// Flags of a (cell, local node) pair for the cell-product kernel.
enum : uint8_t { CELL_FIRST = 1, CELL_FINISH = 2 };

// Optional finishing step of the cell-product kernel (see k_cell_gemm).
struct CellFinish {
  const double *dinv = nullptr;
  double c1 = 0.0, c2 = 0.0, c3 = 0.0;
  const double *Yp = nullptr;
  int64_t ldyp = 0;
  double *Out = nullptr;            // null: no finishing step
  int64_t ldo = 0;
};

// Arguments of the recurrence epilogue (see k_epilogue in cf_ops.hip).
struct EpiArgs {
  int64_t n_h = 0, n_e = 0;
  int N = 0;
  const int32_t *rows = nullptr;    // classical rows to process (null = all n_h)
  int64_t nrows = 0;
  const double *R = nullptr;        // classical rows [n_h][ldr]
  int64_t ldr = 0;
  const double *dR = nullptr;       // per-row scale of R (null = 1)
  const int32_t *qptr = nullptr;    // per classical DOF: range of its enriched-cell
  const int32_t *qidx = nullptr;    //   buffer rows (null = no coupling term)
  const double *Q = nullptr;        // enriched-cell buffer [rows][ldq]
  int64_t ldq = 0;
  const double *dC = nullptr;       // per-row scale of the coupling sum (null = 1)
  const double *Ee = nullptr;       // enrichment rows of the result [n_e][lde]
  int64_t lde = 0;
  double c1 = 1.0;
  const double *Yk = nullptr;
  int64_t ldyk = 0;
  double c2 = 0.0;
  const double *Yp = nullptr;
  int64_t ldyp = 0;
  double c3 = 0.0;
  double *Out = nullptr;
  int64_t ldo = 0;
  int qmax = 0;                     // most buffer rows of one DOF (qptr ranges)
};

// ---- elemental operator kernels (cf_ops.hip)
// Classical elemental products for the cells of one colour:
//   Y[dof(e,a), :] (=|+=) sum_b H_e[a,b] X[dof(e,b), :]
// flag[e*NPAD+a] & CELL_FIRST selects "=" (first touch of that DOF), else "+=";
// CELL_FINISH marks the last touch of a DOF outside the enriched region, which
// takes the recurrence step of f when f.Out is set (see k_cell_gemm).
hipError_t launch_cell_gemm(hipStream_t s, const double *Hp, const int32_t *dofp,
                            const uint8_t *flagp, const int32_t *cells, int ncells,
                            const double *X, int64_t ldx, double *Y, int64_t ldy, int N,
                            const CellFinish &f);

// Coupling partials of the enriched cells (transposed per-cell blocks HT, MT at
// offsets toff with row length tld):
//   P[k0+k, :] = cH sum_a H^ec_e[k,a] X[dof(e,a), :] + cM sum_a M^ec_e[k,a] rs[dof] R[dof(e,a), :]
// Single columns take one workgroup per cell of `cells`; blocks take one per
// item of `items` (position in `cells` * 32 + row-block group, -1 = padding).
hipError_t launch_enr_part(hipStream_t s, const double *HT, const double *MT, const int64_t *toff,
                           const int32_t *tld, const int64_t *eptr, const int32_t *dofp,
                           const int32_t *cells, int ncells, const int32_t *items, int nitems,
                           const double *X, int64_t ldx, double cH, const double *R, int64_t ldr,
                           const double *rs, double cM, double *P, int64_t ldp, int N);

// Transposed coupling products of the enriched cells into the cell-local buffer:
//   Q[128 e' + a, :] = sum_k (cU H^ec_e[k,a] U[idx_k, :] + cV M^ec_e[k,a] V[idx_k, :])
// e' is the cell's position in `cells`; workgroup i takes position order[i]
// (order: a permutation of the positions, or null for the list order).
hipError_t launch_enr_q(hipStream_t s, const double *Hec, const double *Mec, const int64_t *eptr,
                        const int32_t *eidx, const int32_t *cells, const int32_t *order,
                        int ncells, int kmax, const double *U, int64_t ldu, double cU,
                        const double *V, int64_t ldv, double cV, double *Q, int64_t ldq, int N);

// Enrichment rows: out[al,:] = s_p * sum_{k in list(al)} P[k,:] + s_r * R0[al,:]
//                              + sum_be Dn[al,be] * Zd[be,:]     (terms with null pointers skipped)
hipError_t launch_enr_reduce(hipStream_t s, int n_e, const int64_t *aptr, const int32_t *alist,
                             const double *P, int64_t ldp, double s_p, const double *R0,
                             int64_t ldr0, double s_r, const double *Dn, const double *Zd,
                             int64_t ldzd, double *out, int64_t ldo, int N);

// Recurrence epilogue with the node-major coupling (see EpiArgs).
hipError_t launch_epilogue(hipStream_t s, const EpiArgs &g);

// Setup: node-major coupling values of the enriched cells of one colour.
hipError_t launch_csr_fill(hipStream_t s, const double *Hec, const double *Mec,
                           const int64_t *eptr, const int32_t *smap, const int32_t *cells,
                           int ncells, double *hv, double *mv);
// Setup: dense D^-1/2-scaled coupling rows of the enriched region.
hipError_t launch_csr_dense(hipStream_t s, int64_t nreg, const int32_t *regrow,
                            const int32_t *rowptr, const int32_t *ci, const double *hv,
                            const double *mv, const double *dinv, double *BM, double *BH,
                            int64_t ldb);

// ---- reduced-precision operator kernels (cf_lowp.hip): FP32 vectors, FP32
// or BF16 cell matrices, FP32 coupling blocks; enrichment-row sums in FP64.
constexpr int MX_SLOTS = 64;  // words per iterate for the gathered max |Z_k|

// Step scaling of the reduced recurrence: the iterates are kept as
// Z_k = Y_k 2^-s_k, so a step multiplies (c1, c2) by mult[0] = 2^(s_k - s_k+1)
// and c3 by mult[1] = 2^(s_k-1 - s_k+1) (exact: powers of two), and the largest
// |Z_k+1| is gathered into mx[0..MX_SLOTS) (float bits, atomic max per block
// into the block's slot) to choose s_k+2.
struct CellFinishF {
  const double *dinv = nullptr;
  float c1 = 0.f, c2 = 0.f, c3 = 0.f;
  const float *Yp = nullptr;
  int64_t ldyp = 0;
  float *Out = nullptr;             // null: no finishing step
  int64_t ldo = 0;
  const float *mult = nullptr;      // null: no scaling
  unsigned *mx = nullptr;           // null: no max gathering
};

// Recurrence epilogue of the reduced-precision step:
//   Out[i] = c1 * dinv[i] (R[i] + sum_p Q[qidx[p]]) + c2 Yk[i] + c3 Yp[i]  (listed classical rows)
//   Out[i] = c1 * Ee[i - n_h] + c2 Yk[i] + c3 Yp[i]                        (enrichment rows)
struct EpiArgsF {
  int64_t n_h = 0, n_e = 0;
  int N = 0;
  const int32_t *rows = nullptr;
  int64_t nrows = 0;
  const double *dinv = nullptr;
  const float *R = nullptr;
  int64_t ldr = 0;
  const int32_t *qptr = nullptr;
  const int32_t *qidx = nullptr;
  const float *Q = nullptr;
  int64_t ldq = 0;
  const double *Ee = nullptr;
  int64_t lde = 0;
  float c1 = 1.f;
  const float *Yk = nullptr;
  int64_t ldyk = 0;
  float c2 = 0.f;
  const float *Yp = nullptr;
  int64_t ldyp = 0;
  float c3 = 0.f;
  float *Out = nullptr;
  int64_t ldo = 0;
  const float *mult = nullptr;      // as in CellFinishF
  unsigned *mx = nullptr;
};

// As launch_cell_gemm; Hv is [E][NPAD][NPAD] float (bf16 = false) or __bf16 (bf16 = true);
// nsb (1 or 2): 16-column MFMA blocks per column tile (same results, different speed).
hipError_t launch_cell_gemm_lp(hipStream_t s, bool bf16, int nsb, const void *Hv,
                               const int32_t *dofp, const uint8_t *flagp, const int32_t *cells,
                               int ncells, const float *X, int64_t ldx, float *Y, int64_t ldy,
                               int N, const CellFinishF &f);
// As launch_enr_part with FP32 blocks and vectors (rs stays FP64).
// Default map from the row-block count of an enriched cell (1, 2, 3, >= 4
// blocks of 16 functions, 2 bits each) to the FP32 coupling partials' split
// of the workgroup's 8 waves: code 0 -> 1 row block x 8 k parts, 1 -> 2 x 4,
// 2 -> 4 x 2.
constexpr int CPL_BMAP_DEFAULT = 0 | (1 << 2) | (2 << 4) | (2 << 6);
hipError_t launch_enr_part_f32(hipStream_t s, const float *HT, const float *MT,
                               const int64_t *toff, const int32_t *tld, const int64_t *eptr,
                               const int32_t *dofp, const int32_t *cells, int ncells,
                               const float *X, int64_t ldx, float cH, const float *R,
                               int64_t ldr, const double *rs, float cM, float *P, int64_t ldp,
                               int N, int bmap);
// As launch_enr_q with FP32 blocks; U rows FP32, V rows FP64.
hipError_t launch_enr_q_f32(hipStream_t s, const float *Hec, const float *Mec,
                            const int64_t *eptr, const int32_t *eidx, const int32_t *cells,
                            const int32_t *order, int ncells, int kmax, const float *U,
                            int64_t ldu, float cU, const double *V, int64_t ldv, float cV,
                            float *Q, int64_t ldq, int N);
// out[al,:] (FP64) = sum_{k in list(al)} P[k,:] + sum_be Dn[al,be] Zd[be,:]   (P, Zd FP32)
hipError_t launch_enr_reduce_f32(hipStream_t s, int n_e, const int64_t *aptr,
                                 const int32_t *alist, const float *P, int64_t ldp,
                                 const double *Dn, const float *Zd, int64_t ldzd, double *out,
                                 int64_t ldo, int N);
hipError_t launch_epilogue_f32(hipStream_t s, const EpiArgsF &g);
// Conversions: flat arrays and row blocks ([rows][ld], N columns).
hipError_t launch_to_f32(hipStream_t s, int64_t n, const double *x, float *y);
hipError_t launch_to_bf16(hipStream_t s, int64_t n, const double *x, void *y);
hipError_t launch_block_d2f(hipStream_t s, int64_t rows, int N, const double *X, int64_t ldx,
                            float *Y, int64_t ldy);
hipError_t launch_block_f2d(hipStream_t s, int64_t rows, int N, const float *X, int64_t ldx,
                            double *Y, int64_t ldy);
// Scaled recurrence bookkeeping (cf_lowp.hip): reset the max slots mx[0..nslots),
// convert the input block to FP32 while gathering max|X| into mx[0..MX_SLOTS),
// choose the scale of step k (max slots of iterate j at mx[j * MX_SLOTS]), and
// widen Z_m 2^s[m] to FP64.
hipError_t launch_lp_reset(hipStream_t s, unsigned *mx, int nslots);
hipError_t launch_lp_input(hipStream_t s, int64_t rows, int N, const double *X, int64_t ldx,
                           float *Z, int64_t ldz, unsigned *mx0);
hipError_t launch_lp_scale(hipStream_t s, int k, const unsigned *mx, int32_t *sexp, float *mult);
hipError_t launch_lp_output(hipStream_t s, int64_t rows, int N, const float *Z, int64_t ldz,
                            const int32_t *sexp_m, double *Y, int64_t ldy);

// ---- batched reduced-precision recurrence (cf_batch.hip)
// One entry of a batch: the device operator of its problem (shared by the
// entries of one problem), its own FP32 workspace (ld = mc) and the per-call
// block pointers and interval.  The step-k buffers follow the single-problem
// driver: Z_k in F0 (k even) or F1 (k odd).
struct BatchProb {
  const float *Hp32;
  const void *Hp16;
  const int32_t *dofp;
  const uint8_t *flagp;
  const float *HT32, *MT32;
  const int64_t *toff;
  const int32_t *tld;
  const int64_t *eptr;
  const int32_t *ecells;
  const float *Hec32, *Mec32;
  const int32_t *eidx;
  const int64_t *aptr;
  const int32_t *alist;
  const double *Hmod, *Sinv, *dinv;
  const int32_t *qptr, *qidx, *regrows;
  int64_t nregrows, n_h, n_e, n;
  float *R32, *P32, *Q32, *F0, *F1;
  double *Wb, *Zb;
  int64_t mc;
  unsigned *lp_mx;
  int32_t *lp_s;
  float *lp_mult;
  const double *X;
  int64_t ldx;
  double *Y;
  int64_t ldy;
  int N;
  double e, cc;   // t(H~) = e H~ - cc I
};
// Work item of a batched launch: entry p and a cell (or enriched-cell position).
struct BatchItem {
  int32_t p, c;
};
// Launchers; boff / aoff / eoff are prefix sums (count + 1 entries) of the
// row blocks (4 rows each), enrichment rows and epilogue blocks per entry.
hipError_t launch_b_lp_begin(hipStream_t s, const BatchProb *bp, int count, int nslots,
                             const int64_t *boff, int64_t nblocks);
hipError_t launch_b_lp_scale(hipStream_t s, const BatchProb *bp, int count, int k);
hipError_t launch_b_cell(hipStream_t s, bool bf16, int nsb, const BatchProb *bp,
                         const BatchItem *items, int nitems, int k);
hipError_t launch_b_enr(hipStream_t s, const BatchProb *bp, int count, const BatchItem *eitems,
                        int neitems, const int64_t *aoff, int64_t nalpha, int maxN, int kmax,
                        int k, int bmap);
// Raise the dynamic-LDS limit of the batched transposed-coupling kernel for
// the largest per-cell enrichment count (call before any launch or capture).
hipError_t prepare_b_enr(int kmax);
hipError_t launch_b_epilogue(hipStream_t s, const BatchProb *bp, int count, const int64_t *eoff,
                             int64_t nblocks, int k);
hipError_t launch_b_lp_output(hipStream_t s, const BatchProb *bp, int count, const int64_t *boff,
                              int64_t nblocks, int m);

// ---- dense kernels (cf_dense.hip)
// Gram modes: GRAM_SYM  full product, result symmetrised (G + G^T)/2
//             GRAM_UPPER upper tiles only (A = B), mirrored
//             GRAM_FULL  full product, no symmetrisation
enum { GRAM_SYM = 0, GRAM_UPPER = 1, GRAM_FULL = 2 };
// Partial Gram matrices: Gp[c][i*Nb+j] = sum_{rows of chunk c} A[r,i] * B[r,j],
// i < Na, j < Nb (GRAM_UPPER needs Na = Nb).
hipError_t launch_gram_partial(hipStream_t s, const double *A, int64_t lda, const double *B,
                               int64_t ldb, int64_t n, int Na, int Nb, int nchunks,
                               int64_t chunk_rows, double *Gp, int mode);
// G[i*ldg+j] = sum_c Gp[c][i][j], combined as the mode says (SYM/UPPER: Na = Nb).
hipError_t launch_gram_reduce(hipStream_t s, const double *Gp, int nchunks, int Na, int Nb,
                              double *G, int64_t ldg, int mode);
// Lower triangle of a row-major N x N matrix <- its upper triangle.
hipError_t launch_mirror_upper(hipStream_t s, double *G, int N);
// In-place lower Cholesky of the N x N row-major A (ld = N) with optional column
// scaling: A <- chol(S (A + shift*I_diag) S), S = diag(A)^-1/2 when scale != 0;
// s_out[i] receives S_ii (1 when not scaling).  flag[0] = index+1 of a failing
// pivot, 0 on success.
// Only the scaling step of launch_cholesky (scale = 1): sv, S A S + shift I,
// flag[0] = index+1 of a bad diagonal entry.
hipError_t launch_chol_scale(hipStream_t s, double *A, int N, double shift, double *sv, int *flag);
hipError_t launch_cholesky(hipStream_t s, double *A, int N, int scale, double shift_rel,
                           double *s_out, int *flag);
// W (row-major N x N) = diag(sv) * L^-T  (upper triangular), L lower from launch_cholesky
// (sv null: the identity).
hipError_t launch_tri_inv_T(hipStream_t s, const double *L, const double *sv, int N, double *W);
// Small GEMM: C = A * B (row-major, one thread per output).
hipError_t launch_small_gemm(hipStream_t s, int M, int K, int N, const double *A, int64_t lda,
                             const double *B, int64_t ldb, double *C, int64_t ldc);
// Sum of squares / dot product into out[0] (single value, deterministic two-pass).
// x[0..n) = v
hipError_t launch_fill(hipStream_t s, double *x, int64_t n, double v);
hipError_t launch_dot(hipStream_t s, int64_t n, const double *x, const double *y, double *out,
                      double *scratch, int nblk);
// Non-finite detector over a block: flag[0] |= 1 if any element is NaN or Inf.
hipError_t launch_check_finite(hipStream_t s, const double *X, int64_t ldx, int64_t n, int N,
                               int *flag);

// ---- Lanczos helpers (cf_dense.hip); coef[] layout documented there.
hipError_t launch_lanczos_update(hipStream_t s, int64_t n, int j, double *w, const double *v,
                                 const double *vprev, double *coef, double *vnext,
                                 double *scratch, int nblk, int phase);
hipError_t launch_tridiag_bounds(hipStream_t s, const double *coef, const double *unused, int k,
                                 double *out2);
// Independent Lanczos runs as the columns of n x runs blocks (scalars of run r
// at coef[q * runs + r], q as in the single-run layout); bounds of run r into
// out2[2 r], out2[2 r + 1].
hipError_t launch_tridiag_bounds_blk(hipStream_t s, const double *coef, int runs, int k,
                                     double *out2);
hipError_t launch_lanczos_update_blk(hipStream_t s, int64_t n, int runs, int j, double *w,
                                     const double *v, const double *vprev, const double *coef,
                                     double *vnext, int phase);

// ---- Ritz residual helpers (cf_dense.hip)
// R[i][j] -= theta[j] MZ[i][j]  (theta on the device)
hipError_t launch_sub_colscale(hipStream_t s, int64_t n, int N, double *R, int64_t ldr,
                               const double *MZ, int64_t ldm, const double *theta);
// out[j] = sum_i A[i][j] B[i][j]  (part: nchunks * N scratch)
hipError_t launch_coldot(hipStream_t s, int64_t n, int N, const double *A, int64_t lda,
                         const double *B, int64_t ldb, double *part, int nchunks, double *out);

// ---- element blocks of the plain cells (cf_assemble.hip)
// Hp[cells[i]] = K + Btab^T diag(wq .* V[i][:]) Btab over nq points (Btab
// [(nq + 3) & ~3][NPAD] zero-padded, K [NPAD][NPAD] symmetric); the result is
// written exactly symmetric.  One workgroup of 256 threads per cell.
hipError_t launch_assemble_cells(hipStream_t s, const double *Btab, const double *wq,
                                 const double *K, const int *cells, int ncells, const double *V,
                                 int64_t ldv, int nq, double *Hp);

// ---- element blocks of the cells with their own adaptive rule (cf_assemble_enr.hip)
constexpr int EA_MAXNP = 8;       // 1D nodes per axis (degree <= 7)
constexpr int EA_MAXNAP = 256;    // enrichment functions of one cell, padded to 16
constexpr int EA_TPW = 16;        // tiles per wave of an enrichment-row work item
constexpr int EA_TAB_MAX = 256;   // doubles of the shared table (nodes, Gauss rule, shells)
__host__ __device__ constexpr int ea_tab_size(int np1, int ng, int nsh, int nterm) {
  return np1 + 2 * ng + nsh + nsh + 1 + 3 * nterm;
}

struct EnrAsm {
  // listed cells ("slots"): cell index, lower corner, leaf boxes box_ptr[s] ..
  // box_ptr[s+1] (lower corners [3], sides), the potential at the boxes'
  // points (ng^3 per box, x fastest, boxes in order)
  int ncl = 0;
  const int32_t *cell = nullptr;
  const double *lo = nullptr;
  const int64_t *bptr = nullptr;
  const double *blo = nullptr;
  const double *bsz = nullptr;
  const double *V = nullptr;
  int ng = 0, np1 = 0;
  double h = 0.0;
  const double *tab = nullptr;      // nodes [np1], gx [ng], gw [ng], shell l [nsh],
                                    // first term [nsh + 1], terms (c, k, zeta) [nterm]
  int nsh = 0, nterm = 0, npa = 0;
  double r0 = 0.0, t = 0.0;
  const double *centers = nullptr;  // [atoms][3]
  // the context's enrichment layout
  const int64_t *eptr = nullptr;
  const int32_t *eidx = nullptr;
  const int32_t *tld = nullptr;
  const int64_t *toff = nullptr;
  // outputs
  double *Hp = nullptr;
  const double *K = nullptr;        // [NPAD][NPAD] kinetic block
  double *Hec = nullptr, *HT = nullptr;
  double *Pee = nullptr;            // per-slot partial H^ee blocks [nap][nap]
  const int64_t *pee_off = nullptr;
  // enrichment-row work items: slot, first tile, tile count, first point and
  // point count within the slot, partial index (-1: the item covers all of
  // the slot's points and writes the outputs itself)
  const int32_t *item_slot = nullptr, *item_t0 = nullptr, *item_nt = nullptr;
  const int32_t *item_q0 = nullptr, *item_qn = nullptr, *item_pi = nullptr;
  // H^cc items of k_ea_nn (slot, first point, point count, partial index)
  const int32_t *nn_slot = nullptr, *nn_q0 = nullptr, *nn_qn = nullptr, *nn_pi = nullptr;
  // partial tiles of the items of split slots, and the finishing lists: per
  // group, the slot, first tile, tile count, first partial and partial count
  double *Ptile = nullptr, *Pnn = nullptr;
  const int32_t *fin_slot = nullptr, *fin_t0 = nullptr, *fin_nt = nullptr, *fin_p0 = nullptr,
                *fin_np = nullptr;
  const int32_t *nnf_slot = nullptr, *nnf_p0 = nullptr, *nnf_np = nullptr;
};
constexpr int EA_QCHUNK = 4096;   // points per assembly item of a split slot

// H^cc_e = K + sum_q w_q V_q N_a N_b for every slot (exactly symmetric): nitems
// items of whole slots or point chunks (partials), then nfin finishing groups.
hipError_t launch_ea_nn(hipStream_t s, const EnrAsm &a, int nitems, int nfin);
// H^ec_e rows (both stored layouts) and the partial H^ee_e blocks of the items'
// tiles; then the nfin finishing groups of the split slots.
hipError_t launch_ea_erow(hipStream_t s, const EnrAsm &a, int nitems, int nfin);
// Hee[al][be] += sum over the pair's cells of the partial entries (both halves written).
hipError_t launch_ea_ee_reduce(hipStream_t s, const EnrAsm &a, int n_e, int npairs,
                               const int32_t *pair_ij, const int64_t *pair_ptr, const int32_t *pc,
                               double *Hee);
// X[i][j] = (i == j0 + j), i < rows, j < N.
hipError_t launch_unit_cols(hipStream_t s, int64_t rows, int N, int64_t ldx, int64_t j0, double *X);

// ---- self-consistent field quantities (cf_scf.hip)
// Cells of the SCF point set ("SCF cells": the plain cells, then the cells
// with an adaptive rule): cell index, enrichment count, lower corner, the
// range of their points in the point arrays, density-matrix offsets.
struct ScfArgs {
  int64_t n_h = 0;
  int np1 = 0, ng = 0, nsh = 0, npa = 0, ntab = 0;
  double h = 0.0, r0 = 0.0, t = 0.0;
  const double *tab = nullptr;       // EnrAsm::tab layout (nodes first)
  const double *centers = nullptr;
  const int32_t *dofp = nullptr;
  const int64_t *eptr = nullptr;
  const int32_t *eidx = nullptr;
  const int32_t *cell = nullptr;
  const int32_t *cna = nullptr;
  const double *lo = nullptr;
  const int64_t *pofs = nullptr, *pcnt = nullptr;
  const int64_t *doff = nullptr;
  const double *xyz = nullptr, *w = nullptr;
  double cc[3] = {0.0, 0.0, 0.0};    // neutralising Gaussian: centre, width, charge
  double cs = 1.0, Q = 0.0;
};
struct ScfMixCoef {
  double c[8];
};
hipError_t launch_scf_dm(hipStream_t s, const ScfArgs &g, int nitems, const int32_t *item_c,
                         const int32_t *item_t0, const int32_t *item_nt, const double *X,
                         int64_t ldx, int N, const double *f2, double *Dbuf);
// rho at the points of the items' cells from their density matrices; items of
// one launch cover distinct cells; add = 0 writes, 1 adds.
constexpr int SCF_RHO_TILES = 8 * 12;             // upper tiles of D_e per density item
// upper 16 x 16 tiles of a K x K block
__host__ __device__ constexpr int ea_max_tiles(int K) { return (K / 16) * (K / 16 + 1) / 2; }
constexpr int SCF_RHO_QCHUNK = 1024;              // points per density item
hipError_t launch_scf_rho(hipStream_t s, const ScfArgs &g, int nitems, const int32_t *item_c,
                          const int32_t *item_t0, const int32_t *item_nt, const int32_t *item_q0,
                          int add, const double *Dbuf, double *rho);
hipError_t launch_scf_lda(hipStream_t s, int64_t P, const double *rho, const double *w, double *vxc,
                          double *partials, int nblocks);
hipError_t launch_scf_rhs(hipStream_t s, const ScfArgs &g, int ncells, const int32_t *cells,
                          const double *rho, double *b);
hipError_t launch_scf_lap(hipStream_t s, const ScfArgs &g, int ncells, const int32_t *cells,
                          const double *A, const double *x, double *y);
hipError_t launch_scf_cg(hipStream_t s, int64_t n, int op, double alpha, double beta,
                         const double *dinv, double *x, double *r, double *z, double *p,
                         const double *q);
hipError_t launch_scf_cgd(hipStream_t s, int64_t n, int op, double *sc, const double *dinv,
                          double *x, double *r, double *z, double *p, const double *q);
hipError_t launch_scf_veff(hipStream_t s, const ScfArgs &g, int ncells, const double *phi,
                           const double *rho, const double *vext, const double *vxc, double *veff,
                           double *partials);
hipError_t launch_scf_wdot(hipStream_t s, int64_t P, const double *w, const double *a,
                           const double *b, double *partials, int nblocks);
hipError_t launch_scf_mix(hipStream_t s, int64_t P, int m, const ScfMixCoef &cf, double beta,
                          const double *rin, const double *F, int64_t ld, double *out);
hipError_t launch_scf_push(hipStream_t s, int64_t P, const double *rin, const double *rout,
                           double *hin, double *hF);

// ---- data-movement helpers (cf_dense.hip)
hipError_t launch_sub(hipStream_t s, int64_t n, const double *A, const double *B, double *C);
hipError_t launch_transpose(hipStream_t s, int N, const double *In, int64_t ldi, double *Out);
// Batched projection helpers: predicated copy (skip: the entry's 8 status words; nothing is
// written when any of [0..3], [5], [6] is nonzero),
// pencil guard (identity on failure, st[3] on a non-finite pencil) and the
// scatter of the batched eigensolver's info into st[8 e + 2].
hipError_t launch_copy_skip(hipStream_t s, int64_t n, int N, const double *X, int64_t ldx,
                            double *Y, int64_t ldy, const int *skip);
hipError_t launch_rr_guard(hipStream_t s, double *Hh, double *Mh, int N, int *st);
hipError_t launch_rr_info(hipStream_t s, const int *info, const int *slot, int count, int *st);
hipError_t launch_copy(hipStream_t s, int64_t n, int N, const double *X, int64_t ldx, double *Y,
                       int64_t ldy);

}  // namespace cf
