// Device kernels of the Chebyshev-filter library (gfx950).  Host launch
// wrappers are declared here; every wrapper enqueues on the given stream and
// returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cf {

constexpr int NPAD = 128;     // local nodes per cell padded to a multiple of 16 (npc <= 128)
constexpr int CT = 32;        // column tile of the cell and enrichment kernels
constexpr int GT = 64;        // output tile of the Gram / rotation kernels

// ---- elemental operator kernels (cf_ops.hip)
// Classical elemental products for the cells of one colour:
//   Y[dof(e,a), :] (=|+=) sum_b H_e[a,b] X[dof(e,b), :]
// first[e*NPAD+a] != 0 selects "=" (first touch of that DOF), else "+=".
hipError_t launch_cell_gemm(hipStream_t s, const double *Hp, const int32_t *dofp,
                            const uint8_t *firstp, const int32_t *cells, int ncells,
                            const double *X, int64_t ldx, double *Y, int64_t ldy, int N);

// Transposed coupling for the enriched cells of one colour:
//   Y[dof(e,a), :] += sign * sum_k B[k0+k, a] * Z[idx[k0+k], :]
hipError_t launch_enr_T(hipStream_t s, const double *Bp, const int64_t *eptr,
                        const int32_t *eidx, const int32_t *dofp, const int32_t *cells,
                        int ncells, int kmax, const double *Z, int64_t ldz, double *Y,
                        int64_t ldy, int N, double sign);

// Coupling partials for all enriched cells:
//   P[k0+k, :] = sum_a B[k0+k, a] * scale(dof) * Zc[dof(e,a), :]   (scale = 1 if dscale null)
hipError_t launch_enr_N(hipStream_t s, const double *Bp, const int64_t *eptr,
                        const int32_t *dofp, const int32_t *cells, int ncells,
                        const double *Zc, int64_t ldz, const double *dscale, double *P,
                        int64_t ldp, int N);

// Enrichment rows: out[al,:] = s_p * sum_{k in list(al)} P[k,:] + s_r * R0[al,:]
//                              + sum_be Dn[al,be] * Zd[be,:]     (terms with null pointers skipped)
hipError_t launch_enr_reduce(hipStream_t s, int n_e, const int64_t *aptr, const int32_t *alist,
                             const double *P, int64_t ldp, double s_p, const double *R0,
                             int64_t ldr0, double s_r, const double *Dn, const double *Zd,
                             int64_t ldzd, double *out, int64_t ldo, int N);

// Chebyshev step epilogue over all n = n_h + n_e rows:
//   v = (i < n_h) ? dinv[i] * R[i,:] : Ze[i-n_h,:]
//   Out[i,:] = c1 * v + c2 * Yk[i,:] + c3 * Yp[i,:]      (Yk / Yp may be null)
// Out may alias Yp (each element is read before it is written by one thread).
hipError_t launch_epilogue(hipStream_t s, int64_t n_h, int64_t n_e, const double *dinv,
                           const double *R, int64_t ldr, const double *Ze, int64_t ldze,
                           double c1, const double *Yk, int64_t ldyk, double c2,
                           const double *Yp, int64_t ldyp, double c3, double *Out,
                           int64_t ldo, int N);

// Out[i,:] = d[i] * X[i,:] for i < rows (diagonal scaling, Out may alias X).
hipError_t launch_diag_scale(hipStream_t s, int64_t rows, const double *d, const double *X,
                             int64_t ldx, double *Out, int64_t ldo, int N);

// ---- dense kernels (cf_dense.hip)
// Partial Gram matrices: Gp[c][i*ldg+j] = sum_{rows of chunk c} A[r,i] * B[r,j]
hipError_t launch_gram_partial(hipStream_t s, const double *A, int64_t lda, const double *B,
                               int64_t ldb, int64_t n, int N, int nchunks, int64_t chunk_rows,
                               double *Gp, int upper_only);
// G[i][j] = sum_c Gp[c][i][j], symmetrised: G = (G + G^T)/2 (or mirrored when upper_only).
hipError_t launch_gram_reduce(hipStream_t s, const double *Gp, int nchunks, int N, double *G,
                              int upper_only);
// Out[r, j] = sum_k In[r, k] * W[k*wsk + j*wsj]     (out of place)
hipError_t launch_rotate(hipStream_t s, const double *In, int64_t ldi, int64_t n, int N,
                         const double *W, int64_t wsk, int64_t wsj, double *Out, int64_t ldo);
// In-place lower Cholesky of the N x N row-major A (ld = N) with optional column
// scaling: A <- chol(S (A + shift*I_diag) S), S = diag(A)^-1/2 when scale != 0;
// s_out[i] receives S_ii (1 when not scaling).  flag[0] = index+1 of a failing
// pivot, 0 on success.
hipError_t launch_cholesky(hipStream_t s, double *A, int N, int scale, double shift_rel,
                           double *s_out, int *flag);
// W (row-major N x N) = diag(sv) * L^-T  (upper triangular), L lower from launch_cholesky.
hipError_t launch_tri_inv_T(hipStream_t s, const double *L, const double *sv, int N, double *W);
// Small GEMM: C = A * B (row-major, one thread per output).
hipError_t launch_small_gemm(hipStream_t s, int M, int K, int N, const double *A, int64_t lda,
                             const double *B, int64_t ldb, double *C, int64_t ldc);
// Sum of squares / dot product into out[0] (single value, deterministic two-pass).
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

// ---- setup and data-movement helpers (cf_dense.hip)
hipError_t launch_scatter_coupling(hipStream_t s, const double *Bp, const int64_t *eptr,
                                   const int32_t *eidx, const int32_t *dofp,
                                   const int32_t *dof2reg, const int32_t *cells, int ncells,
                                   double *Bt, int64_t ldb);
hipError_t launch_scale_rows_sqrt(hipStream_t s, int64_t rows, const int32_t *regdof,
                                  const double *dinv, double *Bt, int64_t ldb, int ncol);
hipError_t launch_sub(hipStream_t s, int64_t n, const double *A, const double *B, double *C);
hipError_t launch_transpose(hipStream_t s, int N, const double *In, int64_t ldi, double *Out);
hipError_t launch_copy(hipStream_t s, int64_t n, int N, const double *X, int64_t ldx, double *Y,
                       int64_t ldy);

}  // namespace cf
