// Dense kernels of the subspace step (Sec. V): tall-skinny Gram matrices and
// block rotations on FP64 MFMA, a small Cholesky factorisation, triangular
// inverse, small products, reductions and the Lanczos helpers.
#include <math.h>

#include <algorithm>

#include "cf_kernels.h"

namespace cf {

// v_mfma_f64_16x16x4f64 lane layout: A[l % 16][l / 16], B[l / 16][l % 16],
// D[4 * r + l / 16][l % 16] for element r of lane l.
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 d4zero() { d4 z = {0.0, 0.0, 0.0, 0.0}; return z; }

// Number of 64 x 64 output tiles of an Na x Nb product and the (ti, tj) of
// tile t (upper: square products, tiles with ti <= tj only).
__host__ __device__ inline int ntiles_of(int Na, int Nb, int upper) {
  const int Ta = (Na + GT - 1) / GT, Tb = (Nb + GT - 1) / GT;
  return upper ? Ta * (Ta + 1) / 2 : Ta * Tb;
}
__device__ inline void tile_of(int t, int Na, int Nb, int upper, int &ti, int &tj) {
  const int Ta = (Na + GT - 1) / GT, Tb = (Nb + GT - 1) / GT;
  if (!upper) { ti = t / Tb; tj = t % Tb; return; }
  int i = 0;
  while (t >= Ta - i) { t -= Ta - i; ++i; }
  ti = i;
  tj = i + t;
}

// ---------------------------------------------------------------------------
// Partial Gram: Gp[c][i][j] = sum over rows r of chunk c of A[r][i] B[r][j]
// (i < Na, j < Nb; Gp[c] is Na x Nb, row-major).
// 1-D grid of nchunks * ntiles workgroups.  Workgroups that share a row chunk
// are mapped to the same XCD (workgroups are dealt round-robin to the 8 XCDs
// by index), so the chunk is fetched from HBM once into that XCD's L2.  The
// tile's 64 columns of both operands pass through LDS in slabs of 32 rows
// (loaded once per workgroup, the next slab prefetched in registers); each
// wave computes a 32 x 32 quarter of the 64 x 64 tile from LDS.  The rows
// are summed in the same order as a row-by-row MFMA walk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gram_partial(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t n, int Na, int Nb, int nchunks, int64_t chunk_rows, int upper,
    double *__restrict__ Gp) {
  constexpr int KS = 32, LDS = GT + 4;   // row slab, LDS row stride (doubles)
  __shared__ double as[KS * LDS];
  __shared__ double bs[KS * LDS];
  const int ntl = ntiles_of(Na, Nb, upper);   // upper != 0: only tiles with ti <= tj
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int chunk = (slot / ntl) * 8 + xcd;
  const int t = slot % ntl;
  if (chunk >= nchunks) return;
  int ti, tj;
  tile_of(t, Na, Nb, upper, ti, tj);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int ci0 = ti * GT, cj0 = tj * GT;
  const int wi = 32 * (w & 1), wj = 32 * (w >> 1);
  const int64_t r0 = (int64_t)chunk * chunk_rows;
  const int64_t r1 = min(n, r0 + chunk_rows);
  d4 acc[2][2];
  acc[0][0] = acc[0][1] = acc[1][0] = acc[1][1] = d4zero();
  const bool busy = ci0 + wi < Na && cj0 + wj < Nb;
  // 16 x 16 blocks worth computing: inside Na x Nb, and (upper mode) not
  // entirely below the diagonal of a diagonal tile, whose entries the
  // reduction never reads; a skipped block writes zeros that nothing reads
  const bool ra[2] = {ci0 + wi < Na, ci0 + wi + 16 < Na};
  const bool rb[2] = {cj0 + wj < Nb, cj0 + wj + 16 < Nb};
  bool need[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
      need[ib][jb] = ra[ib] && rb[jb] && !(upper && ti == tj && wi + 16 * ib >= wj + 16 * jb + 16);
  // cooperative slab load: column lc of the tile, rows lr + 4p
  const int lc = tid & 63, lr = tid >> 6;
  const bool cva = ci0 + lc < Na, cvb = cj0 + lc < Nb;
  double pa[KS / 4], pb[KS / 4];
  auto load = [&](int64_t rs) {
#pragma unroll
    for (int p = 0; p < KS / 4; ++p) {
      const int64_t r = rs + lr + 4 * p;
      const bool v = r < r1;
      pa[p] = (v && cva) ? A[r * lda + ci0 + lc] : 0.0;
      pb[p] = (v && cvb) ? B[r * ldb + cj0 + lc] : 0.0;
    }
  };
  load(r0);
  for (int64_t rs = r0; rs < r1; rs += KS) {
#pragma unroll
    for (int p = 0; p < KS / 4; ++p) {
      as[(lr + 4 * p) * LDS + lc] = pa[p];
      bs[(lr + 4 * p) * LDS + lc] = pb[p];
    }
    __syncthreads();
    if (rs + KS < r1) load(rs + KS);
    if (busy) {
#pragma unroll
      for (int ks = 0; ks < KS / 4; ++ks) {
        const int kr = (4 * ks + kq) * LDS;
        const double a0 = as[kr + wi + li], a1 = as[kr + wi + 16 + li];
        const double b0 = bs[kr + wj + li], b1 = bs[kr + wj + 16 + li];
        if (need[0][0]) acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
        if (need[0][1]) acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
        if (need[1][0]) acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
        if (need[1][1]) acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
      }
    }
    __syncthreads();
  }
  double *g = Gp + (int64_t)chunk * Na * Nb;
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int j = cj0 + wj + 16 * jb + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ci0 + wi + 16 * ib + kq + 4 * r;
        if (i < Na && j < Nb) g[(int64_t)i * Nb + j] = acc[ib][jb][r];
      }
    }
}

hipError_t launch_gram_partial(hipStream_t s, const double *A, int64_t lda, const double *B,
                               int64_t ldb, int64_t n, int Na, int Nb, int nchunks,
                               int64_t chunk_rows, double *Gp, int mode) {
  if (Na <= 0 || Nb <= 0) return hipSuccess;
  const int upper = mode == GRAM_UPPER;
  if (upper && Na != Nb) return hipErrorInvalidValue;
  const int ntl = ntiles_of(Na, Nb, upper);
  const int nch8 = (nchunks + 7) / 8 * 8;
  hipLaunchKernelGGL(k_gram_partial, dim3(nch8 * ntl), dim3(256), 0, s, A, lda, B, ldb, n, Na, Nb,
                     nchunks, chunk_rows, upper, Gp);
  return hipGetLastError();
}

// G[i][j] (ld ldg) = sum of the chunk partials.  GRAM_FULL: Na x Nb as is;
// GRAM_UPPER / GRAM_SYM (Na = Nb): the upper sums, or the average of the two
// triangles, written to both triangles.
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ Gp, int nchunks,
                                                     int Na, int Nb, double *__restrict__ G,
                                                     int64_t ldg, int mode) {
  const int64_t NN = (int64_t)Na * Nb;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < NN; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / Nb), j = (int)(e % Nb);
    if (mode == GRAM_FULL) {
      double sij = 0.0;
      for (int c = 0; c < nchunks; ++c) sij += Gp[c * NN + (int64_t)i * Nb + j];
      G[(int64_t)i * ldg + j] = sij;
      continue;
    }
    if (j < i) continue;
    double sij = 0.0, sji = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      sij += Gp[c * NN + (int64_t)i * Nb + j];
      if (mode == GRAM_SYM) sji += Gp[c * NN + (int64_t)j * Nb + i];
    }
    const double v = (mode == GRAM_UPPER) ? sij : 0.5 * (sij + sji);
    G[(int64_t)i * ldg + j] = v;
    G[(int64_t)j * ldg + i] = v;
  }
}

hipError_t launch_gram_reduce(hipStream_t s, const double *Gp, int nchunks, int Na, int Nb,
                              double *G, int64_t ldg, int mode) {
  if (Na <= 0 || Nb <= 0) return hipSuccess;
  if (mode != GRAM_FULL && Na != Nb) return hipErrorInvalidValue;
  int64_t blocks = ((int64_t)Na * Nb + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)blocks), dim3(256), 0, s, Gp, nchunks, Na, Nb,
                     G, ldg, mode);
  return hipGetLastError();
}

// Upper triangle of a row-major N x N matrix mirrored onto its lower triangle.
__global__ __launch_bounds__(256) void k_mirror_upper(double *__restrict__ G, int N) {
  const int64_t NN = (int64_t)N * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < NN; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / N), j = (int)(e % N);
    if (j < i) G[e] = G[(int64_t)j * N + i];
  }
}

hipError_t launch_mirror_upper(hipStream_t s, double *G, int N) {
  if (N <= 0) return hipSuccess;
  int64_t blocks = ((int64_t)N * N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_mirror_upper, dim3((unsigned)blocks), dim3(256), 0, s, G, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lower Cholesky of a small SPD matrix (row-major, ld N), one workgroup,
// right-looking in panels of CB = 32 columns:
//   1. the diagonal block is factored in LDS,
//   2. the rows below it are solved against it (one thread per row),
//   3. the trailing lower triangle is updated with the panel (dot products of
//      length CB, one thread per element).
// Optional symmetric scaling S A S with S = diag(A)^-1/2 and a diagonal shift
// are applied first.  flag[0] = index+1 of the first non-positive pivot.
// ---------------------------------------------------------------------------
// The scaling step of k_cholesky alone (for a library factorisation after it):
// sv = diag(A)^-1/2, A <- S A S + shift I; flag[0] = index+1 of a
// non-positive or non-finite diagonal entry (A is then left as it was).
__global__ __launch_bounds__(1024) void k_chol_scale(double *A, int N, double shift, double *sv,
                                                     int *flag) {
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int i = tid; i < N; i += 1024) {
    const double d = A[(int64_t)i * N + i];
    double s = 1.0;
    if (d > 0.0 && isfinite(d)) s = 1.0 / sqrt(d);
    else atomicExch(&bad, i + 1);   // LDS flag only
    sv[i] = s;
  }
  __syncthreads();
  if (bad) { if (tid == 0) flag[0] = bad; return; }
  const int64_t NN = (int64_t)N * N;
  for (int64_t e = tid; e < NN; e += 1024) {
    const int i = (int)(e / N), j = (int)(e % N);
    double v = A[e] * sv[i] * sv[j];
    if (i == j) v += shift;
    A[e] = v;
  }
}

hipError_t launch_chol_scale(hipStream_t s, double *A, int N, double shift, double *sv, int *flag) {
  hipLaunchKernelGGL(k_chol_scale, dim3(1), dim3(1024), 0, s, A, N, shift, sv, flag);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_cholesky(double *A, int N, int scale, double shift,
                                                   double *sv, int *flag) {
  constexpr int CB = 32;
  __shared__ double dblk[CB * (CB + 1)];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int i = tid; i < N; i += 1024) {
    double s = 1.0;
    if (scale) {
      const double d = A[(int64_t)i * N + i];
      if (d > 0.0 && isfinite(d)) s = 1.0 / sqrt(d);
      else atomicExch(&bad, i + 1);   // LDS flag only
    }
    sv[i] = s;
  }
  __syncthreads();
  if (bad) { if (tid == 0) flag[0] = bad; return; }
  const int64_t NN = (int64_t)N * N;
  for (int64_t e = tid; e < NN; e += 1024) {
    const int i = (int)(e / N), j = (int)(e % N);
    double v = A[e] * sv[i] * sv[j];
    if (i == j) v += shift;
    A[e] = v;
  }
  __syncthreads();
  for (int k0 = 0; k0 < N; k0 += CB) {
    const int nb = min(CB, N - k0);
    // 1. diagonal block
    for (int e = tid; e < nb * nb; e += 1024) {
      const int i = e / nb, j = e % nb;
      dblk[i * (CB + 1) + j] = A[(int64_t)(k0 + i) * N + k0 + j];
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
      if (tid == 0) {
        const double d = dblk[k * (CB + 1) + k];
        if (!(d > 0.0) || !isfinite(d)) bad = k0 + k + 1;
        else dblk[k * (CB + 1) + k] = sqrt(d);
      }
      __syncthreads();
      if (bad) { if (tid == 0) flag[0] = bad; return; }
      const double p = dblk[k * (CB + 1) + k];
      if (tid > k && tid < nb) dblk[tid * (CB + 1) + k] /= p;
      __syncthreads();
      for (int e = tid; e < nb * nb; e += 1024) {
        const int i = e / nb, j = e % nb;
        if (j > k && j <= i) dblk[i * (CB + 1) + j] -= dblk[i * (CB + 1) + k] * dblk[j * (CB + 1) + k];
      }
      __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += 1024) {
      const int i = e / nb, j = e % nb;
      if (j <= i) A[(int64_t)(k0 + i) * N + k0 + j] = dblk[i * (CB + 1) + j];
    }
    // 2. panel below: row r solves x L11^T = a in place (one thread per row)
    for (int r = k0 + nb + tid; r < N; r += 1024) {
      double *ar = A + (int64_t)r * N + k0;
      for (int j = 0; j < nb; ++j) {
        double v = ar[j];
        for (int t = 0; t < j; ++t) v -= ar[t] * dblk[j * (CB + 1) + t];
        ar[j] = v / dblk[j * (CB + 1) + j];
      }
    }
    __syncthreads();
    // 3. trailing update of the lower triangle
    const int m = N - k0 - nb;
    const int64_t mm = (int64_t)m * m;
    for (int64_t e = tid; e < mm; e += 1024) {
      const int i = k0 + nb + (int)(e / m), j = k0 + nb + (int)(e % m);
      if (j > i) continue;
      const double *li = A + (int64_t)i * N + k0;
      const double *lj = A + (int64_t)j * N + k0;
      double acc = 0.0;
      for (int t = 0; t < nb; ++t) acc += li[t] * lj[t];
      A[(int64_t)i * N + j] -= acc;
    }
    __syncthreads();
  }
  if (tid == 0) flag[0] = 0;
}

hipError_t launch_cholesky(hipStream_t s, double *A, int N, int scale, double shift_rel,
                           double *s_out, int *flag) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, A, N, scale, shift_rel, s_out, flag);
  return hipGetLastError();
}

// W = diag(sv) L^-T: column c of L^-1 (forward substitution) becomes row c of
// W (upper triangular, zeros below the diagonal).  One single-wave workgroup
// per column: the 64 lanes split each inner product and reduce it with
// cross-lane shuffles; lane 0 stores the solved entry in the output row and a
// workgroup barrier makes it visible before the next inner product.
__global__ __launch_bounds__(64) void k_tri_inv_T(const double *__restrict__ L,
                                                  const double *__restrict__ sv, int N,
                                                  double *__restrict__ W) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  double *x = W + (int64_t)c * N;
  for (int i = lane; i < c; i += 64) x[i] = 0.0;
  for (int i = c; i < N; ++i) {
    const double *Li = L + (int64_t)i * N;
    double acc = 0.0;
    for (int k = c + lane; k < i; k += 64) acc += Li[k] * x[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) x[i] = ((i == c ? 1.0 : 0.0) - acc) / Li[i];
    __syncthreads();
  }
  const double s = sv ? sv[c] : 1.0;
  for (int i = c + lane; i < N; i += 64) x[i] *= s;
}

hipError_t launch_tri_inv_T(hipStream_t s, const double *L, const double *sv, int N, double *W) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_inv_T, dim3(N), dim3(64), 0, s, L, sv, N, W);
  return hipGetLastError();
}

// C[M x N] = A[M x K] B[K x N], row-major; one thread per output element.
__global__ __launch_bounds__(256) void k_small_gemm(int M, int K, int N,
                                                    const double *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ B, int64_t ldb,
                                                    double *__restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  double acc = 0.0;
  const double *a = A + (int64_t)i * lda;
  for (int k = 0; k < K; ++k) acc += a[k] * B[(int64_t)k * ldb + j];
  C[(int64_t)i * ldc + j] = acc;
}

hipError_t launch_small_gemm(hipStream_t s, int M, int K, int N, const double *A, int64_t lda,
                             const double *B, int64_t ldb, double *C, int64_t ldc) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tot = (int64_t)M * N;
  hipLaunchKernelGGL(k_small_gemm, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, K, N,
                     A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic dot product: per-block partial sums, then one block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += x[i] * y[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_final(int nblk, const double *__restrict__ part,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// x[0..n) = v (a kernel, so that clearing needs no memset node under capture).
__global__ __launch_bounds__(256) void k_fill(double *__restrict__ x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    x[i] = v;
}

hipError_t launch_fill(hipStream_t s, double *x, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_dot(hipStream_t s, int64_t n, const double *x, const double *y, double *out,
                      double *scratch, int nblk) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblk), dim3(256), 0, s, n, x, y, scratch);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, nblk, scratch, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_check_finite(const double *__restrict__ X, int64_t ldx,
                                                      int64_t n, int N, int *flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < n; i += (int64_t)gridDim.x * 4)
    for (int j = threadIdx.x; j < N; j += 64)
      if (!isfinite(X[i * ldx + j])) bad = 1;
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_check_finite(hipStream_t s, const double *X, int64_t ldx, int64_t n, int N,
                               int *flag) {
  if (n <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(64, 4), 0, s, X, ldx, n, N,
                     flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lanczos helpers.  coef[] holds the device-side scalars of the run:
//   coef[0]            squared M-norm of the start vector
//   coef[1 + 2j]       alpha_j
//   coef[2 + 2j]       beta_j^2
// phase 0: v = w / sqrt(coef[0])                                  (normalise start)
// phase 1: w -= sqrt(coef[2j]) * vprev   (j > 0)                  (three-term part)
// phase 2: w -= coef[1+2j] * v                                    (alpha part)
// phase 3: vnext = w / sqrt(coef[2+2j])                           (normalise)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lanczos_update(int64_t n, int j, int phase, double *w,
                                                        const double *v, const double *vprev,
                                                        const double *coef, double *vnext) {
  double c = 0.0;
  if (phase == 0) c = 1.0 / sqrt(coef[0]);
  else if (phase == 1) c = sqrt(coef[2 * j]);
  else if (phase == 2) c = coef[1 + 2 * j];
  else c = 1.0 / sqrt(coef[2 + 2 * j]);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (phase == 0) vnext[i] = w[i] * c;
    else if (phase == 1) w[i] -= c * vprev[i];
    else if (phase == 2) w[i] -= c * v[i];
    else vnext[i] = w[i] * c;
  }
}

hipError_t launch_lanczos_update(hipStream_t s, int64_t n, int j, double *w, const double *v,
                                 const double *vprev, double *coef, double *vnext,
                                 double * /*scratch*/, int nblk, int phase) {
  hipLaunchKernelGGL(k_lanczos_update, dim3(nblk), dim3(256), 0, s, n, j, phase, w, v, vprev, coef,
                     vnext);
  return hipGetLastError();
}

// Extreme eigenvalues of the k x k Lanczos tridiagonal by Sturm-sequence
// bisection (one thread).  out2[0] = lambda_min, out2[1] = lambda_max + beta_k.
__device__ int sturm_count(const double *alpha, const double *beta2, int k, double x) {
  int cnt = 0;
  double q = alpha[0] - x;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < k; ++i) {
    const double qq = (q == 0.0) ? 1e-300 : q;
    q = alpha[i] - x - beta2[i - 1] / qq;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Run r = blockIdx.x reads its scalars at coef[q * stride + r] and writes out2[2 r], out2[2 r + 1].
__global__ void k_tridiag_bounds(const double *coef, int k, double *out2, int stride) {
  if (threadIdx.x != 0) return;
  coef += blockIdx.x;
  out2 += 2 * blockIdx.x;
  double alpha[64], beta2[64];
  for (int i = 0; i < k; ++i) {
    alpha[i] = coef[(1 + 2 * i) * stride];
    beta2[i] = coef[(2 + 2 * i) * stride];
  }
  // Gershgorin interval
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    double r = 0.0;
    if (i > 0) r += sqrt(beta2[i - 1]);
    if (i < k - 1) r += sqrt(beta2[i]);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  double res[2];
  for (int which = 0; which < 2; ++which) {
    // which 0: smallest (count >= 1), which 1: largest (count >= k)
    const int target = which == 0 ? 1 : k;
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid == a || mid == b) break;
      if (sturm_count(alpha, beta2, k, mid) >= target) b = mid; else a = mid;
    }
    res[which] = 0.5 * (a + b);
  }
  out2[0] = res[0];
  out2[1] = res[1] + sqrt(beta2[k - 1]);
}

hipError_t launch_tridiag_bounds(hipStream_t s, const double *coef, const double * /*unused*/,
                                 int k, double *out2) {
  hipLaunchKernelGGL(k_tridiag_bounds, dim3(1), dim3(64), 0, s, coef, k, out2, 1);
  return hipGetLastError();
}

hipError_t launch_tridiag_bounds_blk(hipStream_t s, const double *coef, int runs, int k,
                                     double *out2) {
  if (runs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tridiag_bounds, dim3(runs), dim3(64), 0, s, coef, k, out2, runs);
  return hipGetLastError();
}

// The Lanczos update phases (as k_lanczos_update) for `runs` independent runs
// held as the columns of n x runs row-major blocks; run r's scalars sit at
// coef[q * runs + r].
__global__ __launch_bounds__(256) void k_lanczos_update_blk(int64_t n, int runs, int j, int phase,
                                                            double *w, const double *v,
                                                            const double *vprev,
                                                            const double *coef, double *vnext) {
  const int64_t total = n * runs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int r = (int)(e % runs);
    if (phase == 0) vnext[e] = w[e] * (1.0 / sqrt(coef[r]));
    else if (phase == 1) w[e] -= sqrt(coef[2 * j * runs + r]) * vprev[e];
    else if (phase == 2) w[e] -= coef[(1 + 2 * j) * runs + r] * v[e];
    else vnext[e] = w[e] * (1.0 / sqrt(coef[(2 + 2 * j) * runs + r]));
  }
}

hipError_t launch_lanczos_update_blk(hipStream_t s, int64_t n, int runs, int j, double *w,
                                     const double *v, const double *vprev, const double *coef,
                                     double *vnext, int phase) {
  if (n <= 0 || runs <= 0) return hipSuccess;
  int64_t blocks = (n * runs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_lanczos_update_blk, dim3((unsigned)blocks), dim3(256), 0, s, n, runs, j,
                     phase, w, v, vprev, coef, vnext);
  return hipGetLastError();
}

// C = A - B (elementwise, n values)
__global__ __launch_bounds__(256) void k_sub(int64_t n, const double *A, const double *B,
                                             double *C) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    C[i] = A[i] - B[i];
}

hipError_t launch_sub(hipStream_t s, int64_t n, const double *A, const double *B, double *C) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_sub, dim3((unsigned)blocks), dim3(256), 0, s, n, A, B, C);
  return hipGetLastError();
}

// Out[i][j] = In[j][i] for an N x N matrix (Out row-major, ld N).
__global__ __launch_bounds__(256) void k_transpose(int N, const double *In, int64_t ldi,
                                                   double *Out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)N * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  Out[(int64_t)i * N + j] = In[(int64_t)j * ldi + i];
}

hipError_t launch_transpose(hipStream_t s, int N, const double *In, int64_t ldi, double *Out) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)(((int64_t)N * N + 255) / 256)), dim3(256), 0, s,
                     N, In, ldi, Out);
  return hipGetLastError();
}

// Y[i][j] = X[i][j] for an n x N block (copy with leading dimensions).
__global__ __launch_bounds__(256) void k_copy(int64_t n, int N, const double *X, int64_t ldx,
                                              double *Y, int64_t ldy) {
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < n; i += (int64_t)gridDim.x * 4)
    for (int j = threadIdx.x; j < N; j += 64) Y[i * ldy + j] = X[i * ldx + j];
}

hipError_t launch_copy(hipStream_t s, int64_t n, int N, const double *X, int64_t ldx, double *Y,
                       int64_t ldy) {
  if (n <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(64, 4), 0, s, n, N, X, ldx, Y, ldy);
  return hipGetLastError();
}


// Predicated copy for the batched projection: as k_copy, but nothing is
// written when any of the status words [0..3], [5], [6] is nonzero.
__global__ __launch_bounds__(256) void k_copy_skip(int64_t n, int N, const double *X, int64_t ldx,
                                                   double *Y, int64_t ldy,
                                                   const int *__restrict__ skip) {
  if (skip[0] | skip[1] | skip[2] | skip[3] | skip[5] | skip[6]) return;
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < n; i += (int64_t)gridDim.x * 4)
    for (int j = threadIdx.x; j < N; j += 64) Y[i * ldy + j] = X[i * ldx + j];
}

hipError_t launch_copy_skip(hipStream_t s, int64_t n, int N, const double *X, int64_t ldx,
                            double *Y, int64_t ldy, const int *skip) {
  if (n <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_copy_skip, dim3((unsigned)blocks), dim3(64, 4), 0, s, n, N, X, ldx, Y, ldy,
                     skip);
  return hipGetLastError();
}

// Guard of a projected pencil (Hh, Mh, N x N) before the batched eigensolve:
// when the orthonormalisation failed (st[0], st[1], st[5] or st[6] set) or an entry of the
// pencil is not finite, both matrices become the identity, so that the
// eigensolver sees a trivial problem; a non-finite pencil of an entry whose
// orthonormalisation succeeded is recorded in st[3].  One workgroup.
__global__ __launch_bounds__(256) void k_rr_guard(double *__restrict__ Hh, double *__restrict__ Mh,
                                                  int N, int *__restrict__ st) {
  __shared__ int nonfinite;
  if (threadIdx.x == 0) nonfinite = 0;
  __syncthreads();
  const int prior = st[0] | st[1] | st[5] | st[6];
  const int NN = N * N;
  int nf = 0;
  for (int e = threadIdx.x; e < NN; e += 256)
    if (!isfinite(Hh[e]) || !isfinite(Mh[e])) nf = 1;
  if (nf) atomicOr(&nonfinite, 1);   // LDS flag only
  __syncthreads();
  if (!prior && !nonfinite) return;
  for (int e = threadIdx.x; e < NN; e += 256) {
    const double v = (e / N == e % N) ? 1.0 : 0.0;
    Hh[e] = v;
    Mh[e] = v;
  }
  if (threadIdx.x == 0 && !prior) st[3] = 1;
}

hipError_t launch_rr_guard(hipStream_t s, double *Hh, double *Mh, int N, int *st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rr_guard, dim3(1), dim3(256), 0, s, Hh, Mh, N, st);
  return hipGetLastError();
}

// st[8 e + 2] = info[slot[e]] for every entry e with slot[e] >= 0.
__global__ __launch_bounds__(256) void k_rr_info(const int *__restrict__ info,
                                                 const int *__restrict__ slot, int count,
                                                 int *__restrict__ st) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const int k = slot[e];
  if (k >= 0) st[8 * e + 2] = info[k];
}

hipError_t launch_rr_info(hipStream_t s, const int *info, const int *slot, int count, int *st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rr_info, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, info, slot,
                     count, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ritz residuals: R[:, j] -= theta[j] MZ[:, j], then per-column sums
// out[j] = sum_i A[i][j] B[i][j] (row chunks of partial sums, then a fixed-order
// sum of the chunks: deterministic).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sub_colscale(int64_t n, int N, double *__restrict__ R,
                                                      int64_t ldr, const double *__restrict__ MZ,
                                                      int64_t ldm, const double *__restrict__ theta) {
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < n; i += (int64_t)gridDim.x * 4)
    for (int j = threadIdx.x; j < N; j += 64) R[i * ldr + j] -= theta[j] * MZ[i * ldm + j];
}

__global__ __launch_bounds__(256) void k_coldot_partial(int64_t n, int N, int64_t chunk,
                                                        const double *__restrict__ A, int64_t lda,
                                                        const double *__restrict__ B, int64_t ldb,
                                                        double *__restrict__ part) {
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= N) return;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  double acc = 0.0;
  for (int64_t i = r0; i < r1; ++i) acc += A[i * lda + j] * B[i * ldb + j];
  part[(int64_t)blockIdx.x * N + j] = acc;
}

__global__ __launch_bounds__(256) void k_coldot_final(int nchunks, int N, const double *__restrict__ part,
                                                      double *__restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += part[(int64_t)c * N + j];
  out[j] = acc;
}

hipError_t launch_sub_colscale(hipStream_t s, int64_t n, int N, double *R, int64_t ldr,
                               const double *MZ, int64_t ldm, const double *theta) {
  if (n <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_sub_colscale, dim3((unsigned)blocks), dim3(64, 4), 0, s, n, N, R, ldr, MZ, ldm,
                     theta);
  return hipGetLastError();
}

hipError_t launch_coldot(hipStream_t s, int64_t n, int N, const double *A, int64_t lda,
                         const double *B, int64_t ldb, double *part, int nchunks, double *out) {
  if (n <= 0 || N <= 0) return hipSuccess;
  const int64_t chunk = (n + nchunks - 1) / nchunks;
  hipLaunchKernelGGL(k_coldot_partial, dim3(nchunks, (N + 255) / 256), dim3(256), 0, s, n, N, chunk, A,
                     lda, B, ldb, part);
  hipLaunchKernelGGL(k_coldot_final, dim3((N + 255) / 256), dim3(256), 0, s, nchunks, N, part, out);
  return hipGetLastError();
}

}  // namespace cf
